// eqs_probe.hip -- eqsolve_debug_stream: the streaming rate of a plain pointwise kernel with the
// single-sync step's byte mix per cell (11 or 13 FP64 reads, 5 FP64 writes).
//
// The step's HBM rate is read against two figures: the device's nominal peak and what a kernel
// that does nothing but stream the same words reaches.  This kernel is the second: every input is
// read once and every output written once, coalesced, with no stencil, no halo, no LDS and no
// barrier, so its rate is the practical ceiling for any kernel that moves those words.

#include <hip/hip_runtime.h>

#include "eqsolve.h"

namespace {

constexpr int kThreads = 256;
constexpr int kCells = 1;  // cells per thread, kThreads apart (the fastest of 1, 2, 4 cells and 256-1024 threads)
constexpr int kMaxReads = 13, kWrites = 5;

struct StreamArgs {
    const double *in[kMaxReads];
    double *out[kWrites];
};

template <bool NT>
__device__ __forceinline__ void put(double *p, long i, double v) {
    if (NT)
        __builtin_nontemporal_store(v, (__attribute__((address_space(1))) double *)p + i);
    else
        ((__attribute__((address_space(1))) double *)p)[i] = v;
}

// out_w[i] = w + sum_k (k + 1) in_k[i]: every load feeds a store, so none is dropped
template <int NR, bool NT>
__global__ void __launch_bounds__(kThreads) stream_kernel(StreamArgs a, long n) {
    const long base = (long)blockIdx.x * (kThreads * kCells) + threadIdx.x;
    double v[kCells][NR];
#pragma unroll
    for (int c = 0; c < kCells; ++c) {
        const long i = base + (long)c * kThreads;
        const bool ok = i < n;
#pragma unroll
        for (int k = 0; k < NR; ++k) v[c][k] = ok ? ((const __attribute__((address_space(1))) double *)a.in[k])[i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kCells; ++c) {
        const long i = base + (long)c * kThreads;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) s = fma((double)(k + 1), v[c][k], s);
        if (i < n) {
#pragma unroll
            for (int w = 0; w < kWrites; ++w) put<NT>(a.out[w], i, s + (double)w);
        }
    }
}

}  // namespace

extern "C" int eqsolve_debug_stream(const double *const *in, int32_t nr, double *const *out, int32_t nw, int64_t n,
                                    int32_t nontemporal, void *stream) {
    if (!in || !out || n < 1 || (nr != 11 && nr != 13) || nw != kWrites) return EQS_ERR_ARG;
    StreamArgs a{};
    for (int k = 0; k < nr; ++k) {
        if (!in[k]) return EQS_ERR_ARG;
        a.in[k] = in[k];
    }
    for (int w = 0; w < nw; ++w) {
        if (!out[w]) return EQS_ERR_ARG;
        for (int k = 0; k < nr; ++k)
            if ((const void *)out[w] == (const void *)in[k]) return EQS_ERR_ARG;
        a.out[w] = out[w];
    }
    const long blocks = (n + kThreads * kCells - 1) / (kThreads * kCells);
    if (blocks > 0x7fffffffL) return EQS_ERR_ARG;
    const dim3 grid((unsigned)blocks), block(kThreads);
    hipStream_t s = (hipStream_t)stream;
    const bool nt = nontemporal != 0;
    if (nr == 13 && nt)
        hipLaunchKernelGGL((stream_kernel<13, true>), grid, block, 0, s, a, (long)n);
    else if (nr == 13)
        hipLaunchKernelGGL((stream_kernel<13, false>), grid, block, 0, s, a, (long)n);
    else if (nt)
        hipLaunchKernelGGL((stream_kernel<11, true>), grid, block, 0, s, a, (long)n);
    else
        hipLaunchKernelGGL((stream_kernel<11, false>), grid, block, 0, s, a, (long)n);
    return hipGetLastError() == hipSuccess ? EQS_OK : EQS_ERR_HIP;
}
