// simple_internal.h -- launch arguments shared by the SIMPLE-stage kernels and
// their host driver.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace eqsim {

constexpr int kThreads = 256;   // threads per block; one cell per thread
constexpr int kXcds = 8;        // blocks go round-robin to the XCDs of the chip

struct BoxK {
    int32_t nx, ny, nz, pad;
    double hx, hy, hz, rho, mu, dt, gy, v_in, alpha_u, alpha_p;
    // uniform values, formed once on the host in the kernels' own operation order:
    // face areas, cell volume, rho V / dt, diffusion conductances mu A / h, rho A,
    // rho g_y V, 1 - alpha_u
    double Ax, Ay, Az, V, aP0, De, Dn, Dt, rAx, rAy, rAz, rgV, oma;
};

// block q of grid g (nb[g] blocks: u, v, w) forms the contiguous cells [q cpb, (q + 1) cpb) of
// it, 256 at a time, and leaves its partial at partials[nb[0] + ... + nb[g-1] + q]; the grids'
// blocks run interleaved (see form_momentum_kernel)
struct MomArgs {
    BoxK bx;
    const double *u, *v, *w, *p, *u0, *v0, *w0;
    double *a[3][7];
    double *b[3], *d[3];
    double *partials;   // per block: sum of squared row residuals
    int32_t nb[3], cpb[3];
};

struct PresArgs {
    BoxK bx;
    const double *du, *dv, *dw, *u, *v, *w;
    double *a[7];
    double *b;
    double *partials;   // per block: sum of b'^2
    int32_t cpb;        // cells per block (contiguous)
};

// the formation kernels' blocks per grid: at most kFormBlocks, each over a contiguous run of
// cells (a multiple of kThreads).  Measured on the 96 x 384 x 96 bed, one cell per thread (the
// cap above any grid here) forms fastest: runs of 4 or 14 cells per thread took 349 and 344 us
// for the momentum rows against 330 us; the final sum of the ~42k block partials takes ~6 us.
constexpr int kFormBlocks = 1 << 22;
inline int form_cells_per_block(long n) {
    const long per = (n + kFormBlocks - 1) / kFormBlocks;
    return (int)((per + kThreads - 1) / kThreads * kThreads);
}
inline int form_blocks(long n) {
    const long cpb = form_cells_per_block(n);
    return (int)((n + cpb - 1) / cpb);
}

// logical blocks over u, v, w, p in that order
struct CorrArgs {
    BoxK bx;
    const double *du, *dv, *dw, *pp;
    double *u, *v, *w, *p;
    int32_t nb[4];
};

inline int blocks_for(long n) { return (int)((n + kThreads - 1) / kThreads); }

hipError_t launch_form_momentum(const MomArgs &a, hipStream_t s);
hipError_t launch_form_pressure(const PresArgs &a, int nblocks, hipStream_t s);
hipError_t launch_correct(const CorrArgs &a, hipStream_t s);
// out[q] = sum of partials[begin[q] .. begin[q+1]) in a fixed order, q < nq
hipError_t launch_sum_ranges(const double *partials, const int32_t *begin_host, int nq, double *out, hipStream_t s);
hipError_t launch_zero(double *p, long n, hipStream_t s);

}  // namespace eqsim
