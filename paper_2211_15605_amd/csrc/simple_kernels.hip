// simple_kernels.hip -- the pointwise stages of a SIMPLE iteration on the
// gas-only bed box (gfx950): momentum formation, pressure-correction
// formation, correction.
//
// Each stage is one launch over every grid it touches (u, v, w; p'; u, v, w,
// p), one cell per thread, and writes what the solver reads directly: the
// momentum launch forms mass fluxes, upwind and diffusion coefficients,
// boundary conductances, the transient term, pressure force, gravity and
// under-relaxation of a row in registers and stores its 7 diagonals, b and d
// (no face arrays in HBM).  It also takes the row's residual at the incoming
// iterate, since every value that needs is already loaded.  The arithmetic of
// each formula is written in one fixed order with no FMA contraction, so a
// result does not depend on the compiler's choices.
//
// Blocks are handed to the XCDs round-robin; logical block lb = (b % 8) *
// per + b / 8 gives each XCD one contiguous run of cells, so the rows above
// and below a block (its stencil neighbours) sit in the same XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "simple_internal.h"

#pragma clang fp contract(off)

namespace eqsim {
namespace {

__device__ __forceinline__ int logical_block(int total) {
    const int per = (total + kXcds - 1) / kXcds;
    return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

__device__ __forceinline__ double pos(double x) { return fmax(x, 0.0); }

// Store that marks its line for early eviction: the rows a stage writes are read by the next
// launch, not by this one, and left in L2 they evict the fields whose neighbouring planes the
// stage is about to read again.
__device__ __forceinline__ void st_nt(double *p, int i, double v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) double *)p + i);
}

// sum of v over the block, valid in thread 0
__device__ double block_sum(double v) {
    __shared__ double part[kThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) s += part[q];
    return s;
}

// the box's uniform values (formed on the host)
struct Geo {
    double Ax, Ay, Az, aP0, De, Dn, Dt, rAx, rAy, rAz, rgV, oma;
    __device__ explicit Geo(const BoxK &b)
        : Ax(b.Ax), Ay(b.Ay), Az(b.Az), aP0(b.aP0), De(b.De), Dn(b.Dn), Dt(b.Dt), rAx(b.rAx), rAy(b.rAy),
          rAz(b.rAz), rgV(b.rgV), oma(b.oma) {}
};

// a row: coefficients P,E,W,N,S,T,B, right-hand side, d
struct Row {
    double a[7];
    double b, d;
};

__device__ __forceinline__ void fixed_row(const Geo &g, double value, Row &r) {
    r.a[0] = g.aP0;
    for (int q = 1; q < 7; ++q) r.a[q] = 0.0;
    r.b = g.aP0 * value;
    r.d = 0.0;
}

// transient coefficient, under-relaxation with the incoming iterate xs, d
__device__ __forceinline__ void finish(const BoxK &bx, const Geo &g, double aE, double aW, double aN, double aS,
                                       double aT, double aB, double bnd, double src, double xs, double area,
                                       Row &r) {
    const double aP = aE + aW + aN + aS + aT + aB + bnd + g.aP0;
    const double aPr = aP / bx.alpha_u;
    r.a[0] = aPr;
    r.a[1] = aE;
    r.a[2] = aW;
    r.a[3] = aN;
    r.a[4] = aS;
    r.a[5] = aT;
    r.a[6] = aB;
    r.b = src + g.oma * aPr * xs;
    r.d = area * (1.0 / aPr);
}

// grid index helpers: u (nx+1, ny, nz), v (nx, ny+1, nz), w (nx, ny, nz+1), p (nx, ny, nz)
struct Idx {
    int nx, ny, nz;
    __device__ int u(int i, int j, int k) const { return i + (nx + 1) * (j + ny * k); }
    __device__ int v(int i, int j, int k) const { return i + nx * (j + (ny + 1) * k); }
    __device__ int w(int i, int j, int k) const { return i + nx * (j + ny * k); }
    __device__ int p(int i, int j, int k) const { return i + nx * (j + ny * k); }
};

// x-momentum row at u-face (i, j, k)
__device__ void form_u(const MomArgs &A, const Geo &g, const Idx &X, int i, int j, int k, Row &r) {
    const BoxK &bx = A.bx;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    if (i == 0 || i == nx) {
        fixed_row(g, 0.0, r);
        return;
    }
    const double *u = A.u, *v = A.v, *w = A.w, *p = A.p;
    const int c = X.u(i, j, k);
    const double Fe = g.rAx * (u[c] + u[c + 1]) / 2;
    const double Fw = g.rAx * (u[c - 1] + u[c]) / 2;
    const double Fn = g.rAy * (v[X.v(i - 1, j + 1, k)] + v[X.v(i, j + 1, k)]) / 2;
    const double Fs = g.rAy * (v[X.v(i - 1, j, k)] + v[X.v(i, j, k)]) / 2;
    const double Ft = g.rAz * (w[X.w(i - 1, j, k + 1)] + w[X.w(i, j, k + 1)]) / 2;
    const double Fb = g.rAz * (w[X.w(i - 1, j, k)] + w[X.w(i, j, k)]) / 2;
    const double De = g.De, Dn = g.Dn, Dt = g.Dt;
    double bnd = 0.0, aS = 0.0, aT = 0.0, aB = 0.0;
    const double aE = De + pos(-Fe);
    const double aW = De + pos(Fw);
    const double aN = j + 1 < ny ? Dn + pos(-Fn) : 0.0;   // outlet: zero gradient
    if (j > 0) aS = Dn + pos(Fs);
    else bnd = bnd + 2 * Dn + pos(Fs);                      // inlet plane: u = 0 at hy/2
    if (k + 1 < nz) aT = Dt + pos(-Ft);
    else bnd = bnd + 2 * Dt + pos(-Ft);                     // wall z = Lz
    if (k > 0) aB = Dt + pos(Fb);
    else bnd = bnd + 2 * Dt + pos(Fb);                      // wall z = 0
    const double src = g.aP0 * A.u0[c] + (p[X.p(i - 1, j, k)] - p[X.p(i, j, k)]) * g.Ax;
    finish(bx, g, aE, aW, aN, aS, aT, aB, bnd, src, u[c], g.Ax, r);
}

// y-momentum row at v-face (i, j, k); j = ny is the outlet face (p = 0 above)
__device__ void form_v(const MomArgs &A, const Geo &g, const Idx &X, int i, int j, int k, Row &r) {
    const BoxK &bx = A.bx;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    if (j == 0) {
        fixed_row(g, bx.v_in, r);
        return;
    }
    const double *u = A.u, *v = A.v, *w = A.w, *p = A.p;
    const int c = X.v(i, j, k);
    const int jl = j - 1, jh = j < ny ? j : ny - 1;
    const double vn = v[j < ny ? c + nx : c];   // (every load in bounds)
    const double Fn = g.rAy * (j < ny ? (v[c] + vn) / 2 : v[c]);
    const double Fs = g.rAy * (v[c - nx] + v[c]) / 2;
    const double Fe = g.rAx * (u[X.u(i + 1, jl, k)] + u[X.u(i + 1, jh, k)]) / 2;
    const double Fw = g.rAx * (u[X.u(i, jl, k)] + u[X.u(i, jh, k)]) / 2;
    const double Ft = g.rAz * (w[X.w(i, jl, k + 1)] + w[X.w(i, jh, k + 1)]) / 2;
    const double Fb = g.rAz * (w[X.w(i, jl, k)] + w[X.w(i, jh, k)]) / 2;
    const double De = g.De, Dn = g.Dn, Dt = g.Dt;
    double bnd = 0.0, aE = 0.0, aW = 0.0, aT = 0.0, aB = 0.0;
    if (i + 1 < nx) aE = De + pos(-Fe);
    else bnd = bnd + 2 * De + pos(-Fe);
    if (i > 0) aW = De + pos(Fw);
    else bnd = bnd + 2 * De + pos(Fw);
    const double aN = j < ny ? Dn + pos(-Fn) : 0.0;
    const double aS = Dn + pos(Fs);
    if (k + 1 < nz) aT = Dt + pos(-Ft);
    else bnd = bnd + 2 * Dt + pos(-Ft);
    if (k > 0) aB = Dt + pos(Fb);
    else bnd = bnd + 2 * Dt + pos(Fb);
    const double p_hi = p[X.p(i, jh, k)];
    const double p_above = j < ny ? p_hi : 0.0;
    const double src = g.aP0 * A.v0[c] + (p[X.p(i, j - 1, k)] - p_above) * g.Ay + g.rgV;
    finish(bx, g, aE, aW, aN, aS, aT, aB, bnd, src, v[c], g.Ay, r);
}

// z-momentum row at w-face (i, j, k)
__device__ void form_w(const MomArgs &A, const Geo &g, const Idx &X, int i, int j, int k, Row &r) {
    const BoxK &bx = A.bx;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    if (k == 0 || k == nz) {
        fixed_row(g, 0.0, r);
        return;
    }
    const double *u = A.u, *v = A.v, *w = A.w, *p = A.p;
    const int c = X.w(i, j, k), P = nx * ny;
    const double Ft = g.rAz * (w[c] + w[c + P]) / 2;
    const double Fb = g.rAz * (w[c - P] + w[c]) / 2;
    const double Fe = g.rAx * (u[X.u(i + 1, j, k - 1)] + u[X.u(i + 1, j, k)]) / 2;
    const double Fw = g.rAx * (u[X.u(i, j, k - 1)] + u[X.u(i, j, k)]) / 2;
    const double Fn = g.rAy * (v[X.v(i, j + 1, k - 1)] + v[X.v(i, j + 1, k)]) / 2;
    const double Fs = g.rAy * (v[X.v(i, j, k - 1)] + v[X.v(i, j, k)]) / 2;
    const double De = g.De, Dn = g.Dn, Dt = g.Dt;
    double bnd = 0.0, aE = 0.0, aW = 0.0, aS = 0.0;
    if (i + 1 < nx) aE = De + pos(-Fe);
    else bnd = bnd + 2 * De + pos(-Fe);
    if (i > 0) aW = De + pos(Fw);
    else bnd = bnd + 2 * De + pos(Fw);
    const double aN = j + 1 < ny ? Dn + pos(-Fn) : 0.0;
    if (j > 0) aS = Dn + pos(Fs);
    else bnd = bnd + 2 * Dn + pos(Fs);
    const double aT = Dt + pos(-Ft);
    const double aB = Dt + pos(Fb);
    const double src = g.aP0 * A.w0[c] + (p[X.p(i, j, k - 1)] - p[X.p(i, j, k)]) * g.Az;
    finish(bx, g, aE, aW, aN, aS, aT, aB, bnd, src, w[c], g.Az, r);
}

// Logical block lb -> (grid, block of that grid).  The three grids' blocks are interleaved:
// round r holds block r of u, of v and of w, which cover nearly the same cells of the box (the
// grids differ by one face along one axis), then the few blocks one grid has beyond the others.
// Each XCD takes a contiguous run of logical blocks, so the u, v and w rows of one region of
// the box are formed by one XCD and every field is read into one L2 (with the three grids in
// separate runs, each field was fetched from memory by three XCDs).
__device__ __forceinline__ void momentum_block(const MomArgs &A, int lb, int &comp, int &local) {
    const int m = min(A.nb[0], min(A.nb[1], A.nb[2]));
    if (lb < 3 * m) {
        comp = lb % 3;
        local = lb / 3;
        return;
    }
    int rem = lb - 3 * m;
    comp = 0;
    while (comp < 2 && rem >= A.nb[comp] - m) rem -= A.nb[comp++] - m;
    local = m + rem;
}

__global__ void __launch_bounds__(kThreads) form_momentum_kernel(MomArgs A) {
    const int total = A.nb[0] + A.nb[1] + A.nb[2];
    const int lb = logical_block(total);
    if (lb >= total) return;   // whole block: no barrier below is skipped by part of it
    int comp, local;
    momentum_block(A, lb, comp, local);
    const int first = comp == 0 ? 0 : (comp == 1 ? A.nb[0] : A.nb[0] + A.nb[1]);
    const BoxK &bx = A.bx;
    const int NX = bx.nx + (comp == 0), NY = bx.ny + (comp == 1), NZ = bx.nz + (comp == 2);
    const int n = NX * NY * NZ;
    const int cpb = A.cpb[comp];
    const int base = local * cpb;
    const Geo g(bx);
    const Idx X{bx.nx, bx.ny, bx.nz};
    double res2 = 0.0;
    for (int off = 0; off < cpb; off += kThreads) {
        const int c = base + off + (int)threadIdx.x;
        if (c >= n) break;
        const int i = c % NX, q = c / NX, j = q % NY, k = q / NY;
        Row r;
        if (comp == 0) form_u(A, g, X, i, j, k, r);
        else if (comp == 1) form_v(A, g, X, i, j, k, r);
        else form_w(A, g, X, i, j, k, r);
#pragma unroll
        for (int s = 0; s < 7; ++s) st_nt(A.a[comp][s], c, r.a[s]);
        st_nt(A.b[comp], c, r.b);
        st_nt(A.d[comp], c, r.d);
        // row residual at the incoming iterate x (neighbours outside the grid carry no term)
        const double *x = comp == 0 ? A.u : (comp == 1 ? A.v : A.w);
        const int PL = NX * NY;
        double ax = r.a[0] * x[c];
        if (i + 1 < NX) ax -= r.a[1] * x[c + 1];
        if (i > 0) ax -= r.a[2] * x[c - 1];
        if (j + 1 < NY) ax -= r.a[3] * x[c + NX];
        if (j > 0) ax -= r.a[4] * x[c - NX];
        if (k + 1 < NZ) ax -= r.a[5] * x[c + PL];
        if (k > 0) ax -= r.a[6] * x[c - PL];
        const double e = r.b - ax;
        res2 += e * e;
    }
    const double s = block_sum(res2);
    if (threadIdx.x == 0) A.partials[first + local] = s;   // each grid's partials stay contiguous
}

__global__ void __launch_bounds__(kThreads) form_pressure_kernel(PresArgs A, int total) {
    const int lb = logical_block(total);
    if (lb >= total) return;
    const BoxK &bx = A.bx;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int n = nx * ny * nz;
    const Geo g(bx);
    const Idx X{nx, ny, nz};
    double b2 = 0.0;
    for (int off = 0; off < A.cpb; off += kThreads) {
        const int c = lb * A.cpb + off + (int)threadIdx.x;
        if (c >= n) break;
        const int i = c % nx, q = c / nx, j = q % ny, k = q / ny;
        const double rh = bx.rho;
        const double aE = i + 1 < nx ? g.rAx * A.du[X.u(i + 1, j, k)] : 0.0;
        const double aW = i > 0 ? g.rAx * A.du[X.u(i, j, k)] : 0.0;
        const double aN = j + 1 < ny ? g.rAy * A.dv[X.v(i, j + 1, k)] : 0.0;
        const double out = j + 1 == ny ? g.rAy * A.dv[X.v(i, j + 1, k)] : 0.0;
        const double aS = j > 0 ? g.rAy * A.dv[X.v(i, j, k)] : 0.0;
        const double aT = k + 1 < nz ? g.rAz * A.dw[X.w(i, j, k + 1)] : 0.0;
        const double aB = k > 0 ? g.rAz * A.dw[X.w(i, j, k)] : 0.0;
        const double aP = aE + aW + aN + aS + aT + aB + out;
        const double b = rh * ((A.u[X.u(i, j, k)] - A.u[X.u(i + 1, j, k)]) * g.Ax +
                               (A.v[X.v(i, j, k)] - A.v[X.v(i, j + 1, k)]) * g.Ay +
                               (A.w[X.w(i, j, k)] - A.w[X.w(i, j, k + 1)]) * g.Az);
        st_nt(A.a[0], c, aP);
        st_nt(A.a[1], c, aE);
        st_nt(A.a[2], c, aW);
        st_nt(A.a[3], c, aN);
        st_nt(A.a[4], c, aS);
        st_nt(A.a[5], c, aT);
        st_nt(A.a[6], c, aB);
        st_nt(A.b, c, b);
        b2 += b * b;
    }
    const double s = block_sum(b2);
    if (threadIdx.x == 0) A.partials[lb] = s;
}

__global__ void __launch_bounds__(kThreads) correct_kernel(CorrArgs A) {
    const int total = A.nb[0] + A.nb[1] + A.nb[2] + A.nb[3];
    const int lb = logical_block(total);
    if (lb >= total) return;
    int comp = 0, first = 0;
    while (comp < 3 && lb >= first + A.nb[comp]) first += A.nb[comp++];
    const BoxK &bx = A.bx;
    const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
    const int NX = nx + (comp == 0), NY = ny + (comp == 1), NZ = nz + (comp == 2);
    const int c = (lb - first) * kThreads + (int)threadIdx.x;
    if (c >= NX * NY * NZ) return;
    const int i = c % NX, q = c / NX, j = q % NY, k = q / NY;
    const Idx X{nx, ny, nz};
    const double *pp = A.pp;
    if (comp == 0) {
        if (i >= 1 && i <= nx - 1) st_nt(A.u, c, A.u[c] + A.du[c] * (pp[X.p(i - 1, j, k)] - pp[X.p(i, j, k)]));
    } else if (comp == 1) {
        if (j >= 1) {
            const double pa = pp[X.p(i, j < ny ? j : ny - 1, k)];
            const double above = j < ny ? pa : 0.0;
            st_nt(A.v, c, A.v[c] + A.dv[c] * (pp[X.p(i, j - 1, k)] - above));
        }
    } else if (comp == 2) {
        if (k >= 1 && k <= nz - 1) st_nt(A.w, c, A.w[c] + A.dw[c] * (pp[X.p(i, j, k - 1)] - pp[X.p(i, j, k)]));
    } else {
        st_nt(A.p, c, A.p[c] + bx.alpha_p * pp[c]);
    }
}

struct Ranges {
    int32_t begin[5];
};

// one block of kSumThreads: strided partial sums per thread, then a fixed-order tree
constexpr int kSumThreads = 1024;
__global__ void __launch_bounds__(kSumThreads) sum_ranges_kernel(const double *partials, Ranges R, int nq,
                                                                 double *out) {
    __shared__ double part[kSumThreads / 64];
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int t = R.begin[q] + (int)threadIdx.x; t < R.begin[q + 1]; t += kSumThreads) s += partials[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kSumThreads / 64; ++w) t += part[w];
            out[q] = t;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads) zero_kernel(double *p, long n) {
    for (long c = blockIdx.x * (long)kThreads + threadIdx.x; c < n; c += (long)gridDim.x * kThreads) p[c] = 0.0;
}

int grid_for(int total) { return (total + kXcds - 1) / kXcds * kXcds; }

}  // namespace

hipError_t launch_form_momentum(const MomArgs &a, hipStream_t s) {
    const int total = a.nb[0] + a.nb[1] + a.nb[2];
    hipLaunchKernelGGL(form_momentum_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_form_pressure(const PresArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(form_pressure_kernel, dim3(grid_for(nblocks)), dim3(kThreads), 0, s, a, nblocks);
    return hipGetLastError();
}

hipError_t launch_correct(const CorrArgs &a, hipStream_t s) {
    const int total = a.nb[0] + a.nb[1] + a.nb[2] + a.nb[3];
    hipLaunchKernelGGL(correct_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum_ranges(const double *partials, const int32_t *begin_host, int nq, double *out, hipStream_t s) {
    Ranges R{};
    for (int q = 0; q <= nq && q < 5; ++q) R.begin[q] = begin_host[q];
    hipLaunchKernelGGL(sum_ranges_kernel, dim3(1), dim3(kSumThreads), 0, s, partials, R, nq, out);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, long n, hipStream_t s) {
    const long blocks = std::min<long>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::max<long>(blocks, 1)), dim3(kThreads), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace eqsim
