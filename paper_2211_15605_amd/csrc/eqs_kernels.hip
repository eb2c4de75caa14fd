// eqs_kernels.hip -- gfx950 kernels of the equation-set solver.
//
// The solve is Jacobi-preconditioned BiCGSTAB on the 7-point system
//     a_P x_P - sum_nb a_nb x_nb = b
// whose cost per iteration is the stencil product and the global dot
// products (arXiv 2211.15605, Sec. 2.2.2).  The work is bandwidth-bound
// (about 0.2 flop per byte), so there is no MFMA here: every kernel is
// organised to stream each array from HBM once per pass.
//
// One iteration is three fused passes (plus one last-block reduction each):
//   K1  p = r + beta (p - omega v);  p^ = p / a_P;  v = A p^;   (r^, v)
//   K2  s = r - alpha v;             s^ = s / a_P;  t = A s^;   (t, s) (t, t) (s, s)
//   K3  x += alpha p^ + omega s^;    r = s - omega t;           (r^, r) (r, r)
// K1 and K2 compute their stencil operand on the fly, so it never round-trips
// through HBM.  They "march" along k: a tile is a segment of Q = 256*CPT
// consecutive cells of one k-plane (flattened i,j) over KC planes.  For each
// plane the block computes the operand for the segment plus an nx-wide halo
// on both sides (the j-1 and j+1 neighbours) into one of three rotating LDS
// buffers; the k-1 and k+1 neighbours of a thread's own cells stay in
// registers.  One barrier per plane suffices with three buffers.  p and v are
// double-buffered by iteration parity because halo cells read the old p and
// v of neighbouring tiles while those tiles write the new ones.
//
// Dot products: wave64 butterfly, then LDS across the 4 waves, then one
// partial per tile; the last block to finish (agent-scope ticket) sums the
// partials in tile order and runs the scalar update for the next pass.
// Every reduction therefore has a fixed order: results are bitwise
// reproducible, and identical whether a set runs alone or batched.
//
// Blocks are remapped so that each of the 8 XCDs (round-robin dispatch)
// receives a contiguous range of tiles: neighbouring segments, whose halos
// overlap, then share that XCD's L2.

#include <hip/hip_runtime.h>
#include <math.h>

#include "eqs_internal.h"
#include "eqs_launch.h"

namespace eqs {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, rem = nb % X;
    const int xcd = b % X, slot = b / X;
    return xcd * q + min(xcd, rem) + slot;
}

struct TileRef {
    const SetDesc *d;
    int tile;
};

__device__ __forceinline__ TileRef locate(const LaunchSets &ls) {
    const int L = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    int s = 0;
#pragma unroll
    for (int q = 1; q < kMaxSets; ++q)
        if (q < ls.nsets && L >= ls.tile_begin[q]) s = q;
    return TileRef{ls.desc + s, L - ls.tile_begin[s]};
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = ((red[i] + red[NV + i]) + red[2 * NV + i]) + red[3 * NV + i];
    }
}

// Tile partials -> last block sums them in tile order -> fin(state, sums).
template <int NV, class Fin>
__device__ __forceinline__ void reduce_and_finalize(const SetDesc &d, int tile, double (&acc)[NV], Fin fin) {
    __shared__ double red[4 * kMaxRed];
    __shared__ int last;
    block_sum<NV>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            __hip_atomic_store(d.partials + (size_t)tile * NV + i, acc[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t prev =
            __hip_atomic_fetch_add(d.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == (uint32_t)(d.ntiles - 1);
    }
    __syncthreads();
    if (!last) return;
    double s[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] = 0.0;
    for (int b = threadIdx.x; b < d.ntiles; b += kBlock) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            s[i] += __hip_atomic_load(d.partials + (size_t)b * NV + i, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    block_sum<NV>(s, red);
    if (threadIdx.x == 0) {
        fin(d.st, s);
        __hip_atomic_store(d.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ state machine
// (runs in one thread of the finalising block)

__device__ __forceinline__ bool iterating_fp64(int mode) { return mode == MODE_FP64 || mode == MODE_ADJOINT; }

__device__ __forceinline__ void start_fresh(SolveState *st, double rr) {
    st->rho = rr;
    st->rho_prev = 1.0;
    st->alpha = 1.0;
    st->omega = 1.0;
    st->fresh = 1;
    st->half = 0;
    st->active = 1;
}

// stop the BiCGSTAB iteration with a failure code
__device__ __forceinline__ void stop_iter(SolveState *st, int code) {
    st->active = 0;
    if (iterating_fp64(st->mode)) {
        st->status = code;
        st->need_report = 1;
    } else {
        st->inner_done = 1;  // the outer (FP64) residual decides
    }
}

__device__ __forceinline__ void converge_iter(SolveState *st) {
    st->active = 0;
    if (iterating_fp64(st->mode))
        st->converged = 1;  // true-residual recheck next
    else
        st->inner_done = 1;
}

__device__ __forceinline__ double pow2_scale(double rms) {
    if (!(rms > 0.0) || !isfinite(rms)) return 1.0;
    return ldexp(1.0, -ilogb(rms));
}

struct FinSetup {  // sums: (b,b), (r,r), #bad a_P
    const SetDesc *d;
    __device__ void operator()(SolveState *st, const double *s) const {
        st->mode = d->mode;
        st->maxit = d->maxit;
        st->iters = 0;
        st->restarts = 0;
        st->rho_restarts = 0;
        st->outer = 0;
        st->active = 0;
        st->done = 0;
        st->converged = 0;
        st->inner_done = 0;
        st->need_report = 0;
        st->zero_rhs = 0;
        st->half = 0;
        st->fresh = 0;
        st->status = ST_NOT_CONVERGED;
        const double bb = s[0], rr = s[1];
        st->bb = bb;
        st->bb_outer = bb;
        st->lim2 = d->tol * sqrt(bb);  // compared against sqrt((r, r))
        st->lim2_outer = st->lim2;
        st->rr = rr;
        st->rr_true = rr;
        if (s[2] > 0.0) { st->status = ST_ERR_ARG; st->done = 1; return; }
        if (!isfinite(bb) || !isfinite(rr)) { st->status = ST_NONFINITE; st->done = 1; return; }
        if (bb == 0.0) { st->status = ST_OK; st->zero_rhs = 1; st->rr_true = 0.0; st->done = 1; return; }
        if (sqrt(rr) <= st->lim2) { st->status = ST_OK; st->done = 1; return; }
        start_fresh(st, rr);
    }
};

struct FinRecheck {  // sums: (b,b), (r,r), #bad
    __device__ void operator()(SolveState *st, const double *s) const {
        st->converged = 0;
        const double rr = s[1];
        st->rr_true = rr;
        st->rr = rr;
        if (!isfinite(rr)) { st->status = ST_NONFINITE; st->done = 1; return; }
        if (sqrt(rr) <= st->lim2) { st->status = ST_OK; st->done = 1; return; }
        if (st->iters >= st->maxit) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        st->restarts++;
        start_fresh(st, rr);
    }
};

struct FinReport {
    __device__ void operator()(SolveState *st, const double *s) const {
        st->rr_true = s[1];
        st->need_report = 0;
        st->done = 1;
    }
};

struct FinK1 {  // sums: (r^, v)
    __device__ void operator()(SolveState *st, const double *s) const {
        st->iters++;
        st->fresh = 0;
        const double sg = s[0];
        st->sigma = sg;
        if (!isfinite(sg)) { stop_iter(st, ST_NONFINITE); return; }
        if (sg == 0.0) { stop_iter(st, ST_BREAKDOWN); return; }
        st->alpha = st->rho / sg;
    }
};

struct FinK2 {  // sums: (t,s), (t,t), (s,s)
    __device__ void operator()(SolveState *st, const double *s) const {
        st->ts = s[0];
        st->tt = s[1];
        st->ss = s[2];
        if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2])) { stop_iter(st, ST_NONFINITE); return; }
        if (sqrt(s[2]) <= st->lim2) {  // half-step exit: x += alpha p^ only
            st->half = 1;
            st->omega = 0.0;
            return;
        }
        st->omega = s[1] == 0.0 ? 0.0 : s[0] / s[1];
    }
};

struct FinK3 {  // sums: (r^, r), (r, r)
    __device__ void operator()(SolveState *st, const double *s) const {
        const double rho_new = s[0], rr = s[1];
        st->rr = rr;
        if (st->half) { st->half = 0; converge_iter(st); return; }
        if (!isfinite(rho_new) || !isfinite(rr)) { stop_iter(st, ST_NONFINITE); return; }
        if (sqrt(rr) <= st->lim2) { converge_iter(st); return; }
        if (st->omega == 0.0) { stop_iter(st, ST_BREAKDOWN); return; }
        if (st->iters >= st->maxit) { stop_iter(st, ST_NOT_CONVERGED); return; }
        st->rho_prev = st->rho;
        st->rho = rho_new;
        if (rho_new == 0.0) {
            if (st->rho_restarts++ > 0) { stop_iter(st, ST_BREAKDOWN); return; }
            st->restarts++;
            start_fresh(st, rr);  // r^ := r, so rho = (r, r)
        }
    }
};

struct FinCast {  // sums: (b,b), #bad
    const SetDesc *d;
    __device__ void operator()(SolveState *st, const double *s) const {
        st->mode = d->mode;
        st->maxit = d->maxit;
        st->iters = 0;
        st->restarts = 0;
        st->rho_restarts = 0;
        st->outer = 0;
        st->active = 0;
        st->done = 0;
        st->converged = 0;
        st->inner_done = 0;
        st->need_report = 0;
        st->zero_rhs = 0;
        st->half = 0;
        st->fresh = 0;
        st->status = ST_NOT_CONVERGED;
        const double bb = s[0];
        st->bb_outer = bb;
        st->lim2_outer = d->tol * sqrt(bb);
        st->rr_prev = 0.0;
        st->rr_true = bb;
        st->outer_pending = 1;
        if (s[1] > 0.0) { st->status = ST_ERR_ARG; st->done = 1; st->outer_pending = 0; return; }
        if (!isfinite(bb)) { st->status = ST_NONFINITE; st->done = 1; st->outer_pending = 0; return; }
        if (bb == 0.0) { st->status = ST_OK; st->zero_rhs = 1; st->rr_true = 0.0; st->done = 1; st->outer_pending = 0; return; }
        st->scale = pow2_scale(sqrt(bb / (double)d->n));
    }
};

struct FinOuter {  // sums: (r,r) in FP64, (r32, r32)
    const SetDesc *d;
    __device__ void operator()(SolveState *st, const double *s) const {
        st->inner_done = 0;
        st->outer_pending = 0;
        const double rr = s[0], rr32 = s[1];
        st->rr_true = rr;
        if (!isfinite(rr) || !isfinite(rr32)) { st->status = ST_NONFINITE; st->done = 1; return; }
        if (sqrt(rr) <= st->lim2_outer) { st->status = ST_OK; st->done = 1; return; }
        if (st->mode == MODE_FP32 && st->outer >= 1) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        if (st->outer >= 1 && rr > 0.25 * st->rr_prev) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        if (st->iters >= st->maxit) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        if (rr32 == 0.0) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }  // residual below FP32 range
        st->bb = rr32;
        st->lim2 = d->tol_inner * sqrt(rr32);
        st->rr = rr32;
        st->upd_inv_scale = 1.0 / st->scale;  // exact: a power of two
        st->rr_prev = rr;
        st->outer++;
        start_fresh(st, rr32);
        st->scale = pow2_scale(sqrt(rr / (double)d->n) * d->tol_inner);
    }
};

// ------------------------------------------------------------------ stencil

struct Nb {
    bool e, w, n, s;
};

// coefficients paired with the neighbour values xE, xW, xN, xS, xT, xB of
// row idx of A (TR = false) or of A^T (TR = true); zero where the neighbour
// is outside the grid, so out-of-grid slots are never read.
template <typename T, bool TR>
struct Coef6 {
    T e, w, n, s, t, b;
    __device__ __forceinline__ void load(const T *const *a, int idx, int nx, int P, Nb nb, bool up, bool dn) {
        if (!TR) {
            e = nb.e ? a[1][idx] : T(0);
            w = nb.w ? a[2][idx] : T(0);
            n = nb.n ? a[3][idx] : T(0);
            s = nb.s ? a[4][idx] : T(0);
            t = up ? a[5][idx] : T(0);
            b = dn ? a[6][idx] : T(0);
        } else {
            // column idx of A: idx is the west neighbour of idx+1 (a_W[idx+1]),
            // the east neighbour of idx-1 (a_E[idx-1]), and so on.
            e = nb.e ? a[2][idx + 1] : T(0);
            w = nb.w ? a[1][idx - 1] : T(0);
            n = nb.n ? a[4][idx + nx] : T(0);
            s = nb.s ? a[3][idx - nx] : T(0);
            t = up ? a[6][idx + P] : T(0);
            b = dn ? a[5][idx - P] : T(0);
        }
    }
    __device__ __forceinline__ T apply(T ap, T xc, T xE, T xW, T xN, T xS, T xT, T xB) const {
        T acc = ap * xc;
        acc = fma(-e, xE, acc);
        acc = fma(-w, xW, acc);
        acc = fma(-n, xN, acc);
        acc = fma(-s, xS, acc);
        acc = fma(-t, xT, acc);
        acc = fma(-b, xB, acc);
        return acc;
    }
};

// ------------------------------------------------------------------ march skeleton

template <typename T, int CPT, class Ph>
__device__ __forceinline__ void ext_plane(Ph &ph, const SetDesc &d, int k, T *buf, const int *qo,
                                          const bool *ok, int q0, T *vown, typename Ph::Aux *ax) {
    constexpr int Q = kBlock * CPT;
    const int nx = d.nx, P = d.plane;
    const int kb = k * P;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int e = nx + (int)threadIdx.x + kBlock * m;
        T v = T(0);
        if (ok[m]) v = ph.ext_own(qo[m] + kb, ax[m]);
        buf[e] = v;
        vown[m] = v;
    }
    for (int h = threadIdx.x; h < 2 * nx; h += kBlock) {
        const int e = h < nx ? h : h + Q;
        const int q = q0 - nx + e;
        T v = T(0);
        if (q >= 0 && q < P) v = ph.ext_halo(q + kb);
        buf[e] = v;
    }
}

template <typename T, int CPT, class Ph>
__device__ __forceinline__ void march(Ph &ph, const SetDesc &d, int tile, T *lds, double (&acc)[Ph::NV]) {
    constexpr int Q = kBlock * CPT;
    const int tid = threadIdx.x;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane;
    const int seg = tile % d.S, chunk = tile / d.S;
    const int q0 = seg * Q;
    const int k0 = chunk * d.KC;
    const int k1 = min(k0 + d.KC, nz);
    const int L = Q + 2 * nx;

    int qo[CPT];
    bool ok[CPT];
    Nb nb[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int q = q0 + tid + kBlock * m;
        qo[m] = q;
        ok[m] = q < P;
        const int j = q / nx, i = q - j * nx;
        nb[m] = Nb{i + 1 < nx, i > 0, j + 1 < ny, j > 0};
    }
    T vm[CPT], vc[CPT], vp[CPT];
    typename Ph::Aux axc[CPT], axp[CPT];
    typename Ph::Pre pre[CPT];

    if (k0 > 0) {
#pragma unroll
        for (int m = 0; m < CPT; ++m) vm[m] = ok[m] ? ph.value_only(qo[m] + (k0 - 1) * P) : T(0);
    } else {
#pragma unroll
        for (int m = 0; m < CPT; ++m) vm[m] = T(0);
    }
    ext_plane<T, CPT>(ph, d, k0, lds, qo, ok, q0, vc, axc);

    int bc = 0;  // buffer of plane k
    for (int k = k0; k < k1; ++k) {
        const bool up = k + 1 < nz, dn = k > 0;
        const int bn = bc == 2 ? 0 : bc + 1;
        // operands of the centre pass of plane k, issued before the barrier
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            if (ok[m]) ph.pre(qo[m] + k * P, nb[m], up, dn, pre[m]);
        if (up && k + 1 < k1) {
            ext_plane<T, CPT>(ph, d, k + 1, lds + bn * L, qo, ok, q0, vp, axp);
        } else if (up) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) vp[m] = ok[m] ? ph.value_only(qo[m] + (k + 1) * P) : T(0);
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m) vp[m] = T(0);
        }
        __syncthreads();
        const T *bufc = lds + bc * L;
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (ok[m]) {
                const int e = nx + tid + kBlock * m;
                const T xE = nb[m].e ? bufc[e + 1] : T(0);
                const T xW = nb[m].w ? bufc[e - 1] : T(0);
                const T xN = nb[m].n ? bufc[e + nx] : T(0);
                const T xS = nb[m].s ? bufc[e - nx] : T(0);
                const T xT = up ? vp[m] : T(0);
                const T xB = dn ? vm[m] : T(0);
                ph.center(qo[m] + k * P, pre[m], axc[m], vc[m], xE, xW, xN, xS, xT, xB, acc);
            }
        }
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            vm[m] = vc[m];
            vc[m] = vp[m];
            axc[m] = axp[m];
        }
        bc = bn;
    }
}

// ------------------------------------------------------------------ phases

template <typename T>
struct Vecs;
template <>
struct Vecs<double> {
    __device__ static const double *const *a(const SetDesc &d) { return d.a; }
    __device__ static double *r(const SetDesc &d) { return d.r; }
    __device__ static double *rh(const SetDesc &d) { return d.rh; }
    __device__ static double *p(const SetDesc &d, int i) { return d.p[i]; }
    __device__ static double *v(const SetDesc &d, int i) { return d.v[i]; }
    __device__ static double *t(const SetDesc &d) { return d.t; }
    __device__ static double *x(const SetDesc &d) { return d.x; }
};
template <>
struct Vecs<float> {
    __device__ static const float *const *a(const SetDesc &d) { return (const float *const *)d.a32; }
    __device__ static float *r(const SetDesc &d) { return d.r32; }
    __device__ static float *rh(const SetDesc &d) { return d.rh32; }
    __device__ static float *p(const SetDesc &d, int i) { return d.p32[i]; }
    __device__ static float *v(const SetDesc &d, int i) { return d.v32[i]; }
    __device__ static float *t(const SetDesc &d) { return d.t32; }
    __device__ static float *x(const SetDesc &d) { return d.d32; }
};

// K1: p = r + beta (p - omega v); p^ = p / a_P; v = A p^; (r^, v)
template <typename T, bool TR>
struct PhK1 {
    static constexpr int NV = 1;
    struct Aux { T ap; };
    struct Pre { Coef6<T, TR> c; T rh; };
    const T *const *a;
    const T *r, *rhd, *pold, *vold;
    T *pnew, *vnew, *rhw;
    T beta, omega;
    int nx, P;
    bool fresh;
    __device__ __forceinline__ T pval(int idx, T rv) const {
        return fresh ? rv : fma(beta, fma(-omega, vold[idx], pold[idx]), rv);
    }
    __device__ __forceinline__ T ext_own(int idx, Aux &ax) {
        const T rv = r[idx];
        const T p = pval(idx, rv);
        const T ap = a[0][idx];
        pnew[idx] = p;
        if (fresh) rhw[idx] = rv;
        ax.ap = ap;
        return p / ap;
    }
    __device__ __forceinline__ T ext_halo(int idx) const { return pval(idx, r[idx]) / a[0][idx]; }
    __device__ __forceinline__ T value_only(int idx) const { return pval(idx, r[idx]) / a[0][idx]; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, nb, up, dn);
        pr.rh = rhd[idx];
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &ax, T xc, T xE, T xW, T xN,
                                           T xS, T xT, T xB, double (&acc)[NV]) {
        const T v = pr.c.apply(ax.ap, xc, xE, xW, xN, xS, xT, xB);
        vnew[idx] = v;
        acc[0] += (double)pr.rh * (double)v;
    }
};

// K2: s = r - alpha v; s^ = s / a_P; t = A s^; (t, s), (t, t), (s, s)
template <typename T, bool TR>
struct PhK2 {
    static constexpr int NV = 3;
    struct Aux { T ap, s; };
    struct Pre { Coef6<T, TR> c; };
    const T *const *a;
    const T *r, *v;
    T *tout;
    T alpha;
    int nx, P;
    __device__ __forceinline__ T ext_own(int idx, Aux &ax) {
        const T s = fma(-alpha, v[idx], r[idx]);
        const T ap = a[0][idx];
        ax.ap = ap;
        ax.s = s;
        return s / ap;
    }
    __device__ __forceinline__ T ext_halo(int idx) const { return fma(-alpha, v[idx], r[idx]) / a[0][idx]; }
    __device__ __forceinline__ T value_only(int idx) const { return fma(-alpha, v[idx], r[idx]) / a[0][idx]; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, nb, up, dn);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &ax, T xc, T xE, T xW, T xN,
                                           T xS, T xT, T xB, double (&acc)[NV]) {
        const T t = pr.c.apply(ax.ap, xc, xE, xW, xN, xS, xT, xB);
        tout[idx] = t;
        const double td = (double)t, sd = (double)ax.s;
        acc[0] += td * sd;
        acc[1] += td * td;
        acc[2] += sd * sd;
    }
};

// r = b - A x (FP64).  SETUP and RECHECK write r and r^ = r; REPORT only sums.
template <bool TR>
struct PhRes {
    static constexpr int NV = 3;
    struct Aux {};
    struct Pre { Coef6<double, TR> c; double ap, b; };
    const double *const *a;
    const double *x, *b;
    double *r, *rh;
    int nx, P;
    bool write;
    __device__ __forceinline__ double ext_own(int idx, Aux &) { return x[idx]; }
    __device__ __forceinline__ double ext_halo(int idx) const { return x[idx]; }
    __device__ __forceinline__ double value_only(int idx) const { return x[idx]; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, nb, up, dn);
        pr.ap = a[0][idx];
        pr.b = b[idx];
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double ax = pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
        const double rv = pr.b - ax;
        if (write) {
            r[idx] = rv;
            rh[idx] = rv;
        }
        acc[0] += pr.b * pr.b;
        acc[1] += rv * rv;
        acc[2] += (pr.ap == 0.0 || !isfinite(pr.ap)) ? 1.0 : 0.0;
    }
};

// refinement residual: r = b - A x in FP64, emitted as FP32 r * scale (also r^ and a zero inner iterate)
struct PhOuter {
    static constexpr int NV = 2;
    struct Aux {};
    struct Pre { Coef6<double, false> c; double ap, b; };
    const double *const *a;
    const double *x, *b;
    float *r32, *rh32, *d32;
    double scale;
    int nx, P;
    __device__ __forceinline__ double ext_own(int idx, Aux &) { return x[idx]; }
    __device__ __forceinline__ double ext_halo(int idx) const { return x[idx]; }
    __device__ __forceinline__ double value_only(int idx) const { return x[idx]; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, nb, up, dn);
        pr.ap = a[0][idx];
        pr.b = b[idx];
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double rv = pr.b - pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
        const float f = (float)(rv * scale);
        r32[idx] = f;
        rh32[idx] = f;
        d32[idx] = 0.0f;
        acc[0] += rv * rv;
        acc[1] += (double)f * (double)f;
    }
};

// y = A x or A^T x (FP64, no reduction)
template <bool TR>
struct PhApply {
    static constexpr int NV = 1;
    struct Aux {};
    struct Pre { Coef6<double, TR> c; double ap; };
    const double *const *a;
    const double *x;
    double *y;
    int nx, P;
    __device__ __forceinline__ double ext_own(int idx, Aux &) { return x[idx]; }
    __device__ __forceinline__ double ext_halo(int idx) const { return x[idx]; }
    __device__ __forceinline__ double value_only(int idx) const { return x[idx]; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, nb, up, dn);
        pr.ap = a[0][idx];
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&)[NV]) {
        y[idx] = pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
    }
};

// ------------------------------------------------------------------ march kernels

template <typename T>
__device__ __forceinline__ T *lds_base() {
    extern __shared__ __align__(16) unsigned char eqs_smem[];
    return reinterpret_cast<T *>(eqs_smem);
}

template <typename T, int CPT, bool TR>
__global__ void __launch_bounds__(kBlock) k1_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (!st->active) return;
    const int par = st->iters & 1;
    PhK1<T, TR> ph;
    ph.a = Vecs<T>::a(d);
    ph.r = Vecs<T>::r(d);
    ph.fresh = st->fresh != 0;
    ph.rhd = ph.fresh ? Vecs<T>::r(d) : Vecs<T>::rh(d);
    ph.rhw = Vecs<T>::rh(d);
    ph.pold = Vecs<T>::p(d, par);
    ph.vold = Vecs<T>::v(d, par);
    ph.pnew = Vecs<T>::p(d, par ^ 1);
    ph.vnew = Vecs<T>::v(d, par ^ 1);
    ph.beta = (T)((st->rho / st->rho_prev) * (st->alpha / st->omega));
    ph.omega = (T)st->omega;
    ph.nx = d.nx;
    ph.P = d.plane;
    double acc[1] = {0.0};
    march<T, CPT>(ph, d, tr.tile, lds_base<T>(), acc);
    reduce_and_finalize<1>(d, tr.tile, acc, FinK1{});
}

template <typename T, int CPT, bool TR>
__global__ void __launch_bounds__(kBlock) k2_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (!st->active) return;
    const int par = st->iters & 1;
    PhK2<T, TR> ph;
    ph.a = Vecs<T>::a(d);
    ph.r = Vecs<T>::r(d);
    ph.v = Vecs<T>::v(d, par);
    ph.tout = Vecs<T>::t(d);
    ph.alpha = (T)st->alpha;
    ph.nx = d.nx;
    ph.P = d.plane;
    double acc[3] = {0.0, 0.0, 0.0};
    march<T, CPT>(ph, d, tr.tile, lds_base<T>(), acc);
    reduce_and_finalize<3>(d, tr.tile, acc, FinK2{});
}

// mode: 0 setup, 1 recheck, 2 report
template <int CPT, bool TR>
__global__ void __launch_bounds__(kBlock) res_kernel(LaunchSets ls, int mode) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (mode == 1 && !st->converged) return;
    if (mode == 2 && !st->need_report) return;
    PhRes<TR> ph;
    ph.a = d.a;
    ph.x = d.x;
    ph.b = d.b;
    ph.r = d.r;
    ph.rh = d.rh;
    ph.write = mode != 2;
    ph.nx = d.nx;
    ph.P = d.plane;
    double acc[3] = {0.0, 0.0, 0.0};
    march<double, CPT>(ph, d, tr.tile, lds_base<double>(), acc);
    if (mode == 0)
        reduce_and_finalize<3>(d, tr.tile, acc, FinSetup{&d});
    else if (mode == 1)
        reduce_and_finalize<3>(d, tr.tile, acc, FinRecheck{});
    else
        reduce_and_finalize<3>(d, tr.tile, acc, FinReport{});
}

template <int CPT>
__global__ void __launch_bounds__(kBlock) outer_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (st->done || !(st->outer_pending || st->inner_done)) return;
    PhOuter ph;
    ph.a = d.a;
    ph.x = d.x;
    ph.b = d.b;
    ph.r32 = d.r32;
    ph.rh32 = d.rh32;
    ph.d32 = d.d32;
    ph.scale = st->scale;
    ph.nx = d.nx;
    ph.P = d.plane;
    double acc[2] = {0.0, 0.0};
    march<double, CPT>(ph, d, tr.tile, lds_base<double>(), acc);
    reduce_and_finalize<2>(d, tr.tile, acc, FinOuter{&d});
}

template <int CPT, bool TR>
__global__ void __launch_bounds__(kBlock) apply_kernel(LaunchSets ls, const double *x, double *y) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    PhApply<TR> ph;
    ph.a = d.a;
    ph.x = x;
    ph.y = y;
    ph.nx = d.nx;
    ph.P = d.plane;
    double acc[1] = {0.0};
    march<double, CPT>(ph, d, tr.tile, lds_base<double>(), acc);
}

// ------------------------------------------------------------------ pointwise kernels (same tiles)

// visits the tile's own cells: for each plane of the chunk, the segment's cells
template <int CPT, class F>
__device__ __forceinline__ void for_tile_cells(const SetDesc &d, int tile, F f) {
    constexpr int Q = kBlock * CPT;
    const int seg = tile % d.S, chunk = tile / d.S;
    const int q0 = seg * Q;
    const int k0 = chunk * d.KC;
    const int k1 = min(k0 + d.KC, d.nz);
    for (int k = k0; k < k1; ++k) {
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int q = q0 + (int)threadIdx.x + kBlock * m;
            if (q < d.plane) f(q + k * d.plane, q, k);
        }
    }
}

// K3: x += alpha p^ + omega s^; r = s - omega t; (r^, r), (r, r)
template <typename T, int CPT>
__global__ void __launch_bounds__(kBlock) k3_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (!st->active) return;
    const int par = st->iters & 1;
    const T *a0 = Vecs<T>::a(d)[0];
    const T *p = Vecs<T>::p(d, par);
    const T *v = Vecs<T>::v(d, par);
    const T *t = Vecs<T>::t(d);
    const T *rh = Vecs<T>::rh(d);
    T *r = Vecs<T>::r(d);
    T *x = Vecs<T>::x(d);
    const T alpha = (T)st->alpha, omega = (T)st->omega;
    double acc[2] = {0.0, 0.0};
    for_tile_cells<CPT>(d, tr.tile, [&](int idx, int, int) {
        const T ap = a0[idx];
        const T s = fma(-alpha, v[idx], r[idx]);
        const T ph = p[idx] / ap, sh = s / ap;
        x[idx] = x[idx] + fma(alpha, ph, omega * sh);
        const T rn = fma(-omega, t[idx], s);
        r[idx] = rn;
        acc[0] += (double)rh[idx] * (double)rn;
        acc[1] += (double)rn * (double)rn;
    });
    reduce_and_finalize<2>(d, tr.tile, acc, FinK3{});
}

// FP64 -> FP32 coefficient copies (round to nearest even), (b, b), a_P check
template <int CPT>
__global__ void __launch_bounds__(kBlock) cast_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    double acc[2] = {0.0, 0.0};
    for_tile_cells<CPT>(d, tr.tile, [&](int idx, int, int) {
#pragma unroll
        for (int s = 0; s < 7; ++s) d.a32[s][idx] = (float)d.a[s][idx];
        const double ap = d.a[0][idx], bv = d.b[idx];
        acc[0] += bv * bv;
        acc[1] += (ap == 0.0 || !isfinite(ap) || (float)ap == 0.0f) ? 1.0 : 0.0;
    });
    reduce_and_finalize<2>(d, tr.tile, acc, FinCast{&d});
}

// x += d32 / scale (FP64), for sets whose inner solve has finished
template <int CPT>
__global__ void __launch_bounds__(kBlock) update_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st = d.st;
    if (st->done || !st->inner_done) return;
    const double is = st->upd_inv_scale;
    for_tile_cells<CPT>(d, tr.tile, [&](int idx, int, int) { d.x[idx] = fma(is, (double)d.d32[idx], d.x[idx]); });
}

// x = 0 where b = 0 (flagged by setup), or unconditionally (force)
template <int CPT>
__global__ void __launch_bounds__(kBlock) zero_kernel(LaunchSets ls, int force) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    if (!force && !d.st->zero_rhs) return;
    for_tile_cells<CPT>(d, tr.tile, [&](int idx, int, int) { d.x[idx] = 0.0; });
}

// adjoint gradients: g_P = -lambda x; g_nb = lambda x_nb (0 out of the grid)
template <int CPT>
__global__ void __launch_bounds__(kBlock) grad_kernel(LaunchSets ls) {
    const TileRef tr = locate(ls);
    const SetDesc &d = *tr.d;
    const double *lam = d.x, *xf = d.xf;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane;
    for_tile_cells<CPT>(d, tr.tile, [&](int idx, int q, int k) {
        const int j = q / nx, i = q - j * nx;
        const double l = lam[idx];
        if (d.g[0]) d.g[0][idx] = -l * xf[idx];
        if (d.g[1]) d.g[1][idx] = i + 1 < nx ? l * xf[idx + 1] : 0.0;
        if (d.g[2]) d.g[2][idx] = i > 0 ? l * xf[idx - 1] : 0.0;
        if (d.g[3]) d.g[3][idx] = j + 1 < ny ? l * xf[idx + nx] : 0.0;
        if (d.g[4]) d.g[4][idx] = j > 0 ? l * xf[idx - nx] : 0.0;
        if (d.g[5]) d.g[5][idx] = k + 1 < nz ? l * xf[idx + P] : 0.0;
        if (d.g[6]) d.g[6][idx] = k > 0 ? l * xf[idx - P] : 0.0;
    });
}

// ------------------------------------------------------------------ host launchers

size_t march_lds_bytes(int cpt, int max_nx, int elem) {
    return (size_t)3 * (size_t)(kBlock * cpt + 2 * max_nx) * (size_t)elem;
}

#define EQS_DISPATCH_CPT(cpt, BODY)                                   \
    do {                                                              \
        if ((cpt) == 1) { constexpr int C = 1; BODY; }                \
        else if ((cpt) == 2) { constexpr int C = 2; BODY; }           \
        else { constexpr int C = 4; BODY; }                           \
    } while (0)

hipError_t launch_kernel(Kern k, const LaunchSets &ls, int ntiles, int cpt, int max_nx, bool fp32, bool trans,
                         hipStream_t stream, const double *x, double *y, int arg) {
    const dim3 grid(ntiles), block(kBlock);
    const size_t lds64 = march_lds_bytes(cpt, max_nx, 8), lds32 = march_lds_bytes(cpt, max_nx, 4);
    switch (k) {
    case K_K1:
        if (fp32) {
            if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k1_kernel<float, C, true>), grid, block, lds32, stream, ls));
            else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k1_kernel<float, C, false>), grid, block, lds32, stream, ls));
        } else {
            if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k1_kernel<double, C, true>), grid, block, lds64, stream, ls));
            else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k1_kernel<double, C, false>), grid, block, lds64, stream, ls));
        }
        break;
    case K_K2:
        if (fp32) {
            if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k2_kernel<float, C, true>), grid, block, lds32, stream, ls));
            else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k2_kernel<float, C, false>), grid, block, lds32, stream, ls));
        } else {
            if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k2_kernel<double, C, true>), grid, block, lds64, stream, ls));
            else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k2_kernel<double, C, false>), grid, block, lds64, stream, ls));
        }
        break;
    case K_K3:
        if (fp32) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k3_kernel<float, C>), grid, block, 0, stream, ls));
        else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((k3_kernel<double, C>), grid, block, 0, stream, ls));
        break;
    case K_SETUP:
    case K_RECHECK:
    case K_REPORT: {
        const int mode = k == K_SETUP ? 0 : (k == K_RECHECK ? 1 : 2);
        if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((res_kernel<C, true>), grid, block, lds64, stream, ls, mode));
        else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((res_kernel<C, false>), grid, block, lds64, stream, ls, mode));
        break;
    }
    case K_OUTER:
        EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((outer_kernel<C>), grid, block, lds64, stream, ls));
        break;
    case K_CAST:
        EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((cast_kernel<C>), grid, block, 0, stream, ls));
        break;
    case K_UPDATE:
        EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((update_kernel<C>), grid, block, 0, stream, ls));
        break;
    case K_ZERO:
        EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((zero_kernel<C>), grid, block, 0, stream, ls, arg));
        break;
    case K_GRAD:
        EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((grad_kernel<C>), grid, block, 0, stream, ls));
        break;
    case K_APPLY:
        if (trans) EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((apply_kernel<C, true>), grid, block, lds64, stream, ls, x, y));
        else EQS_DISPATCH_CPT(cpt, hipLaunchKernelGGL((apply_kernel<C, false>), grid, block, lds64, stream, ls, x, y));
        break;
    }
    return hipGetLastError();
}

}  // namespace eqs
