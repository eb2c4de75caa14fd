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
#include <hip/hip_ext.h>
#include <math.h>

#include <algorithm>

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

// block -> (set, index in the set's list) over the launch's concatenated lists (begin: each set's
// first index, begin[nsets] the total).  The hardware hands block b to XCD b % 8, so XCD x runs
// floor(n / 8) blocks, one more if x < n % 8.  Contiguous map (xcd_remap): XCD x takes one run of
// the concatenated list, so neighbouring tiles, which read each other's halo cells, share its L2,
// but a set's tiles then sit on one or two XCDs only, and a launch in which only some sets have work
// (the others return at once) leaves the other XCDs idle.  Balanced map (bal): XCD x takes a run of
// every set instead, set q giving each XCD floor(T_q / 8) of its T_q tiles and its T_q % 8 extra
// ones to consecutive XCDs, the extras of the sets dealt round the eight XCDs in turn; that gives
// each XCD exactly the number of blocks the hardware hands it.  Either map is a bijection, and each
// block's partial sums go to its tile's slot, so results do not depend on the map.
__device__ __forceinline__ TileRef locate_in(const LaunchSets &ls, const int32_t *begin, bool bal) {
    const int b = (int)blockIdx.x;
    if (bal) {
        const int x = b % 8, slot = b / 8;
        int c = 0, o = 0;  // XCD x's slots taken by the sets before q; extras dealt so far, mod 8
#pragma unroll
        for (int q = 0; q < kMaxSets; ++q) {
            const int T = begin[q + 1] - begin[q], k = T >> 3, r = T & 7;
            const int a = k + (((x - o) & 7) < r ? 1 : 0);  // set q's tiles on XCD x
            if (q < ls.nsets && (slot < c + a || q == ls.nsets - 1)) {
                int before = x * k;  // set q's tiles on the XCDs before x
                for (int y = 0; y < x; ++y) before += ((y - o) & 7) < r ? 1 : 0;
                return TileRef{ls.desc + q, before + slot - c};
            }
            c += a;
            o = (o + r) & 7;
        }
    }
    const int L = xcd_remap(b, (int)gridDim.x);
    int s = 0;
#pragma unroll
    for (int q = 1; q < kMaxSets; ++q)
        if (q < ls.nsets && L >= begin[q]) s = q;
    return TileRef{ls.desc + s, L - begin[s]};
}

// block -> (set, tile) for march kernels (FLAT = false) or (set, block) for pointwise ones
template <bool FLAT>
__device__ __forceinline__ TileRef locate(const LaunchSets &ls) {
    return FLAT ? locate_in(ls, ls.flat_begin, (ls.xbal & 2) != 0) : locate_in(ls, ls.tile_begin, (ls.xbal & 1) != 0);
}

// block -> (set, tile) for the single-sync step (its own tiling)
__device__ __forceinline__ TileRef locate_fused(const LaunchSets &ls) {
    return locate_in(ls, ls.ftile_begin, (ls.xbal & 4) != 0);
}

// global-address-space accessors: pointers taken from the set table are
// generic; these make every access a global (not flat) memory operation
template <typename T>
__device__ __forceinline__ T ld(const T *p, int i) {
    return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <typename T>
__device__ __forceinline__ void st(T *p, int i, T v) {
    ((__attribute__((address_space(1))) T *)p)[i] = v;
}
// a nontemporal store: for vectors no block of the same launch reads back (the single-sync step
// writes the buffer slot its neighbours do not read), so they need not be kept in L2
template <typename T>
__device__ __forceinline__ void st_nt(T *p, int i, T v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T *)p + i);
}

template <int NV, int NT = kBlock>
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
        for (int i = 0; i < NV; ++i) {
            double t = ((red[i] + red[NV + i]) + red[2 * NV + i]) + red[3 * NV + i];
#pragma unroll
            for (int w = 4; w < NT / 64; ++w) t += red[w * NV + i];
            v[i] = t;
        }
    }
}

// Per-block partials -> the last of the set's `count` blocks sums them in
// block order -> fin(state, sums).
//
// Visibility: the partials are written with agent-scope atomic stores, which
// go through to the device's coherence point, and read back by the last
// block with agent-scope atomic loads.  A block therefore only has to wait
// until its partial stores are complete (vmcnt = 0) before taking its
// ticket; an agent-scope release there would write back the XCD's whole L2,
// once per block.  Nothing else written by the kernel is read by the last
// block.
template <int NV, class Fin, int NT = kBlock>
__device__ __forceinline__ void reduce_and_finalize(const SetDesc &d, int tile, int count, double (&acc)[NV],
                                                    Fin fin) {
    __shared__ double red[(NT / 64) * kMaxRed];
    __shared__ int last;
    double *partials = d.partials;
    uint32_t *counter = d.counter;
    block_sum<NV, NT>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            __hip_atomic_store(partials + (size_t)tile * NV + i, acc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);  // all counters zero: the partial stores are complete
        const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == (uint32_t)(count - 1);
    }
    __syncthreads();
    if (!last) return;
    double s[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] = 0.0;
    for (int b = threadIdx.x; b < count; b += NT) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            s[i] += __hip_atomic_load(partials + (size_t)b * NV + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    block_sum<NV, NT>(s, red);
    if (threadIdx.x == 0) {
        fin(d.st, s);
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    st->redo = 0;
    st->half = 0;
    st->active = 1;
    st->fpar = 0;     // the residual is in slot 0 of s
    st->need_f = 1;   // single-sync iteration: f = M^T r^ before the first step
    st->mat = 0;
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
        st->mat = 0;
        st->need_f = 0;
        st->fpar = 0;
        st->maxit = d->maxit;
        st->iters = 0;
        st->restarts = 0;
        st->sig_restarts = 0;
        st->sig_inner = 0;
        st->sig_redos = 0;
        st->redo = 0;
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
        st->mat = 0;
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
        st->mat = 0;
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

// Single-sync iteration (see fused_kernel).  After a fresh start: sums (f, r^),
// (r^, r^) with f = M^T r^, so sigma_0 = (r^, M p_0) = (f, r_0) (p_0 = r_0 = r^).
struct FinFSetup {
    __device__ void operator()(SolveState *st, const double *s) const {
        st->need_f = 0;
        st->mat = 0;
        st->fpar = 0;
        st->fresh = 1;
        st->redo = 0;
        const double sg = s[0], rr = s[1];
        st->rho = rr;
        st->sigma = sg;
        if (!isfinite(sg) || !isfinite(rr)) { stop_iter(st, ST_NONFINITE); return; }
        if (sg == 0.0) {  // breakdown in the first half-step of the iteration about to start
            st->iters++;
            stop_iter(st, ST_BREAKDOWN);
            return;
        }
        st->alpha = rr / sg;
    }
};

// sigma-consistency restarts one BiCGSTAB solve may take (each inner solve of the refinement has
// its own budget) before it reports BREAKDOWN
constexpr int kMaxSigmaRestarts = 32;

// After launch j of the single-sync iteration: sums (f,p_j), (f,v_j), (f,s_j),
// (f,t_j), (r^,s_j), (r^,t_j), (t_j,s_j), (t_j,t_j), (r_j,r_j), (s_j,s_j), (r^,v_j).
struct FinFused {
    double sig_tol;
    int redo_on;
    __device__ void operator()(SolveState *st, const double *s) const {
        const double fp = s[0], fv = s[1], fs = s[2], ft = s[3], rs = s[4], rt = s[5];
        const double ts = s[6], tt = s[7], rr = s[8], ss = s[9];
        const int was_fresh = st->fresh;
        st->fpar ^= 1;  // step j's s, t, p, v are in the other slot now
        if (!st->fresh) {
            // r_j (formed by this launch) decides convergence; y_j is stored
            st->rr = rr;
            if (!isfinite(rr)) { stop_iter(st, ST_NONFINITE); return; }
            if (sqrt(rr) <= st->lim2) { converge_iter(st); return; }
        }
        st->fresh = 0;
        st->ts = ts;
        st->tt = tt;
        st->ss = ss;
        bool fin = true;
        for (int i = 0; i < 11; ++i) fin = fin && isfinite(s[i]);
        if (!fin) { stop_iter(st, ST_NONFINITE); return; }
        // alpha_j came from sigma_j expanded over the previous step's vectors; (r^, v_j) taken
        // directly must agree with it.  Where the expansion's terms cancel (in FP32 above all),
        // they can part, and a step with the wrong alpha derails the iteration: start afresh
        // from the current iterate instead (r_j = s_j + alpha_j v_j, r^ = r_j).
        const double sd = s[10];
        // FP64 solves check at most kMaxSigmaRestarts times a solve; past that the iteration goes
        // on with the expanded sigma (a relative gap of the FP64 threshold is harmless).  An FP32
        // inner solve past its budget ends, and the refinement's FP64 residual decides.
        const bool check = !iterating_fp64(st->mode) || st->sig_inner < kMaxSigmaRestarts;
        if (check && fabs(sd - st->sigma) > sig_tol * fabs(sd)) {
            if (redo_on && sd != 0.0) {
                // Run step j again with alpha_j = rho_j / (r^, v_j): its inputs are still in the
                // slot this launch read, p_j and v_j come out the same bit for bit (so the rerun
                // passes this check), and y_j, which this launch formed from step j-1's values,
                // stays as it is.  omega, beta and alpha_prev still hold step j-1's values.
                st->fpar ^= 1;
                st->fresh = was_fresh;
                st->sigma = sd;
                st->alpha = st->rho / sd;
                st->redo = 1;
                st->sig_redos++;
                return;
            }
            if (st->sig_inner >= kMaxSigmaRestarts) { stop_iter(st, ST_BREAKDOWN); return; }
            st->restarts++;
            st->sig_restarts++;
            st->sig_inner++;
            st->mat = 4;
            st->need_f = 1;
            return;
        }
        st->redo = 0;
        st->iters++;
        st->alpha_prev = st->alpha;  // alpha_j
        if (sqrt(ss) <= st->lim2) {  // half-step exit: x = y_j + alpha_j p_j
            st->mat = 1;
            converge_iter(st);
            return;
        }
        const double om = tt == 0.0 ? 0.0 : ts / tt;
        st->omega = om;
        if (om == 0.0) { st->mat = 2; stop_iter(st, ST_BREAKDOWN); return; }
        if (st->iters >= st->maxit) {  // y_{j+1} formed, then the true residual decides
            st->mat = 2;
            converge_iter(st);
            return;
        }
        const double rho_new = rs - om * rt;  // (r^, r_{j+1}) with r_{j+1} = s_j - omega_j t_j
        if (!isfinite(rho_new)) { st->mat = 2; stop_iter(st, ST_NONFINITE); return; }
        if (rho_new == 0.0) {
            if (st->rho_restarts++ > 0) { st->mat = 2; stop_iter(st, ST_BREAKDOWN); return; }
            st->restarts++;
            st->mat = 3;  // y_{j+1}, r_{j+1}, r^ := r_{j+1}, then a fresh start
            st->need_f = 1;
            return;
        }
        const double beta = (rho_new / st->rho) * (st->alpha_prev / om);
        // (r^, M p_{j+1}) = (f, p_{j+1}), p_{j+1} = s_j - omega t_j + beta (p_j - omega v_j)
        const double sg = fs - om * ft + beta * (fp - om * fv);
        st->sigma = sg;
        if (!isfinite(sg) || sg == 0.0) { st->mat = 2; stop_iter(st, sg == 0.0 ? ST_BREAKDOWN : ST_NONFINITE); return; }
        st->beta = beta;
        st->rho_prev = st->rho;
        st->rho = rho_new;
        st->alpha = rho_new / sg;
    }
};

struct FinCast {  // sums: (b,b), #bad, #asymmetric rows
    const SetDesc *d;
    int sym_on;
    __device__ void operator()(SolveState *st, const double *s) const {
        st->sym = (sym_on && s[2] == 0.0) ? 1 : 0;
        st->mode = d->mode;
        st->weak_outer = 0;
        st->mat = 0;
        st->need_f = 0;
        st->fpar = 0;
        st->maxit = d->maxit;
        st->iters = 0;
        st->restarts = 0;
        st->sig_restarts = 0;
        st->sig_inner = 0;
        st->sig_redos = 0;
        st->redo = 0;
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
        st->sig_inner = 0;  // the next inner solve has its own restart budget
        st->outer_pending = 0;
        st->mat = 0;
        const double rr = s[0], rr32 = s[1];
        st->rr_true = rr;
        if (!isfinite(rr) || !isfinite(rr32)) { st->status = ST_NONFINITE; st->done = 1; return; }
        if (sqrt(rr) <= st->lim2_outer) { st->status = ST_OK; st->done = 1; return; }
        if (st->mode == MODE_FP32 && st->outer >= 1) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        // a refinement step should cut ||r|| at least in half; an inner FP32 solve can fail
        // to (rounding), and the next step starts afresh from the new residual, so only
        // three such steps in a row stop the solve
        if (st->outer >= 1 && rr > 0.25 * st->rr_prev) {
            if (++st->weak_outer >= 3) { st->status = ST_NOT_CONVERGED; st->done = 1; return; }
        } else {
            st->weak_outer = 0;
        }
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
// is outside the grid, so out-of-grid slots never contribute.  The loads
// are unconditional (indices clamped into the array) and masked afterwards,
// so a block's loads issue together without control flow between them.
template <typename T, bool TR>
struct Coef6 {
    T e, w, n, s, t, b;
    __device__ __forceinline__ void load(const T *const *a, int idx, int nx, int P, int ncell, Nb nb, bool up,
                                         bool dn) {
        if (!TR) {
            e = ld(a[1], idx);
            w = ld(a[2], idx);
            n = ld(a[3], idx);
            s = ld(a[4], idx);
            t = ld(a[5], idx);
            b = ld(a[6], idx);
        } else {
            // column idx of A: idx is the west neighbour of idx+1 (a_W[idx+1]),
            // the east neighbour of idx-1 (a_E[idx-1]), and so on.
            e = ld(a[2], min(idx + 1, ncell - 1));
            w = ld(a[1], max(idx - 1, 0));
            n = ld(a[4], min(idx + nx, ncell - 1));
            s = ld(a[3], max(idx - nx, 0));
            t = ld(a[6], min(idx + P, ncell - 1));
            b = ld(a[5], max(idx - P, 0));
        }
        e = nb.e ? e : T(0);
        w = nb.w ? w : T(0);
        n = nb.n ? n : T(0);
        s = nb.s ? s : T(0);
        t = up ? t : T(0);
        b = dn ? b : T(0);
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

// a row's six neighbour coefficients; with sym (an exactly symmetric matrix) the W, S and B terms
// are read from the E, N and T arrays at the neighbouring cell, a_W(c) = a_E(c-1) and so on, so a
// pass streams four coefficient arrays instead of seven.  Sources and indices are selected, not
// branched on, so every load stays unconditional.
template <typename T>
__device__ __forceinline__ void load_row6(Coef6<T, false> &c, const T *const *a, int idx, int nx, int P, Nb nb,
                                          bool up, bool dn, bool sym) {
    const T *wp = sym ? a[1] : a[2], *sp = sym ? a[3] : a[4], *bp = sym ? a[5] : a[6];
    const int wi = sym ? max(idx - 1, 0) : idx, si = sym ? max(idx - nx, 0) : idx, bi = sym ? max(idx - P, 0) : idx;
    c.e = ld(a[1], idx);
    c.w = ld(wp, wi);
    c.n = ld(a[3], idx);
    c.s = ld(sp, si);
    c.t = ld(a[5], idx);
    c.b = ld(bp, bi);
    c.e = nb.e ? c.e : T(0);
    c.w = nb.w ? c.w : T(0);
    c.n = nb.n ? c.n : T(0);
    c.s = nb.s ? c.s : T(0);
    c.t = up ? c.t : T(0);
    c.b = dn ? c.b : T(0);
}

// ------------------------------------------------------------------ march skeleton
//
// Geometry and pointers are copied into registers at kernel entry: the set
// table lives in global memory, and after the first store the compiler could
// no longer keep table fields in registers (it cannot rule out aliasing), so
// every reload would drain the loads in flight.
struct Geo {
    int nx, ny, nz, P, n, S, KC;
};
__device__ __forceinline__ Geo geo_of(const SetDesc &d) {
    return Geo{d.nx, d.ny, d.nz, d.plane, d.n, d.S, d.KC};
}
//
// A phase Ph supplies:
//   Raw  load(idx, q, k)           raw inputs of the stencil operand at cell idx
//                                  (in-plane index q, plane k)
//   T    own(raw, idx, Aux&)       operand value of an own cell (+ its stores)
//   T    halo(raw)                 operand value of any other cell (no stores)
//   void pre(idx, nb, up, dn, Pre&)  loads for the centre pass of an own cell
//   void center(idx, Pre, Aux, xc, xE..xB, acc)
// Every step issues all of its loads (centre operands of plane k, raw inputs
// of plane k+2 for the own cells and H halo slots per thread) before any
// store, so they are in flight together.  load() must not read what own() or
// center() write: the raw inputs of a plane are read a step before its stores.

// raw inputs of plane k (own cells; H halo slots per thread: the row below and the row above
// the segment), at indices clamped into the plane
template <int CPT, int H, class Ph>
__device__ __forceinline__ void load_plane(const Ph &ph, const Geo &d, int k, const int *qo, int q0,
                                           typename Ph::Raw *ro, typename Ph::Raw *rh) {
    constexpr int Q = kBlock * CPT;
    const int nx = d.nx, P = d.P;
    const int kb = k * P;
#pragma unroll
    for (int m = 0; m < CPT; ++m) ro[m] = ph.load(min(qo[m], P - 1) + kb, min(qo[m], P - 1), k);
#pragma unroll
    for (int hh = 0; hh < H; ++hh) {
        const int h = (int)threadIdx.x + kBlock * hh;
        const int e = h < nx ? h : h + Q;
        const int q = min(max(q0 - nx + e, 0), P - 1);
        rh[hh] = ph.load(q + kb, q, k);
    }
}

// plane k into an LDS buffer from its raw inputs: operand values of the own cells (with their
// stores) and of the halo slots (out-of-grid cells hold 0)
template <typename T, int CPT, int H, class Ph>
__device__ __forceinline__ void store_plane(Ph &ph, const Geo &d, int k, T *buf, const int *qo, const bool *ok,
                                            int q0, T *vown, typename Ph::Aux *ax, const typename Ph::Raw *ro,
                                            const typename Ph::Raw *rh) {
    constexpr int Q = kBlock * CPT;
    const int nx = d.nx, P = d.P;
    const int kb = k * P;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int e = nx + (int)threadIdx.x + kBlock * m;
        const T v = ok[m] ? ph.own(ro[m], qo[m] + kb, ax[m]) : T(0);
        buf[e] = v;
        vown[m] = v;
    }
#pragma unroll
    for (int hh = 0; hh < H; ++hh) {
        const int h = (int)threadIdx.x + kBlock * hh;
        const int e = h < nx ? h : h + Q;
        const int q = q0 - nx + e;
        if (h < 2 * nx) buf[e] = (q >= 0 && q < P) ? ph.halo(rh[hh]) : T(0);
    }
}

// The march of a tile through its chunk of planes.  Step k forms the products on plane k
// from the LDS buffer of plane k; before its barrier it stores plane k + 1 into the next
// buffer from raw inputs loaded one step earlier, and issues the loads of plane k + 2, which
// are then in flight through the step (its barrier waits for LDS only).
template <typename T, int CPT, int H, class Ph>
__device__ __forceinline__ void march(Ph &ph, const Geo &d, int tile, T *lds, double (&acc)[Ph::NV]) {
    constexpr int Q = kBlock * CPT;
    const int tid = threadIdx.x;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.P;
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

    {
        typename Ph::Raw rb[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) rb[m] = ph.load(min(qo[m], P - 1) + max(k0 - 1, 0) * P, min(qo[m], P - 1), max(k0 - 1, 0));
#pragma unroll
        for (int m = 0; m < CPT; ++m) vm[m] = (k0 > 0 && ok[m]) ? ph.halo(rb[m]) : T(0);
    }
    typename Ph::Raw rco[CPT], rch[H];  // raw inputs of plane k + 1 (clamped into the grid)
    load_plane<CPT, H>(ph, d, k0, qo, q0, rco, rch);
    store_plane<T, CPT, H>(ph, d, k0, lds, qo, ok, q0, vc, axc, rco, rch);
    load_plane<CPT, H>(ph, d, min(k0 + 1, nz - 1), qo, q0, rco, rch);

    int bc = 0;  // buffer of plane k
    for (int k = k0; k < k1; ++k) {
        const bool up = k + 1 < nz, dn = k > 0;
        const int bn = bc == 2 ? 0 : bc + 1;
#pragma unroll
        for (int m = 0; m < CPT; ++m) ph.pre(min(qo[m], P - 1) + k * P, nb[m], up, dn, pre[m]);
        typename Ph::Raw rno[CPT], rnh[H];
        load_plane<CPT, H>(ph, d, min(k + 2, nz - 1), qo, q0, rno, rnh);
        if (up && k + 1 < k1) {
            store_plane<T, CPT, H>(ph, d, k + 1, lds + bn * L, qo, ok, q0, vp, axp, rco, rch);
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m) vp[m] = (up && ok[m]) ? ph.halo(rco[m]) : T(0);
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
            rco[m] = rno[m];
        }
#pragma unroll
        for (int hh = 0; hh < H; ++hh) rch[hh] = rnh[hh];
        bc = bn;
    }
}

// ------------------------------------------------------------------ phases
//
// The BiCGSTAB iteration runs on the column-scaled operator A D^-1 (unit
// diagonal, D = diag(a_P)) with iterate y = D x: this is right-Jacobi
// BiCGSTAB on A with the preconditioner folded into the matrix once per
// solve, so the iteration reads six coefficient arrays, never a_P, and
// divides nowhere.  (A D^-1 y)[c] = y[c] - sum_nb s_nb[c] y[nb(c)] with
// s_nb[c] = a_nb[c] / a_P[nb(c)].

template <typename T>
struct Vecs;
template <>
struct Vecs<double> {
    __device__ static double *const *as(const SetDesc &d) { return d.as; }
    __device__ static double *r(const SetDesc &d) { return d.r; }
    __device__ static double *rh(const SetDesc &d) { return d.rh; }
    __device__ static double *p(const SetDesc &d, int i) { return i ? d.p[1] : d.p[0]; }
    __device__ static double *v(const SetDesc &d, int i) { return i ? d.v[1] : d.v[0]; }
    __device__ static double *t(const SetDesc &d) { return d.t; }
    __device__ static double *y(const SetDesc &d) { return d.y; }
    __device__ static double *s(const SetDesc &d, int i) { return i ? d.s1 : d.r; }
    __device__ static double *t(const SetDesc &d, int i) { return i ? d.t1 : d.t; }
    __device__ static double *f(const SetDesc &d) { return d.f; }
    // symmetric form: a_E, a_N, a_T (the caller's arrays), 1/a_P
    __device__ static const double *sy(const SetDesc &d, int i) {
        return i == 0 ? d.a[1] : i == 1 ? d.a[3] : i == 2 ? d.a[5] : d.dinv;
    }
};
template <>
struct Vecs<float> {
    __device__ static float *const *as(const SetDesc &d) { return d.as32; }
    __device__ static float *r(const SetDesc &d) { return d.r32; }
    __device__ static float *rh(const SetDesc &d) { return d.rh32; }
    __device__ static float *p(const SetDesc &d, int i) { return i ? d.p32[1] : d.p32[0]; }
    __device__ static float *v(const SetDesc &d, int i) { return i ? d.v32[1] : d.v32[0]; }
    __device__ static float *t(const SetDesc &d) { return d.t32; }
    __device__ static float *y(const SetDesc &d) { return d.d32; }
    __device__ static float *s(const SetDesc &d, int i) { return i ? d.s1_32 : d.r32; }
    __device__ static float *t(const SetDesc &d, int i) { return i ? d.t1_32 : d.t32; }
    __device__ static float *f(const SetDesc &d) { return d.f32; }
    __device__ static const float *sy(const SetDesc &d, int i) { return d.sym32[i]; }
};

// the six scaled coefficients of a row, zero where the neighbour is outside
// the grid (loads unconditional, masked afterwards, as in Coef6)
template <typename T>
struct Unit6 {
    T e, w, n, s, t, b;
    __device__ __forceinline__ void load(const T *const *as, int idx, Nb nb, bool up, bool dn) {
        e = ld(as[0], idx);
        w = ld(as[1], idx);
        n = ld(as[2], idx);
        s = ld(as[3], idx);
        t = ld(as[4], idx);
        b = ld(as[5], idx);
        e = nb.e ? e : T(0);
        w = nb.w ? w : T(0);
        n = nb.n ? n : T(0);
        s = nb.s ? s : T(0);
        t = up ? t : T(0);
        b = dn ? b : T(0);
    }
    // in-plane links of row idx of an exactly symmetric matrix: a_W(idx) = a_E(idx-1) and
    // a_S(idx) = a_N(idx-nx), so two arrays hold all four (the neighbour's entries are read from
    // cache lines the neighbouring rows bring in); the T and B links are set by the caller
    __device__ __forceinline__ void load_sym_plane(const T *aE, const T *aN, int idx, int nx, Nb nb) {
        e = ld(aE, idx);
        w = ld(aE, max(idx - 1, 0));
        n = ld(aN, idx);
        s = ld(aN, max(idx - nx, 0));
        e = nb.e ? e : T(0);
        w = nb.w ? w : T(0);
        n = nb.n ? n : T(0);
        s = nb.s ? s : T(0);
    }
    // row idx of M^T: the link to neighbour nb is row nb's coefficient towards idx
    __device__ __forceinline__ void load_transposed(const T *const *as, int idx, int nx, int P, int ncell, Nb nb,
                                                    bool up, bool dn) {
        e = ld(as[1], min(idx + 1, ncell - 1));
        w = ld(as[0], max(idx - 1, 0));
        n = ld(as[3], min(idx + nx, ncell - 1));
        s = ld(as[2], max(idx - nx, 0));
        t = ld(as[5], min(idx + P, ncell - 1));
        b = ld(as[4], max(idx - P, 0));
        e = nb.e ? e : T(0);
        w = nb.w ? w : T(0);
        n = nb.n ? n : T(0);
        s = nb.s ? s : T(0);
        t = up ? t : T(0);
        b = dn ? b : T(0);
    }
    __device__ __forceinline__ T apply(T xc, T xE, T xW, T xN, T xS, T xT, T xB) const {
        T acc = xc;
        acc = fma(-e, xE, acc);
        acc = fma(-w, xW, acc);
        acc = fma(-n, xN, acc);
        acc = fma(-s, xS, acc);
        acc = fma(-t, xT, acc);
        acc = fma(-b, xB, acc);
        return acc;
    }
};

// K1: p = r + beta (p - omega v); v = (A D^-1) p; (r^, v)
template <typename T>
struct PhK1 {
    static constexpr int NV = 1;
    struct Raw { T r, p, v; };
    struct Aux {};
    struct Pre { Unit6<T> c; T rh; };
    const T *as[6];
    const T *r, *rhd, *pold, *vold;
    T *pnew, *vnew, *rhw;
    T beta, omega;
    bool fresh;
    __device__ __forceinline__ Raw load(int idx, int, int) const {
        Raw w;
        w.r = ld(r, idx);
        w.p = ld(pold, idx);
        w.v = ld(vold, idx);
        return w;
    }
    __device__ __forceinline__ T pval(const Raw &w) const {
        return fresh ? w.r : fma(beta, fma(-omega, w.v, w.p), w.r);
    }
    __device__ __forceinline__ T own(const Raw &w, int idx, Aux &) {
        const T p = pval(w);
        st(pnew, idx, p);
        if (fresh) st(rhw, idx, w.r);
        return p;
    }
    __device__ __forceinline__ T halo(const Raw &w) const { return pval(w); }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(as, idx, nb, up, dn);
        pr.rh = ld(rhd, idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, T xc, T xE, T xW, T xN, T xS,
                                           T xT, T xB, double (&acc)[NV]) {
        const T v = pr.c.apply(xc, xE, xW, xN, xS, xT, xB);
        st(vnew, idx, v);
        acc[0] += (double)pr.rh * (double)v;
    }
};

// K2: s = r - alpha v; t = (A D^-1) s; (t, s), (t, t), (s, s)
template <typename T>
struct PhK2 {
    static constexpr int NV = 3;
    struct Raw { T r, v; };
    struct Aux { T s; };
    struct Pre { Unit6<T> c; };
    const T *as[6];
    const T *r, *v;
    T *tout;
    T alpha;
    __device__ __forceinline__ Raw load(int idx, int, int) const {
        Raw w;
        w.r = ld(r, idx);
        w.v = ld(v, idx);
        return w;
    }
    __device__ __forceinline__ T own(const Raw &w, int, Aux &ax) {
        ax.s = fma(-alpha, w.v, w.r);
        return ax.s;
    }
    __device__ __forceinline__ T halo(const Raw &w) const { return fma(-alpha, w.v, w.r); }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(as, idx, nb, up, dn);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &ax, T xc, T xE, T xW, T xN, T xS,
                                           T xT, T xB, double (&acc)[NV]) {
        const T t = pr.c.apply(xc, xE, xW, xN, xS, xT, xB);
        st(tout, idx, t);
        const double td = (double)t, sd = (double)ax.s;
        acc[0] += td * sd;
        acc[1] += td * td;
        acc[2] += sd * sd;
    }
};

// stencil operand = x itself (residual and product phases, original operator)
struct RawX { double x; };

template <bool TR>
struct PhRes {
    static constexpr int NV = 3;
    using Raw = RawX;
    struct Aux {};
    struct Pre { Coef6<double, TR> c; double ap, b; };
    const double *a[7];
    const double *x, *b;
    double *r, *rh, *y, *dinv;
    int nx, P, ncell;
    bool write, wdinv;
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(x, idx)}; }
    __device__ __forceinline__ double own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ double halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, ncell, nb, up, dn);
        pr.ap = ld(a[0], idx);
        pr.b = ld(b, idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double ax = pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
        const double rv = pr.b - ax;
        if (write) {
            st(r, idx, rv);
            st(rh, idx, rv);
            st(y, idx, pr.ap * xc);  // the scaled iterate y = D x that the iteration continues from
            if (wdinv) st(dinv, idx, 1.0 / pr.ap);  // for the raw form of the single-sync step
        }
        acc[0] += pr.b * pr.b;
        acc[1] += rv * rv;
        acc[2] += (pr.ap == 0.0 || !isfinite(pr.ap)) ? 1.0 : 0.0;
    }
};

// refinement residual: r = b - A x in FP64, emitted as FP32 r * scale (also r^ and a zero inner iterate)
struct PhOuter {
    static constexpr int NV = 2;
    using Raw = RawX;
    struct Aux {};
    struct Pre { Coef6<double, false> c; double ap, b; };
    const double *a[7];
    const double *x, *b;
    float *r32, *rh32, *d32;
    double scale;
    int nx, P, ncell;
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(x, idx)}; }
    __device__ __forceinline__ double own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ double halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, ncell, nb, up, dn);
        pr.ap = ld(a[0], idx);
        pr.b = ld(b, idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double rv = pr.b - pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
        const float f = (float)(rv * scale);
        st(r32, idx, f);
        st(rh32, idx, f);
        st(d32, idx, 0.0f);
        acc[0] += rv * rv;
        acc[1] += (double)f * (double)f;
    }
};

// y = A x or A^T x (FP64, no reduction)
template <bool TR>
struct PhApply {
    static constexpr int NV = 1;
    using Raw = RawX;
    struct Aux {};
    struct Pre { Coef6<double, TR> c; double ap; };
    const double *a[7];
    const double *x;
    double *y;
    int nx, P, ncell;
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(x, idx)}; }
    __device__ __forceinline__ double own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ double halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, ncell, nb, up, dn);
        pr.ap = ld(a[0], idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&)[NV]) {
        st(y, idx, pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB));
    }
};

// f = M^T r^ (M the scaled operator), (f, r^), (r^, r^): set-up of the single-sync iteration
template <typename T>
struct PhFSet {
    static constexpr int NV = 2;
    struct Raw { T x; };
    struct Aux {};
    struct Pre { Unit6<T> c; };
    const T *as[6];
    const T *rh;
    T *f;
    int nx, P, ncell;
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(rh, idx)}; }
    __device__ __forceinline__ T own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ T halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load_transposed(as, idx, nx, P, ncell, nb, up, dn);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, T xc, T xE, T xW, T xN, T xS,
                                           T xT, T xB, double (&acc)[NV]) {
        const T fv = pr.c.apply(xc, xE, xW, xN, xS, xT, xB);
        st(f, idx, fv);
        acc[0] += (double)fv * (double)xc;
        acc[1] += (double)xc * (double)xc;
    }
};

// f = M^T r^ from the caller's coefficients (the raw form of the single-sync step): row c of
// M^T = D^-1 A^T is r^_c - (1/a_P)_c sum_nb a_{nb->c} r^_nb, the link from neighbour nb being row
// nb's coefficient towards c
struct PhFSetRaw {
    static constexpr int NV = 2;
    struct Raw { double x; };
    struct Aux {};
    struct Pre { Coef6<double, true> c; double g; };
    const double *a[7];
    const double *rh, *dinv;
    double *f;
    int nx, P, ncell;
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(rh, idx)}; }
    __device__ __forceinline__ double own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ double halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        pr.c.load(a, idx, nx, P, ncell, nb, up, dn);
        pr.g = ld(dinv, idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double q = pr.c.apply(0.0, xc, xE, xW, xN, xS, xT, xB);  // -sum_nb a_{nb->c} r^_nb
        const double fv = fma(pr.g, q, xc);
        st(f, idx, fv);
        acc[0] += fv * xc;
        acc[1] += xc * xc;
    }
};

// ------------------------------------------------------------------ march kernels

template <typename T>
__device__ __forceinline__ T *lds_base() {
    extern __shared__ __align__(16) unsigned char eqs_smem[];
    return reinterpret_cast<T *>(eqs_smem);
}

template <typename T, int CPT, int H>
__global__ void __launch_bounds__(kBlock) k1_kernel(LaunchSets ls) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    const int par = st_->iters & 1;
    PhK1<T> ph;
    for (int k = 0; k < 6; ++k) ph.as[k] = Vecs<T>::as(d)[k];
    ph.r = Vecs<T>::r(d);
    ph.fresh = st_->fresh != 0;
    ph.rhd = ph.fresh ? Vecs<T>::r(d) : Vecs<T>::rh(d);
    ph.rhw = Vecs<T>::rh(d);
    ph.pold = Vecs<T>::p(d, par);
    ph.vold = Vecs<T>::v(d, par);
    ph.pnew = Vecs<T>::p(d, par ^ 1);
    ph.vnew = Vecs<T>::v(d, par ^ 1);
    ph.beta = (T)((st_->rho / st_->rho_prev) * (st_->alpha / st_->omega));
    ph.omega = (T)st_->omega;
    double acc[1] = {0.0};
    march<T, CPT, H>(ph, geo_of(d), tr.tile, lds_base<T>(), acc);
    reduce_and_finalize<1>(d, tr.tile, d.ntiles, acc, FinK1{});
}

template <typename T, int CPT, int H>
__global__ void __launch_bounds__(kBlock) k2_kernel(LaunchSets ls) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    const int par = st_->iters & 1;
    PhK2<T> ph;
    for (int k = 0; k < 6; ++k) ph.as[k] = Vecs<T>::as(d)[k];
    ph.r = Vecs<T>::r(d);
    ph.v = Vecs<T>::v(d, par);
    ph.tout = Vecs<T>::t(d);
    ph.alpha = (T)st_->alpha;
    double acc[3] = {0.0, 0.0, 0.0};
    march<T, CPT, H>(ph, geo_of(d), tr.tile, lds_base<T>(), acc);
    reduce_and_finalize<3>(d, tr.tile, d.ntiles, acc, FinK2{});
}

// mode: 0 setup, 1 recheck, 2 report
template <int CPT, int H, bool TR>
__global__ void __launch_bounds__(kBlock) res_kernel(LaunchSets ls, int mode, int wdinv) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (mode == 1 && !st_->converged) return;
    if (mode == 2 && !st_->need_report) return;
    PhRes<TR> ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = d.a[k];
    ph.x = d.x;
    ph.b = d.b;
    ph.r = d.r;
    ph.rh = d.rh;
    ph.y = d.y;
    ph.dinv = d.dinv;
    ph.write = mode != 2;
    ph.wdinv = wdinv != 0;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[3] = {0.0, 0.0, 0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
    if (mode == 0)
        reduce_and_finalize<3>(d, tr.tile, d.ntiles, acc, FinSetup{&d});
    else if (mode == 1)
        reduce_and_finalize<3>(d, tr.tile, d.ntiles, acc, FinRecheck{});
    else
        reduce_and_finalize<3>(d, tr.tile, d.ntiles, acc, FinReport{});
}

template <int CPT, int H>
__global__ void __launch_bounds__(kBlock) outer_kernel(LaunchSets ls) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (st_->done || !(st_->outer_pending || st_->inner_done)) return;
    PhOuter ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = d.a[k];
    ph.x = d.x;
    ph.b = d.b;
    ph.r32 = d.r32;
    ph.rh32 = d.rh32;
    ph.d32 = d.d32;
    ph.scale = st_->scale;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[2] = {0.0, 0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
    reduce_and_finalize<2>(d, tr.tile, d.ntiles, acc, FinOuter{&d});
}

template <int CPT, int H, bool TR>
__global__ void __launch_bounds__(kBlock) apply_kernel(LaunchSets ls, const double *x, double *y) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    PhApply<TR> ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = d.a[k];
    ph.x = x;
    ph.y = y;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[1] = {0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
}

template <typename T, int CPT, int H>
__global__ void __launch_bounds__(kBlock) fsetup_kernel(LaunchSets ls) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (st_->done || !st_->active || !st_->need_f) return;
    PhFSet<T> ph;
    for (int k = 0; k < 6; ++k) ph.as[k] = Vecs<T>::as(d)[k];
    ph.rh = Vecs<T>::rh(d);
    ph.f = Vecs<T>::f(d);
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[2] = {0.0, 0.0};
    march<T, CPT, H>(ph, geo_of(d), tr.tile, lds_base<T>(), acc);
    reduce_and_finalize<2>(d, tr.tile, d.ntiles, acc, FinFSetup{});
}

template <int CPT, int H>
__global__ void __launch_bounds__(kBlock) fsetup_raw_kernel(LaunchSets ls) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (st_->done || !st_->active || !st_->need_f) return;
    PhFSetRaw ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = d.a[k];
    ph.rh = d.rh;
    ph.dinv = d.dinv;
    ph.f = d.f;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[2] = {0.0, 0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
    reduce_and_finalize<2>(d, tr.tile, d.ntiles, acc, FinFSetup{});
}

// ------------------------------------------------------------------ single-sync iteration
//
// One launch per BiCGSTAB step j on the scaled operator M = A D^-1.  From
// step j-1's s, t, p, v (slot st->fpar) and scalars it forms, per cell,
//   r_j = s_{j-1} - omega_{j-1} t_{j-1}
//   y_j = y_{j-1} + alpha_{j-1} p_{j-1} + omega_{j-1} s_{j-1}
//   p_j = r_j + beta_{j-1} (p_{j-1} - omega_{j-1} v_{j-1})
//   v_j = M p_j,   s_j = r_j - alpha_j v_j,   t_j = M s_j
// (at a fresh start r_0 is the stored residual, p_0 = r_0, y unchanged) and
// the ten sums of FinFused, from which the finalising block gets omega_j,
// rho_{j+1} = (r^, s_j) - omega_j (r^, t_j) and sigma_{j+1} = (r^, M p_{j+1})
// = (f, p_{j+1}) with f = M^T r^, expanded over step j's vectors.  The
// products and vector updates are those of BiCGSTAB; only the grouping of
// the dot products differs, so one grid-wide reduction serves a step and
// the six coefficient arrays are read once for both products.
//
// Tile: a segment of Q = 256 CPT cells of a plane (flat in-plane index q0 ..
// q0+Q-1) times the planes k0 .. k1-1.  t needs s one row (nx cells) and one
// plane beyond the tile, and s there needs p one more row and plane out, so
// p is formed on the segment widened by 2 nx cells each side (index e = q -
// q0 + 2 nx in [0, Q + 4 nx)), v and s on the segment widened by nx, t on
// the segment itself.  Step kt forms p on plane kt + 2d, v and s on plane
// kt + d and t on plane kt, with d = +1 (upward march) or -1 (downward); four
// lead-in steps start the pipeline two planes outside the chunk.  Tiles are
// numbered chunk-fastest, so the chunks of a column of segments are
// neighbours in the launch (the same XCD: see xcd_remap), and odd chunks march
// downward: two chunks that share a boundary then read the planes on either
// side of it at the same time, and the second read finds them in L2.
// p and s planes rotate through three LDS buffers each.  Each thread owns
// CPT cells of the segment and H cells of each of two halo rings: the inner
// ring (the nx cells next to the segment on each side: v and s needed there)
// and the outer ring (p only).
// how the single-sync step forms its products (see fused_step)
constexpr int kFormScaled = 0, kFormSym = 1, kFormRaw = 2;

// x where c holds, else +0, as a bitwise mask: a use of x that does not depend on
// c, so the compiler cannot move x's loads under a per-lane branch (whose join
// would wait for every load in flight), and a NaN or Inf in x never leaks out
__device__ __forceinline__ double keep_if(bool c, double x) {
    return __longlong_as_double(__double_as_longlong(x) & (c ? ~0ll : 0ll));
}
__device__ __forceinline__ float keep_if(bool c, float x) {
    return __int_as_float(__float_as_int(x) & (c ? ~0 : 0));
}

// FORM (kFormScaled, kFormSym, kFormRaw) is how the step forms the products of M = A D^-1:
//  - scaled: from the six coefficients of M written by the per-solve scale pass, p in LDS;
//  - symmetric: the planes in LDS hold p D^-1 and s D^-1 (each value times 1/a_P of its
//    cell), the products take a_E, a_N, a_T and the neighbours' a_E, a_N, a_T for the W, S, B
//    links, (A D^-1 p)_c = p_c - sum_nb a_nb(c) (p/a_P)_nb, and the own cells' p and s come
//    from registers: 4 coefficient words per cell instead of 6;
//  - raw (FP64): the same with the caller's six coefficients of the row itself, so no scale
//    pass is needed (1/a_P comes from the setup pass): 7 coefficient words per cell instead of 6,
//    for solves of a few steps, where the per-solve pass costs more than the extra word.
template <typename T, int CPT, int H, int FORM, int NT>
__device__ __forceinline__ void fused_step(const TileRef &tr) {
    constexpr bool SYM = FORM == kFormSym, RAW = FORM == kFormRaw;
    constexpr bool PD = SYM || RAW;  // LDS planes hold p D^-1 and s D^-1
    static_assert(!RAW || sizeof(T) == 8, "the raw form runs in FP64");
    constexpr int Q = NT * CPT;
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    const int in = st_->fpar, out = in ^ 1;
    const bool fresh = st_->fresh != 0;
    const bool redo = st_->redo != 0;  // y_j is formed already: a rerun of the step leaves it
    const T al = (T)st_->alpha, ap = (T)st_->alpha_prev, om = (T)st_->omega, be = (T)st_->beta;
    const T *as[6];
    for (int k = 0; k < 6; ++k) as[k] = RAW ? (const T *)d.a[k + 1] : Vecs<T>::as(d)[k];
    const T *aE = Vecs<T>::sy(d, 0), *aN = Vecs<T>::sy(d, 1), *aT = Vecs<T>::sy(d, 2), *gv = Vecs<T>::sy(d, 3);
    const T *sI = Vecs<T>::s(d, in), *tI = Vecs<T>::t(d, in), *pI = Vecs<T>::p(d, in), *vI = Vecs<T>::v(d, in);
    T *sO = Vecs<T>::s(d, out), *tO = Vecs<T>::t(d, out), *pO = Vecs<T>::p(d, out), *vO = Vecs<T>::v(d, out);
    T *yv = Vecs<T>::y(d);
    const T *fv = Vecs<T>::f(d), *rhv = Vecs<T>::rh(d);
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, KC = d.KC, NKC = d.NKC;
    // every other step runs the tiles in reverse order and each march in the
    // opposite direction, so a step starts on the planes the previous one
    // touched last (still in the MALL, the memory-side cache) and ends on those
    // the next step will start from
    const bool flip = in != 0;
    const int tl = flip ? d.fntiles - 1 - tr.tile : tr.tile;
    // chunk-fastest: the chunks of a column of segments are neighbours in the launch; segment-
    // fastest: the segments of a chunk are, so neighbouring segments (whose rings read each
    // other's cells) start together and march in step
    const int chunk = d.ford ? tl / d.fS : tl % NKC, seg = d.ford ? tl % d.fS : tl / NKC;
    const int q0 = seg * Q, k0 = chunk * KC, k1 = min(k0 + KC, nz);
    const bool down = ((chunk & 1) != 0) != flip;
    const int dk = down ? -1 : 1;
    const int W = Q + 4 * nx;
    T *Pb = lds_base<T>();
    T *Sb = Pb + 3 * W;
    T *pad = Sb + 3 * W;  // one cell per thread: the target of unused ring slots
    const int tid = threadIdx.x;

    // own cells
    int qo[CPT], eo[CPT];
    bool oko[CPT];
    Nb nbo[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int q = q0 + tid + NT * m;
        qo[m] = min(q, P - 1);
        eo[m] = 2 * nx + tid + NT * m;
        oko[m] = q < P;
        const int j = qo[m] / nx, i = qo[m] - j * nx;
        nbo[m] = Nb{i + 1 < nx, i > 0, j + 1 < ny, j > 0};
    }
    // ring cells: slot h covers ring position hh = tid + 256 h < 2 nx; an unused
    // slot writes its (ignored) values to the thread's pad cell
    int qi[H], qr[H];
    int ei[H], er[H];   // LDS offsets within a plane buffer, -1 for an unused slot
    bool oki[H], okr[H];
    Nb nbi[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int hh = tid + NT * h;
        const bool use = hh < 2 * nx;
        // inner ring: e in [nx, 2nx) and [Q + 2nx, Q + 3nx)
        const int e1 = hh < nx ? nx + hh : Q + nx + hh;
        const int q1 = q0 - 2 * nx + e1;
        ei[h] = use ? e1 : -1;
        oki[h] = use && q1 >= 0 && q1 < P;
        qi[h] = min(max(q1, 0), P - 1);
        const int j = qi[h] / nx, i = qi[h] - j * nx;
        nbi[h] = Nb{i + 1 < nx, i > 0, j + 1 < ny, j > 0};
        // outer ring: e in [0, nx) and [Q + 3nx, Q + 4nx)
        const int e2 = hh < nx ? hh : Q + 2 * nx + hh;
        const int q2 = q0 - 2 * nx + e2;
        er[h] = use ? e2 : -1;
        okr[h] = use && q2 >= 0 && q2 < P;
        qr[h] = min(max(q2, 0), P - 1);
    }

    // values carried between steps (own cells): f on planes kt+d / kt,
    // r^ and the coefficients on plane kt, r on plane kt+d (also inner ring)
    T fB[CPT], fC[CPT], rhC[CPT], rBo[CPT], rBi[H];
    // symmetric form: p and 1/a_P on plane kt+d (own cells, inner ring), s on plane kt (own);
    // a_T of the plane loaded at the previous step (own cells, inner ring)
    T pBo[CPT], pBi[H], gBo[CPT], gBi[H], sCo[CPT], tLo[CPT], tLi[H];
    Unit6<T> cC[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        fB[m] = fC[m] = rhC[m] = rBo[m] = T(0);
        pBo[m] = gBo[m] = sCo[m] = tLo[m] = T(0);
        cC[m] = Unit6<T>{T(0), T(0), T(0), T(0), T(0), T(0)};
    }
#pragma unroll
    for (int h = 0; h < H; ++h) rBi[h] = pBi[h] = gBi[h] = tLi[h] = T(0);
    double acc[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) acc[i] = 0.0;
    // At a fresh start r = s (the stored residual) and p = r: the terms of step
    // j-1 are masked off bitwise (their buffers may hold anything) and their
    // scalars zeroed, so no branch depends on `fresh` either.
    const T omf = fresh ? T(0) : om, bef = fresh ? T(0) : be;
    const bool cont = !fresh;

    // The previous step's vectors that step `it` reads on plane kp (own cells and both rings),
    // y and f (own cells) and, in the symmetric form, 1/a_P there.  Step it issues these loads
    // for step it + 1 as soon as its p planes are in LDS, so they are in flight while it forms
    // the products (its barriers wait for LDS only); the first step's are issued before the
    // loop.  Every load is unconditional, at a plane index clamped into the grid (y, f: into
    // the chunk), so the extra loads after the last step stay in bounds.  FP64 with four halo
    // slots per ring issues them at the top of their own step instead: the values held a step
    // longer would take it past 256 VGPRs and halve its occupancy.
    constexpr bool PF = sizeof(T) == 4 || H <= 2;
    // the rings' loads (mostly L2 hits: the neighbouring segments load the same cells) go a
    // step ahead too with one halo slot per ring, except in the FP64 symmetric form, which has
    // no registers to spare (FP64 with two slots: 251 VGPRs with the own cells' loads a step
    // ahead, past 256 with the rings' as well)
    constexpr bool PFR = (sizeof(T) == 4 || H == 1) && !(PD && sizeof(T) == 8);
    struct VecLoads {
        T s[CPT], t[CPT], p[CPT], v[CPT], y[CPT], f[CPT], g[CPT];
        T si[H], ti[H], pi[H], vi[H], gi[H], sr[H], tr[H], pr[H], vr[H], gr[H];
    };
    auto load_own = [&](int it, VecLoads &L) {
        const int kp = (down ? k1 + 3 - it : k0 - 4 + it) + 2 * dk;
        const int kpb = min(max(kp, 0), nz - 1) * P;
        const int kyb = min(max(kp, k0), k1 - 1) * P;  // y, f: own planes
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int i = qo[m] + kpb;
            L.s[m] = ld(sI, i); L.t[m] = ld(tI, i); L.p[m] = ld(pI, i); L.v[m] = ld(vI, i);
            L.y[m] = ld(yv, qo[m] + kyb);
            L.f[m] = ld(fv, qo[m] + kyb);
            L.g[m] = PD ? ld(gv, i) : T(0);
        }
    };
    auto load_rings = [&](int it, VecLoads &L) {
        const int kp = (down ? k1 + 3 - it : k0 - 4 + it) + 2 * dk;
        const int kpb = min(max(kp, 0), nz - 1) * P;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int i = qi[h] + kpb, r = qr[h] + kpb;
            L.si[h] = ld(sI, i); L.ti[h] = ld(tI, i); L.pi[h] = ld(pI, i); L.vi[h] = ld(vI, i);
            L.sr[h] = ld(sI, r); L.tr[h] = ld(tI, r); L.pr[h] = ld(pI, r); L.vr[h] = ld(vI, r);
            L.gi[h] = PD ? ld(gv, i) : T(0);
            L.gr[h] = PD ? ld(gv, r) : T(0);
        }
    };
    VecLoads nextv;
    if (PF) load_own(0, nextv);
    if (PFR) load_rings(0, nextv);

    int bt = 0, bv = 1, bp = 2;  // LDS slots of planes kt, kt+d, kt+2d (kt-d shares kt+2d's slot)
    const int nsteps = k1 - k0 + 4;
    for (int it = 0; it < nsteps; ++it) {
        const int kt = down ? k1 + 3 - it : k0 - 4 + it;
        const int kp = kt + 2 * dk, kv = kt + dk;
        const bool pin = kp >= 0 && kp < nz, pown = kp >= k0 && kp < k1;
        const bool do2 = it >= 2, vin = kv >= 0 && kv < nz, vown = kv >= k0 && kv < k1;
        const bool do3 = it >= 4;
        const int kpb = min(max(kp, 0), nz - 1) * P, kvb = min(max(kv, 0), nz - 1) * P;

        // ---- loads: coefficients and r^ on plane kv (the vectors on plane kp are in flight
        // since the previous step).  Every load is unconditional, at a plane index clamped into
        // the range where it is used; what a step outside that range loads is read again when
        // the range is reached.
        if (!PF) load_own(it, nextv);
        if (!PFR) load_rings(it, nextv);
        const VecLoads cv = nextv;
        T rhN[CPT];
        Unit6<T> cN[CPT], cI[H];
        {
            const int krb = min(max(kv, k0), k1 - 1) * P;  // r^: own planes
            const int kcb = min(max(min(max(kv, k0 - 1), k1), 0), nz - 1) * P;  // coefficients: k0-1 .. k1
            const bool up = kv + 1 < nz, dn = kv > 0;
            // symmetric form: the T and B links of plane kv are a_T on planes kv and kv - 1, which
            // consecutive steps share: each step loads one of them (plane kv going up, kv - 1 going
            // down, planes clamped into the grid) and takes the other from the previous step's load
            const int ktb = min(max(down ? kv - 1 : kv, 0), nz - 1) * P;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (SYM) {
                    cN[m].load_sym_plane(aE, aN, qo[m] + kcb, nx, nbo[m]);
                    const T tl = ld(aT, qo[m] + ktb);
                    cN[m].t = up ? (down ? tLo[m] : tl) : T(0);
                    cN[m].b = dn ? (down ? tl : tLo[m]) : T(0);
                    tLo[m] = tl;
                } else {
                    cN[m].load(as, qo[m] + kcb, nbo[m], up, dn);
                }
                rhN[m] = ld(rhv, qo[m] + krb);
            }
#pragma unroll
            for (int h = 0; h < H; ++h) {
                if (SYM) {
                    cI[h].load_sym_plane(aE, aN, qi[h] + kcb, nx, nbi[h]);
                    const T tl = ld(aT, qi[h] + ktb);
                    cI[h].t = up ? (down ? tLi[h] : tl) : T(0);
                    cI[h].b = dn ? (down ? tl : tLi[h]) : T(0);
                    tLi[h] = tl;
                } else {
                    cI[h].load(as, qi[h] + kcb, nbi[h], up, dn);
                }
            }
        }

        // ---- p_j on plane kp (segment + both rings), r_j kept for plane kp
        T rAo[CPT], rAi[H], pAo[CPT], pAi[H];
        T *pw = Pb + bp * W;
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const bool ok = pin && oko[m];
            const T r = keep_if(ok, fma(-omf, keep_if(cont, cv.t[m]), cv.s[m]));
            const T pv = keep_if(ok, fma(bef, keep_if(cont, fma(-om, cv.v[m], cv.p[m])), r));
            pw[eo[m]] = PD ? keep_if(ok, pv * cv.g[m]) : pv;
            pAo[m] = pv;
            rAo[m] = r;
            const bool own = pown && oko[m];
            const T yn = cv.y[m] + fma(ap, cv.p[m], om * cv.s[m]);
            asm volatile("" ::"v"(yn));  // formed on every lane, before the branch (no sunk loads)
            if (own) {
                const int i = qo[m] + kpb;
                st_nt(pO, i, pv);
                if (!fresh && !redo) st_nt(yv, i, yn);
            }
            acc[0] += (double)keep_if(own, cv.f[m]) * (double)pv;
            acc[8] += (double)keep_if(own, r) * (double)r;
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const bool ok = pin && oki[h];
            const T r = keep_if(ok, fma(-omf, keep_if(cont, cv.ti[h]), cv.si[h]));
            const T pv = keep_if(ok, fma(bef, keep_if(cont, fma(-om, cv.vi[h], cv.pi[h])), r));
            rAi[h] = r;
            pAi[h] = pv;
            (ei[h] >= 0 ? pw[ei[h]] : pad[tid]) = PD ? keep_if(ok, pv * cv.gi[h]) : pv;
            const bool ok2 = pin && okr[h];
            const T r2 = keep_if(ok2, fma(-omf, keep_if(cont, cv.tr[h]), cv.sr[h]));
            const T pv2 = keep_if(ok2, fma(bef, keep_if(cont, fma(-om, cv.vr[h], cv.pr[h])), r2));
            (er[h] >= 0 ? pw[er[h]] : pad[tid]) = PD ? keep_if(ok2, pv2 * cv.gr[h]) : pv2;
        }
        __syncthreads();
        if (PF) load_own(it + 1, nextv);  // in flight while the products below are formed
        if (PFR) load_rings(it + 1, nextv);

        // ---- v_j = M p_j and s_j = r_j - alpha_j v_j on plane kv (segment + inner ring)
        T sNo[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) sNo[m] = T(0);
        if (do2) {
            // plane kv's neighbours: kv + d = kp, kv - d = kt
            const T *pc = Pb + bv * W, *pu = Pb + (down ? bt : bp) * W, *pd = Pb + (down ? bp : bt) * W;
            T *sw = Sb + bv * W;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int e = eo[m];
                const T xc = PD ? pBo[m] : pc[e];
                const T v = cN[m].apply(xc, pc[e + 1], pc[e - 1], pc[e + nx], pc[e - nx], pu[e], pd[e]);
                const bool ok = vin && oko[m];
                const T sv = keep_if(ok, fma(-al, v, rBo[m]));
                sw[e] = PD ? keep_if(ok, sv * gBo[m]) : sv;
                sNo[m] = sv;
                const bool own = vown && oko[m];
                if (own) {
                    const int i = qo[m] + kvb;
                    st_nt(vO, i, v);
                    st_nt(sO, i, sv);
                }
                const T vk = keep_if(own, v), sk = keep_if(own, sv);
                acc[1] += (double)fB[m] * (double)vk;
                acc[2] += (double)fB[m] * (double)sk;
                acc[4] += (double)keep_if(own, rhN[m]) * (double)sk;
                acc[9] += (double)sk * (double)sk;
                acc[10] += (double)keep_if(own, rhN[m]) * (double)vk;  // sigma_j taken directly
            }
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int e = ei[h] >= 0 ? ei[h] : 2 * nx;  // an unused slot reads a valid cell, writes its pad
                const T xc = PD ? pBi[h] : pc[e];
                const T v = cI[h].apply(xc, pc[e + 1], pc[e - 1], pc[e + nx], pc[e - nx], pu[e], pd[e]);
                const bool ok = vin && oki[h];
                const T sv = keep_if(ok, fma(-al, v, rBi[h]));
                (ei[h] >= 0 ? sw[e] : pad[tid]) = PD ? keep_if(ok, sv * gBi[h]) : sv;
            }
        }
        __syncthreads();

        // ---- t_j = M s_j on plane kt (segment)
        if (do3) {
            // plane kt's neighbours: kt + d = kv, kt - d (slot of kt + 2d)
            const T *sc = Sb + bt * W, *su = Sb + (down ? bp : bv) * W, *sd = Sb + (down ? bv : bp) * W;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int e = eo[m];
                const T s0 = PD ? sCo[m] : sc[e];
                const T t = cC[m].apply(s0, sc[e + 1], sc[e - 1], sc[e + nx], sc[e - nx], su[e], sd[e]);
                if (oko[m]) st_nt(tO, qo[m] + kt * P, t);
                const T tk = keep_if(oko[m], t);
                acc[3] += (double)fC[m] * (double)tk;
                acc[5] += (double)rhC[m] * (double)tk;
                acc[6] += (double)tk * (double)s0;
                acc[7] += (double)tk * (double)tk;
            }
        }

        // ---- rotate
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            fC[m] = fB[m];
            fB[m] = cv.f[m];
            rhC[m] = rhN[m];
            cC[m] = cN[m];
            rBo[m] = rAo[m];
            pBo[m] = pAo[m];
            gBo[m] = cv.g[m];
            sCo[m] = sNo[m];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
            rBi[h] = rAi[h];
            pBi[h] = pAi[h];
            gBi[h] = cv.gi[h];
        }
        const int b0 = bt;
        bt = bv;
        bv = bp;
        bp = b0;
    }
    reduce_and_finalize<11, FinFused, NT>(d, tr.tile, d.fntiles, acc, FinFused{d.sigma_tol[sizeof(T) == 4 ? 1 : 0], d.sig_redo});
}

// FORM is chosen on the host (symmetric: every set of the launch exactly symmetric; raw: asked
// for on the context); NT (256 or 512 threads) by the launch shape
template <typename T, int CPT, int H, int FORM, int NT>
__global__ void __launch_bounds__(NT) fused_kernel(LaunchSets ls) {
    const TileRef tr = locate_fused(ls);
    const SolveState *st_ = tr.d->st;
    if (!st_->active || st_->need_f) return;
    fused_step<T, CPT, H, FORM, NT>(tr);
}

// ------------------------------------------------------------------ pointwise kernels
//
// Block b of a set takes chunks b, b + nflat, ... of kFlatChunk cells; each
// thread loads all kFlatU cells of a chunk (strided by the block size) before
// computing and storing.


// K3: y += alpha p + omega s; r = s - omega t; (r^, r), (r, r)
template <typename T>
__global__ void __launch_bounds__(kBlock) k3_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    const int par = st_->iters & 1;
    const T *p = Vecs<T>::p(d, par);
    const T *v = Vecs<T>::v(d, par);
    const T *t = Vecs<T>::t(d);
    const T *rh = Vecs<T>::rh(d);
    T *r = Vecs<T>::r(d);
    T *y = Vecs<T>::y(d);
    const T alpha = (T)st_->alpha, omega = (T)st_->omega;
    const int n = d.n, nflat = d.nflat;
    double acc[2] = {0.0, 0.0};
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        T Pv[kFlatU], V[kFlatU], R[kFlatU], Tt[kFlatU], Y[kFlatU], RH[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            Pv[u] = ld(p, i); V[u] = ld(v, i); R[u] = ld(r, i);
            Tt[u] = ld(t, i); Y[u] = ld(y, i); RH[u] = ld(rh, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) {
                const T s = fma(-alpha, V[u], R[u]);
                st(y, i, Y[u] + fma(alpha, Pv[u], omega * s));
                const T rn = fma(-omega, Tt[u], s);
                st(r, i, rn);
                acc[0] += (double)RH[u] * (double)rn;
                acc[1] += (double)rn * (double)rn;
            }
        }
    }
    reduce_and_finalize<2>(d, tr.tile, nflat, acc, FinK3{});
}

// Leaving the single-sync iteration (st->mat): y += alpha p (1), y += alpha p +
// omega s (2), and for a restart (3) also r = s - omega t into slot 0 and r^ = r,
// with step j's vectors (slot st->fpar) and scalars (alpha_prev, omega).
template <typename T>
__global__ void __launch_bounds__(kBlock) mat_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    const int mode = st_->mat;
    if (!mode) return;
    const int cur = st_->fpar;
    if (mode == 4) {  // restart at the current iterate: r = s + alpha v into slot 0, r^ = r
        const T al = (T)st_->alpha;
        const T *s = Vecs<T>::s(d, cur), *v = Vecs<T>::v(d, cur);
        T *r0 = Vecs<T>::s(d, 0), *rh = Vecs<T>::rh(d);
        const int n = d.n, nflat = d.nflat;
        for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
            const int base = ch * kFlatChunk + (int)threadIdx.x;
            T Sv[kFlatU], V[kFlatU];
#pragma unroll
            for (int u = 0; u < kFlatU; ++u) {
                const int i = min(base + kBlock * u, n - 1);
                Sv[u] = ld(s, i);
                V[u] = ld(v, i);
            }
#pragma unroll
            for (int u = 0; u < kFlatU; ++u) {
                const int i = base + kBlock * u;
                if (i < n) {
                    const T rv = fma(al, V[u], Sv[u]);
                    st(r0, i, rv);
                    st(rh, i, rv);
                }
            }
        }
        return;
    }
    const T a = (T)st_->alpha_prev, om = mode == 1 ? T(0) : (T)st_->omega;
    const T *p = Vecs<T>::p(d, cur), *s = Vecs<T>::s(d, cur), *t = Vecs<T>::t(d, cur);
    T *y = Vecs<T>::y(d), *r0 = Vecs<T>::s(d, 0), *rh = Vecs<T>::rh(d);
    const int n = d.n, nflat = d.nflat;
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        T Y[kFlatU], Pv[kFlatU], Sv[kFlatU], Tt[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            Y[u] = ld(y, i);
            Pv[u] = ld(p, i);
            Sv[u] = ld(s, i);
            Tt[u] = mode == 3 ? ld(t, i) : T(0);  // t only for a restart residual
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) {
                st(y, i, mode == 1 ? fma(a, Pv[u], Y[u]) : Y[u] + fma(a, Pv[u], om * Sv[u]));
                if (mode == 3) {
                    const T rv = fma(-om, Tt[u], Sv[u]);
                    st(r0, i, rv);
                    st(rh, i, rv);
                }
            }
        }
    }
}

// coefficients of A D^-1 (TR = false) or A^T D^-1 (TR = true), FP64 (for the
// FP64 iteration) or FP32 (for the refinement's inner iteration, rounded
// once from the FP64 quotient)
template <bool TR, typename T>
__device__ __forceinline__ void scaled_row(const double *const *a, int idx, int i, int j, int k, int nx, int ny,
                                           int nz, int P, T (&o)[6]) {
    const bool e = i + 1 < nx, w = i > 0, nn = j + 1 < ny, ss = j > 0, up = k + 1 < nz, dn = k > 0;
    double c[6];
    if (!TR) {
        c[0] = e ? ld(a[1], idx) / ld(a[0], idx + 1) : 0.0;
        c[1] = w ? ld(a[2], idx) / ld(a[0], idx - 1) : 0.0;
        c[2] = nn ? ld(a[3], idx) / ld(a[0], idx + nx) : 0.0;
        c[3] = ss ? ld(a[4], idx) / ld(a[0], idx - nx) : 0.0;
        c[4] = up ? ld(a[5], idx) / ld(a[0], idx + P) : 0.0;
        c[5] = dn ? ld(a[6], idx) / ld(a[0], idx - P) : 0.0;
    } else {
        // row idx of A^T D^-1: the link to neighbour nb is row nb's coefficient towards idx, over a_P[nb]
        c[0] = e ? ld(a[2], idx + 1) / ld(a[0], idx + 1) : 0.0;
        c[1] = w ? ld(a[1], idx - 1) / ld(a[0], idx - 1) : 0.0;
        c[2] = nn ? ld(a[4], idx + nx) / ld(a[0], idx + nx) : 0.0;
        c[3] = ss ? ld(a[3], idx - nx) / ld(a[0], idx - nx) : 0.0;
        c[4] = up ? ld(a[6], idx + P) / ld(a[0], idx + P) : 0.0;
        c[5] = dn ? ld(a[5], idx - P) / ld(a[0], idx - P) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = (T)c[q];
}

// 1 if a link of cell idx = (i, j, k) towards W, S or B inside the grid differs from the
// neighbour's link back (a_W(c) != a_E(c-1) and so on), else 0
__device__ __forceinline__ double asym_row(const double *const *a, int idx, int i, int j, int k, int nx, int P) {
    const bool w = i > 0, ss = j > 0, dn = k > 0;
    const double wv = ld(a[2], idx), sv = ld(a[4], idx), bv = ld(a[6], idx);
    const double ev = ld(a[1], max(idx - 1, 0)), nv = ld(a[3], max(idx - nx, 0)), tv = ld(a[5], max(idx - P, 0));
    return ((w && wv != ev) || (ss && sv != nv) || (dn && bv != tv)) ? 1.0 : 0.0;
}

// sums: #asymmetric rows; the set takes the symmetric form of the single-sync step when
// there are none (and the form is enabled)
struct FinSym {
    int on;
    __device__ void operator()(SolveState *st, const double *s) const { st->sym = (on && s[0] == 0.0) ? 1 : 0; }
};

template <bool TR>
__global__ void __launch_bounds__(kBlock) scale_kernel(LaunchSets ls, int sym_on) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, n = d.n, nflat = d.nflat;
    const bool chk = !TR && sym_on;
    const double *a[7];
    double *as[6];
    double *dinv = d.dinv;
    for (int q = 0; q < 7; ++q) a[q] = d.a[q];
    for (int q = 0; q < 6; ++q) as[q] = d.as[q];
    double acc[1] = {0.0};
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int idx = base + kBlock * u;
            if (idx < n) {
                const int k = idx / P, q = idx - k * P, j = q / nx, i = q - j * nx;
                double o[6];
                scaled_row<TR>(a, idx, i, j, k, nx, ny, nz, P, o);
#pragma unroll
                for (int z = 0; z < 6; ++z) st(as[z], idx, o[z]);
                st(dinv, idx, 1.0 / ld(a[0], idx));
                if (chk) acc[0] += asym_row(a, idx, i, j, k, nx, P);
            }
        }
    }
    reduce_and_finalize<1>(d, tr.tile, nflat, acc, FinSym{chk ? 1 : 0});
}

// x = y / a_P for sets about to be rechecked or reported
__global__ void __launch_bounds__(kBlock) unscale_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->converged && !st_->need_report) return;
    const int n = d.n, nflat = d.nflat;
    const double *a0 = d.a[0], *y = d.y;
    double *x = d.x;
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        double Y[kFlatU], A[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            Y[u] = ld(y, i);
            A[u] = ld(a0, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) st(x, i, Y[u] / A[u]);
        }
    }
}

// FP32 coefficients of A D^-1 (each rounded to nearest once from the FP64
// quotient), (b, b), a_P check; with sym_on also the symmetry check and the
// FP32 a_E, a_N, a_T and 1/a_P of the symmetric form of the step
__global__ void __launch_bounds__(kBlock) cast_kernel(LaunchSets ls, int sym_on) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, n = d.n, nflat = d.nflat;
    const double *a[7];
    float *as32[6], *sy[4];
    for (int q = 0; q < 7; ++q) a[q] = d.a[q];
    for (int q = 0; q < 6; ++q) as32[q] = d.as32[q];
    for (int q = 0; q < 4; ++q) sy[q] = d.sym32[q];
    const double *bvec = d.b;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int idx = base + kBlock * u;
            if (idx < n) {
                const int k = idx / P, q = idx - k * P, j = q / nx, i = q - j * nx;
                float o[6];
                scaled_row<false>(a, idx, i, j, k, nx, ny, nz, P, o);
#pragma unroll
                for (int z = 0; z < 6; ++z) st(as32[z], idx, o[z]);
                const double ap = ld(a[0], idx), bv = ld(bvec, idx);
                acc[0] += bv * bv;
                acc[1] += (ap == 0.0 || !isfinite(ap)) ? 1.0 : 0.0;
                if (sym_on) {
                    st(sy[0], idx, (float)ld(a[1], idx));
                    st(sy[1], idx, (float)ld(a[3], idx));
                    st(sy[2], idx, (float)ld(a[5], idx));
                    st(sy[3], idx, (float)(1.0 / ap));
                    acc[2] += asym_row(a, idx, i, j, k, nx, P);
                }
            }
        }
    }
    reduce_and_finalize<3>(d, tr.tile, nflat, acc, FinCast{&d, sym_on});
}

// x += (d32 / scale) / a_P (FP64), for sets whose inner solve has finished
// (d32 is the inner iterate of the scaled system, D times the correction)
__global__ void __launch_bounds__(kBlock) update_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (st_->done || !st_->inner_done) return;
    const double is = st_->upd_inv_scale;
    const int n = d.n, nflat = d.nflat;
    double *xv = d.x;
    const float *dv = d.d32;
    const double *a0 = d.a[0];
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        double X[kFlatU], A[kFlatU];
        float D[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            X[u] = ld(xv, i);
            D[u] = ld(dv, i);
            A[u] = ld(a0, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) st(xv, i, X[u] + (is * (double)D[u]) / A[u]);
        }
    }
}

// x = 0 where b = 0 (flagged by setup), or unconditionally (force)
__global__ void __launch_bounds__(kBlock) zero_kernel(LaunchSets ls, int force) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    if (!force && !d.st->zero_rhs) return;
    const int n = d.n, nflat = d.nflat;
    double *xv = d.x;
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) st(xv, i, 0.0);
        }
    }
}

// The rows of A^T in the Patankar form of A: a_P on the diagonal, and the links of row c of A^T
// are the links pointing at c in the neighbouring rows of A, aT_E(c) = a_W(c+1), aT_W(c) = a_E(c-1),
// aT_N(c) = a_S(c+nx), aT_S(c) = a_N(c-nx), aT_T(c) = a_B(c+P), aT_B(c) = a_T(c-P) (0 where that
// neighbour is outside the grid).  Written into the set's six scaled-coefficient buffers, which the
// multigrid iteration does not use, so the multigrid solve of A^T x = b runs on them unchanged.
__global__ void __launch_bounds__(kBlock) transpose_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, n = d.n, nflat = d.nflat;
    const double *E = d.a[1], *Wc = d.a[2], *N = d.a[3], *S = d.a[4], *T = d.a[5], *B = d.a[6];
    double *o[6];
    for (int q = 0; q < 6; ++q) o[q] = d.as[q];
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int idx = base + kBlock * u;
            if (idx < n) {
                const int k = idx / P, q = idx - k * P, j = q / nx, i = q - j * nx;
                st(o[0], idx, i + 1 < nx ? ld(Wc, idx + 1) : 0.0);
                st(o[1], idx, i > 0 ? ld(E, idx - 1) : 0.0);
                st(o[2], idx, j + 1 < ny ? ld(S, idx + nx) : 0.0);
                st(o[3], idx, j > 0 ? ld(N, idx - nx) : 0.0);
                st(o[4], idx, k + 1 < nz ? ld(B, idx + P) : 0.0);
                st(o[5], idx, k > 0 ? ld(T, idx - P) : 0.0);
            }
        }
    }
}

// adjoint gradients: g_P = -lambda x; g_nb = lambda x_nb (0 out of the grid)
__global__ void __launch_bounds__(kBlock) grad_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const double *lam = d.x, *xf = d.xf;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, n = d.n, nflat = d.nflat;
    double *g[7];
    for (int s = 0; s < 7; ++s) g[s] = d.g[s];
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int idx = base + kBlock * u;
            if (idx < n) {
                const int k = idx / P, q = idx - k * P, j = q / nx, i = q - j * nx;
                const double l = ld(lam, idx);
                const double xc = ld(xf, idx);
                const double xE = i + 1 < nx ? ld(xf, idx + 1) : 0.0;
                const double xW = i > 0 ? ld(xf, idx - 1) : 0.0;
                const double xN = j + 1 < ny ? ld(xf, idx + nx) : 0.0;
                const double xS = j > 0 ? ld(xf, idx - nx) : 0.0;
                const double xT = k + 1 < nz ? ld(xf, idx + P) : 0.0;
                const double xB = k > 0 ? ld(xf, idx - P) : 0.0;
                if (g[0]) st(g[0], idx, -l * xc);
                if (g[1]) st(g[1], idx, l * xE);
                if (g[2]) st(g[2], idx, l * xW);
                if (g[3]) st(g[3], idx, l * xN);
                if (g[4]) st(g[4], idx, l * xS);
                if (g[5]) st(g[5], idx, l * xT);
                if (g[6]) st(g[6], idx, l * xB);
            }
        }
    }
}


// ------------------------------------------------------------------ one-block persistent solve (tiny sets)
//
// For a set of at most kSmallThreads * 4 cells, one 512-thread block runs the
// whole FP64 solve in a single launch: every cell's coefficients and vectors
// live in registers (cell c = tid + kSmallThreads * m), the stencil operand is
// exchanged through LDS, and the scalar updates are the same state-machine
// functions the multi-kernel path uses.  Several tiny sets of one call run as
// independent blocks of one launch.

constexpr int kSmallThreads = 512;  // 2 waves per SIMD: up to 256 VGPRs per lane for the register-resident vectors
constexpr int kSmallMaxCells = kSmallThreads * 4;

template <int NV>
__device__ __forceinline__ void small_block_sum(double (&v)[NV], double *red) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double t = 0.0;
            for (int w = 0; w < kSmallThreads / 64; ++w) t += red[w * NV + i];
            v[i] = t;
        }
    }
}

template <int CPC, bool TR>
__global__ void __launch_bounds__(kSmallThreads) small_kernel(LaunchSets ls) {
    const SetDesc &d = ls.desc[blockIdx.x];
    SolveState *st_ = d.st;
    const int nx = d.nx, ny = d.ny, nz = d.nz, P = d.plane, n = d.n;
    __shared__ double op[kSmallMaxCells];
    __shared__ double red[(kSmallThreads / 64) * 4];
    const double *a[7];
    for (int q = 0; q < 7; ++q) a[q] = d.a[q];
    const double *bp = d.b;
    double *xp = d.x, *rhp = d.rh;
    const int tid = threadIdx.x;

    // r, p, v and t of this thread's cells stay in registers; x, r^ and the
    // coefficients are read from L2 (the whole set is L2-resident) when needed
    double r[CPC], p[CPC], v[CPC], t[CPC];
#pragma unroll
    for (int m = 0; m < CPC; ++m) p[m] = v[m] = t[m] = r[m] = 0.0;
    auto valid = [&](int m) { return tid + kSmallThreads * m < n; };
    // A applied to the operand held in op[] at cell c of the m-th slot
    auto stencil = [&](int m) {
        const int c = min(tid + kSmallThreads * m, n - 1);
        const int k = c / P, q = c - k * P, j = q / nx, i = q - j * nx;
        const Nb nb{i + 1 < nx, i > 0, j + 1 < ny, j > 0};
        const bool up = k + 1 < nz, dn = k > 0;
        Coef6<double, TR> cf;
        cf.load(a, c, nx, P, n, nb, up, dn);
        const double xE = nb.e ? op[c + 1] : 0.0, xW = nb.w ? op[c - 1] : 0.0;
        const double xN = nb.n ? op[c + nx] : 0.0, xS = nb.s ? op[c - nx] : 0.0;
        const double xT = up ? op[c + P] : 0.0, xB = dn ? op[c - P] : 0.0;
        return cf.apply(ld(a[0], c), op[c], xE, xW, xN, xS, xT, xB);
    };
    auto diag = [&](int m) { return ld(a[0], min(tid + kSmallThreads * m, n - 1)); };
    // r = b - A x with setup semantics (mode 0), recheck (1) or report (2)
    auto residual = [&](int mode) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < CPC; ++m)
            if (valid(m)) op[tid + kSmallThreads * m] = ld(xp, tid + kSmallThreads * m);
        __syncthreads();
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < CPC; ++m) {
            if ((m & 3) == 0) __builtin_amdgcn_sched_barrier(0);
            if (!valid(m)) continue;
            const int c = tid + kSmallThreads * m;
            const double bv = ld(bp, c), apv = ld(a[0], c);
            const double rv = bv - stencil(m);
            if (mode != 2) {
                r[m] = rv;
                st(rhp, c, rv);
            }
            acc[0] += bv * bv;
            acc[1] += rv * rv;
            acc[2] += (apv == 0.0 || !isfinite(apv)) ? 1.0 : 0.0;
        }
        small_block_sum<3>(acc, red);
        if (tid == 0) {
            if (mode == 0) FinSetup{&d}(st_, acc);
            else if (mode == 1) FinRecheck{}(st_, acc);
            else FinReport{}(st_, acc);
        }
        __syncthreads();
    };

    residual(0);
    const long guard = 4l * (long)d.maxit + 16;
    for (long turn = 0; turn < guard; ++turn) {
        // keep the coefficient loads inside the loop (re-read from L2 each pass)
        // rather than hoisted into registers for all cells
        __asm__ volatile("" ::: "memory");
        if (st_->done) break;
        if (st_->converged) { residual(1); continue; }
        if (st_->need_report) { residual(2); continue; }
        if (!st_->active) break;
        // K1: p update, p^ = p / a_P into LDS, v = A p^, (r^, v)
        const bool fresh = st_->fresh != 0;
        const double beta = (st_->rho / st_->rho_prev) * (st_->alpha / st_->omega), omega0 = st_->omega;
#pragma unroll
        for (int m = 0; m < CPC; ++m) {
            p[m] = fresh ? r[m] : fma(beta, fma(-omega0, v[m], p[m]), r[m]);
            if (valid(m)) {
                op[tid + kSmallThreads * m] = p[m] / diag(m);
                if (fresh) st(rhp, tid + kSmallThreads * m, r[m]);
            }
        }
        __syncthreads();
        double a1[1] = {0.0};
#pragma unroll
        for (int m = 0; m < CPC; ++m) {
            if (valid(m)) {
                v[m] = stencil(m);
                a1[0] += ld(rhp, tid + kSmallThreads * m) * v[m];
            }
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight (registers)
        }
        small_block_sum<1>(a1, red);
        if (tid == 0) FinK1{}(st_, a1);
        __syncthreads();
        if (!st_->active) continue;
        // K2: s = r - alpha v, s^ into LDS (after every thread has read p^), t = A s^
        const double alpha = st_->alpha;
#pragma unroll
        for (int m = 0; m < CPC; ++m)
            if (valid(m)) op[tid + kSmallThreads * m] = fma(-alpha, v[m], r[m]) / diag(m);
        __syncthreads();
        double a2[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < CPC; ++m) {
            if (valid(m)) {
                const double sv = fma(-alpha, v[m], r[m]);
                t[m] = stencil(m);
                a2[0] += t[m] * sv;
                a2[1] += t[m] * t[m];
                a2[2] += sv * sv;
            }
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        small_block_sum<3>(a2, red);
        if (tid == 0) FinK2{}(st_, a2);
        __syncthreads();
        if (!st_->active) continue;
        // K3: x += alpha p^ + omega s^, r = s - omega t, (r^, r), (r, r)
        const double om = st_->omega;
        double a3[2] = {0.0, 0.0};
#pragma unroll
        for (int m = 0; m < CPC; ++m) {
            if (!valid(m)) continue;
            const int c = tid + kSmallThreads * m;
            const double apv = diag(m), sv = fma(-alpha, v[m], r[m]);
            st(xp, c, ld(xp, c) + fma(alpha, p[m] / apv, om * (sv / apv)));
            r[m] = fma(-om, t[m], sv);
            a3[0] += ld(rhp, c) * r[m];
            a3[1] += r[m] * r[m];
        }
        small_block_sum<2>(a3, red);
        if (tid == 0) FinK3{}(st_, a3);
        __syncthreads();
    }
    if (st_->zero_rhs) {
#pragma unroll
        for (int m = 0; m < CPC; ++m)
            if (valid(m)) st(xp, tid + kSmallThreads * m, 0.0);
    }
}

// p[0..n) = v (synthetic systems for the tuner)
__global__ void __launch_bounds__(kBlock) fill_kernel(double *p, long n, double v) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) p[i] = v;
}

// ------------------------------------------------------------------ multigrid preconditioner
//
// Aggregation V-cycle B^{-1} (right preconditioner of the FP64 solve).  Level
// l + 1 aggregates the cells (i, j, k) of level l with equal (i/2, j/2, k/2);
// interpolation is piecewise constant, restriction its transpose (the sum
// over an aggregate), the coarse operators are the Galerkin products (again
// 7-point).  V-cycle on level l with right-hand side r, D = diag(a_P):
//   coarsest level: z = 0, then coarse_sweeps times z += omega D^-1 (r - A z)
//   otherwise:      z1 = omega D^-1 r; e = V-cycle(l+1, R (r - A z1));
//                   z2 = z1 + gamma P e;  z = z2 + omega D^-1 (r - A z2)
// The kernels take the operations in that order, with FMA contraction off,
// and sum an aggregate's cells in index order, so the V-cycle equals a plain
// sequential evaluation of the definition to the last bit.

// the coefficients of level l as the V-cycle sees them: level 0 from its FP32 copy
// (widened exactly to FP64), coarser levels from their FP64 Galerkin arrays
// A level's coefficients.  Where the level-0 matrix is exactly symmetric (st->sym), every coarse
// level is too, bit for bit: a coarse a_E and the a_W of the next coarse cell sum the same fine
// links (a_W(c) = a_E(c-1)) in the same order.  Coarse levels then read W, S and B as the E, N
// and T coefficients of the neighbouring cell (sym), four coefficient streams instead of seven.
// A W/S/B coefficient is only read for a neighbour inside the grid.
struct LevCoef {
    const double *d[7];
    const float *f[7];
    bool f32, sym;
    int nx, P;
    __device__ __forceinline__ double operator()(int q, int c) const {
        if (f32) return (double)ld(f[q], c);
        if (q == 2 || q == 4 || q == 6) {
            const int off = q == 2 ? 1 : (q == 4 ? nx : P);
            return sym ? ld(d[q - 1], c - off) : ld(d[q], c);
        }
        return ld(d[q], c);
    }
};

__device__ __forceinline__ LevCoef mg_coef(const MgLevel &L, int l, bool sym = false) {
    LevCoef k;
    k.f32 = l == 0;
    k.sym = sym && l > 0;
    k.nx = L.nx;
    k.P = L.nx * L.ny;
    for (int q = 0; q < 7; ++q) {
        k.d[q] = L.a[q];
        k.f[q] = L.a32[q];
    }
    return k;
}

// row c = (i, j, k) of A applied to x: a_P x_c, then minus each present
// neighbour's term in the order E, W, N, S, T, B; xat(cell, i, j, k) gives x
template <class F>
__device__ __forceinline__ double mg_row(const LevCoef &a, int nx, int ny, int nz, int i, int j, int k, int c,
                                         F xat) {
#pragma clang fp contract(off)
    const int P = nx * ny;
    double acc = a(0, c) * xat(c, i, j, k);
    if (i + 1 < nx) acc -= a(1, c) * xat(c + 1, i + 1, j, k);
    if (i > 0) acc -= a(2, c) * xat(c - 1, i - 1, j, k);
    if (j + 1 < ny) acc -= a(3, c) * xat(c + nx, i, j + 1, k);
    if (j > 0) acc -= a(4, c) * xat(c - nx, i, j - 1, k);
    if (k + 1 < nz) acc -= a(5, c) * xat(c + P, i, j, k + 1);
    if (k > 0) acc -= a(6, c) * xat(c - P, i, j, k - 1);
    return acc;
}

// exact symmetry of the set's matrix, once per solve: st->sym = on, then cleared by any block
// that finds a pair inside the grid with a_W(c) != a_E(c-1), a_S(c) != a_N(c-nx) or
// a_B(c) != a_T(c-P) (coefficients pointing out of the grid are never used)
__global__ void mg_symflag_kernel(const SetDesc *d, int on) {
    if (blockIdx.x == 0 && threadIdx.x == 0) d->st->sym = on;
}

__global__ void __launch_bounds__(kBlock) mg_symcheck_kernel(const SetDesc *d) {
    const int nx = d->nx, n = d->n, P = d->plane;
    const double *E = d->a[1], *W = d->a[2], *N = d->a[3], *S = d->a[4], *T = d->a[5], *B = d->a[6];
    int bad = 0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < n; c += gridDim.x * kBlock) {
        const int k = c / P, q = c - k * P, j = q / nx, i = q - j * nx;
        if (i > 0 && ld(W, c) != ld(E, c - 1)) bad = 1;
        if (j > 0 && ld(S, c) != ld(N, c - nx)) bad = 1;
        if (k > 0 && ld(B, c) != ld(T, c - P)) bad = 1;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicAnd(&d->st->sym, 0);
}

// level 0's FP32 copy of the set's coefficients (round to nearest), once per solve
__global__ void __launch_bounds__(kBlock) mg_round0_kernel(const SetDesc *d, const MgLevel *lev) {
    const MgLevel F = lev[0];
    const double *a[7];
    for (int q = 0; q < 7; ++q) a[q] = d->a[q];
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < F.n; c += gridDim.x * kBlock)
#pragma unroll
        for (int q = 0; q < 7; ++q) st(F.a32[q], c, (float)ld(a[q], c));
}

// Galerkin coarse operator of level l + 1, one thread per coarse cell
__global__ void __launch_bounds__(kBlock) mg_coarsen_kernel(const SetDesc *d, const MgLevel *lev, int l) {
#pragma clang fp contract(off)
    const MgLevel F = lev[l], C = lev[l + 1];
    const LevCoef a = mg_coef(F, l);
    const int nx = F.nx, ny = F.ny, nz = F.nz, cx = C.nx, cy = C.ny;
    for (int cc = blockIdx.x * kBlock + threadIdx.x; cc < C.n; cc += gridDim.x * kBlock) {
        const int I = cc % cx, t = cc / cx, J = t % cy, K = t / cy;
        double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 2 * K; k < min(2 * K + 2, nz); ++k)
            for (int j = 2 * J; j < min(2 * J + 2, ny); ++j)
                for (int i = 2 * I; i < min(2 * I + 2, nx); ++i) {
                    const int c = i + nx * (j + ny * k);
                    acc[0] += a(0, c);
                    const int ni[6] = {i + 1, i - 1, i, i, i, i};
                    const int nj[6] = {j, j, j + 1, j - 1, j, j};
                    const int nk[6] = {k, k, k, k, k + 1, k - 1};
                    for (int dd = 0; dd < 6; ++dd) {
                        if (ni[dd] < 0 || ni[dd] >= nx || nj[dd] < 0 || nj[dd] >= ny || nk[dd] < 0 || nk[dd] >= nz)
                            continue;
                        const double coef = a(1 + dd, c);
                        if (ni[dd] / 2 == I && nj[dd] / 2 == J && nk[dd] / 2 == K)
                            acc[0] -= coef;  // link inside the aggregate
                        else
                            acc[1 + dd] += coef;
                    }
                }
        for (int q = 0; q < 7; ++q) st(C.a[q], cc, acc[q]);
    }
}

// R (r - A z1) with z1 = omega D^-1 r, into level l + 1's right-hand side.
// Eight consecutive lanes take the eight cells of one aggregate (lane bits:
// i, j, k offsets), so a wave reads rows of 16 consecutive cells; lane 0 of
// the group sums the group's values in cell-index order (the definition's).
// gt: the thread's index among the nt threads taking the level; out(cc, sum) stores a coarse value
template <class Out>
__device__ __forceinline__ void mg_restrict_body(const MgLevel &F, const MgLevel &C, const LevCoef &a,
                                                 const double *rin, double w, int gt, int nt, Out out) {
#pragma clang fp contract(off)
    const int nx = F.nx, ny = F.ny, nz = F.nz, cx = C.nx, cy = C.ny;
    auto z1 = [&](int x, int, int, int) { return w * ld(rin, x) / a(0, x); };
    const int g8 = gt & 7, di = g8 & 1, dj = (g8 >> 1) & 1, dk = g8 >> 2;
    const int stride = nt >> 3;
    // the loop bound is uniform over a wave (the shuffles need every lane of a group)
    for (int w0 = (gt & ~63) >> 3; w0 < C.n; w0 += stride) {
        const int cc = w0 + ((gt & 63) >> 3);
        const bool inC = cc < C.n;
        const int ccl = min(cc, C.n - 1);
        const int I = ccl % cx, t = ccl / cx, J = t % cy, K = t / cy;
        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
        const bool ok = inC && i < nx && j < ny && k < nz;
        double q = 0.0;
        if (ok) {
            const int c = i + nx * (j + ny * k);
            q = ld(rin, c) - mg_row(a, nx, ny, nz, i, j, k, c, z1);
        }
        double qs[8];
        int oks[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            qs[m] = __shfl(q, m, 8);
            oks[m] = __shfl(ok ? 1 : 0, m, 8);
        }
        if (g8 == 0 && inC) {
            double sum = 0.0;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (oks[m]) sum += qs[m];
            out(cc, sum);
        }
    }
}

// The coarse-level kernels take the sets of a launch along blockIdx.y (set blockIdx.y of the
// table `desc`, its level table at lev + blockIdx.y * kMgMaxLevels, its level count in cnt); a set
// without the level returns at once.

// a V-cycle's input (which = 0: p, 1: s, 2: the diagnostic's r) and output (p^, s^, t)
__device__ __forceinline__ const double *mg_in(const SetDesc &d, int which) {
    return which == 0 ? d.p[0] : (which == 1 ? d.s1 : d.r);
}
__device__ __forceinline__ double *mg_out(const SetDesc &d, int which) {
    return which == 0 ? d.p[1] : (which == 1 ? d.v[1] : d.t);
}

__global__ void __launch_bounds__(kBlock) mg_restrict_kernel(const SetDesc *desc, const MgLevel *levs, MgCounts cnt,
                                                             int l, MgParams prm, int gated) {
    if (l > cnt.n[blockIdx.y] - 2) return;
    const SetDesc *d = desc + blockIdx.y;
    const MgLevel *lev = levs + (size_t)blockIdx.y * kMgMaxLevels;
    if (gated && !d->st->active) return;
    const MgLevel F = lev[l], C = lev[l + 1];
    const LevCoef a = mg_coef(F, l, prm.coarse_sym && d->st->sym != 0);
    double *cr = C.r;
    mg_restrict_body(F, C, a, F.r, prm.omega, (int)(blockIdx.x * kBlock + threadIdx.x), (int)(gridDim.x * kBlock),
                     [&](int cc, double v) { st(cr, cc, v); });
}

// z = z2 + omega D^-1 (r - A z2) with z2 = omega D^-1 r + gamma P e, e = level l + 1's result
// eat(cc) gives the coarse level's result at coarse cell cc
template <class E>
__device__ __forceinline__ void mg_prolong_body(const MgLevel &F, const MgLevel &C, const LevCoef &a,
                                                const double *rin, double *zout, double w, double gm, int gt,
                                                int nt, E eat) {
#pragma clang fp contract(off)
    const int nx = F.nx, ny = F.ny, nz = F.nz, cx = C.nx, cy = C.ny;
    auto z2 = [&](int x, int i, int j, int k) {
        return w * ld(rin, x) / a(0, x) + gm * eat(i / 2 + cx * (j / 2 + cy * (k / 2)));
    };
    for (int c = gt; c < F.n; c += nt) {
        const int i = c % nx, t = c / nx, j = t % ny, k = t / ny;
        const double q = mg_row(a, nx, ny, nz, i, j, k, c, z2);
        st(zout, c, z2(c, i, j, k) + w * (ld(rin, c) - q) / a(0, c));
    }
}

__global__ void __launch_bounds__(kBlock) mg_prolong_kernel(const SetDesc *desc, const MgLevel *levs, MgCounts cnt,
                                                            int l, MgParams prm, int gated) {
    if (l > cnt.n[blockIdx.y] - 2) return;
    const SetDesc *d = desc + blockIdx.y;
    const MgLevel *lev = levs + (size_t)blockIdx.y * kMgMaxLevels;
    if (gated && !d->st->active) return;
    const MgLevel F = lev[l], C = lev[l + 1];
    const LevCoef a = mg_coef(F, l, prm.coarse_sym && d->st->sym != 0);
    const double *e = C.z;
    mg_prolong_body(F, C, a, F.r, F.z, prm.omega, prm.gamma, (int)(blockIdx.x * kBlock + threadIdx.x),
                    (int)(gridDim.x * kBlock), [&](int cc) { return ld(e, cc); });
}

// coarsest level: coarse_sweeps damped-Jacobi sweeps from zero in one block;
// a thread keeps its cells' coefficients and right-hand side in registers
constexpr int kMgCoarseThreads = 1024;
constexpr int kMgCoarseCells = kMgCoarsestMax / kMgCoarseThreads;
// rat(c): the level's right-hand side at cell c; the result is left in zb[returned slot]
template <class R>
__device__ __forceinline__ int mg_coarsest_body(const MgLevel &F, const LevCoef &a, double w, int sweeps,
                                                double (*zb)[kMgCoarsestMax], R rat) {
#pragma clang fp contract(off)
    const int nx = F.nx, ny = F.ny, nz = F.nz, n = F.n, P = nx * ny;
    double co[kMgCoarseCells][7], rr[kMgCoarseCells];
    int cell[kMgCoarseCells];
    bool has[kMgCoarseCells][6];
#pragma unroll
    for (int m = 0; m < kMgCoarseCells; ++m) {
        const int c = threadIdx.x + kMgCoarseThreads * m;
        cell[m] = c;
        const int cl = min(c, n - 1);
        const int i = cl % nx, t = cl / nx, j = t % ny, k = t / ny;
        has[m][0] = i + 1 < nx;
        has[m][1] = i > 0;
        has[m][2] = j + 1 < ny;
        has[m][3] = j > 0;
        has[m][4] = k + 1 < nz;
        has[m][5] = k > 0;
        co[m][0] = a(0, cl);
        for (int q = 1; q < 7; ++q) co[m][q] = has[m][q - 1] ? a(q, cl) : 0.0;  // (unused where absent)
        rr[m] = rat(cl);
        if (c < n) zb[0][c] = 0.0;
    }
    __syncthreads();
    const int off[6] = {1, -1, nx, -nx, P, -P};
    int cur = 0;
    for (int it = 0; it < sweeps; ++it) {
        const double *zc = zb[cur];
#pragma unroll
        for (int m = 0; m < kMgCoarseCells; ++m) {
            const int c = cell[m];
            if (c < n) {
                double acc = co[m][0] * zc[c];  // a_P z, then E, W, N, S, T, B in order
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    if (has[m][q]) acc -= co[m][1 + q] * zc[c + off[q]];
                zb[cur ^ 1][c] = zc[c] + w * (rr[m] - acc) / co[m][0];
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

// one block per set (set blockIdx.x), each on its own coarsest level
__global__ void __launch_bounds__(kMgCoarseThreads) mg_coarsest_kernel(const SetDesc *desc, const MgLevel *levs,
                                                                       MgCounts cnt, int which, MgParams prm,
                                                                       int gated) {
    const SetDesc *d = desc + blockIdx.x;
    if (gated && !d->st->active) return;
    __shared__ double zb[2][kMgCoarsestMax];
    const MgLevel *lev = levs + (size_t)blockIdx.x * kMgMaxLevels;
    const int l = cnt.n[blockIdx.x] - 1;
    const MgLevel F = lev[l];
    const double *rin = l == 0 ? mg_in(*d, which) : F.r;
    double *zout = l == 0 ? mg_out(*d, which) : F.z;
    const LevCoef a = mg_coef(F, l, prm.coarse_sym && d->st->sym != 0);
    const int cur = mg_coarsest_body(F, a, prm.omega, prm.coarse_sweeps, zb, [&](int c) { return ld(rin, c); });
    for (int c = threadIdx.x; c < F.n; c += kMgCoarseThreads) st(zout, c, zb[cur][c]);
}

// ---- finest level through the k-march (operands staged in LDS like the
// iteration's stencil passes): the residual of the pre-smoothed iterate, and
// the prolongation with its smoothing step.  Same operations and order as the
// per-cell kernels above (an absent neighbour's coefficient is zero, so its
// term subtracts an exact zero).

// q = r - A z1 with z1 = omega D^-1 r, per cell (summed over aggregates by mg_aggregate_kernel).
// With sfused the V-cycle's input is the iteration's s = r - alpha v, formed here from r and v (the
// operation of pc_s_kernel, the same bits) on every cell the pass reads, and stored for the own
// cells (the prolongation and the products read it later): one pass less per iteration.
struct PhMgResid {
    static constexpr int NV = 1;
    struct Raw { double r, v, ap; };
    struct Aux { double r, ap; };
    struct Pre { Coef6<float, false> c; };  // level 0's FP32 coefficients, widened in use
    const float *a[7];
    const double *rin, *vin;
    double *res, *sout;
    double w, al;
    bool sym, sfused;
    int nx, P, ncell;
    __device__ __forceinline__ Raw load(int idx, int, int) const {
        return Raw{ld(rin, idx), sfused ? ld(vin, idx) : 0.0, ld(a[0], idx)};
    }
    __device__ __forceinline__ double rval(const Raw &v) const { return sfused ? fma(-al, v.v, v.r) : v.r; }
    __device__ __forceinline__ double zval(const Raw &v) const {
#pragma clang fp contract(off)
        return w * rval(v) / v.ap;
    }
    __device__ __forceinline__ double own(const Raw &v, int idx, Aux &ax) {
        ax.r = rval(v);
        ax.ap = v.ap;
        if (sfused) st(sout, idx, ax.r);
        return zval(v);
    }
    __device__ __forceinline__ double halo(const Raw &v) const { return zval(v); }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        load_row6(pr.c, a, idx, nx, P, nb, up, dn, sym);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &ax, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&)[NV]) {
#pragma clang fp contract(off)
        double q = ax.ap * xc;
        q -= pr.c.e * xE;
        q -= pr.c.w * xW;
        q -= pr.c.n * xN;
        q -= pr.c.s * xS;
        q -= pr.c.t * xT;
        q -= pr.c.b * xB;
        st(res, idx, ax.r - q);
    }
};

// z = z2 + omega D^-1 (r - A z2) with z2 = omega D^-1 r + gamma e(aggregate)
struct PhMgProlong {
    static constexpr int NV = 1;
    struct Raw { double r, ap, e; };
    struct Aux { double r, ap; };
    struct Pre { Coef6<float, false> c; };  // level 0's FP32 coefficients, widened in use
    const float *a[7];
    const double *rin, *e;
    double *zout;
    double w, g;
    bool sym;
    int nx, P, ncell, cx, cy;
    __device__ __forceinline__ Raw load(int idx, int q, int k) const {
        const int j = q / nx, i = q - j * nx;
        return Raw{ld(rin, idx), ld(a[0], idx), ld(e, (i >> 1) + cx * ((j >> 1) + cy * (k >> 1)))};
    }
    __device__ __forceinline__ double zval(const Raw &v) const {
#pragma clang fp contract(off)
        return w * v.r / v.ap + g * v.e;
    }
    __device__ __forceinline__ double own(const Raw &v, int, Aux &ax) {
        ax.r = v.r;
        ax.ap = v.ap;
        return zval(v);
    }
    __device__ __forceinline__ double halo(const Raw &v) const { return zval(v); }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        load_row6(pr.c, a, idx, nx, P, nb, up, dn, sym);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &ax, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&)[NV]) {
#pragma clang fp contract(off)
        double q = ax.ap * xc;
        q -= pr.c.e * xE;
        q -= pr.c.w * xW;
        q -= pr.c.n * xN;
        q -= pr.c.s * xS;
        q -= pr.c.t * xT;
        q -= pr.c.b * xB;
        st(zout, idx, xc + w * (ax.r - q) / ax.ap);
    }
};

template <int CPT, int H>
__global__ void __launch_bounds__(kBlock) mg_resid0_kernel(LaunchSets ls, const MgLevel *levs, MgCounts cnt, int which,
                                                           MgParams prm, int gated) {
    const TileRef tr = locate<false>(ls);
    const int si = (int)(tr.d - ls.desc);
    if (cnt.n[si] < 2) return;
    const SetDesc &d = *tr.d;
    const MgLevel *lev = levs + (size_t)si * kMgMaxLevels;
    if (gated && !d.st->active) return;
    PhMgResid ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = lev[0].a32[k];
    ph.sym = d.st->sym != 0;
    // the s-cycle of the iteration forms s = r - alpha v itself (pc_s_kernel skips such sets)
    ph.sfused = which == 1;
    ph.rin = ph.sfused ? d.r : mg_in(d, which);
    ph.vin = d.v[0];
    ph.sout = d.s1;
    ph.al = d.st->alpha;
    ph.res = d.y;  // the per-cell residual (the y buffer is unused by this iteration)
    ph.w = prm.omega;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[1] = {0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
}

template <int CPT, int H>
__global__ void __launch_bounds__(kBlock) mg_prolong0_kernel(LaunchSets ls, const MgLevel *levs, MgCounts cnt,
                                                             int which, MgParams prm, int gated) {
    const TileRef tr = locate<false>(ls);
    const int si = (int)(tr.d - ls.desc);
    if (cnt.n[si] < 2) return;
    const SetDesc &d = *tr.d;
    const MgLevel *lev = levs + (size_t)si * kMgMaxLevels;
    if (gated && !d.st->active) return;
    PhMgProlong ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = lev[0].a32[k];
    ph.sym = d.st->sym != 0;
    ph.rin = mg_in(d, which);
    ph.e = lev[1].z;
    ph.zout = mg_out(d, which);
    ph.w = prm.omega;
    ph.g = prm.gamma;
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    ph.cx = lev[1].nx;
    ph.cy = lev[1].ny;
    double acc[1] = {0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
}

// level 1's right-hand side: the sum of res over each aggregate of level 0, in
// cell-index order (i fastest, then j, then k), one thread per aggregate
__global__ void __launch_bounds__(kBlock) mg_aggregate_kernel(const SetDesc *desc, const MgLevel *levs, MgCounts cnt,
                                                              int gated) {
#pragma clang fp contract(off)
    if (cnt.n[blockIdx.y] < 2) return;
    const SetDesc *d = desc + blockIdx.y;
    const MgLevel *lev = levs + (size_t)blockIdx.y * kMgMaxLevels;
    if (gated && !d->st->active) return;
    const double *res = d->y;
    const MgLevel F = lev[0], C = lev[1];
    const int nx = F.nx, ny = F.ny, nz = F.nz, cx = C.nx, cy = C.ny;
    for (int cc = blockIdx.x * kBlock + threadIdx.x; cc < C.n; cc += gridDim.x * kBlock) {
        const int I = cc % cx, t = cc / cx, J = t % cy, K = t / cy;
        double sum = 0.0;
        for (int k = 2 * K; k < min(2 * K + 2, nz); ++k)
            for (int j = 2 * J; j < min(2 * J + 2, ny); ++j)
                for (int i = 2 * I; i < min(2 * I + 2, nx); ++i) sum += ld(res, i + nx * (j + ny * k));
        st(C.r, cc, sum);
    }
}

// ---- BiCGSTAB with the V-cycle as right preconditioner (FP64, original A, x updated in place).
// Buffers: p = p[0], v = v[0], p^ = p[1], s = s1, s^ = v[1], t, r, r^; the finalisers are
// those of the three-launch iteration (FinK1: alpha; FinK2: omega and the half-step exit;
// FinK3: convergence, rho and restarts).

// p = r + beta (p - omega v); at a fresh start p = r and r^ = r
__global__ void __launch_bounds__(kBlock) pc_p_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    const bool fresh = st_->fresh != 0;
    const double beta = (st_->rho / st_->rho_prev) * (st_->alpha / st_->omega), om = st_->omega;
    const double *r = d.r, *v = d.v[0];
    double *p = d.p[0], *rh = d.rh;
    const int n = d.n, nflat = d.nflat;
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        double R[kFlatU], Pv[kFlatU], V[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            R[u] = ld(r, i);
            Pv[u] = ld(p, i);
            V[u] = ld(v, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) {
                st(p, i, fresh ? R[u] : fma(beta, fma(-om, V[u], Pv[u]), R[u]));
                if (fresh) st(rh, i, R[u]);
            }
        }
    }
}

// stencil operand x at a cell for the products of the preconditioned iteration
struct PhPc {
    static constexpr int NV = 3;
    using Raw = RawX;
    struct Aux {};
    struct Pre { Coef6<double, false> c; double ap, w; };
    const double *a[7];
    const double *x, *wv;  // operand; second vector of the sums ((r^) for v, (s) for t)
    double *y;
    int nx, P, ncell;
    bool tstep;
    bool sym;              // exactly symmetric matrix: W, S, B read as E, N, T of the neighbour            // false: v = A p^, sum (r^, v); true: t = A s^, sums (t,s), (t,t), (s,s)
    __device__ __forceinline__ Raw load(int idx, int, int) const { return Raw{ld(x, idx)}; }
    __device__ __forceinline__ double own(const Raw &w, int, Aux &) { return w.x; }
    __device__ __forceinline__ double halo(const Raw &w) const { return w.x; }
    __device__ __forceinline__ void pre(int idx, Nb nb, bool up, bool dn, Pre &pr) const {
        load_row6(pr.c, a, idx, nx, P, nb, up, dn, sym);
        pr.ap = ld(a[0], idx);
        pr.w = ld(wv, idx);
    }
    __device__ __forceinline__ void center(int idx, const Pre &pr, const Aux &, double xc, double xE, double xW,
                                           double xN, double xS, double xT, double xB, double (&acc)[NV]) {
        const double yv = pr.c.apply(pr.ap, xc, xE, xW, xN, xS, xT, xB);
        st(y, idx, yv);
        if (!tstep) {
            acc[0] += pr.w * yv;
        } else {
            acc[0] += yv * pr.w;
            acc[1] += yv * yv;
            acc[2] += pr.w * pr.w;
        }
    }
};

template <int CPT, int H>
__global__ void __launch_bounds__(kBlock) pc_prod_kernel(LaunchSets ls, int tstep) {
    const TileRef tr = locate<false>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    PhPc ph;
    for (int k = 0; k < 7; ++k) ph.a[k] = d.a[k];
    ph.tstep = tstep != 0;
    ph.sym = st_->sym != 0;
    ph.x = ph.tstep ? d.v[1] : d.p[1];
    ph.wv = ph.tstep ? d.s1 : d.rh;
    ph.y = ph.tstep ? d.t : d.v[0];
    ph.nx = d.nx;
    ph.P = d.plane;
    ph.ncell = d.n;
    double acc[3] = {0.0, 0.0, 0.0};
    march<double, CPT, H>(ph, geo_of(d), tr.tile, lds_base<double>(), acc);
    if (ph.tstep) {
        reduce_and_finalize<3>(d, tr.tile, d.ntiles, acc, FinK2{});
    } else {
        double sig[1] = {acc[0]};
        reduce_and_finalize<1>(d, tr.tile, d.ntiles, sig, FinK1{});
    }
}

// s = r - alpha v (only for sets whose V-cycle has no finest-level pass, i.e. a single level: the
// others form s in the V-cycle's residual pass)
__global__ void __launch_bounds__(kBlock) pc_s_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active || d.mg_levels >= 2) return;
    const double al = st_->alpha;
    const double *r = d.r, *v = d.v[0];
    double *s = d.s1;
    const int n = d.n, nflat = d.nflat;
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        double R[kFlatU], V[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            R[u] = ld(r, i);
            V[u] = ld(v, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) st(s, i, fma(-al, V[u], R[u]));
        }
    }
}

// x += alpha p^ + omega s^; r = s - omega t; (r^, r), (r, r)
__global__ void __launch_bounds__(kBlock) pc_x_kernel(LaunchSets ls) {
    const TileRef tr = locate<true>(ls);
    const SetDesc &d = *tr.d;
    const SolveState *st_ = d.st;
    if (!st_->active) return;
    const double al = st_->alpha, om = st_->omega;
    const double *ph = d.p[1], *sh = d.v[1], *s = d.s1, *t = d.t, *rh = d.rh;
    double *x = d.x, *r = d.r;
    const int n = d.n, nflat = d.nflat;
    double acc[2] = {0.0, 0.0};
    for (int ch = tr.tile; ch * kFlatChunk < n; ch += nflat) {
        const int base = ch * kFlatChunk + (int)threadIdx.x;
        double X[kFlatU], PH[kFlatU], SH[kFlatU], S[kFlatU], Tt[kFlatU], RH[kFlatU];
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = min(base + kBlock * u, n - 1);
            X[u] = ld(x, i); PH[u] = ld(ph, i); SH[u] = ld(sh, i);
            S[u] = ld(s, i); Tt[u] = ld(t, i); RH[u] = ld(rh, i);
        }
#pragma unroll
        for (int u = 0; u < kFlatU; ++u) {
            const int i = base + kBlock * u;
            if (i < n) {
                st(x, i, X[u] + fma(al, PH[u], om * SH[u]));
                const double rn = fma(-om, Tt[u], S[u]);
                st(r, i, rn);
                acc[0] += RH[u] * rn;
                acc[1] += rn * rn;
            }
        }
    }
    reduce_and_finalize<2>(d, tr.tile, nflat, acc, FinK3{});
}

// ------------------------------------------------------------------ host launchers

hipError_t launch_small(const LaunchSets &ls, int max_n, bool trans, hipStream_t stream) {
    const dim3 grid(ls.nsets), block(kSmallThreads);
    const int cpc = (max_n + kSmallThreads - 1) / kSmallThreads;
    if (max_n > kSmallMaxCells || cpc < 1) return hipErrorInvalidValue;
    if (cpc == 1) {
        if (trans) hipLaunchKernelGGL((small_kernel<1, true>), grid, block, 0, stream, ls);
        else hipLaunchKernelGGL((small_kernel<1, false>), grid, block, 0, stream, ls);
    } else if (cpc == 2) {
        if (trans) hipLaunchKernelGGL((small_kernel<2, true>), grid, block, 0, stream, ls);
        else hipLaunchKernelGGL((small_kernel<2, false>), grid, block, 0, stream, ls);
    } else {
        if (trans) hipLaunchKernelGGL((small_kernel<4, true>), grid, block, 0, stream, ls);
        else hipLaunchKernelGGL((small_kernel<4, false>), grid, block, 0, stream, ls);
    }
    return hipGetLastError();
}

static dim3 mg_grid(int n) { return dim3((unsigned)std::max(1, std::min((n + kBlock - 1) / kBlock, 8192))); }

hipError_t launch_mg_symcheck(const SetDesc *d, int n, int on, hipStream_t stream) {
    hipLaunchKernelGGL(mg_symflag_kernel, dim3(1), dim3(64), 0, stream, d, on);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !on) return e;
    hipLaunchKernelGGL(mg_symcheck_kernel, mg_grid(n), dim3(kBlock), 0, stream, d);
    return hipGetLastError();
}

hipError_t launch_mg_round0(const SetDesc *d, const MgLevel *lev, int n, hipStream_t stream) {
    hipLaunchKernelGGL(mg_round0_kernel, mg_grid(n), dim3(kBlock), 0, stream, d, lev);
    return hipGetLastError();
}

hipError_t launch_mg_coarsen(const SetDesc *d, const MgLevel *lev, int l, int nc, hipStream_t stream) {
    hipLaunchKernelGGL(mg_coarsen_kernel, mg_grid(nc), dim3(kBlock), 0, stream, d, lev, l);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int l, int nc,
                              MgParams prm, bool gated, hipStream_t stream) {
    // eight lanes per coarse cell of the largest set's level l + 1
    dim3 grid = mg_grid(8 * nc);
    grid.y = (unsigned)nsets;
    hipLaunchKernelGGL(mg_restrict_kernel, grid, dim3(kBlock), 0, stream, desc, levs, cnt, l, prm, gated ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_mg_coarsest(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int which,
                              MgParams prm, bool gated, hipStream_t stream) {
    hipLaunchKernelGGL(mg_coarsest_kernel, dim3((unsigned)nsets), dim3(kMgCoarseThreads), 0, stream, desc, levs, cnt,
                       which, prm, gated ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_mg_prolong(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int l, int n,
                             MgParams prm, bool gated, hipStream_t stream) {
    dim3 grid = mg_grid(n);
    grid.y = (unsigned)nsets;
    hipLaunchKernelGGL(mg_prolong_kernel, grid, dim3(kBlock), 0, stream, desc, levs, cnt, l, prm, gated ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, long n, double v, hipStream_t stream) {
    hipLaunchKernelGGL(fill_kernel, dim3(2048), dim3(kBlock), 0, stream, p, n, v);
    return hipGetLastError();
}

size_t march_lds_bytes(int cpt, int max_nx, int elem) {
    return (size_t)3 * (size_t)(kBlock * cpt + 2 * max_nx) * (size_t)elem;
}

int halo_slots(int max_nx, int nt) {
    const int need = (2 * max_nx + nt - 1) / nt;
    return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : -1;
}

size_t fused_lds_bytes(int cpt, int max_nx, int elem, int nt) {
    // p and s: three planes each of nt * cpt + 4 nx values; plus one pad cell per thread; the
    // block's reduction scratch is static
    return ((size_t)6 * (size_t)(nt * cpt + 4 * max_nx) + (size_t)nt) * (size_t)elem;
}

bool fused_shape_ok(int cpt, int max_nx, int nt) {
    const int h = halo_slots(max_nx, nt);
    if (nt == 256) return (cpt == 1 || cpt == 2) && h >= 1 && h <= 4;
    return nt == 512 && (cpt == 1 || cpt == 2) && h >= 1 && h <= 2;
}

// the single-sync kernel: 256 threads with 1 or 2 cells per thread and 1, 2 or 4 halo slots per
// ring, or 512 threads with 1 or 2 cells per thread and 1 or 2 halo slots
#define EQS_DISPATCH_FUSED(cpt, h, nt, BODY)                                         \
    do {                                                                             \
        if ((nt) == 512 && (cpt) == 1) {                                             \
            constexpr int C = 1, NTT = 512;                                          \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else { constexpr int HH = 2; BODY; }                                     \
        } else if ((nt) == 512) {                                                    \
            constexpr int C = 2, NTT = 512;                                          \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else { constexpr int HH = 2; BODY; }                                     \
        } else if ((cpt) == 1) {                                                     \
            constexpr int C = 1, NTT = 256;                                          \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else if ((h) == 2) { constexpr int HH = 2; BODY; }                       \
            else { constexpr int HH = 4; BODY; }                                     \
        } else {                                                                     \
            constexpr int C = 2, NTT = 256;                                          \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else if ((h) == 2) { constexpr int HH = 2; BODY; }                       \
            else { constexpr int HH = 4; BODY; }                                     \
        }                                                                            \
    } while (0)

// Dynamic LDS beyond 64 KB must be allowed per kernel: every instantiation of the single-sync step
// may take up to `bytes` (the device's per-block limit)
hipError_t allow_fused_lds(size_t bytes) {
    hipError_t e = hipSuccess;
    auto allow = [&](const void *f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    };
    auto all_forms = [&](int cpt, int h, int nt) {
        EQS_DISPATCH_FUSED(cpt, h, nt, {
            allow((const void *)fused_kernel<double, C, HH, kFormScaled, NTT>);
            allow((const void *)fused_kernel<double, C, HH, kFormSym, NTT>);
            allow((const void *)fused_kernel<double, C, HH, kFormRaw, NTT>);
            allow((const void *)fused_kernel<float, C, HH, kFormScaled, NTT>);
            allow((const void *)fused_kernel<float, C, HH, kFormSym, NTT>);
        });
    };
    for (int cpt = 1; cpt <= 2; ++cpt) {
        for (int h : {1, 2, 4}) all_forms(cpt, h, 256);
        for (int h : {1, 2}) all_forms(cpt, h, 512);
    }
    return e;
}

#define EQS_DISPATCH(cpt, h, BODY)                                                   \
    do {                                                                             \
        if ((cpt) == 1) {                                                            \
            constexpr int C = 1;                                                     \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else if ((h) == 2) { constexpr int HH = 2; BODY; }                       \
            else if ((h) == 4) { constexpr int HH = 4; BODY; }                       \
            else { constexpr int HH = 8; BODY; }                                     \
        } else {                                                                     \
            constexpr int C = 2;                                                     \
            if ((h) == 1) { constexpr int HH = 1; BODY; }                            \
            else if ((h) == 2) { constexpr int HH = 2; BODY; }                       \
            else if ((h) == 4) { constexpr int HH = 4; BODY; }                       \
            else { constexpr int HH = 8; BODY; }                                     \
        }                                                                            \
    } while (0)

// With a start/stop event pair the launch goes through hipExtLaunchKernel, which
// stamps the events with the dispatch's own start and end times (the kernel's
// duration alone, as a kernel trace reports it); such launches are never captured.
#define EQS_LAUNCH(KERN, GRID, BLOCK, LDS, ...)                                                  \
    do {                                                                                         \
        if (e0) hipExtLaunchKernelGGL(KERN, GRID, BLOCK, LDS, stream, e0, e1, 0u, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERN, GRID, BLOCK, LDS, stream, __VA_ARGS__);                   \
    } while (0)

hipError_t launch_mg_fine(const LaunchSets &ls, const MgLevel *levs, const MgCounts &cnt, int ntiles, int cpt,
                          int max_nx, int which, bool resid, MgParams prm, bool gated, hipStream_t stream) {
    const dim3 grid(ntiles), block(kBlock);
    const int h = halo_slots(max_nx, kBlock);
    if (h < 0 || (cpt != 1 && cpt != 2)) return hipErrorInvalidValue;
    const size_t lds64 = march_lds_bytes(cpt, max_nx, 8);
    if (resid)
        EQS_DISPATCH(cpt, h, hipLaunchKernelGGL((mg_resid0_kernel<C, HH>), grid, block, lds64, stream, ls, levs, cnt,
                                                which, prm, gated ? 1 : 0));
    else
        EQS_DISPATCH(cpt, h, hipLaunchKernelGGL((mg_prolong0_kernel<C, HH>), grid, block, lds64, stream, ls, levs,
                                                cnt, which, prm, gated ? 1 : 0));
    return hipGetLastError();
}

hipError_t launch_mg_aggregate(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int nc,
                               bool gated, hipStream_t stream) {
    dim3 grid = mg_grid(nc);
    grid.y = (unsigned)nsets;
    hipLaunchKernelGGL(mg_aggregate_kernel, grid, dim3(kBlock), 0, stream, desc, levs, cnt, gated ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_kernel(Kern k, const LaunchSets &ls, int ntiles, int nflat, int cpt, int max_nx, bool fp32,
                         bool trans, hipStream_t stream, const double *x, double *y, int arg, hipEvent_t e0,
                         hipEvent_t e1) {
    const dim3 grid(ntiles), fgrid(nflat), block(kBlock);
    const int h = halo_slots(max_nx, kBlock);
    if (h < 0 || (cpt != 1 && cpt != 2)) return hipErrorInvalidValue;
    const size_t lds64 = march_lds_bytes(cpt, max_nx, 8), lds32 = march_lds_bytes(cpt, max_nx, 4);
    switch (k) {
    case K_K1:  // the scaled operator needs no transpose variant
        if (fp32) EQS_DISPATCH(cpt, h, EQS_LAUNCH((k1_kernel<float, C, HH>), grid, block, lds32, ls));
        else EQS_DISPATCH(cpt, h, EQS_LAUNCH((k1_kernel<double, C, HH>), grid, block, lds64, ls));
        break;
    case K_K2:
        if (fp32) EQS_DISPATCH(cpt, h, EQS_LAUNCH((k2_kernel<float, C, HH>), grid, block, lds32, ls));
        else EQS_DISPATCH(cpt, h, EQS_LAUNCH((k2_kernel<double, C, HH>), grid, block, lds64, ls));
        break;
    case K_SCALE:
        if (trans) EQS_LAUNCH((scale_kernel<true>), fgrid, block, 0, ls, 0);
        else EQS_LAUNCH((scale_kernel<false>), fgrid, block, 0, ls, arg);
        break;
    case K_UNSCALE:
        EQS_LAUNCH(unscale_kernel, fgrid, block, 0, ls);
        break;
    case K_K3:
        if (fp32) EQS_LAUNCH((k3_kernel<float>), fgrid, block, 0, ls);
        else EQS_LAUNCH((k3_kernel<double>), fgrid, block, 0, ls);
        break;
    case K_SETUP:
    case K_RECHECK:
    case K_REPORT: {
        const int mode = k == K_SETUP ? 0 : (k == K_RECHECK ? 1 : 2);
        const int wd = k == K_SETUP && arg == 1;  // the setup writes 1/a_P for the raw form
        if (trans) EQS_DISPATCH(cpt, h, EQS_LAUNCH((res_kernel<C, HH, true>), grid, block, lds64, ls, mode, wd));
        else EQS_DISPATCH(cpt, h, EQS_LAUNCH((res_kernel<C, HH, false>), grid, block, lds64, ls, mode, wd));
        break;
    }
    case K_OUTER:
        EQS_DISPATCH(cpt, h, EQS_LAUNCH((outer_kernel<C, HH>), grid, block, lds64, ls));
        break;
    case K_CAST:
        EQS_LAUNCH(cast_kernel, fgrid, block, 0, ls, arg);
        break;
    case K_UPDATE:
        EQS_LAUNCH(update_kernel, fgrid, block, 0, ls);
        break;
    case K_ZERO:
        EQS_LAUNCH(zero_kernel, fgrid, block, 0, ls, arg);
        break;
    case K_GRAD:
        EQS_LAUNCH(grad_kernel, fgrid, block, 0, ls);
        break;
    case K_TRANSPOSE:
        EQS_LAUNCH(transpose_kernel, fgrid, block, 0, ls);
        break;
    case K_APPLY:
        if (trans) EQS_DISPATCH(cpt, h, EQS_LAUNCH((apply_kernel<C, HH, true>), grid, block, lds64, ls, x, y));
        else EQS_DISPATCH(cpt, h, EQS_LAUNCH((apply_kernel<C, HH, false>), grid, block, lds64, ls, x, y));
        break;
    case K_FUSED: {  // the scaled operator needs no transpose variant; arg: the form (kForm*)
        const int nt = ls.fnt, fh = halo_slots(max_nx, nt);
        if (!fused_shape_ok(cpt, max_nx, nt) || arg < kFormScaled || arg > kFormRaw || (fp32 && arg == kFormRaw))
            return hipErrorInvalidValue;
        const dim3 fg(ls.ftile_begin[ls.nsets]), fb(nt);
        const size_t fl = fused_lds_bytes(cpt, max_nx, fp32 ? 4 : 8, nt);
        if (arg == kFormSym) {  // every set of the launch exactly symmetric
            if (fp32) EQS_DISPATCH_FUSED(cpt, fh, nt, EQS_LAUNCH((fused_kernel<float, C, HH, kFormSym, NTT>), fg, fb, fl, ls));
            else EQS_DISPATCH_FUSED(cpt, fh, nt, EQS_LAUNCH((fused_kernel<double, C, HH, kFormSym, NTT>), fg, fb, fl, ls));
        } else if (arg == kFormRaw) {
            EQS_DISPATCH_FUSED(cpt, fh, nt, EQS_LAUNCH((fused_kernel<double, C, HH, kFormRaw, NTT>), fg, fb, fl, ls));
        } else {
            if (fp32) EQS_DISPATCH_FUSED(cpt, fh, nt, EQS_LAUNCH((fused_kernel<float, C, HH, kFormScaled, NTT>), fg, fb, fl, ls));
            else EQS_DISPATCH_FUSED(cpt, fh, nt, EQS_LAUNCH((fused_kernel<double, C, HH, kFormScaled, NTT>), fg, fb, fl, ls));
        }
        break;
    }
    case K_FSETUP:  // arg: the form of the step that follows (kFormRaw: from the caller's coefficients)
        if (fp32) EQS_DISPATCH(cpt, h, EQS_LAUNCH((fsetup_kernel<float, C, HH>), grid, block, lds32, ls));
        else if (arg == kFormRaw) EQS_DISPATCH(cpt, h, EQS_LAUNCH((fsetup_raw_kernel<C, HH>), grid, block, lds64, ls));
        else EQS_DISPATCH(cpt, h, EQS_LAUNCH((fsetup_kernel<double, C, HH>), grid, block, lds64, ls));
        break;
    case K_MAT:
        if (fp32) EQS_LAUNCH((mat_kernel<float>), fgrid, block, 0, ls);
        else EQS_LAUNCH((mat_kernel<double>), fgrid, block, 0, ls);
        break;
    case K_PC_P:
        EQS_LAUNCH(pc_p_kernel, fgrid, block, 0, ls);
        break;
    case K_PC_V:
    case K_PC_T:
        EQS_DISPATCH(cpt, h, EQS_LAUNCH((pc_prod_kernel<C, HH>), grid, block, lds64, ls, k == K_PC_T ? 1 : 0));
        break;
    case K_PC_S:
        EQS_LAUNCH(pc_s_kernel, fgrid, block, 0, ls);
        break;
    case K_PC_X:
        EQS_LAUNCH(pc_x_kernel, fgrid, block, 0, ls);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace eqs
