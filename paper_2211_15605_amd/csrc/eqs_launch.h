// eqs_launch.h -- host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>

#include "eqs_internal.h"

namespace eqs {

enum Kern {
    K_SETUP,    // r = b - A x, r^ = r, (b,b), (r,r), a_P check; initialises the state
    K_RECHECK,  // true residual after recursive convergence (restart if above tol)
    K_REPORT,   // true residual of the final iterate (no writes)
    K_K1,       // p update + Jacobi + product + (r^, v)
    K_K2,       // s + Jacobi + product + (t,s), (t,t), (s,s)
    K_K3,       // x and r updates + (r^, r), (r, r)
    K_CAST,     // FP64 -> FP32 coefficients, (b,b), a_P check (FP32 forms)
    K_OUTER,    // FP64 residual -> scaled FP32 inner right-hand side (FP32 forms)
    K_UPDATE,   // x += d / scale (FP32 forms)
    K_ZERO,     // x = 0 (b = 0, or forced)
    K_GRAD,     // adjoint gradients
    K_APPLY,    // y = A x or A^T x
    K_SCALE,    // coefficients of A D^-1 (or A^T D^-1), FP64
    K_UNSCALE,  // x = y / a_P (before a recheck or a final report)
    K_FUSED,    // single-sync iteration: both products and all ten dot products in one launch
    K_FSETUP,   // f = M^T r^, (f, r^), (r^, r^) after a fresh start (single-sync iteration)
    K_MAT,      // form the iterate (and a restart residual) on leaving the single-sync iteration
    K_PC_P,     // multigrid-preconditioned iteration: p = r + beta (p - omega v)
    K_PC_V,     // v = A p^, (r^, v)
    K_PC_S,     // s = r - alpha v
    K_PC_T,     // t = A s^, (t,s), (t,t), (s,s)
    K_PC_X,     // x += alpha p^ + omega s^, r = s - omega t, (r^, r), (r, r)
    K_MG,       // one V-cycle level step (restriction, coarsest sweeps or prolongation + smoothing)
    K_TRANSPOSE // the six neighbour coefficients of A^T into the set's scaled-coefficient buffers
};

// multigrid setup of set `set` (d: its device table entry, lev: its device level table)
hipError_t launch_mg_symcheck(const SetDesc *d, int n, int on, hipStream_t stream);
hipError_t launch_mg_round0(const SetDesc *d, const MgLevel *lev, int n, hipStream_t stream);
hipError_t launch_mg_coarsen(const SetDesc *d, const MgLevel *lev, int l, int nc, hipStream_t stream);
// The V-cycle over the nsets sets of a launch (desc: the device table entry of its first set, levs:
// that set's level table, the next sets' following kMgMaxLevels apart, cnt: each set's number of
// levels; a set without the level returns).
// which: the V-cycle's input and output, 0: p -> p^, 1: s -> s^, 2: r -> t (diagnostics).
// restriction from level l to l + 1 (nc: the largest set's cells on level l + 1)
hipError_t launch_mg_restrict(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int l, int nc,
                              MgParams prm, bool gated, hipStream_t stream);
// each set's coarsest level (at most kMgCoarsestMax cells): coarse_sweeps damped-Jacobi sweeps from
// zero, one block per set
constexpr int kMgCoarsestMax = 2048;
hipError_t launch_mg_coarsest(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int which,
                              MgParams prm, bool gated, hipStream_t stream);
// finest level through the k-march (the launch's tiles): resid: the per-cell residual r - A z1 into
// each set's y buffer; else the prolongation of level 1's result + one smoothing step
hipError_t launch_mg_fine(const LaunchSets &ls, const MgLevel *levs, const MgCounts &cnt, int ntiles, int cpt,
                          int max_nx, int which, bool resid, MgParams prm, bool gated, hipStream_t stream);
// level 1's right-hand side from the per-cell residual of level 0 (nc: the largest set's level-1 cells)
hipError_t launch_mg_aggregate(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int nc,
                               bool gated, hipStream_t stream);
// prolongation of level l + 1's result and one smoothing sweep on level l (n: the largest set's cells)
hipError_t launch_mg_prolong(const SetDesc *desc, const MgLevel *levs, const MgCounts &cnt, int nsets, int l, int n,
                             MgParams prm, bool gated, hipStream_t stream);

// LDS bytes of the single-sync kernel with nt threads per block (p and s, three planes each of
// nt * cpt + 4 nx values, and a pad cell per thread)
size_t fused_lds_bytes(int cpt, int max_nx, int elem, int nt);

// the single-sync kernel has an instantiation for this shape (nt = 256: up to 4 halo slots;
// nt = 512: up to 2; cpt 1 or 2)
bool fused_shape_ok(int cpt, int max_nx, int nt);

// let every instantiation of the single-sync kernel take up to `bytes` of dynamic LDS
hipError_t allow_fused_lds(size_t bytes);

// LDS bytes of a march kernel (three plane buffers of Q + 2 nx values)
size_t march_lds_bytes(int cpt, int max_nx, int elem);

// halo cells per thread per plane for blocks of nt threads (1, 2, 4 or 8), or -1 if nx is too wide
int halo_slots(int max_nx, int nt);

// cells of the largest set the one-block persistent solve takes
constexpr int kSmallSolveMaxCells = 2048;

// one-block persistent FP64 solve of every set of the launch table (each
// at most kSmallSolveMaxCells cells): one block per set, one launch
hipError_t launch_small(const LaunchSets &ls, int max_n, bool trans, hipStream_t stream);

// p[0..n) = v on `stream`
hipError_t launch_fill(double *p, long n, double v, hipStream_t stream);

// Launch kernel k: march kernels over ntiles blocks (the sum of the sets'
// tile counts), pointwise kernels over nflat blocks (the sum of their nflat).
// A non-null e0/e1 pair receives the kernel's own start and end timestamps
// (not for use under stream capture).
hipError_t launch_kernel(Kern k, const LaunchSets &ls, int ntiles, int nflat, int cpt, int max_nx, bool fp32,
                         bool trans, hipStream_t stream, const double *x, double *y, int arg,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

}  // namespace eqs
