// eqs_internal.h -- structures shared by the host driver and the gfx950 kernels.
//
// Every equation set owns one SetDesc (device-resident table entry) and one
// SolveState.  Kernels take a launch table (LaunchSets) by value that maps
// the blocks of one launch onto the tiles of one or more sets, so a single
// set and the whole batch of a time step go through the same kernels, with
// the same tiles and the same reduction order: per-set results do not depend
// on how many sets share a launch.
#pragma once

#include <stdint.h>

namespace eqs {

constexpr int kBlock = 256;      // threads per block (4 wave64)
constexpr int kMaxSets = 8;      // sets per launch table
constexpr int kMaxRed = 11;      // reduction values per tile
constexpr int kFlatU = 4;        // pointwise kernels: cells per thread per chunk
constexpr int kFlatChunk = kBlock * kFlatU;
constexpr int kMaxFlatBlocks = 4096;

// per-set iteration mode
enum : int32_t { MODE_FP64 = 0, MODE_REFINE = 1, MODE_FP32 = 2, MODE_ADJOINT = 3 };

// computed statuses (the public EQS_* codes)
enum : int32_t { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3, ST_ERR_ARG = -1 };

// Device-side state of one set's solve.  Written only by the finalising
// block of a launch (after all tiles' partial sums are in) and read by every
// block at the start of the next launch.
struct SolveState {
    double bb;        // (b, b) of the system being iterated
    double lim2;      // tol_iter * sqrt(bb): stop when sqrt((r, r)) <= lim2
    double rho, rho_prev, alpha, omega;
    double sigma, ts, tt, ss, rr;   // latest reductions
    double rr_true;   // (b - A x, b - A x) in FP64 of the returned x
    double bb_outer;  // (b, b) of the FP64 system (refinement)
    double lim2_outer;
    double rr_prev;   // outer residual of the previous refinement step
    double scale;     // power of two applied to the residual cast to FP32
    double upd_inv_scale;  // 1/scale of the inner solve being applied
    // single-sync iteration: the scalars of the previous step (alpha_prev,
    // omega, beta) with which the next launch forms r, p and y
    double alpha_prev, beta;
    int32_t iters;    // BiCGSTAB iterations so far (inner, for the FP32 forms)
    int32_t maxit;
    int32_t active;   // BiCGSTAB iterating
    int32_t done;     // final status reached
    int32_t status;
    int32_t fresh;    // next K1 starts afresh: p = r, r^ = r
    int32_t half;     // half-step exit taken in this iteration
    int32_t converged;    // FP64: recursive residual met tol; true-residual recheck pending
    int32_t inner_done;   // FP32 forms: inner solve finished; update + outer residual pending
    int32_t need_report;  // final true residual pending
    int32_t rho_restarts; // fresh starts forced by rho = 0
    int32_t restarts;     // all fresh starts after the first
    int32_t outer;        // refinement steps started
    int32_t zero_rhs;     // b = 0: x must be set to 0
    int32_t mode;
    int32_t outer_pending;  // FP32 forms: first outer residual pending
    // single-sync iteration
    int32_t fpar;     // buffer slot (0/1) holding the latest s, t, p, v
    int32_t need_f;   // f = M^T r^ and sigma_0 pending (after a fresh start)
    int32_t mat;      // iterate to form before leaving the iteration: 1 y += alpha p;
                      // 2 y += alpha p + omega s; 3 as 2, plus r = s - omega t, r^ = r (restart);
                      // 4 no y change, r = s + alpha v, r^ = r (restart at the current iterate)
    int32_t weak_outer;  // consecutive refinement steps that reduced ||r|| by less than 2x
    int32_t sym;      // the matrix is exactly symmetric (checked per solve): the single-sync step and
                      // the multigrid finest-level passes read a_W, a_S, a_B as a_E, a_N, a_T of the
                      // neighbour
    // single-sync iteration: restarts forced by the sigma consistency check, over the whole solve
    // and within the current inner solve (FP32 forms: each refinement step's solve has its own
    // budget; FP64: the solve's)
    int32_t sig_restarts;
    int32_t sig_inner;
    // single-sync iteration: the next launch runs the last step again, with alpha from the
    // directly summed sigma (its inputs are intact; y, which the first run formed, is kept)
    int32_t redo;
    int32_t sig_redos;   // such reruns over the whole solve
};

struct MgLevel;

struct SetDesc {
    int32_t nx, ny, nz, plane, n;
    // march tiling: S segments of Q = kBlock*cpt cells per plane, KC planes per chunk
    int32_t S, KC, NKC, ntiles;
    // the single-sync step's own tiling: fS segments of fnt*cpt cells per plane (fnt = its block
    // size, LaunchSets::fnt), the same chunks, fntiles tiles numbered chunk-fastest (ford = 0) or
    // segment-fastest (ford = 1)
    int32_t fS, fntiles, ford;
    int32_t sig_redo;   // a sigma mismatch reruns the step (1) or restarts the iteration (0)
    // multigrid: the set's level table (device) and its number of levels (0: none)
    const MgLevel *mg;
    int32_t mg_levels, mg_pad;
    // pointwise kernels: nflat blocks, block b takes chunks b, b + nflat, ... of kFlatChunk cells
    int32_t nflat;
    int32_t mode;
    double tol, tol_inner;
    double sigma_tol[2];  // single-sync iteration: largest relative gap between sigma taken
                          // directly and the expanded one it ran with, FP64 [0] and FP32 [1]
    int32_t maxit, pad;
    // caller arrays
    const double *a[7];
    const double *b;
    double *x;
    // FP64 work (r^ = rh); p and v are double-buffered by iteration parity.
    // The iteration runs on the column-scaled operator A D^-1 (unit diagonal,
    // D = diag(a_P)): as[0..5] hold its E, W, N, S, T, B coefficients (for
    // the adjoint, those of A^T D^-1) and y = D x is its iterate.
    double *r, *rh, *p[2], *v[2], *t, *y;
    double *as[6];
    // symmetric matrices: 1/a_P, with which the single-sync step forms the products of
    // A D^-1 from the caller's a_E, a_N, a_T (FP32 forms: sym32 = those three rounded
    // to FP32, then 1/a_P rounded)
    double *dinv;
    float *sym32[4];
    // single-sync iteration: s and t double-buffered with r (slot 0 of s) and
    // t (slot 0 of t); f = M^T r^ with M the scaled operator
    double *s1, *t1, *f;
    // FP32 work (refinement): scaled coefficients, vectors, d32 = inner iterate (scaled)
    float *as32[6];
    float *r32, *rh32, *p32[2], *v32[2], *t32, *d32;
    float *s1_32, *t1_32, *f32;
    // adjoint: forward solution and gradient outputs (grad_b is the iterate x)
    const double *xf;
    double *g[7];
    // reductions
    double *partials;   // [max(ntiles, nflat) * kMaxRed]
    uint32_t *counter;  // last-block ticket
    SolveState *st;
};

// One level of a set's multigrid hierarchy (the aggregation V-cycle used as
// the right preconditioner of the FP64 solve).  Level 0 is the system itself
// (its coefficients are the caller's arrays in the set table); level l + 1
// aggregates 2 x 2 x 2 cells of level l.
constexpr int kMgMaxLevels = 16;
struct MgLevel {
    int32_t nx, ny, nz, n;
    double *a[7];   // Galerkin coefficients (levels >= 1)
    double *r, *z;  // right-hand side and result of the level's V-cycle (levels >= 1)
    float *a32[7];  // level 0: the system's coefficients rounded to FP32, the operator the
                    // V-cycle takes on that level (and coarsens from); arithmetic stays FP64
};
// number of multigrid levels of each set of a launch (a kernel argument: no load before the first
// level-table access)
struct MgCounts {
    int32_t n[kMaxSets];
};
struct MgParams {
    double omega;         // damped-Jacobi weight
    double gamma;         // scale of the coarse correction
    int32_t coarse_sweeps;
    int32_t coarse_cells;
    int32_t coarse_sym;   // coarse levels of an exactly symmetric matrix read W, S, B as E, N, T
    int32_t pad;
};

// blocks of one launch -> (set, tile); set s owns logical tiles [tile_begin[s], tile_begin[s+1])
// (pointwise kernels use flat_begin over the sets' nflat blocks instead)
struct LaunchSets {
    int32_t nsets;
    int32_t tile_begin[kMaxSets + 1];
    int32_t flat_begin[kMaxSets + 1];
    int32_t ftile_begin[kMaxSets + 1];  // the single-sync step's tiles (SetDesc::fntiles)
    int32_t fnt;                        // threads per block of the single-sync step (256 or 512)
    const SetDesc *desc;   // device table, nsets entries
    // bit 0: tiles, bit 1: pointwise blocks, bit 2: the single-sync step's tiles -- each XCD runs a
    // share of every set (the balanced map of locate_in) instead of one run of the launch
    int32_t xbal;
};

}  // namespace eqs
