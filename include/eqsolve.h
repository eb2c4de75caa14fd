/*
 * eqsolve.h -- C ABI of the MI355X (gfx950) equation-set solver.
 *
 * The operation: each equation set of a time step (u, v, w momentum and the
 * pressure correction) is one linear system that equation decomposition
 * hands, whole, to one device (Woo et al., arXiv 2211.15605, Sec. 2.2.2).
 * Its cost is the system's stencil product and the global dot products the
 * Krylov solver takes on every iteration (Sec. 2.2.2).  This library solves
 * such a system on one GPU with Jacobi-preconditioned BiCGSTAB, in FP64
 * (the paper's precision, Sec. 3.1), in FP32 with FP64 iterative refinement,
 * or in FP32 alone, for one set or for all sets of a time step in one call
 * (the single-device assignment "111[1]" of Sec. 2.2.2), and gives the
 * adjoint (gradients of a loss with respect to b and the coefficients).
 *
 * System (Patankar form of the 7-point finite-volume discretisation):
 *     a_P[c] x[c] - sum_{nb in E,W,N,S,T,B} a_nb[c] x[nb(c)] = b[c]
 * on an nx*ny*nz structured grid, flat cell index c = i + nx*(j + ny*k)
 * (i fastest; fields are flat rank-1 arrays, Sec. 2.2.3).  E/W = +x/-x,
 * N/S = +y/-y, T/B = +z/-z.  A neighbour outside the grid contributes
 * nothing: coefficients that point out of the grid are ignored, whatever
 * they hold.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (the device current when the
 *    context was created) to contiguous FP64 arrays of n = nx*ny*nz entries.
 *    The caller owns them; they must stay valid until the call returns.
 *  - diag[7] is an array of 7 device pointers in the order P, E, W, N, S, T, B.
 *  - x must not alias b or any diag array.
 *  - Work is enqueued on the context's stream; every call returns only after
 *    its results are complete (one small device-to-host copy of the status).
 *  - A context is bound to one stream and is not thread-safe.
 *  - Return value: < 0 is an error found before any work was done (x is
 *    untouched); 0 means converged; > 0 means x holds a computed iterate that
 *    did not meet the tolerance (see the EQS_* codes).
 *  - Convergence: ||b - A x||_2 <= tol * ||b||_2, recomputed in FP64 from the
 *    final x.  b = 0 gives x = 0.
 */
#ifndef EQSOLVE_H
#define EQSOLVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eqs_ctx eqs_ctx;

typedef struct {
    int32_t nx, ny, nz;
} eqs_grid;

/* precision of the iteration */
enum {
    EQS_FP64 = 0,        /* plain FP64 BiCGSTAB */
    EQS_FP32_REFINE = 1, /* FP32 inner BiCGSTAB, FP64 residual / update / norms */
    EQS_FP32 = 2         /* one FP32 BiCGSTAB solve of the FP64 residual system */
};

/* result codes */
enum {
    EQS_OK = 0,
    EQS_NOT_CONVERGED = 1, /* maxit reached, or refinement stopped reducing ||r|| */
    EQS_BREAKDOWN = 2,     /* (r^, v) = 0, omega = 0, or rho = 0 twice */
    EQS_NONFINITE = 3,     /* NaN/Inf in b, x0 or an iterate (x: last iterate, or untouched if in b/x0) */
    EQS_ERR_ARG = -1,      /* bad argument: null pointer, bad sizes, tol not in (0,1), maxit < 1, a_P = 0 */
    EQS_ERR_NOMEM = -2,    /* device allocation failed in eqsolve_create */
    EQS_ERR_HIP = -3,      /* a HIP runtime call failed */
    EQS_ERR_STATE = -4,    /* context unusable (null, or a previous HIP failure) */
    EQS_ERR_SIZE = -5      /* eqsolve_solve_noalloc: the system exceeds its static workspace */
};

typedef struct {
    int32_t status;  /* EQS_* of this set */
    int32_t iters;   /* BiCGSTAB iterations (inner iterations for the FP32 forms) */
    int32_t outer;   /* refinement steps (FP32 forms), restarts (FP64) */
    int32_t flags;   /* EQS_INFO_* bits describing how the solve ran */
    double rel_res;  /* ||b - A x||_2 / ||b||_2 of the returned x, in FP64 */
    int32_t sigma_restarts; /* fresh starts the single-sync iteration took when its expanded (r^, M p)
                               parted from the directly summed one (all inner solves of the FP32 forms).
                               FP64: at most 32 a solve, then the check is off for the rest of it; an
                               FP32 inner solve: at most 32, then it ends and the refinement decides */
    int32_t sigma_reruns;   /* with EQS_SIGMA_REDO=1 at eqsolve_create, such steps run a second time
                               with alpha from the directly summed value instead of restarting (a rerun
                               reads the same inputs and is not counted in iters) */
} eqs_info;

/*
 * eqs_info.flags: EQS_INFO_SYMMETRIC -- the matrix was found exactly symmetric
 * (a_W(c) = a_E(c-1), a_S(c) = a_N(c-nx), a_B(c) = a_T(c-nx*ny) wherever both
 * cells are in the grid; checked once per solve, on the device) and the
 * single-sync iteration ran in its symmetric form, reading a_E, a_N, a_T and
 * 1/a_P instead of six scaled coefficients.  Set for a solve whose launch held
 * only such sets (in a batched call: every set); EQS_SYM=0 in the environment
 * at eqsolve_create turns the form off.  EQS_INFO_UNSCALED -- the solve ran the
 * single-sync iteration in its unscaled form (eqsolve_set_step_form).
 */
enum { EQS_INFO_SYMMETRIC = 1, EQS_INFO_UNSCALED = 2 };

/*
 * Create a context for nsets equation sets with the given grids (the sets
 * of one time step, e.g. p', u, v, w on their staggered grids).  Allocates
 * all device workspace for `precision` once (no allocation happens in the
 * solve calls).  hip_stream is a hipStream_t (NULL = the default stream).
 * Grids need 1 <= nx <= 1024 (a stencil pass stages one row of nx cells on
 * each side of a plane segment in LDS), 1 <= ny, nz and nx*ny*nz < 2^31;
 * 1 <= nsets <= 8.  Returns EQS_OK, EQS_ERR_ARG (grids, nsets, precision),
 * EQS_ERR_NOMEM or EQS_ERR_HIP; *ctx is NULL unless EQS_OK.  The argument
 * checks come before any HIP call.
 */
int eqsolve_create(eqs_ctx **ctx, const eqs_grid *grids, int32_t nsets, int32_t precision,
                   void *hip_stream);

/*
 * Solve set `set` of the context: x (x0 on entry, solution on return).
 * tol in (0, 1); maxit >= 1 (for the FP32 forms: the cap on total inner
 * iterations).  info (host pointer) receives the outcome.
 */
int eqsolve_solve(eqs_ctx *ctx, int32_t set, const double *const diag[7], const double *b,
                  double *x, double tol, int32_t maxit, eqs_info *info);

/*
 * Solve all nsets sets of the context in one call, sharing every launch
 * (the time step's equation sets on one device).  diag[s][7], b[s], x[s],
 * tol[s], maxit[s] and info[s] are host arrays indexed by set.  Each set
 * converges on its own; a converged set does no further work.  Per-set
 * results equal eqsolve_solve's bit for bit.
 */
int eqsolve_solve_batched(eqs_ctx *ctx, const double *const *const *diag, const double *const *b,
                          double *const *x, const double *tol, const int32_t *maxit,
                          eqs_info *info);

/*
 * Adjoint of x = A^{-1} b for a loss L(x): given x (the converged forward
 * solution) and w = dL/dx, solve A^T lambda = w in FP64 BiCGSTAB (Jacobi on
 * the same a_P; with EQS_PRECOND_MG selected, the multigrid V-cycle of A^T,
 * whose rows -- a_P and the links pointing at each cell -- are formed into
 * the context's workspace first) and return
 *     grad_b = lambda,
 *     grad_diag[P][c] = -lambda[c] x[c],
 *     grad_diag[nb][c] = +lambda[c] x[nb(c)]  (0 where nb(c) is outside the grid),
 * i.e. the gradients with respect to the arrays as passed (Patankar signs).
 * grad_b also serves as the solver's iterate (its input value is ignored).
 * Any grad_diag[k] may be NULL to skip it.
 */
int eqsolve_adjoint(eqs_ctx *ctx, int32_t set, const double *const diag[7], const double *x,
                    const double *w, double *grad_b, double *const grad_diag[7], double tol,
                    int32_t maxit, eqs_info *info);

/*
 * y = A x (transpose = 0) or y = A^T x (transpose = 1) for set `set`, in FP64.
 * y must not alias x.
 */
int eqsolve_apply(eqs_ctx *ctx, int32_t set, const double *const diag[7], const double *x, double *y,
                  int32_t transpose);

/*
 * Pick the launch shape of every set by measurement: for each candidate
 * (cells per thread of the stencil passes, planes per k-chunk, then the block
 * count of the pointwise pass) time `iters` BiCGSTAB iterations with HIP
 * events on a synthetic system of the set's exact shape in the context's
 * precision, and keep the fastest.  A context of several sets then also times
 * the batched launch (eqsolve_solve_batched) under that choice and under one
 * common number of planes per chunk for every set, and keeps the fastest for
 * the context.  The result applies to the context at once; the per-set choice
 * is appended to the JSON-lines file cache_path (or $EQS_TUNE_CACHE if
 * cache_path is NULL; nothing is written if both are unset), which
 * eqsolve_create consults when $EQS_TUNE_CACHE is set.  Allocates and frees
 * 9 temporary arrays of the largest set while it runs.  Returns EQS_OK,
 * EQS_ERR_NOMEM or EQS_ERR_HIP / EQS_ERR_STATE.
 */
int eqsolve_autotune(eqs_ctx *ctx, const char *cache_path, int32_t iters);

/* Release the context and its workspace (NULL is allowed). */
int eqsolve_destroy(eqs_ctx *ctx);

/* How the single-sync iteration of the FP64 forward solves forms its products. */
enum { EQS_STEP_SCALED = 0, EQS_STEP_UNSCALED = 1 };

/*
 * The iteration runs on M = A D^-1 (D = diag(a_P), the right Jacobi
 * preconditioner; Woo et al. Sec. 2.2.2 for the per-set solve).  EQS_STEP_SCALED
 * (the default): a pass at the start of every solve writes M's six
 * off-diagonal coefficients a_nb(c) / a_P(nb(c)) (and checks for exact
 * symmetry, which selects the symmetric form), and every step reads those six.
 * EQS_STEP_UNSCALED: no such pass; every step reads the caller's six arrays and
 * 1/a_P (written by the setup pass) and forms (M p)_c = p_c - sum_nb a_nb(c)
 * (p / a_P)_nb -- one word per cell more per step, about fourteen less per
 * solve, so it pays for systems that converge in a few steps, such as the
 * momentum rows of a SIMPLE iteration, whose transient term dominates.  Both
 * give the same iterates up to rounding.  For EQS_FP64 contexts only; the
 * adjoint and the multigrid-preconditioned solves are unaffected.  Returns
 * EQS_OK, EQS_ERR_ARG (form, or a context that is not EQS_FP64) or
 * EQS_ERR_STATE.
 */
int eqsolve_set_step_form(eqs_ctx *ctx, int32_t form);

/* Preconditioners of the FP64 solves (forward and adjoint). */
enum { EQS_PRECOND_JACOBI = 0, EQS_PRECOND_MG = 1 };

/* Parameters of the multigrid V-cycle (see eqsolve_set_preconditioner). */
typedef struct {
    double omega;          /* damped-Jacobi weight, in (0, 2); default 0.8 */
    double gamma;          /* scale of the coarse correction, in (0, 4]; default 1 */
    int32_t coarse_sweeps; /* damped-Jacobi sweeps on the coarsest level, >= 1; default 30 */
    int32_t coarse_cells;  /* coarsen until a level has at most this many cells, 1..2048; default 512 */
} eqs_mg_params;

/*
 * Choose the right preconditioner of the solves of an EQS_FP64 context
 * (eqsolve_solve, eqsolve_solve_batched and eqsolve_adjoint, whose A^T solve
 * then runs the V-cycle built from A^T).  EQS_PRECOND_JACOBI is the default.  EQS_PRECOND_MG is an
 * aggregation multigrid V-cycle, an addition to the paper's method aimed at
 * the pressure-correction system, whose Jacobi iteration count grows with
 * the grid: levels of 2 x 2 x 2 aggregates (dimensions halved, rounding up)
 * down to at most coarse_cells cells, piecewise-constant interpolation,
 * restriction by summing an aggregate, Galerkin coarse operators (again
 * 7-point), one damped-Jacobi step before and after the coarse correction
 * (scaled by gamma) and coarse_sweeps damped-Jacobi sweeps on the coarsest
 * level.  The iteration runs on the original A, with x updated in place; a
 * batched call iterates its sets together (every launch over all of them).
 * The finest level's operator is the system's with its coefficients rounded
 * to FP32 (arithmetic stays FP64); when a call's matrix is exactly symmetric
 * (a_W(c) = a_E(c-1), a_S(c) = a_N(c-nx), a_B(c) = a_T(c-P), checked per
 * call) its finest-level passes read W, S, B from the E, N, T arrays.
 * Selecting multigrid also re-tiles the context's sets to at most 8 planes
 * per chunk (the fine-level passes need more blocks than the Jacobi step;
 * $EQS_MG_KC overrides); selecting Jacobi again restores the tuned tiling.
 * params NULL selects the defaults.  Allocates the level hierarchy (about
 * 1.3 words per cell, plus 7 FP32 words per finest cell) here, not in the
 * solves.  Returns EQS_OK, EQS_ERR_ARG
 * (kind, params, or a context that is not EQS_FP64), EQS_ERR_NOMEM,
 * EQS_ERR_HIP or EQS_ERR_STATE.
 */
int eqsolve_set_preconditioner(eqs_ctx *ctx, int32_t kind, const eqs_mg_params *params);

/*
 * Diagnostics: z = B^-1 r, one V-cycle of the multigrid preconditioner of set
 * `set`, built from the diagonals diag (device arrays as in eqsolve_solve;
 * r and z device arrays of the set's size, z not aliasing r).  *levels (host,
 * may be NULL) receives the number of levels.  Returns EQS_OK, EQS_ERR_ARG
 * (multigrid not selected, bad pointers), EQS_ERR_HIP or EQS_ERR_STATE.
 */
int eqsolve_debug_precond(eqs_ctx *ctx, int32_t set, const double *const diag[7], const double *r, double *z,
                          int32_t *levels);

/*
 * Largest system eqsolve_solve_noalloc takes: EQS_NOALLOC_MAX_CELLS cells, and
 * a workspace (18 FP64 words per cell, per-block reduction partials, the set
 * table and state block) of at most EQS_NOALLOC_BYTES bytes.
 */
#define EQS_NOALLOC_MAX_CELLS 262144
#define EQS_NOALLOC_BYTES (40u << 20)

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the plain FP64 solve of
 * eqsolve_solve (Jacobi-preconditioned BiCGSTAB, the single-sync iteration)
 * for one system on grid *grid, with no context.  Its workspace is a static
 * device array of EQS_NOALLOC_BYTES bytes in this library, one per GPU, held
 * from the first call on that GPU until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or host heap), launches its kernels one by
 * one on hip_stream (a hipStream_t; NULL = the default stream) and returns
 * after they complete.  The caller passes the inputs and the output exactly
 * as for eqsolve_solve: diag[7], b and x (x0 on entry, solution on return)
 * are device arrays of nx*ny*nz FP64 values on the current device; tol in
 * (0, 1), maxit >= 1; info (host, may be NULL) receives the outcome.
 * Every call on one GPU shares that GPU's array and clears the part it uses
 * first: calls that overlap on one GPU (two threads, or two streams) race,
 * and must not be made.
 * Returns the EQS_* code of the solve, EQS_ERR_ARG (bad pointers, sizes, tol
 * or maxit, aliasing; checked before any HIP call), EQS_ERR_SIZE (more than
 * EQS_NOALLOC_MAX_CELLS cells, or a workspace beyond EQS_NOALLOC_BYTES), or
 * EQS_ERR_HIP.
 */
int eqsolve_solve_noalloc(const eqs_grid *grid, const double *const diag[7], const double *b, double *x,
                          double tol, int32_t maxit, eqs_info *info, void *hip_stream);

/* Static description of a result code. */
const char *eqsolve_strerror(int code);

/*
 * Diagnostics: the launch layout of set `set` (chosen at create time or by
 * eqsolve_autotune).  out8 (host, 12 entries) receives cells per thread,
 * segments per plane, planes per chunk, chunks, tiles, the number of host
 * state readbacks so far, the grid-wide reductions per BiCGSTAB step of the
 * iteration in use (1: one fused launch per step; 3: three launches), the
 * blocks of the pointwise kernels, and for the single-sync step its threads per
 * block (256 or 512), segments per plane, tiles, and tile order (0: chunks of a
 * segment adjacent in the launch, 1: segments of a chunk adjacent).  Returns
 * EQS_OK or EQS_ERR_ARG.
 */
int eqsolve_debug_layout(const eqs_ctx *ctx, int32_t set, int32_t *out8);

/*
 * Diagnostics: every `every`-th launch of a kernel kind whose bit is set in
 * kind_mask (bit k for kind k, see eqsolve_debug_kernel_stats) is bracketed
 * by two HIP events on the context's stream, and its duration is added to a
 * per-kind total (resolved at each state readback).  kind_mask 0 turns timing
 * off.  Any call resets the totals.  Returns EQS_OK, EQS_ERR_ARG (every < 1)
 * or EQS_ERR_STATE.
 */
int eqsolve_debug_profile(eqs_ctx *ctx, int32_t kind_mask, int32_t every);

/*
 * Diagnostics: launches and total milliseconds recorded for kernel `kind`
 * (for the BiCGSTAB iteration kernels, only launches that did work: those
 * enqueued past a set's convergence are left out)
 * (0 setup, 1 recheck, 2 report, 3 K1, 4 K2, 5 K3, 6 cast, 7 outer residual,
 * 8 update, 9 zero, 10 gradient, 11 product, 12 scaling, 13 unscaling,
 * 14 fused single-sync step, 15 its set-up product f = M^T r^, 16 forming the
 * iterate on leaving it) in FP32 (fp32 = 1) or FP64.  Returns EQS_OK or
 * EQS_ERR_ARG (kind outside 0..31).
 */
int eqsolve_debug_kernel_stats(const eqs_ctx *ctx, int32_t kind, int32_t fp32, int64_t *count,
                               double *total_ms);

/*
 * Diagnostics, for reading the single-sync step's HBM rate: one launch of a
 * plain pointwise kernel over n cells that reads nr FP64 device arrays
 * in[0..nr) and writes nw FP64 device arrays out[0..nw), every word once and
 * coalesced (no stencil, halo, LDS or barrier); out[w][i] = w + sum_k (k+1)
 * in[k][i].  nr = 13 or 11 with nw = 5 is the per-cell mix of the step's
 * general or symmetric form; nontemporal != 0 writes with nontemporal stores,
 * as the step does.  Its rate is the practical streaming ceiling for those
 * words on the device.  in and out are host arrays of device pointers, each
 * array n values, no output aliasing an input; stream is a hipStream_t (NULL:
 * the default stream); the call enqueues and returns.  Returns EQS_OK,
 * EQS_ERR_ARG (null pointers, n < 1, another mix, aliasing) or EQS_ERR_HIP.
 */
int eqsolve_debug_stream(const double *const *in, int32_t nr, double *const *out, int32_t nw, int64_t n,
                         int32_t nontemporal, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EQSOLVE_H */
