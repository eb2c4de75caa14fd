/*
 * eqsimple.h -- C ABI of the SIMPLE iteration on a gas-only bed box (gfx950).
 *
 * The operation: one time step of the paper's gas phase (arXiv 2211.15605,
 * Sec. 2.1, Eqs. (1)-(2), with no parcels: volume fraction 1 and no drag
 * term) advanced by SIMPLE iterations as MFiX does (Sec. 2.2.2): form and
 * solve the u, v and w momentum systems, form and solve the
 * pressure-correction system p', correct pressure and velocities.  Matrix
 * formation and solves both stay on the device (Sec. 2.2.2), the three
 * momentum systems go through one batched solve (the single-device
 * assignment "111[1]"), the p' system through its own solve.
 *
 * The box (Sec. 3, verification case, without particles): gravity along -y;
 * gas enters through the bottom plane y = 0 at a uniform speed v_in and
 * leaves through the top plane y = Ly, where the pressure of a ghost cell
 * above the last row is 0 and every velocity has zero gradient; the four
 * vertical planes are no-slip walls.  Staggered finite volumes: p and p' at
 * cell centres (nx*ny*nz), u on x-faces ((nx+1)*ny*nz), v on y-faces
 * (nx*(ny+1)*nz), w on z-faces (nx*ny*(nz+1)); every array is flat with
 * index i + NX*(j + NY*k) over its own grid dimensions (NX, NY, NZ).
 * First-order upwind convection, central diffusion (mu times the Laplacian),
 * implicit Euler in time (Patankar 1980, ch. 5-6).  Each momentum row:
 *     a_P x_P - sum a_nb x_nb = b
 * with a_P = (sum a_nb + conductances towards boundary values + rho V/dt)
 * / alpha_u and b = rho V/dt x_old + pressure force + gravity
 * + (1 - alpha_u) a_P x*, x* the incoming iterate; d = A / a_P is the face
 * velocity change per unit p' difference.  Velocities on walls and on the
 * inlet are fixed-value rows (a_P = rho V/dt, b = a_P * value, d = 0).  The
 * p' rows are the continuity balance of each cell with every face velocity
 * written as its predicted value plus d times the p' difference across it
 * (symmetric, a_P = sum a_nb plus the outlet term).  Correction: each face
 * velocity takes d times the p' difference across it, p takes alpha_p p'.
 *
 * Conventions as in eqsolve.h: DEVICE pointers to contiguous FP64 arrays on
 * the context's device, owned by the caller; work is enqueued on the
 * context's stream; a context is bound to one stream and not thread-safe;
 * < 0 return = error found before any work was done (nothing written).
 */
#ifndef EQSIMPLE_H
#define EQSIMPLE_H

#include <stdint.h>

#include "eqsolve.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eqsimple_ctx eqsimple_ctx;

typedef struct {
    int32_t nx, ny, nz;  /* pressure cells; 1 <= nx <= 1023, ny, nz >= 1, every grid < 2^30 cells */
    int32_t pad;
    double hx, hy, hz;   /* cell sizes (m), > 0 */
    double rho;          /* gas density (kg/m^3), > 0 */
    double mu;           /* gas viscosity (Pa s), >= 0 */
    double dt;           /* time step (s), > 0 */
    double gy;           /* gravity along y (m/s^2; negative = downwards) */
    double v_in;         /* inlet speed at y = 0 (m/s) */
    double alpha_u;      /* momentum under-relaxation, in (0, 1] */
    double alpha_p;      /* pressure under-relaxation, in (0, 1] */
} eqs_box;

typedef struct {
    int32_t status;          /* worst EQS_* status (>= 0) of the call's solves */
    int32_t iters[4];        /* BiCGSTAB iterations of the last SIMPLE iteration's solves: p', u, v, w */
    int32_t simple_iters;    /* SIMPLE iterations the call ran */
    double mom_residual[3];  /* ||b - A x*||_2 of the u, v, w rows at the incoming iterate x* */
    double mass_residual;    /* ||b'||_2: mass imbalance of the predicted velocities (kg/s) */
} eqs_simple_info;

/*
 * Create a context for one box: two solver contexts on `hip_stream` (the
 * three momentum grids, in `precision`, one EQS_* precision of eqsolve.h;
 * the p' grid in FP64) and the work arrays of one SIMPLE iteration (8 FP64
 * arrays per system, 3 d arrays, p', partial sums) and of a time step (the
 * 3 old-time velocity fields).  Returns EQS_OK,
 * EQS_ERR_ARG (box values out of range, precision), EQS_ERR_NOMEM or
 * EQS_ERR_HIP; *ctx is NULL unless EQS_OK.
 */
int eqsimple_create(eqsimple_ctx **ctx, const eqs_box *box, int32_t precision, void *hip_stream);

/*
 * Momentum formation (fused: mass fluxes, upwind and diffusion coefficients,
 * boundary conductances, transient term, pressure force, gravity and
 * under-relaxation in one pass, no intermediate face arrays).
 * vel[3] = u, v, w (the incoming iterate x*), p, old[3] = u, v, w at the old
 * time level.  Outputs: diag[21] = the 7 diagonals (P, E, W, N, S, T, B) of
 * u, then of v, then of w; b[3]; d[3].  res2 (host, may be NULL): the
 * squared norms ||b - A x*||^2 of the three systems; when given, the call
 * returns after the work is complete, otherwise it only enqueues it.
 * Outputs must not alias inputs.  Returns EQS_OK, EQS_ERR_ARG (null
 * pointer), EQS_ERR_HIP or EQS_ERR_STATE.
 */
int eqsimple_form_momentum(eqsimple_ctx *ctx, const double *const vel[3], const double *p,
                           const double *const old[3], double *const diag[21], double *const b[3],
                           double *const d[3], double res2[3]);

/*
 * Pressure-correction formation: from d[3] and the predicted velocities
 * vel[3], the 7 diagonals and right-hand side (the mass imbalance) of p'.
 * mass2 (host, may be NULL): ||b'||^2, as for res2 above.  Returns as
 * eqsimple_form_momentum.
 */
int eqsimple_form_pressure(eqsimple_ctx *ctx, const double *const d[3], const double *const vel[3],
                           double *const diag[7], double *b, double *mass2);

/*
 * Correction, in place: vel[3] (u, v, w) take d times the p' difference
 * across their face, p takes alpha_p pp.  Enqueues only.  Returns EQS_OK,
 * EQS_ERR_ARG (null pointer), EQS_ERR_HIP or EQS_ERR_STATE.
 */
int eqsimple_correct(eqsimple_ctx *ctx, const double *const d[3], const double *pp, double *const vel[3],
                     double *p);

/*
 * niter SIMPLE iterations of one time step, in place on vel[3] and p, with
 * old[3] the old-time velocities: each forms the momentum systems, solves
 * them batched from the current velocities (tol[0], maxit[0]), forms p',
 * solves it from 0 (tol[1], maxit[1]) and corrects.  A solve that stops
 * short of its tolerance does not stop the iterations (MFiX likewise goes on
 * with partially converged solves); info (host, may be NULL) describes the
 * last iteration.  Returns EQS_OK, EQS_ERR_ARG (null pointer, niter < 1,
 * tol not in (0,1), maxit < 1), EQS_ERR_HIP or EQS_ERR_STATE, or the first
 * negative code of a solve (then the fields hold the iteration's partial
 * work).
 */
int eqsimple_iterate(eqsimple_ctx *ctx, double *const vel[3], double *p, const double *const old[3],
                     int32_t niter, const double tol[2], const int32_t maxit[2], eqs_simple_info *info);

/*
 * One time step in one call (the paper's one call into the device graph per
 * time step, Sec. 2.2.2): the current velocities vel[3] become the old-time
 * fields (copied into the context), then SIMPLE iterations as in
 * eqsimple_iterate run in place on vel[3] and p, at most max_iter, stopping
 * after the first iteration whose mass imbalance ||b'|| is at most mass_tol
 * times the first iteration's (mass_tol = 0: all max_iter).  info reports the
 * SIMPLE iterations run.  Returns as eqsimple_iterate; EQS_ERR_ARG also for
 * max_iter < 1 or mass_tol outside [0, 1).
 */
int eqsimple_step(eqsimple_ctx *ctx, double *const vel[3], double *p, int32_t max_iter, double mass_tol,
                  const double tol[2], const int32_t maxit[2], eqs_simple_info *info);

/*
 * Preconditioner of the p' solves (eqsolve_set_preconditioner on the
 * context's p' solver).  Returns its codes.
 */
int eqsimple_set_pressure_preconditioner(eqsimple_ctx *ctx, int32_t kind, const eqs_mg_params *params);

/* Free the context (waits for its stream first).  NULL is accepted. */
int eqsimple_destroy(eqsimple_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* EQSIMPLE_H */
