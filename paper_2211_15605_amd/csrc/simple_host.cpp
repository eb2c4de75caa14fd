// simple_host.cpp -- the eqsimple C ABI: SIMPLE iterations of a gas-only bed
// box on one device.
//
// A context owns the systems of one SIMPLE iteration (7 diagonals and b of
// u, v, w and p', d of u, v, w, p', partial sums) and two solver contexts on
// the caller's stream: one for the three momentum grids (solved in one
// batched call) and one for the p' grid.  An iteration enqueues the
// momentum formation, the batched momentum solve (from the current
// velocities), the p' formation, the p' solve (from 0) and the correction;
// fields and systems never leave the device, only the solvers' status words
// and four residual norms cross to the host (arXiv 2211.15605, Sec. 2.2.2:
// formation and solve on the device, one call per time step).

#include <hip/hip_runtime_api.h>
#include <stdlib.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "eqsimple.h"
#include "simple_internal.h"

using namespace eqsim;

// the uniform values of BoxK are formed exactly as the kernels would form them
#pragma clang fp contract(off)

struct eqsimple_ctx {
    eqs_box box{};
    BoxK bk{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool broken = false;
    eqs_ctx *mom = nullptr, *prs = nullptr;
    long n[4] = {0, 0, 0, 0};   // cells of u, v, w, p'
    int nb[4] = {0, 0, 0, 0};   // blocks of u, v, w, p' at one cell per thread (correction)
    int nf[4] = {0, 0, 0, 0};   // blocks of the formation kernels
    int cpb[4] = {0, 0, 0, 0};  // their cells per block
    double *pool = nullptr;     // every work array below, one allocation
    double *a[4][7] = {};       // diagonals: u, v, w, p'
    double *b[4] = {};
    double *d[3] = {};
    double *pp = nullptr;
    double *old[3] = {};        // old-time velocities of eqsimple_step
    double *partials = nullptr;
    double *sums = nullptr;     // 4 device doubles
    double *sums_host = nullptr;  // pinned
};

namespace {

bool finite_pos(double x) { return isfinite(x) && x > 0; }

bool box_ok(const eqs_box *b) {
    if (!b) return false;
    if (b->nx < 1 || b->ny < 1 || b->nz < 1 || b->nx > 1023) return false;
    const double lim = (double)(1 << 30);
    const double nx = b->nx, ny = b->ny, nz = b->nz;
    if ((nx + 1) * ny * nz > lim || nx * (ny + 1) * nz > lim || nx * ny * (nz + 1) > lim) return false;
    if (!finite_pos(b->hx) || !finite_pos(b->hy) || !finite_pos(b->hz) || !finite_pos(b->rho) || !finite_pos(b->dt))
        return false;
    if (!isfinite(b->mu) || b->mu < 0 || !isfinite(b->gy) || !isfinite(b->v_in)) return false;
    if (!(b->alpha_u > 0 && b->alpha_u <= 1) || !(b->alpha_p > 0 && b->alpha_p <= 1)) return false;
    return true;
}

BoxK to_k(const eqs_box &b) {
    BoxK k{};
    k.nx = b.nx;
    k.ny = b.ny;
    k.nz = b.nz;
    k.hx = b.hx;
    k.hy = b.hy;
    k.hz = b.hz;
    k.rho = b.rho;
    k.mu = b.mu;
    k.dt = b.dt;
    k.gy = b.gy;
    k.v_in = b.v_in;
    k.alpha_u = b.alpha_u;
    k.alpha_p = b.alpha_p;
    k.Ax = b.hy * b.hz;
    k.Ay = b.hx * b.hz;
    k.Az = b.hx * b.hy;
    k.V = b.hx * b.hy * b.hz;
    k.aP0 = b.rho * k.V / b.dt;
    k.De = b.mu * k.Ax / b.hx;
    k.Dn = b.mu * k.Ay / b.hy;
    k.Dt = b.mu * k.Az / b.hz;
    k.rAx = b.rho * k.Ax;
    k.rAy = b.rho * k.Ay;
    k.rAz = b.rho * k.Az;
    k.rgV = b.rho * b.gy * k.V;
    k.oma = 1.0 - b.alpha_u;
    return k;
}

int usable(const eqsimple_ctx *c) {
    if (!c || c->broken) return EQS_ERR_STATE;
    return EQS_OK;
}

int hip_fail(eqsimple_ctx *c) {
    c->broken = true;
    return EQS_ERR_HIP;
}

template <typename T>
bool all_set(const T *const *p, int k) {
    if (!p) return false;
    for (int q = 0; q < k; ++q)
        if (!p[q]) return false;
    return true;
}

hipError_t enqueue_form_momentum(eqsimple_ctx *c, const double *const vel[3], const double *p,
                                 const double *const old[3], double *const diag[21], double *const b[3],
                                 double *const d[3]) {
    MomArgs A{};
    A.bx = c->bk;
    A.u = vel[0];
    A.v = vel[1];
    A.w = vel[2];
    A.p = p;
    A.u0 = old[0];
    A.v0 = old[1];
    A.w0 = old[2];
    for (int s = 0; s < 3; ++s) {
        for (int q = 0; q < 7; ++q) A.a[s][q] = diag[7 * s + q];
        A.b[s] = b[s];
        A.d[s] = d[s];
        A.nb[s] = c->nf[s];
        A.cpb[s] = c->cpb[s];
    }
    A.partials = c->partials;
    hipError_t e = launch_form_momentum(A, c->stream);
    if (e != hipSuccess) return e;
    const int32_t begin[4] = {0, c->nf[0], c->nf[0] + c->nf[1], c->nf[0] + c->nf[1] + c->nf[2]};
    return launch_sum_ranges(c->partials, begin, 3, c->sums, c->stream);
}

hipError_t enqueue_form_pressure(eqsimple_ctx *c, const double *const d[3], const double *const vel[3],
                                 double *const diag[7], double *b) {
    PresArgs A{};
    A.bx = c->bk;
    A.du = d[0];
    A.dv = d[1];
    A.dw = d[2];
    A.u = vel[0];
    A.v = vel[1];
    A.w = vel[2];
    for (int q = 0; q < 7; ++q) A.a[q] = diag[q];
    A.b = b;
    A.partials = c->partials;
    A.cpb = c->cpb[3];
    hipError_t e = launch_form_pressure(A, c->nf[3], c->stream);
    if (e != hipSuccess) return e;
    const int32_t begin[2] = {0, c->nf[3]};
    return launch_sum_ranges(c->partials, begin, 1, c->sums + 3, c->stream);
}

hipError_t enqueue_correct(eqsimple_ctx *c, const double *const d[3], const double *pp, double *const vel[3],
                           double *p) {
    CorrArgs A{};
    A.bx = c->bk;
    A.du = d[0];
    A.dv = d[1];
    A.dw = d[2];
    A.pp = pp;
    A.u = vel[0];
    A.v = vel[1];
    A.w = vel[2];
    A.p = p;
    for (int s = 0; s < 4; ++s) A.nb[s] = c->nb[s];
    return launch_correct(A, c->stream);
}

// copy the 4 sums to the host and wait
hipError_t read_sums(eqsimple_ctx *c) {
    hipError_t e = hipMemcpyAsync(c->sums_host, c->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

// up to niter SIMPLE iterations; with mass_tol > 0 they stop once the mass imbalance of an
// iteration's predicted velocities is at most mass_tol times the first iteration's
int run_iterations(eqsimple_ctx *c, double *const vel[3], double *p, const double *const old[3], int32_t niter,
                   double mass_tol, const double tol[2], const int32_t maxit[2], eqs_simple_info *info) {
    int rc;
    double *diag_m[21];
    double *bm[3];
    for (int s = 0; s < 3; ++s) {
        for (int q = 0; q < 7; ++q) diag_m[7 * s + q] = c->a[s][q];
        bm[s] = c->b[s];
    }
    const double *const *vel_c = (const double *const *)vel;
    const double *diag_sets[3][7];
    const double *const *diag_ptrs[3];
    const double *b_sets[3];
    for (int s = 0; s < 3; ++s) {
        for (int q = 0; q < 7; ++q) diag_sets[s][q] = c->a[s][q];
        diag_ptrs[s] = diag_sets[s];
        b_sets[s] = c->b[s];
    }
    const double tols[3] = {tol[0], tol[0], tol[0]};
    const int32_t maxits[3] = {maxit[0], maxit[0], maxit[0]};
    const double *diag_p[7];
    for (int q = 0; q < 7; ++q) diag_p[q] = c->a[3][q];
    eqs_info mi[3], pi{};
    int worst = EQS_OK, done = 0;
    double mass0 = -1.0;
    for (int it = 0; it < niter; ++it) {
        if (enqueue_form_momentum(c, vel_c, p, old, diag_m, bm, c->d) != hipSuccess) return hip_fail(c);
        rc = eqsolve_solve_batched(c->mom, diag_ptrs, b_sets, vel, tols, maxits, mi);
        if (rc < 0) return rc;
        if (enqueue_form_pressure(c, c->d, vel_c, c->a[3], c->b[3]) != hipSuccess) return hip_fail(c);
        if (launch_zero(c->pp, c->n[3], c->stream) != hipSuccess) return hip_fail(c);
        rc = eqsolve_solve(c->prs, 0, diag_p, c->b[3], c->pp, tol[1], maxit[1], &pi);
        if (rc < 0) return rc;
        if (enqueue_correct(c, c->d, c->pp, vel, p) != hipSuccess) return hip_fail(c);
        worst = std::max({worst, pi.status, mi[0].status, mi[1].status, mi[2].status});
        ++done;
        if (mass_tol > 0) {
            if (read_sums(c) != hipSuccess) return hip_fail(c);
            const double m = sqrt(c->sums_host[3]);
            if (mass0 < 0) mass0 = m;
            if (m <= mass_tol * mass0) break;
        }
    }
    if (read_sums(c) != hipSuccess) return hip_fail(c);
    if (info) {
        memset(info, 0, sizeof(*info));
        info->status = worst;
        info->simple_iters = done;
        info->iters[0] = pi.iters;
        for (int s = 0; s < 3; ++s) {
            info->iters[1 + s] = mi[s].iters;
            info->mom_residual[s] = sqrt(c->sums_host[s]);
        }
        info->mass_residual = sqrt(c->sums_host[3]);
    }
    return EQS_OK;
}

bool solve_args_ok(const double tol[2], const int32_t maxit[2]) {
    if (!tol || !maxit) return false;
    for (int q = 0; q < 2; ++q)
        if (!(tol[q] > 0 && tol[q] < 1) || maxit[q] < 1) return false;
    return true;
}

}  // namespace

extern "C" {

int eqsimple_create(eqsimple_ctx **out, const eqs_box *box, int32_t precision, void *hip_stream) {
    if (!out) return EQS_ERR_ARG;
    *out = nullptr;
    if (!box_ok(box)) return EQS_ERR_ARG;
    if (precision != EQS_FP64 && precision != EQS_FP32_REFINE && precision != EQS_FP32) return EQS_ERR_ARG;
    eqsimple_ctx *c = new eqsimple_ctx;
    c->box = *box;
    c->bk = to_k(*box);
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return EQS_ERR_HIP;
    }
    const long nx = box->nx, ny = box->ny, nz = box->nz;
    c->n[0] = (nx + 1) * ny * nz;
    c->n[1] = nx * (ny + 1) * nz;
    c->n[2] = nx * ny * (nz + 1);
    c->n[3] = nx * ny * nz;
    for (int s = 0; s < 4; ++s) {
        c->nb[s] = blocks_for(c->n[s]);
        c->nf[s] = form_blocks(c->n[s]);
        c->cpb[s] = form_cells_per_block(c->n[s]);
    }
    const eqs_grid mg[3] = {{box->nx + 1, box->ny, box->nz}, {box->nx, box->ny + 1, box->nz},
                            {box->nx, box->ny, box->nz + 1}};
    const eqs_grid pg = {box->nx, box->ny, box->nz};
    int rc = eqsolve_create(&c->mom, mg, 3, precision, hip_stream);
    if (rc == EQS_OK) rc = eqsolve_create(&c->prs, &pg, 1, EQS_FP64, hip_stream);
    // The momentum rows converge in a step or two (their transient term dominates), so their FP64
    // solves skip the per-solve scale pass and read the formed coefficients directly
    // (EQS_SIMPLE_SCALED_MOM=1 keeps the scaled form, for comparison).
    if (rc == EQS_OK && precision == EQS_FP64) {
        const char *e = getenv("EQS_SIMPLE_SCALED_MOM");
        rc = eqsolve_set_step_form(c->mom, e && atoi(e) != 0 ? EQS_STEP_SCALED : EQS_STEP_UNSCALED);
    }
    if (rc != EQS_OK) {
        eqsolve_destroy(c->mom);
        eqsolve_destroy(c->prs);
        delete c;
        return rc;
    }
    // 8 arrays per system; d and the old-time velocity of u, v, w; p'; partials; sums
    // (each rounded up to 32 doubles)
    auto up = [](long v) { return (v + 31) / 32 * 32; };
    long total = 0;
    for (int s = 0; s < 4; ++s) total += 8 * up(c->n[s]);
    for (int s = 0; s < 3; ++s) total += 2 * up(c->n[s]);   // d, old-time velocity
    total += up(c->n[3]);
    const long nparts = std::max((long)c->nf[0] + c->nf[1] + c->nf[2], (long)c->nf[3]);
    total += up(nparts) + 32;
    if (hipMalloc((void **)&c->pool, total * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        eqsolve_destroy(c->mom);
        eqsolve_destroy(c->prs);
        delete c;
        return EQS_ERR_NOMEM;
    }
    double *q = c->pool;
    for (int s = 0; s < 4; ++s) {
        for (int k = 0; k < 7; ++k) {
            c->a[s][k] = q;
            q += up(c->n[s]);
        }
        c->b[s] = q;
        q += up(c->n[s]);
    }
    for (int s = 0; s < 3; ++s) {
        c->d[s] = q;
        q += up(c->n[s]);
        c->old[s] = q;
        q += up(c->n[s]);
    }
    c->pp = q;
    q += up(c->n[3]);
    c->partials = q;
    q += up(nparts);
    c->sums = q;
    q += 32;
    if (q - c->pool != total) {   // the layout above covers the allocation exactly (internal check)
        (void)hipFree(c->pool);
        eqsolve_destroy(c->mom);
        eqsolve_destroy(c->prs);
        delete c;
        return EQS_ERR_STATE;
    }
    if (hipHostMalloc((void **)&c->sums_host, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(c->pool);
        eqsolve_destroy(c->mom);
        eqsolve_destroy(c->prs);
        delete c;
        return EQS_ERR_NOMEM;
    }
    *out = c;
    return EQS_OK;
}

int eqsimple_form_momentum(eqsimple_ctx *c, const double *const vel[3], const double *p, const double *const old[3],
                           double *const diag[21], double *const b[3], double *const d[3], double res2[3]) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    if (!all_set(vel, 3) || !p || !all_set(old, 3) || !all_set(diag, 21) || !all_set(b, 3) || !all_set(d, 3))
        return EQS_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c);
    if (enqueue_form_momentum(c, vel, p, old, diag, b, d) != hipSuccess) return hip_fail(c);
    if (res2) {
        if (read_sums(c) != hipSuccess) return hip_fail(c);
        for (int s = 0; s < 3; ++s) res2[s] = c->sums_host[s];
    }
    return EQS_OK;
}

int eqsimple_form_pressure(eqsimple_ctx *c, const double *const d[3], const double *const vel[3],
                           double *const diag[7], double *b, double *mass2) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    if (!all_set(d, 3) || !all_set(vel, 3) || !all_set(diag, 7) || !b) return EQS_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c);
    if (enqueue_form_pressure(c, d, vel, diag, b) != hipSuccess) return hip_fail(c);
    if (mass2) {
        if (read_sums(c) != hipSuccess) return hip_fail(c);
        *mass2 = c->sums_host[3];
    }
    return EQS_OK;
}

int eqsimple_correct(eqsimple_ctx *c, const double *const d[3], const double *pp, double *const vel[3], double *p) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    if (!all_set(d, 3) || !pp || !all_set(vel, 3) || !p) return EQS_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c);
    if (enqueue_correct(c, d, pp, vel, p) != hipSuccess) return hip_fail(c);
    return EQS_OK;
}

int eqsimple_iterate(eqsimple_ctx *c, double *const vel[3], double *p, const double *const old[3], int32_t niter,
                     const double tol[2], const int32_t maxit[2], eqs_simple_info *info) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    if (!all_set(vel, 3) || !p || !all_set(old, 3) || niter < 1 || !solve_args_ok(tol, maxit)) return EQS_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c);
    return run_iterations(c, vel, p, old, niter, 0.0, tol, maxit, info);
}

int eqsimple_step(eqsimple_ctx *c, double *const vel[3], double *p, int32_t max_iter, double mass_tol,
                  const double tol[2], const int32_t maxit[2], eqs_simple_info *info) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    if (!all_set(vel, 3) || !p || max_iter < 1 || !(mass_tol >= 0 && mass_tol < 1) || !solve_args_ok(tol, maxit))
        return EQS_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c);
    for (int s = 0; s < 3; ++s)
        if (hipMemcpyAsync(c->old[s], vel[s], c->n[s] * sizeof(double), hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess)
            return hip_fail(c);
    const double *old_c[3] = {c->old[0], c->old[1], c->old[2]};
    return run_iterations(c, vel, p, old_c, max_iter, mass_tol, tol, maxit, info);
}

int eqsimple_set_pressure_preconditioner(eqsimple_ctx *c, int32_t kind, const eqs_mg_params *params) {
    int rc = usable(c);
    if (rc != EQS_OK) return rc;
    return eqsolve_set_preconditioner(c->prs, kind, params);
}

int eqsimple_destroy(eqsimple_ctx *c) {
    if (!c) return EQS_OK;
    int rc = EQS_OK;
    if (hipSetDevice(c->device) != hipSuccess) rc = EQS_ERR_HIP;
    if (c->stream && hipStreamSynchronize(c->stream) != hipSuccess) rc = EQS_ERR_HIP;
    eqsolve_destroy(c->mom);
    eqsolve_destroy(c->prs);
    if (c->pool && hipFree(c->pool) != hipSuccess) rc = EQS_ERR_HIP;
    if (c->sums_host && hipHostFree(c->sums_host) != hipSuccess) rc = EQS_ERR_HIP;
    delete c;
    return rc;
}

}  // extern "C"
