/*
 * orc.c -- CPU oracle for the per-equation-set linear solve of equation
 * decomposition (Woo et al., "Development of an Equation-based
 * Parallelization Method for Multiphase Particle-in-Cell Simulations",
 * arXiv 2211.15605).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, constant or helper with
 * the HIP library; the two meet only through the seeded input generators.
 *
 * What it computes, and where that comes from:
 *  - Sec. 2.2.2: each equation set (u, v, w momentum, pressure correction)
 *    is one linear system solved by its own device; the solver's cost is its
 *    matrix-vector product and the dot products it needs every iteration.
 *  - Sec. 2.2.3: fields are flat rank-1 arrays over a structured mesh.
 *  - Sec. 3.1: verification runs in 64-bit precision, so everything here is
 *    double precision.
 *  - The paper names no Krylov method.  The method taken here is
 *    BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) with a
 *    right Jacobi preconditioner M = diag(a_P), in the preconditioned form of
 *    Barrett et al., "Templates for the Solution of Linear Systems", 1994.
 *    Right preconditioning keeps r the true residual b - A x.  M = I (the
 *    paper's own verification setting, Sec. 3: no preconditioner) is
 *    reachable with jacobi = 0.
 *
 * Discretised equation (Patankar form, 7-point finite-volume stencil):
 *     a_P[c] x[c] - sum_{nb in E,W,N,S,T,B} a_nb[c] x[nb(c)] = b[c]
 * flat index c = i + nx*(j + ny*k), i fastest; E/W = +-x, N/S = +-y,
 * T/B = +-z.  A neighbour outside the grid contributes nothing (its
 * coefficient is ignored).
 *
 * Dot products are summed in fixed 4096-element chunks, then the chunk sums
 * in index order, so every result is independent of the OpenMP thread count.
 *
 * Addition beyond the paper (its solver is unpreconditioned or Jacobi): an
 * aggregation multigrid V-cycle as a second right preconditioner, aimed at
 * the pressure-correction system, whose Jacobi iteration count grows with
 * the grid (Sec. 3.1 notes the pressure equation needs many more iterations
 * than momentum).  Its definition is below (orc_mg_*).
 *
 * Every function here is pinned by tests that do not retype it: closed-form
 * eigenpairs of constant-coefficient tridiagonal-Toeplitz Kronecker sums, the
 * adjoint identity, row-sum invariants, dense LU, banded LU, exact finite
 * termination, and central finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* coefficient slots of the 7-array argument */
#define SLOT_P 0
#define SLOT_E 1
#define SLOT_W 2
#define SLOT_N 3
#define SLOT_S 4
#define SLOT_T 5
#define SLOT_B 6

/* result codes (same meaning as the library's, defined independently) */
#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_BREAKDOWN 2
#define ORC_NONFINITE 3
#define ORC_BAD_ARG (-1)
#define ORC_NOMEM (-2)

#define ORC_CHUNK 4096

typedef struct {
    int32_t status;   /* ORC_* */
    int32_t iters;    /* number of products v = A p^ taken */
    int32_t restarts; /* fresh starts after the first (rho = 0, failed recheck) */
    int32_t half_exit;/* 1 if the last exit was on the s half-step test */
    double rel_res;   /* ||b - A x||_2 / ||b||_2, recomputed at exit */
} orc_info;

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* y = A x (transpose = 0) or y = A^T x (transpose = 1). */
void orc_apply(int nx, int ny, int nz, const double *const *a, const double *x,
               double *y, int transpose)
{
    const long sx = 1, sy = nx, sz = (long)nx * ny;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                long c = i + sy * j + sz * k;
                double acc = a[SLOT_P][c] * x[c];
                if (!transpose) {
                    /* row c of A */
                    if (i + 1 < nx) acc -= a[SLOT_E][c] * x[c + sx];
                    if (i > 0)      acc -= a[SLOT_W][c] * x[c - sx];
                    if (j + 1 < ny) acc -= a[SLOT_N][c] * x[c + sy];
                    if (j > 0)      acc -= a[SLOT_S][c] * x[c - sy];
                    if (k + 1 < nz) acc -= a[SLOT_T][c] * x[c + sz];
                    if (k > 0)      acc -= a[SLOT_B][c] * x[c - sz];
                } else {
                    /* row c of A^T = column c of A: cell c is the east
                     * neighbour of c-1, the west neighbour of c+1, the north
                     * neighbour of c-nx, and so on. */
                    if (i > 0)      acc -= a[SLOT_E][c - sx] * x[c - sx];
                    if (i + 1 < nx) acc -= a[SLOT_W][c + sx] * x[c + sx];
                    if (j > 0)      acc -= a[SLOT_N][c - sy] * x[c - sy];
                    if (j + 1 < ny) acc -= a[SLOT_S][c + sy] * x[c + sy];
                    if (k > 0)      acc -= a[SLOT_T][c - sz] * x[c - sz];
                    if (k + 1 < nz) acc -= a[SLOT_B][c + sz] * x[c + sz];
                }
                y[c] = acc;
            }
        }
    }
}

/* (u, v) summed in fixed chunks, chunk sums added in index order. */
double orc_dot(long n, const double *u, const double *v)
{
    long nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    if (nch == 0) return 0.0;
    double *part = (double *)malloc((size_t)nch * sizeof(double));
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nch; q++) {
        long lo = q * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        double s = 0.0;
        for (long c = lo; c < hi; c++) s += u[c] * v[c];
        part[q] = s;
    }
    double s = 0.0;
    for (long q = 0; q < nch; q++) s += part[q];
    free(part);
    return s;
}

/* r = b - A x (or b - A^T x); returns (r, r). */
static double residual(int nx, int ny, int nz, const double *const *a, int transpose,
                       const double *b, const double *x, double *r)
{
    long n = (long)nx * ny * nz;
    orc_apply(nx, ny, nz, a, x, r, transpose);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) r[c] = b[c] - r[c];
    return orc_dot(n, r, r);
}

/* ---------------------------------------------------------------- multigrid
 *
 * Aggregation multigrid V-cycle B^{-1}, used as a right preconditioner.
 *
 * Levels: level 0 is the system as passed; level l+1 has dimensions
 * ((nx+1)/2, (ny+1)/2, (nz+1)/2) (a dimension of 1 stays 1) and aggregates
 * the fine cells (i, j, k) with (i/2, j/2, k/2) equal.  Coarsening stops at
 * a level of at most coarse_cells cells (or 1 x 1 x 1).
 *
 * Interpolation P is piecewise constant (a coarse value copied to every
 * cell of its aggregate), restriction is R = P^T (sum over the aggregate)
 * and the coarse operator is the Galerkin product P^T A P, which is again a
 * 7-point operator in the same Patankar form:
 *   coarse a_P(C)  = sum over c in C of a_P(c), minus a_nb(c) for every link
 *                    from c to a neighbour inside C;
 *   coarse a_nb(C) = sum of a_nb(c) over the links from c in C to cells of
 *                    the neighbouring aggregate in direction nb.
 *
 * V-cycle at level l on right-hand side r (D = diag(a_P), weight omega):
 *   coarsest level: z = 0, then coarse_sweeps times z += omega D^{-1} (r - A z);
 *   otherwise:      z1 = omega D^{-1} r
 *                   e  = V-cycle at level l+1 on R (r - A z1)
 *                   z2 = z1 + gamma P e
 *                   z  = z2 + omega D^{-1} (r - A z2)
 * A fixed number of sweeps everywhere makes B^{-1} a fixed linear map, as
 * BiCGSTAB's preconditioner must be.
 */
typedef struct {
    double omega;       /* damped-Jacobi weight */
    double gamma;       /* scale of the coarse correction */
    int32_t coarse_sweeps;
    int32_t coarse_cells;
} orc_mg_params;

#define ORC_MG_MAX_LEVELS 24

typedef struct {
    int nlev;
    int dims[ORC_MG_MAX_LEVELS][3];
    double *coef[ORC_MG_MAX_LEVELS][7];  /* level 0 points at the caller's arrays */
    double *work;                          /* per level: q, z1, rc, e (largest level size) */
    orc_mg_params prm;
} orc_mg;

/* Galerkin coarse operator of one level (see above); returns 0, or ORC_BAD_ARG */
int orc_mg_coarsen(int nx, int ny, int nz, const double *const *a, int *cdims, double *const *ac)
{
    if (nx < 1 || ny < 1 || nz < 1 || !a || !cdims || !ac) return ORC_BAD_ARG;
    const int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
    cdims[0] = cx;
    cdims[1] = cy;
    cdims[2] = cz;
    const long nc = (long)cx * cy * cz;
    for (int q = 0; q < 7; q++) memset(ac[q], 0, (size_t)nc * sizeof(double));
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const long c = i + (long)nx * (j + (long)ny * k);
                const long C = i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2));
                ac[SLOT_P][C] += a[SLOT_P][c];
                /* each link: direction slot, neighbour (i2, j2, k2) */
                const int nbi[6] = {i + 1, i - 1, i, i, i, i};
                const int nbj[6] = {j, j, j + 1, j - 1, j, j};
                const int nbk[6] = {k, k, k, k, k + 1, k - 1};
                for (int d = 0; d < 6; d++) {
                    const int i2 = nbi[d], j2 = nbj[d], k2 = nbk[d];
                    if (i2 < 0 || i2 >= nx || j2 < 0 || j2 >= ny || k2 < 0 || k2 >= nz) continue;
                    const double coef = a[SLOT_E + d][c];
                    if (i2 / 2 == i / 2 && j2 / 2 == j / 2 && k2 / 2 == k / 2)
                        ac[SLOT_P][C] -= coef;        /* link inside the aggregate */
                    else
                        ac[SLOT_E + d][C] += coef;    /* link to the neighbouring aggregate */
                }
            }
    return 0;
}

static void mg_free(orc_mg *m)
{
    for (int l = 1; l < m->nlev; l++)
        free(m->coef[l][0]);
    free(m->work);
}

static int mg_build(orc_mg *m, int nx, int ny, int nz, const double *const *a, const orc_mg_params *prm)
{
    memset(m, 0, sizeof(*m));
    m->prm = *prm;
    m->nlev = 1;
    m->dims[0][0] = nx;
    m->dims[0][1] = ny;
    m->dims[0][2] = nz;
    for (int q = 0; q < 7; q++) m->coef[0][q] = (double *)a[q];
    for (;;) {
        const int l = m->nlev - 1;
        const int *dm = m->dims[l];
        const long n = (long)dm[0] * dm[1] * dm[2];
        if (n <= prm->coarse_cells || n == 1 || m->nlev == ORC_MG_MAX_LEVELS) break;
        const long nc = (long)((dm[0] + 1) / 2) * ((dm[1] + 1) / 2) * ((dm[2] + 1) / 2);
        double *blk = (double *)malloc((size_t)nc * 7 * sizeof(double));
        if (!blk) { mg_free(m); return ORC_NOMEM; }
        for (int q = 0; q < 7; q++) m->coef[l + 1][q] = blk + q * nc;
        orc_mg_coarsen(dm[0], dm[1], dm[2], (const double *const *)m->coef[l], m->dims[l + 1], m->coef[l + 1]);
        m->nlev++;
    }
    long tot = 0;
    for (int l = 0; l < m->nlev; l++) tot += 4L * m->dims[l][0] * m->dims[l][1] * m->dims[l][2];
    m->work = (double *)malloc((size_t)tot * sizeof(double));
    if (!m->work) { mg_free(m); return ORC_NOMEM; }
    return 0;
}

static void mg_vcycle(const orc_mg *m, int l, double *wk, const double *r, double *z)
{
    const int nx = m->dims[l][0], ny = m->dims[l][1], nz = m->dims[l][2];
    const long n = (long)nx * ny * nz;
    const double *const *a = (const double *const *)m->coef[l];
    const double *ap = a[SLOT_P];
    const double w = m->prm.omega;
    double *q = wk, *z1 = wk + n;
    if (l == m->nlev - 1) {
        for (long c = 0; c < n; c++) z[c] = 0.0;
        for (int it = 0; it < m->prm.coarse_sweeps; it++) {
            orc_apply(nx, ny, nz, a, z, q, 0);
            for (long c = 0; c < n; c++) z[c] += w * (r[c] - q[c]) / ap[c];
        }
        return;
    }
    const int cx = m->dims[l + 1][0], cy = m->dims[l + 1][1];
    const long nc = (long)cx * cy * m->dims[l + 1][2];
    double *rc = wk + 2 * n, *e = rc + nc, *wk_next = e + nc;
    for (long c = 0; c < n; c++) z1[c] = w * r[c] / ap[c];
    orc_apply(nx, ny, nz, a, z1, q, 0);
    for (long C = 0; C < nc; C++) rc[C] = 0.0;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const long c = i + (long)nx * (j + (long)ny * k);
                rc[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))] += r[c] - q[c];
            }
    mg_vcycle(m, l + 1, wk_next, rc, e);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const long c = i + (long)nx * (j + (long)ny * k);
                z1[c] += m->prm.gamma * e[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))];
            }
    orc_apply(nx, ny, nz, a, z1, q, 0);
    for (long c = 0; c < n; c++) z[c] = z1[c] + w * (r[c] - q[c]) / ap[c];
}

/* z = B^{-1} r: one V-cycle of the hierarchy built for this system.  levels, if
 * not NULL, receives the number of levels. */
int orc_mg_apply(int nx, int ny, int nz, const double *const *a, const orc_mg_params *prm, const double *r,
                 double *z, int *levels)
{
    if (nx < 1 || ny < 1 || nz < 1 || !a || !prm || !r || !z || prm->coarse_sweeps < 1 || prm->coarse_cells < 1)
        return ORC_BAD_ARG;
    orc_mg m;
    int rc = mg_build(&m, nx, ny, nz, a, prm);
    if (rc) return rc;
    /* the work layout of a level holds the next level's after its own q, z1, rc, e */
    mg_vcycle(&m, 0, m.work, r, z);
    if (levels) *levels = m.nlev;
    mg_free(&m);
    return 0;
}

/* the preconditioner of the BiCGSTAB below */
typedef struct {
    int kind;             /* 0: M = I, 1: Jacobi, 2: multigrid */
    const double *ap;
    const orc_mg *mg;
} orc_pc;

/* w = M^{-1} u */
static void precond(long n, const orc_pc *pc, const double *u, double *w)
{
    if (pc->kind == 2) {
        mg_vcycle(pc->mg, 0, pc->mg->work, u, w);
        return;
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; c++) w[c] = pc->kind == 1 ? u[c] / pc->ap[c] : u[c];
}

static int all_finite(long n, const double *u)
{
    int ok = 1;
#pragma omp parallel for reduction(&& : ok) schedule(static)
    for (long c = 0; c < n; c++) ok = ok && isfinite(u[c]);
    return ok;
}

/*
 * Right-preconditioned BiCGSTAB (van der Vorst 1992; Templates 1994).
 *
 *   r = b - A x0, r^ = r; stop at once if ||b|| = 0 (x = 0) or ||r|| <= tol ||b||.
 *   rho_prev = alpha = omega = 1, p = v = 0, then repeat:
 *     rho  = (r^, r)                          [rho = 0: fresh start once]
 *     beta = (rho / rho_prev) (alpha / omega)
 *     p    = r + beta (p - omega v);  p^ = M^{-1} p;  v = A p^
 *     alpha = rho / (r^, v)                   [(r^, v) = 0: breakdown]
 *     s    = r - alpha v                      [||s|| <= tol ||b||: x += alpha p^, stop]
 *     s^   = M^{-1} s;  t = A s^
 *     omega = (t, s) / (t, t)                 [(t, t) = 0: omega = 0]
 *     x   += alpha p^ + omega s^;  r = s - omega t
 *                                             [||r|| <= tol ||b||: stop]
 *                                             [omega = 0: breakdown]
 *   On a stop by the recursive residual, r = b - A x is recomputed; if it is
 *   above tol the iteration starts afresh from it (r^ = r), within maxit.
 *
 * transpose = 1 solves A^T x = b instead (the adjoint system); the Jacobi
 * preconditioner is the same, since A and A^T share their diagonal.
 * x holds x0 on entry and the last iterate on return.  hist, if not NULL,
 * receives ||r||_2 / ||b||_2 after every iteration (maxit entries).
 */
static int bicgstab_core(int nx, int ny, int nz, const double *const *a, const double *b, double *x, double tol,
                         int maxit, orc_pc *pc, int transpose, orc_info *info, double *hist);

int orc_bicgstab(int nx, int ny, int nz, const double *const *a, const double *b,
                 double *x, double tol, int maxit, int jacobi, int transpose,
                 orc_info *info, double *hist)
{
    orc_pc pc = {jacobi ? 1 : 0, a ? a[SLOT_P] : NULL, NULL};
    return bicgstab_core(nx, ny, nz, a, b, x, tol, maxit, &pc, transpose, info, hist);
}

/* The same BiCGSTAB with the multigrid V-cycle (orc_mg_params) as the right
 * preconditioner; the hierarchy is built once, from the system's diagonals.
 * levels, if not NULL, receives the number of levels. */
int orc_bicgstab_mg(int nx, int ny, int nz, const double *const *a, const double *b, double *x, double tol,
                    int maxit, const orc_mg_params *prm, orc_info *info, double *hist, int *levels)
{
    orc_info loc;
    if (!info) info = &loc;
    memset(info, 0, sizeof(*info));
    if (nx < 1 || ny < 1 || nz < 1 || !a || !prm || prm->coarse_sweeps < 1 || prm->coarse_cells < 1) {
        info->status = ORC_BAD_ARG;
        return info->status;
    }
    for (int q = 0; q < 7; q++)
        if (!a[q]) { info->status = ORC_BAD_ARG; return info->status; }
    orc_mg m;
    if (mg_build(&m, nx, ny, nz, a, prm)) { info->status = ORC_NOMEM; return info->status; }
    if (levels) *levels = m.nlev;
    orc_pc pc = {2, a[SLOT_P], &m};
    int st = bicgstab_core(nx, ny, nz, a, b, x, tol, maxit, &pc, 0, info, hist);
    mg_free(&m);
    return st;
}

static int bicgstab_core(int nx, int ny, int nz, const double *const *a, const double *b, double *x, double tol,
                         int maxit, orc_pc *pc, int transpose, orc_info *info, double *hist)
{
    orc_info loc;
    if (!info) info = &loc;
    memset(info, 0, sizeof(*info));
    if (nx < 1 || ny < 1 || nz < 1 || !a || !b || !x || !(tol > 0.0 && tol < 1.0) || maxit < 1) {
        info->status = ORC_BAD_ARG;
        return info->status;
    }
    for (int q = 0; q < 7; q++)
        if (!a[q]) { info->status = ORC_BAD_ARG; return info->status; }
    long n = (long)nx * ny * nz;
    if (pc->kind != 0) {
        for (long c = 0; c < n; c++)
            if (a[SLOT_P][c] == 0.0 || !isfinite(a[SLOT_P][c])) {
                info->status = ORC_BAD_ARG;
                return info->status;
            }
    }

    double *buf = (double *)malloc((size_t)n * 8 * sizeof(double));
    if (!buf) { info->status = ORC_NOMEM; return info->status; }
    double *r = buf, *rh = buf + n, *p = buf + 2 * n, *v = buf + 3 * n;
    double *ph = buf + 4 * n, *s = buf + 5 * n, *sh = buf + 6 * n, *t = buf + 7 * n;

    double bb = orc_dot(n, b, b);
    if (!isfinite(bb) || !all_finite(n, x)) {
        info->status = ORC_NONFINITE;
        info->rel_res = NAN;
        free(buf);
        return info->status;
    }
    if (bb == 0.0) {
        /* b = 0: the solution of a nonsingular system is x = 0 */
        memset(x, 0, (size_t)n * sizeof(double));
        info->status = ORC_OK;
        info->rel_res = 0.0;
        free(buf);
        return info->status;
    }
    const double bnorm = sqrt(bb);
    const double lim = tol * bnorm;

    double rr = residual(nx, ny, nz, a, transpose, b, x, r);
    if (!isfinite(rr)) {
        info->status = ORC_NONFINITE;
        info->rel_res = NAN;
        free(buf);
        return info->status;
    }

    int status = ORC_NOT_CONVERGED;
    int rho_zero_restarts = 0;
    int iters = 0;
    int fresh = 1;
    double rho = 0.0, rho_prev = 1.0, alpha = 1.0, omega = 1.0;

    if (sqrt(rr) <= lim) {
        status = ORC_OK;
        goto done;
    }

    for (;;) {
        if (fresh) {
            /* fresh start from the current r */
            memcpy(rh, r, (size_t)n * sizeof(double));
            memset(p, 0, (size_t)n * sizeof(double));
            memset(v, 0, (size_t)n * sizeof(double));
            rho_prev = alpha = omega = 1.0;
            fresh = 0;
        }
        if (iters >= maxit) { status = ORC_NOT_CONVERGED; break; }

        rho = orc_dot(n, rh, r);
        if (!isfinite(rho)) { status = ORC_NONFINITE; break; }
        if (rho == 0.0) {
            /* r has become orthogonal to the shadow residual */
            if (rho_zero_restarts++ > 0) { status = ORC_BREAKDOWN; break; }
            info->restarts++;
            fresh = 1;
            continue;
        }
        double beta = (rho / rho_prev) * (alpha / omega);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) p[c] = r[c] + beta * (p[c] - omega * v[c]);
        precond(n, pc, p, ph);
        orc_apply(nx, ny, nz, a, ph, v, transpose);
        iters++;

        double sigma = orc_dot(n, rh, v);
        if (!isfinite(sigma)) { status = ORC_NONFINITE; break; }
        if (sigma == 0.0) { status = ORC_BREAKDOWN; break; }
        alpha = rho / sigma;
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) s[c] = r[c] - alpha * v[c];

        double ss = orc_dot(n, s, s);
        if (!isfinite(ss)) { status = ORC_NONFINITE; break; }
        if (sqrt(ss) <= lim) {
            /* half-step exit: x_{k+1/2} already meets the tolerance */
#pragma omp parallel for schedule(static)
            for (long c = 0; c < n; c++) x[c] += alpha * ph[c];
            if (hist) hist[iters - 1] = sqrt(ss) / bnorm;
            info->half_exit = 1;
            goto recheck;
        }

        precond(n, pc, s, sh);
        orc_apply(nx, ny, nz, a, sh, t, transpose);
        double ts = orc_dot(n, t, s);
        double tt = orc_dot(n, t, t);
        if (!isfinite(ts) || !isfinite(tt)) { status = ORC_NONFINITE; break; }
        omega = tt == 0.0 ? 0.0 : ts / tt;
#pragma omp parallel for schedule(static)
        for (long c = 0; c < n; c++) {
            x[c] += alpha * ph[c] + omega * sh[c];
            r[c] = s[c] - omega * t[c];
        }
        rr = orc_dot(n, r, r);
        if (!isfinite(rr)) { status = ORC_NONFINITE; break; }
        if (hist) hist[iters - 1] = sqrt(rr) / bnorm;
        if (sqrt(rr) <= lim) {
            info->half_exit = 0;
            goto recheck;
        }
        if (omega == 0.0) { status = ORC_BREAKDOWN; break; }
        rho_prev = rho;
        continue;

    recheck:
        /* the recursive residual met tol: confirm with the true residual */
        rr = residual(nx, ny, nz, a, transpose, b, x, r);
        if (!isfinite(rr)) { status = ORC_NONFINITE; break; }
        if (sqrt(rr) <= lim) { status = ORC_OK; break; }
        if (iters >= maxit) { status = ORC_NOT_CONVERGED; break; }
        info->restarts++;
        fresh = 1;
    }

done:
    rr = residual(nx, ny, nz, a, transpose, b, x, r);
    info->status = status;
    info->iters = iters;
    info->rel_res = sqrt(rr) / bnorm;
    free(buf);
    return status;
}

/*
 * Gradient of a loss L(x) through x = A^{-1} b, given lambda = A^{-T} dL/dx.
 * With A_cc = a_P[c] and A_{c,nb} = -a_nb[c]:
 *     dL/db      = lambda
 *     dL/da_P[c] = -lambda[c] x[c]
 *     dL/da_nb[c] = +lambda[c] x[nb(c)], and 0 where nb(c) is outside the grid.
 * g[slot] receives dL/da_slot in the slot order P, E, W, N, S, T, B.
 */
void orc_grad(int nx, int ny, int nz, const double *lam, const double *x, double *const *g)
{
    const long sy = nx, sz = (long)nx * ny;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                long c = i + sy * j + sz * k;
                double l = lam[c];
                g[SLOT_P][c] = -l * x[c];
                g[SLOT_E][c] = i + 1 < nx ? l * x[c + 1] : 0.0;
                g[SLOT_W][c] = i > 0 ? l * x[c - 1] : 0.0;
                g[SLOT_N][c] = j + 1 < ny ? l * x[c + sy] : 0.0;
                g[SLOT_S][c] = j > 0 ? l * x[c - sy] : 0.0;
                g[SLOT_T][c] = k + 1 < nz ? l * x[c + sz] : 0.0;
                g[SLOT_B][c] = k > 0 ? l * x[c - sz] : 0.0;
            }
        }
    }
}
