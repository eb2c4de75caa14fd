"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something that does not come from the
oracle's own code: closed-form eigenpairs of tridiagonal-Toeplitz Kronecker
sums, the adjoint identity, row-sum invariants of the generators, LAPACK
dense and banded solves, exact finite termination of Krylov methods,
a-posteriori error certificates, and central finite differences of a dense
solve.  ``test_oracle_mutants.py`` shows that plausible mistakes planted in a
copy of the oracle fail these pins.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from paper_2211_15605_amd import workloads as W

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- stencil product

def toeplitz_mode(n, p, sub, sup):
    """Eigenvector of tridiag(sub, 0, sup) (n x n): v_i = (sub/sup)^(i/2) sin(i p pi/(n+1)),
    eigenvalue 2 sqrt(sub*sup) cos(p pi/(n+1)); i = 1..n."""
    i = np.arange(1, n + 1)
    th = p * math.pi / (n + 1)
    return (sub / sup) ** (i / 2.0) * np.sin(i * th), 2.0 * math.sqrt(sub * sup) * math.cos(th)


def const_coeffs(shape, c, e, w):
    """Every slot constant, including slots that point out of the grid (must be ignored)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    return [np.full(n, c), np.full(n, e[0]), np.full(n, w[0]), np.full(n, e[1]), np.full(n, w[1]),
            np.full(n, e[2]), np.full(n, w[2])]


@pytest.mark.parametrize("shape", [(5, 4, 3), (7, 6, 5), (9, 2, 4)])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_closed_form_eigenpairs(orc, shape, transpose):
    # A = c I - (S_x (+) S_y (+) S_z), S_d = tridiag(a_W, 0, a_E) along axis d:
    # a Kronecker sum, so its eigenvectors are outer products of the 1-D modes.
    c = 13.0
    e = (0.7, 1.9, 0.35)   # a_E, a_N, a_T
    w = (2.3, 0.45, 1.6)   # a_W, a_S, a_B
    diags = const_coeffs(shape, c, e, w)
    nx, ny, nz = shape
    for modes in [(1, 1, 1), (2, 1, 1), (1, 2, 3), (nx, ny, nz)]:
        vs, lam = [], c
        for d, (n, p) in enumerate(zip(shape, modes)):
            sub, sup = (e[d], w[d]) if transpose else (w[d], e[d])
            v, mu = toeplitz_mode(n, min(p, n), sub, sup)
            vs.append(v)
            lam -= mu
        V = np.einsum("k,j,i->kji", vs[2], vs[1], vs[0]).ravel()
        AV = orc.apply(shape, diags, V, transpose=transpose)
        assert np.max(np.abs(AV - lam * V)) <= 64 * EPS * (c + sum(e) + sum(w)) * np.max(np.abs(V))


def test_apply_dirichlet_laplacian_eigenpair(orc):
    # the constant-coefficient 7-point Laplacian with zero ghost values
    shape = (6, 5, 4)
    diags = const_coeffs(shape, 6.0, (1, 1, 1), (1, 1, 1))
    p = (2, 3, 1)
    vs = [np.sin(np.pi * pp * np.arange(1, n + 1) / (n + 1)) for n, pp in zip(shape, p)]
    V = np.einsum("k,j,i->kji", vs[2], vs[1], vs[0]).ravel()
    lam = sum(2 - 2 * np.cos(np.pi * pp / (n + 1)) for n, pp in zip(shape, p))
    np.testing.assert_allclose(orc.apply(shape, diags, V), lam * V, atol=1e-13)


@pytest.mark.parametrize("recipe,margin", [("cd", 0.1), ("sym", 1e-3)])
def test_apply_row_sums_of_generated_systems(orc, recipe, margin):
    # the generators set a_P = sum(in-grid a_nb) + margin, so A 1 = margin in every row
    g = W.Grid(9, 7, 5)
    diags = W.coefficients(g, recipe, W.rng_for(7, 0))
    r = orc.apply(g.shape, diags, np.ones(g.n))
    np.testing.assert_allclose(r, margin, atol=32 * EPS * np.max(diags[0]))


def test_apply_row_sums_ignore_outward_slots(orc):
    # random values in every slot, outward ones included; a_P = sum(in-grid) + 0.5
    g = W.Grid(6, 5, 4)
    diags = W.random_general(g, seed=3)
    r = orc.apply(g.shape, diags, np.ones(g.n))
    np.testing.assert_allclose(r, 0.5, atol=1e-14)


@pytest.mark.parametrize("shape", [(6, 5, 4), (1, 7, 3), (8, 1, 1)])
def test_apply_adjoint_identity(orc, shape):
    g = W.Grid(*shape)
    diags = W.random_general(g, seed=5)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(g.n), rng.standard_normal(g.n)
    lhs = np.dot(orc.apply(shape, diags, y, transpose=True), x)
    rhs = np.dot(y, orc.apply(shape, diags, x))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_apply_symmetric_recipe_is_self_adjoint(orc):
    g = W.Grid(7, 6, 5)
    diags = W.coefficients(g, "sym", W.rng_for(7, 1))
    x = np.random.default_rng(2).standard_normal(g.n)
    np.testing.assert_allclose(orc.apply(g.shape, diags, x, True), orc.apply(g.shape, diags, x),
                               rtol=0, atol=1e-13)


def test_dot_against_exactly_rounded_sum(orc):
    rng = np.random.default_rng(3)
    n = 100_003
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    exact = math.fsum((u * v).tolist())
    nch = -(-n // 4096)
    bound = (4096 + nch) * EPS * float(np.sum(np.abs(u * v)))
    assert abs(orc.dot(u, v) - exact) <= bound


def test_dot_independent_of_thread_count(orc):
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(300_001), rng.standard_normal(300_001)
    old = orc.get_threads()
    try:
        orc.set_threads(1)
        d1 = orc.dot(u, v)
        orc.set_threads(5)
        d5 = orc.dot(u, v)
    finally:
        orc.set_threads(old)
    assert d1 == d5


# ---------------------------------------------------------------- solve

def dense_of(orc, g, diags):
    return orc.dense(g.shape, diags)


@pytest.mark.parametrize("side", [8, 16])
def test_bicgstab_matches_dense_lu(orc, side):
    g = W.Grid(side, side, side)
    s = W.make_set(0, 0, grid=g)
    A = dense_of(orc, g, s["diags"])
    b = A @ s["x_star"]
    x_lu = np.linalg.solve(A, b)
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=1e-13, maxit=1000)
    assert info["status"] == 0
    assert np.linalg.norm(b - A @ x) <= 1e-13 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_lu) <= 1e-10 * np.linalg.norm(x_lu)


@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-12])
@pytest.mark.parametrize("cfg", [0, 1])
def test_bicgstab_residual_invariant_and_certificate(orc, tol, cfg):
    g = W.Grid(12, 20, 10)
    s = W.make_set(cfg, 0, grid=g)
    A = scipy.sparse.csr_matrix(dense_of(orc, g, s["diags"]))
    b = A @ s["x_star"]
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=tol, maxit=5000)
    assert info["status"] == 0
    rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel <= tol
    assert abs(rel - info["rel_res"]) <= 1e-3 * rel + 1e-16
    # Varah: ||x - x*||_inf <= ||b - A x||_inf / min_c(a_P - sum|a_nb|)
    margin = 0.1 if cfg == 0 else 1e-3
    cert = np.max(np.abs(b - A @ x)) / margin
    assert np.max(np.abs(x - s["x_star"])) <= cert * (1 + 1e-6) + 1e-15


def test_bicgstab_jacobi_off_matches_lu(orc):
    # the paper's verification setting: no preconditioner
    g = W.Grid(8, 8, 8)
    s = W.make_set(0, 0, grid=g)
    A = dense_of(orc, g, s["diags"])
    b = A @ s["x_star"]
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=1e-13, maxit=2000, jacobi=False)
    assert info["status"] == 0
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-10)


def test_bicgstab_one_dimensional_matches_banded_lu(orc):
    g = W.Grid(40, 1, 1)
    s = W.make_set(0, 0, grid=g)
    P, E, Wd = s["diags"][0], s["diags"][1], s["diags"][2]
    n = g.n
    ab = np.zeros((3, n))
    ab[0, 1:] = -E[:-1]   # superdiagonal: row c, column c+1
    ab[1, :] = P
    ab[2, :-1] = -Wd[1:]  # subdiagonal: row c+1, column c
    b = np.random.default_rng(5).uniform(-1, 1, n)
    x_band = scipy.linalg.solve_banded((1, 1), ab, b)
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=1e-14, maxit=200)
    assert info["status"] == 0
    np.testing.assert_allclose(x, x_band, rtol=0, atol=1e-12)


def test_bicgstab_diagonal_system_exits_after_one_half_step(orc):
    # a_nb = 0: A M^{-1} = I, so s = r - alpha A p^ = 0 after the first product
    g = W.Grid(5, 4, 3)
    rng = np.random.default_rng(6)
    P = rng.uniform(1, 3, g.n)
    diags = [P] + [np.zeros(g.n)] * 6
    b = rng.uniform(-1, 1, g.n)
    x, info = orc.bicgstab(g.shape, diags, b, tol=1e-12, maxit=10)
    assert info["status"] == 0 and info["iters"] == 1 and info["half_exit"] == 1
    np.testing.assert_allclose(x, b / P, rtol=4 * EPS, atol=0)


@pytest.mark.parametrize("nx", [2, 3])
def test_bicgstab_finite_termination(orc, nx):
    # Krylov methods are exact after at most n steps in exact arithmetic
    g = W.Grid(nx, 1, 1)
    diags = W.random_general(g, seed=7 + nx)
    b = np.random.default_rng(8).uniform(-1, 1, g.n)
    x, info = orc.bicgstab(g.shape, diags, b, tol=1e-14, maxit=nx)
    A = dense_of(orc, g, diags)
    assert info["status"] == 0 and info["iters"] <= nx
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-13, atol=1e-14)


def test_bicgstab_exact_initial_guess_takes_no_iteration(orc):
    g = W.Grid(6, 6, 6)
    s = W.make_set(0, 0, grid=g)
    b = orc.apply(g.shape, s["diags"], s["x_star"])
    x, info = orc.bicgstab(g.shape, s["diags"], b, x0=s["x_star"], tol=1e-10)
    assert info["status"] == 0 and info["iters"] == 0
    assert np.array_equal(x, s["x_star"])


def test_bicgstab_zero_rhs_gives_zero(orc):
    g = W.Grid(4, 4, 4)
    s = W.make_set(0, 0, grid=g)
    x, info = orc.bicgstab(g.shape, s["diags"], np.zeros(g.n), x0=np.ones(g.n))
    assert info["status"] == 0 and info["iters"] == 0 and not np.any(x)


def test_bicgstab_status_codes(orc):
    g = W.Grid(6, 6, 6)
    s = W.make_set(0, 0, grid=g)
    b = orc.apply(g.shape, s["diags"], s["x_star"])
    # maxit too small: computed, not converged
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=1e-12, maxit=1)
    assert info["status"] == 1 and info["iters"] == 1 and info["rel_res"] > 1e-12
    # NaN in b
    bn = b.copy(); bn[7] = np.nan
    _, info = orc.bicgstab(g.shape, s["diags"], bn)
    assert info["status"] == 3
    # zero diagonal is an argument error
    d = [a.copy() for a in s["diags"]]; d[0][3] = 0.0
    _, info = orc.bicgstab(g.shape, d, b)
    assert info["status"] == -1
    # bad tolerance / maxit
    assert orc.bicgstab(g.shape, s["diags"], b, tol=0.0)[1]["status"] == -1
    assert orc.bicgstab(g.shape, s["diags"], b, maxit=0)[1]["status"] == -1


def test_bicgstab_breakdown_on_exact_integer_system(orc):
    # A = [[1, -2], [0, 1]] (a_P = 1, a_E(0) = 2), b = (1, 1), x0 = 0:
    # r = r^ = (1, 1) and (r^, A M^{-1} r) = 1 + 1 - 2 = 0 exactly.
    g = W.Grid(2, 1, 1)
    z = np.zeros(2)
    diags = [np.ones(2), np.array([2.0, 0.0]), z, z, z, z, z]
    x, info = orc.bicgstab(g.shape, diags, np.ones(2), tol=1e-10, maxit=10)
    assert info["status"] == 2 and info["iters"] == 1


def test_bicgstab_agrees_with_scipy_bicgstab(orc):
    # run-only cross-check against an independent library implementation
    g = W.Grid(10, 16, 8)
    s = W.make_set(1, 0, grid=g)
    A = scipy.sparse.csr_matrix(dense_of(orc, g, s["diags"]))
    b = A @ s["x_star"]
    Minv = scipy.sparse.diags(1.0 / s["diags"][0])
    xs, flag = scipy.sparse.linalg.bicgstab(A, b, rtol=1e-12, atol=0, maxiter=5000, M=Minv)
    assert flag == 0
    x, info = orc.bicgstab(g.shape, s["diags"], b, tol=1e-12, maxit=5000)
    assert info["status"] == 0
    xl = scipy.sparse.linalg.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xl) <= 1e-6 * np.linalg.norm(xl)
    assert np.linalg.norm(xs - xl) <= 1e-6 * np.linalg.norm(xl)


def test_bicgstab_thread_count_does_not_change_result(orc):
    g = W.Grid(20, 24, 16)
    s = W.make_set(0, 0, grid=g)
    b = orc.apply(g.shape, s["diags"], s["x_star"])
    old = orc.get_threads()
    try:
        orc.set_threads(1)
        x1, i1 = orc.bicgstab(g.shape, s["diags"], b)
        orc.set_threads(7)
        x7, i7 = orc.bicgstab(g.shape, s["diags"], b)
    finally:
        orc.set_threads(old)
    assert i1 == i7 and np.array_equal(x1, x7)


# ---------------------------------------------------------------- gradient

def test_grad_matches_finite_differences_of_dense_solve(orc):
    # L(a) = w . A(a)^{-1} b, differentiated entry by entry with central differences
    g = W.Grid(3, 3, 2)
    diags = W.random_general(g, seed=11)
    rng = np.random.default_rng(12)
    b, w = rng.standard_normal(g.n), rng.standard_normal(g.n)

    def loss(ds, bb):
        return float(w @ np.linalg.solve(orc.dense(g.shape, ds), bb))

    A = orc.dense(g.shape, diags)
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, w)
    G = orc.grad(g.shape, lam, x)
    h = 1e-6
    for slot in range(7):
        for c in range(g.n):
            dp = [a.copy() for a in diags]; dm = [a.copy() for a in diags]
            dp[slot][c] += h; dm[slot][c] -= h
            fd = (loss(dp, b) - loss(dm, b)) / (2 * h)
            assert abs(fd - G[slot][c]) <= 1e-7 * (1 + abs(fd)), (slot, c, fd, G[slot][c])
    # dL/db = lambda
    for c in range(g.n):
        bp = b.copy(); bm = b.copy(); bp[c] += h; bm[c] -= h
        assert abs((loss(diags, bp) - loss(diags, bm)) / (2 * h) - lam[c]) <= 1e-7 * (1 + abs(lam[c]))


def test_grad_through_oracle_solves_matches_directional_fd(orc):
    # the whole adjoint path on the oracle: x by BiCGSTAB, lambda by BiCGSTAB on A^T
    g = W.Grid(8, 8, 8)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    diags, w = s["diags"], s["w"]
    b = orc.apply(g.shape, diags, s["x_star"])
    x, i1 = orc.bicgstab(g.shape, diags, b, tol=1e-15, maxit=2000)
    rng = np.random.default_rng(13)
    # lambda = A^{-T} w by the oracle's transpose product and a dense solve of it
    AT = orc.dense(g.shape, diags, transpose=True)
    lam = np.linalg.solve(AT, w)
    G = orc.grad(g.shape, lam, x)
    h = 1e-6
    for _ in range(4):
        dirs = [rng.choice([-1.0, 0.0, 1.0], g.n, p=[0.05, 0.9, 0.05]) for _ in range(7)]
        dirs[0] = np.abs(dirs[0])
        db = rng.choice([-1.0, 0.0, 1.0], g.n, p=[0.05, 0.9, 0.05])
        pred = sum(float(G[k] @ dirs[k]) for k in range(7)) + float(lam @ db)

        def L(sign):
            d2 = [a + sign * h * dd for a, dd in zip(diags, dirs)]
            xx, ii = orc.bicgstab(g.shape, d2, b + sign * h * db, x0=x, tol=1e-15, maxit=2000)
            return float(w @ xx)

        fd = (L(+1) - L(-1)) / (2 * h)
        assert abs(fd - pred) <= 1e-5 * max(1.0, abs(pred)), (fd, pred)


# ---------------------------------------------------------------- helpers

def test_matching_digits_equation_6(orc):
    ref = np.array([1.0, 2.0, -3.0, 0.0])
    val = np.array([1.0 + 1e-9, 2.0, -3.003, 5.0])
    d = orc.matching_digits(ref, val)
    assert d.size == 3
    assert abs(d[0] - 9.0) < 1e-6 and d[1] == 17.0 and abs(d[2] - 3.0) < 1e-9


def test_bicgstab_transpose_matches_dense_lu(orc):
    # the adjoint system A^T lam = w against LAPACK on the numpy transpose of A
    g = W.Grid(8, 6, 5)
    s = W.make_set(3, 0, grid=g, with_weights=True)
    A = orc.dense(g.shape, s["diags"])
    lam, info = orc.bicgstab(g.shape, s["diags"], s["w"], tol=1e-13, maxit=1000, transpose=True)
    assert info["status"] == 0
    np.testing.assert_allclose(lam, np.linalg.solve(A.T, s["w"]), rtol=0, atol=1e-10)


# ---------------------------------------------------------------- multigrid preconditioner
# (an addition beyond the paper's method: aggregation multigrid as the right preconditioner)

def _aggregation_matrix(shape):
    """Piecewise-constant interpolation from the aggregate definition: fine cell (i, j, k)
    belongs to coarse cell (i // 2, j // 2, k // 2) of the ((nx+1)//2, (ny+1)//2, (nz+1)//2) grid."""
    nx, ny, nz = shape
    cx, cy, cz = (nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2
    P = np.zeros((nx * ny * nz, cx * cy * cz))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                P[i + nx * (j + ny * k), i // 2 + cx * (j // 2 + cy * (k // 2))] = 1.0
    return P


def _transposed_diagonals(shape, diags):
    """Diagonals of A^T in the same Patankar form: row c of A^T links to c+1 with A's
    coefficient from c+1 towards c (a_W[c+1]), and so on; a_P is shared."""
    nx, ny, nz = shape
    P_, E, Wd, N, S, T, B = [np.asarray(d, dtype=np.float64).reshape(nz, ny, nx) for d in diags]
    out = [P_.copy()] + [np.zeros_like(P_) for _ in range(6)]
    out[1][:, :, :-1] = Wd[:, :, 1:]
    out[2][:, :, 1:] = E[:, :, :-1]
    out[3][:, :-1, :] = S[:, 1:, :]
    out[4][:, 1:, :] = N[:, :-1, :]
    out[5][:-1, :, :] = B[1:, :, :]
    out[6][1:, :, :] = T[:-1, :, :]
    return [o.ravel() for o in out]


@pytest.mark.parametrize("shape", [(5, 3, 4), (4, 4, 4), (1, 6, 3), (7, 1, 1), (3, 5, 1), (2, 2, 2)])
def test_mg_coarse_operator_is_galerkin_product(orc, shape):
    g = W.Grid(*shape)
    diags = W.random_general(g, seed=31)
    A = orc.dense(shape, diags)
    Pm = _aggregation_matrix(shape)
    cshape, cd = orc.mg_coarsen(shape, diags)
    Ac = orc.dense(cshape, cd)
    ref = Pm.T @ A @ Pm
    assert np.max(np.abs(Ac - ref)) <= 1e-13 * np.max(np.abs(A))


def _mg_params(levels_small=True):
    from oracle import oracle as O
    return O.mg_params(omega=0.8, gamma=1.6, coarse_sweeps=5, coarse_cells=16 if levels_small else 512)


@pytest.mark.parametrize("recipe", ["cd", "sym"])
def test_mg_vcycle_transpose_identity(orc, recipe):
    # with R = P^T and Galerkin coarse operators, the V-cycle built for A^T is the
    # transpose of the one built for A: (u, B_A^{-1} v) = (B_{A^T}^{-1} u, v); for a
    # symmetric system that is the symmetry of B^{-1}
    shape = (11, 9, 7)
    g = W.Grid(*shape)
    diags = W.coefficients(g, recipe, W.rng_for(0, 5))
    dT = _transposed_diagonals(shape, diags)
    A = orc.dense((5, 4, 3), W.random_general(W.Grid(5, 4, 3), seed=2))
    AT = orc.dense((5, 4, 3), _transposed_diagonals((5, 4, 3), W.random_general(W.Grid(5, 4, 3), seed=2)))
    assert np.array_equal(A.T, AT)  # the helper itself is right
    rng = np.random.default_rng(7)
    u, v = rng.standard_normal(g.n), rng.standard_normal(g.n)
    zA, lev = orc.mg_apply(shape, diags, v, _mg_params())
    zT, _ = orc.mg_apply(shape, dT, u, _mg_params())
    assert lev >= 3
    lhs, rhs = float(u @ zA), float(zT @ v)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(zA)


def test_mg_vcycle_exact_on_diagonal_system_with_unit_weight(orc):
    from oracle import oracle as O
    g = W.Grid(9, 6, 5)
    rng = np.random.default_rng(3)
    ap = rng.uniform(1, 3, g.n)
    diags = [ap] + [np.zeros(g.n)] * 6
    r = rng.uniform(-1, 1, g.n)
    z, lev = orc.mg_apply(g.shape, diags, r, O.mg_params(omega=1.0, gamma=1.6, coarse_sweeps=3, coarse_cells=8))
    assert lev >= 3
    np.testing.assert_allclose(z, r / ap, rtol=4 * np.finfo(float).eps, atol=0)


def test_mg_bicgstab_matches_dense_lu(orc):
    g = W.Grid(8, 8, 8)
    s = W.make_set(0, 0, grid=g)
    A = orc.dense(g.shape, s["diags"])
    b = A @ s["x_star"]
    xd = np.linalg.solve(A, b)
    x, info = orc.bicgstab_mg(g.shape, s["diags"], b, tol=1e-13, maxit=200, params=_mg_params())
    assert info["status"] == 0 and info["levels"] >= 2
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("cfg,shape", [(1, (16, 32, 16)), (0, (16, 16, 16))])
def test_mg_bicgstab_residual_invariant_and_iterations(orc, cfg, shape):
    from oracle import oracle as O
    g = W.Grid(*shape)
    s = W.make_set(cfg, 0, grid=g)
    b = orc.apply(g.shape, s["diags"], s["x_star"])
    x, info = orc.bicgstab_mg(g.shape, s["diags"], b, tol=1e-10, maxit=500, params=O.mg_params())
    assert info["status"] == 0
    assert orc.rel_residual(g.shape, s["diags"], b, x) <= 1e-10
    _, jinfo = orc.bicgstab(g.shape, s["diags"], b, tol=1e-10, maxit=2000)
    assert 4 * info["iters"] <= jinfo["iters"], (info, jinfo)


def _dense_vcycle(A_levels, P_levels, r, omega, gamma, sweeps):
    """The V-cycle written as dense matrix algebra on an explicit hierarchy: A_levels[l] is
    level l's matrix, P_levels[l] the piecewise-constant interpolation from level l + 1.
    Level l < last: z1 = omega D^-1 r; e = V_{l+1}(P^T (r - A z1)); z2 = z1 + gamma P e;
    z = z2 + omega D^-1 (r - A z2).  Last level: `sweeps` damped-Jacobi sweeps from zero."""
    def vc(l, rl):
        A = A_levels[l]
        dinv = 1.0 / np.diag(A)
        if l == len(A_levels) - 1:
            z = np.zeros_like(rl)
            for _ in range(sweeps):
                z = z + omega * dinv * (rl - A @ z)
            return z
        P = P_levels[l]
        z1 = omega * dinv * rl
        e = vc(l + 1, P.T @ (rl - A @ z1))
        z2 = z1 + gamma * (P @ e)
        return z2 + omega * dinv * (rl - A @ z2)
    return vc(0, r)


@pytest.mark.parametrize("recipe,shape,coarse_cells,gamma,sweeps", [
    ("cd", (7, 6, 5), 8, 1.6, 3),
    ("sym", (6, 5, 4), 4, 0.7, 2),
    ("general", (5, 4, 6), 10, 1.3, 4),
])
def test_mg_vcycle_matches_dense_definition(orc, recipe, shape, coarse_cells, gamma, sweeps):
    # The hierarchy is rebuilt here from the dense matrix alone (Galerkin products with the
    # aggregation matrix, dimensions halved rounding up until at most coarse_cells cells), and the
    # V-cycle applied as matrix algebra, with gamma != 1 and several coarsest-level sweeps so that
    # the coarse-correction scale and the sweep count both show in the result.
    from oracle import oracle as O
    g = W.Grid(*shape)
    diags = W.random_general(g, seed=41) if recipe == "general" else W.coefficients(g, recipe, W.rng_for(0, 6))
    A_levels, P_levels, sh = [orc.dense(shape, diags)], [], shape
    while sh[0] * sh[1] * sh[2] > coarse_cells:
        Pm = _aggregation_matrix(sh)
        P_levels.append(Pm)
        A_levels.append(Pm.T @ A_levels[-1] @ Pm)
        sh = ((sh[0] + 1) // 2, (sh[1] + 1) // 2, (sh[2] + 1) // 2)
    assert len(A_levels) >= 3
    rng = np.random.default_rng(11)
    r = rng.standard_normal(g.n)
    prm = O.mg_params(omega=0.8, gamma=gamma, coarse_sweeps=sweeps, coarse_cells=coarse_cells)
    z, lev = orc.mg_apply(shape, diags, r, prm)
    ref = _dense_vcycle(A_levels, P_levels, r, 0.8, gamma, sweeps)
    assert lev == len(A_levels)
    assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the same V-cycle with gamma or the sweep count changed differs by far more than that
    alt_g = _dense_vcycle(A_levels, P_levels, r, 0.8, 1.0, sweeps)
    alt_s = _dense_vcycle(A_levels, P_levels, r, 0.8, gamma, sweeps - 1)
    assert np.max(np.abs(alt_g - ref)) > 1e-6 * np.max(np.abs(ref))
    assert np.max(np.abs(alt_s - ref)) > 1e-6 * np.max(np.abs(ref))


# ---------------------------------------------------------------- forward-error certificate

@pytest.mark.parametrize("recipe,margin", [("cd", 0.1), ("sym", 1e-3)])
def test_diag_dominance_margin_of_generated_systems(orc, recipe, margin):
    # both recipes give every row a_P = sum(in-grid a_nb) + margin with a_nb >= 0, so the
    # smallest row excess a_P - sum |a_nb| is the margin itself, up to the rounding of a_P
    from oracle import oracle as O
    g = W.Grid(9, 7, 6)
    diags = W.coefficients(g, recipe, W.rng_for(0, 7))
    m = O.diag_dominance_margin(g.shape, diags)
    assert abs(m - margin) <= 16 * EPS * float(np.max(diags[0]))
    # brute force over the dense matrix: the same minimum row excess
    A = orc.dense(g.shape, diags)
    excess = np.abs(np.diag(A)) - (np.sum(np.abs(A), axis=1) - np.abs(np.diag(A)))
    assert abs(m - float(np.min(excess))) <= 16 * EPS * float(np.max(diags[0]))


def test_diag_dominance_margin_ignores_outward_slots_and_finds_the_worst_row(orc):
    from oracle import oracle as O
    g = W.Grid(5, 4, 3)
    diags = W.random_general(g, seed=12, diag_shift=0.25)   # outward slots hold nonzero junk
    A = orc.dense(g.shape, diags)
    excess = np.abs(np.diag(A)) - (np.sum(np.abs(A), axis=1) - np.abs(np.diag(A)))
    np.testing.assert_allclose(excess, 0.25, rtol=0, atol=32 * EPS * float(np.max(diags[0])))
    # make one row the worst: raise a single in-grid link of cell (2, 1, 1)
    c = 2 + 5 * (1 + 4 * 1)
    bumped = [d.copy() for d in diags]
    bumped[5][c] += 0.2   # its T link (k + 1 = 2 is inside the grid)
    assert abs(O.diag_dominance_margin(g.shape, bumped) - 0.05) <= 64 * EPS
    bumped = [d.copy() for d in diags]
    bumped[2][0] += 0.2   # the W slot of cell i = 0 points out of the grid: no change
    assert abs(O.diag_dominance_margin(g.shape, bumped) - 0.25) <= 64 * EPS


def test_forward_error_certificate_bounds_the_true_error(orc):
    # Varah (1975): ||A^-1||_inf <= 1 / margin for a strictly row-dominant A, so
    # ||x - A^-1 b||_inf <= ||b - A x||_inf / margin for any x
    g = W.Grid(6, 5, 4)
    s = W.make_set(0, 0, grid=g)
    A = orc.dense(g.shape, s["diags"])
    assert np.max(np.sum(np.abs(np.linalg.inv(A)), axis=1)) <= 1.0 / 0.1 * (1 + 1e-12)
    b = A @ s["x_star"]
    xd = np.linalg.solve(A, b)
    rng = np.random.default_rng(5)
    for scale in (1e-3, 1e-8):
        x = xd + scale * rng.standard_normal(g.n)
        cert = orc.forward_error_certificate(g.shape, s["diags"], b, x)
        err = float(np.max(np.abs(x - xd)))
        assert err <= cert * (1 + 1e-10)
        assert cert <= 1e4 * err   # and not vacuous
    # a diagonal system: the certificate is exact where the residual and the smallest a_P meet
    ap = np.full(g.n, 2.0)
    ap[7] = 0.5
    dg = [ap] + [np.zeros(g.n)] * 6
    x = np.zeros(g.n)
    bb = np.zeros(g.n)
    bb[7] = 1.0
    assert orc.forward_error_certificate(g.shape, dg, bb, x) == 2.0
