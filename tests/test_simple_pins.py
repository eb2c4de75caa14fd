"""Pins of the SIMPLE-iteration oracle (oracle/simple.py) against facts that do
not come from its own formulas.

* The coefficient rows of the three momentum systems against a face-by-face
  flux balance of each control volume, written here from cell positions:
  mass fluxes by trilinear interpolation of the staggered velocity fields at
  face centres (clamped past the last sample: zero gradient), neighbours
  classified by whether the adjacent control volume exists, boundary values at
  half a cell.  Both are the finite-volume balance of Eq. (2) of Sec. 2.1 with
  upwind convection; they must give the same residual for any field.
* Continuity (Eq. (1)) of the corrected velocities after an exact p' solve:
  the defining property of the pressure-correction step.
* The hydrostatic state is a fixed point of a SIMPLE iteration.
* A one-cell-wide column has a closed-form steady state (plug flow, linear
  pressure balancing gravity and wall friction), which is a fixed point and
  which repeated SIMPLE iterations reach from p = 0.
"""
import numpy as np
import pytest

from oracle import simple as S

ORIGIN = dict(u=(0.0, 0.5, 0.5), v=(0.5, 0.0, 0.5), w=(0.5, 0.5, 0.0))   # sample offsets in cells (x, y, z)
AXIS = dict(u=0, v=1, w=2)


def random_state(bx, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    st = {c: scale * rng.uniform(-1, 1, sh) for c, sh in bx.shapes().items()}
    for c in "uvw":
        st[c + "0"] = scale * rng.uniform(-1, 1, bx.shapes()[c])
    st["p"] = rng.uniform(-1, 1, bx.shapes()["p"]) * 1e-3
    return st


def sample(bx, field, comp, x, y, z):
    """Trilinear interpolation of a staggered velocity component at (x, y, z),
    clamped to the sample range along each axis."""
    nz, ny, nx = field.shape
    h = (bx.hx, bx.hy, bx.hz)
    pos = []
    for a, (coord, n) in enumerate(zip((x, y, z), (nx, ny, nz))):
        f = coord / h[a] - ORIGIN[comp][a]
        f = min(max(f, 0.0), n - 1.0)
        i0 = min(int(np.floor(f)), n - 2) if n > 1 else 0
        t = f - i0 if n > 1 else 0.0
        pos.append((i0, t))
    (i0, tx), (j0, ty), (k0, tz) = pos
    val = 0.0
    for dk, wz in ((0, 1 - tz), (1, tz)):
        for dj, wy in ((0, 1 - ty), (1, ty)):
            for di, wx in ((0, 1 - tx), (1, tx)):
                wgt = wx * wy * wz
                if wgt != 0.0:
                    val += wgt * field[k0 + dk, j0 + dj, i0 + di]
    return val


def fixed_row(bx, comp, k, j, i):
    return (comp == "u" and i in (0, bx.nx)) or (comp == "v" and j == 0) or (comp == "w" and k in (0, bx.nz))


def flux_balance(bx, st, comp, x):
    """Residual of the momentum balance of every control volume of `comp`,
    evaluated at the field x (fluxes from the state st), face by face.
    Returns (residual, a_P before relaxation) on the non-fixed rows (others 0)."""
    shape = bx.shapes()[comp]
    h = np.array([bx.hx, bx.hy, bx.hz])
    area = np.array([bx.hy * bx.hz, bx.hx * bx.hz, bx.hx * bx.hy])
    V = bx.hx * bx.hy * bx.hz
    vel = dict(u=st["u"], v=st["v"], w=st["w"])
    R = np.zeros(shape)
    AP = np.zeros(shape)
    ax_c = AXIS[comp]
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                if fixed_row(bx, comp, k, j, i):
                    continue
                idx = np.array([i, j, k])
                centre = (idx + np.array(ORIGIN[comp])) * h
                ap = bx.rho * V / bx.dt
                r = bx.rho * V / bx.dt * (x[k, j, i] - st[comp + "0"][k, j, i])
                for a in range(3):
                    for side in (+1, -1):
                        face = centre.copy()
                        face[a] += side * h[a] / 2
                        nb = idx.copy()
                        nb[a] += side
                        n_a = shape[2 - a]
                        normal = "uvw"[a]
                        F_out = side * bx.rho * area[a] * sample(bx, vel[normal], normal, *face)
                        D = bx.mu * area[a] / h[a]
                        if 0 <= nb[a] < n_a:
                            cnd = D + max(-F_out, 0.0)
                            r += cnd * (x[k, j, i] - x[nb[2], nb[1], nb[0]])
                        elif a == 1 and side == +1:
                            continue                      # outlet: zero gradient
                        else:
                            cnd = 2 * D + max(-F_out, 0.0)
                            r += cnd * (x[k, j, i] - 0.0)
                        ap += cnd
                # pressure force: p at the cell centres half a cell either side
                lo = centre.copy()
                lo[ax_c] -= h[ax_c] / 2
                hi = centre.copy()
                hi[ax_c] += h[ax_c] / 2
                p_lo = st["p"][tuple(int(round(c / hh - 0.5)) for c, hh in zip(lo[::-1], h[::-1]))]
                ijk_hi = tuple(int(round(c / hh - 0.5)) for c, hh in zip(hi[::-1], h[::-1]))
                p_hi = st["p"][ijk_hi] if ijk_hi[1] < bx.ny else 0.0
                r -= (p_lo - p_hi) * area[ax_c]
                if comp == "v":
                    r -= bx.rho * bx.gy * V
                R[k, j, i] = r
                AP[k, j, i] = ap
    return R, AP


def row_residual(diags, b, x):
    """a_P x_c - sum a_nb x_nb - b by explicit neighbour loops."""
    nz, ny, nx = x.shape
    out = np.zeros_like(x)
    nbs = [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = diags[0][k, j, i] * x[k, j, i] - b[k, j, i]
                for q, (dk, dj, di) in enumerate(nbs, start=1):
                    kk, jj, ii = k + dk, j + dj, i + di
                    if 0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx:
                        s -= diags[q][k, j, i] * x[kk, jj, ii]
                out[k, j, i] = s
    return out


BOXES = [S.Box(3, 4, 2, 0.01, 0.012, 0.009), S.Box(2, 3, 3, 0.02, 0.01, 0.015), S.Box(1, 3, 1, 0.01, 0.01, 0.01)]


@pytest.mark.parametrize("comp", ["u", "v", "w"])
@pytest.mark.parametrize("bi", range(len(BOXES)))
def test_momentum_rows_equal_face_flux_balance(comp, bi):
    """Unrelaxed rows: a_P x - sum a_nb x_nb - b equals the face-by-face
    balance for an arbitrary x; fixed rows hold their boundary value."""
    bx = BOXES[bi].with_(alpha_u=1.0, mu=0.3, dt=0.05)   # conductances of the order of the fluxes
    st = random_state(bx, 10 + bi)
    diags, b, d = S.form_momentum(bx, st, comp)
    x = np.random.default_rng(99).uniform(-1, 1, bx.shapes()[comp])
    R, AP = flux_balance(bx, st, comp, x)
    got = row_residual(diags, b, x)
    mask = np.zeros(x.shape, bool)
    for k, j, i in np.ndindex(*x.shape):
        mask[k, j, i] = not fixed_row(bx, comp, k, j, i)
    if mask.any():   # (a one-cell-wide box has only wall faces in x and z)
        scale = np.abs(R[mask]).max()
        assert np.abs(got[mask] - R[mask]).max() <= 1e-12 * scale
        np.testing.assert_allclose(diags[0][mask], AP[mask], rtol=1e-13)
    # fixed rows: only a_P, value = b / a_P
    fr = ~mask
    for q in range(1, 7):
        assert np.all(diags[q][fr] == 0)
    val = bx.v_in if comp == "v" else 0.0
    np.testing.assert_allclose(b[fr] / diags[0][fr], val)
    assert np.all(d[fr] == 0)
    area = dict(u=bx.hy * bx.hz, v=bx.hx * bx.hz, w=bx.hx * bx.hy)[comp]
    np.testing.assert_allclose(d[mask], area / diags[0][mask], rtol=1e-15)


@pytest.mark.parametrize("comp", ["u", "v", "w"])
def test_momentum_under_relaxation(comp):
    """Relaxed rows: residual at x equals the unrelaxed balance plus
    (1/alpha - 1) a_P (x - x*), with x* the incoming iterate."""
    bx = BOXES[0].with_(alpha_u=0.6, mu=0.3, dt=0.05)
    st = random_state(bx, 5)
    diags, b, _ = S.form_momentum(bx, st, comp)
    x = np.random.default_rng(7).uniform(-1, 1, bx.shapes()[comp])
    R, AP = flux_balance(bx, st, comp, x)
    want = R + (1 / 0.6 - 1) * AP * (x - st[comp])
    got = row_residual(diags, b, x)
    mask = AP > 0
    assert np.abs(got[mask] - want[mask]).max() <= 1e-12 * np.abs(want[mask]).max()
    # the velocity change per unit p' difference belongs to the relaxed row
    _, _, d = S.form_momentum(bx, st, comp)
    area = dict(u=bx.hy * bx.hz, v=bx.hx * bx.hz, w=bx.hx * bx.hy)[comp]
    np.testing.assert_allclose(d[mask], area * 0.6 / AP[mask], rtol=1e-13)


def test_pressure_relaxation_scales_only_the_pressure_update():
    """alpha_p enters the pressure update alone: velocities after one
    iteration do not depend on it, the pressure change is proportional to it."""
    bx = BOXES[0]
    st = random_state(bx, 31)
    a, _ = S.simple_iteration(bx.with_(alpha_p=0.8), st)
    b, _ = S.simple_iteration(bx.with_(alpha_p=1.0), st)
    for c in "uvw":
        np.testing.assert_allclose(a[c], b[c], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(a["p"] - st["p"], 0.8 * (b["p"] - st["p"]), rtol=1e-10, atol=1e-18)


@pytest.mark.parametrize("bi", range(len(BOXES)))
def test_pressure_correction_restores_continuity(bi):
    """After an exact p' solve the corrected velocities conserve mass in every
    cell; the mass imbalance before it is the right-hand side of the p' rows."""
    bx = BOXES[bi]
    st = random_state(bx, 20 + bi)
    new, dg = S.simple_iteration(bx, st)
    pd, pb = dg["pressure"]
    pred = dg["predicted"]
    np.testing.assert_allclose(pb, S.continuity(bx, pred), rtol=1e-12, atol=1e-18)
    flux_scale = bx.rho * max(bx.hx * bx.hy, bx.hy * bx.hz, bx.hx * bx.hz) * max(np.abs(x).max() for x in pred)
    div = S.continuity(bx, (new["u"], new["v"], new["w"]))
    assert np.abs(div).max() <= 1e-12 * flux_scale
    # p' matrix symmetric, with a_P at least the sum of its neighbours
    A = S.to_sparse(pd)
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    offsum = sum(pd[q] for q in range(1, 7))
    assert np.all(pd[0] >= offsum * (1 - 1e-15))
    assert np.any(pd[0] > offsum * (1 + 1e-6))      # the outlet row makes the system nonsingular


def hydrostatic(bx):
    j = np.arange(bx.ny)
    p = -bx.rho * bx.gy * bx.hy * (bx.ny - j)
    return np.broadcast_to(p[None, :, None], bx.shapes()["p"]).copy()


def test_hydrostatic_state_is_a_fixed_point():
    bx = S.Box(3, 5, 2, 0.01, 0.02, 0.015, v_in=0.0)
    st = {c: np.zeros(sh) for c, sh in bx.shapes().items()}
    for c in "uvw":
        st[c + "0"] = np.zeros(bx.shapes()[c])
    st["p"] = hydrostatic(bx)
    new, dg = S.simple_iteration(bx, st)
    for c in "uvw":
        assert np.abs(new[c]).max() <= 1e-13
    np.testing.assert_allclose(new["p"], st["p"], rtol=1e-12, atol=1e-14)
    assert dg["mass_residual"] <= 1e-15


def column_steady_state(bx):
    """One cell wide in x and z: plug flow v = v_in and a linear pressure that
    balances gravity and the friction of the four walls."""
    Ax, Ay, Az = bx.hy * bx.hz, bx.hx * bx.hz, bx.hx * bx.hy
    V = bx.hx * bx.hy * bx.hz
    walls = 4 * bx.mu * Ax / bx.hx + 4 * bx.mu * Az / bx.hz
    dp = (walls * bx.v_in - bx.rho * bx.gy * V) / Ay
    j = np.arange(bx.ny)
    return (bx.ny - j)[None, :, None] * dp * np.ones(bx.shapes()["p"])


def column_state(bx, p):
    st = {c: np.zeros(sh) for c, sh in bx.shapes().items()}
    st["v"][:] = bx.v_in
    for c in "uvw":
        st[c + "0"] = st[c].copy()
    st["p"] = p
    return st


def test_column_closed_form_is_a_fixed_point():
    bx = S.Box(1, 6, 1, 0.01, 0.02, 0.012, mu=1e-3)
    st = column_state(bx, column_steady_state(bx))
    new, _ = S.simple_iteration(bx, st)
    np.testing.assert_allclose(new["v"], bx.v_in, rtol=1e-13)
    np.testing.assert_allclose(new["p"], st["p"], rtol=1e-12)


def test_column_iterations_reach_the_closed_form():
    bx = S.Box(1, 6, 1, 0.01, 0.02, 0.012, mu=1e-3)
    st = column_state(bx, np.zeros(bx.shapes()["p"]))
    for _ in range(60):
        st, _ = S.simple_iteration(bx, st)
    np.testing.assert_allclose(st["p"], column_steady_state(bx), rtol=1e-9)
    np.testing.assert_allclose(st["v"], bx.v_in, rtol=1e-12)


def test_sparse_matrix_matches_row_loops():
    """to_sparse (used by the exact solves) against the explicit loops."""
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    diags = [rng.uniform(1, 2, shape)] + [rng.uniform(0, 1, shape) for _ in range(6)]
    x = rng.uniform(-1, 1, shape)
    b = np.zeros(shape)
    want = row_residual(diags, b, x)
    got = (S.to_sparse(diags) @ x.ravel()).reshape(shape)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)
