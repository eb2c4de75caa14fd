"""CPU oracle for one SIMPLE iteration on a gas-only bed box (arXiv 2211.15605).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the HIP library.

What is computed.  The paper's gas phase (Sec. 2.1, Eqs. (1)-(2)) with no
parcels (volume fraction 1, no drag term F): constant-density continuity and
momentum with pressure, viscous stress (mu times the Laplacian of the velocity,
which is the divergence of the stress tensor for constant mu and a
divergence-free field) and gravity.  The box follows the verification case of
Sec. 3: gravity along -y, gas entering through the bottom plane y = 0 at a
uniform speed, leaving through the top plane y = Ly at a fixed pressure, and
no-slip walls on the four vertical planes.  MFiX advances such a state with
SIMPLE iterations (Sec. 2.2.2): form and solve the u, v and w momentum
systems, then form and solve the pressure-correction system p', then correct
pressure and velocities.  The discretisation is the standard staggered
finite-volume one (Patankar, Numerical Heat Transfer and Fluid Flow, 1980,
ch. 5-6): first-order upwind convection, central diffusion, implicit Euler in
time, momentum under-relaxation folded into the coefficients.

Grids (all arrays indexed [k, j, i], i fastest in memory):
  p, p'  (nz,   ny,   nx)    cell centres
  u      (nz,   ny,   nx+1)  x-faces; i = 0 and i = nx are walls
  v      (nz,   ny+1, nx)    y-faces; j = 0 is the inlet, j = ny the outlet
  w      (nz+1, ny,   nx)    z-faces; k = 0 and k = nz are walls

Each momentum row is written in Patankar form a_P x_P - sum a_nb x_nb = b.
A velocity on a wall or inlet face is a fixed-value row (a_P = rho V / dt,
b = a_P * value, no neighbours) so that every row has the scale of the
transient term.  A face whose control volume reaches a boundary plane that
carries a tangential wall or inlet value takes that value (zero) at half a
cell, with twice the diffusion conductance, folded into a_P.  The top plane
is an outlet: zero gradient of every velocity (no term) and p = 0 in a ghost
cell above the last row.

Every function is pinned by ``tests/test_simple_pins.py``: the coefficient
form of the momentum rows against an independent face-by-face flux balance
written from cell positions and trilinear interpolation; continuity of the
corrected velocities after an exact p' solve; the hydrostatic state as a
fixed point; the closed-form steady state of a one-cell-wide column.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass(frozen=True)
class Box:
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    rho: float = 1.093      # gas density of the verification case (Sec. 3)
    mu: float = 1.9e-5      # gas viscosity of the verification case (Sec. 3)
    dt: float = 1e-3        # initial time step of the verification case (Sec. 3.1)
    gy: float = -9.81       # gravity along y
    v_in: float = 0.5       # inlet speed, inside the 0.3-1.0 m/s range of Sec. 3
    alpha_u: float = 0.5    # momentum under-relaxation
    alpha_p: float = 0.8    # pressure under-relaxation

    def shapes(self):
        """[k, j, i] array shapes of p, u, v, w."""
        nx, ny, nz = self.nx, self.ny, self.nz
        return dict(p=(nz, ny, nx), u=(nz, ny, nx + 1), v=(nz, ny + 1, nx), w=(nz + 1, ny, nx))

    def with_(self, **kw):
        return replace(self, **kw)


def _geometry(bx):
    Ax, Ay, Az = bx.hy * bx.hz, bx.hx * bx.hz, bx.hx * bx.hy
    V = bx.hx * bx.hy * bx.hz
    return Ax, Ay, Az, V


def _fixed_row(bx, value):
    """A fixed-value row: a_P = rho V / dt, no neighbours, b = a_P value."""
    aP0 = bx.rho * _geometry(bx)[3] / bx.dt
    return [aP0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0], aP0 * value, 0.0


def _finish(bx, a, bnd, src, x_star):
    """a = [aE, aW, aN, aS, aT, aB] of the neighbours in the grid, bnd = the
    conductances towards boundary values (all zero), src = the explicit source
    (old-time term, pressure force, gravity).  Adds the transient coefficient,
    under-relaxes with the current iterate x_star and returns (row, b, d/A)."""
    aE, aW, aN, aS, aT, aB = a
    aP0 = bx.rho * _geometry(bx)[3] / bx.dt
    aP = aE + aW + aN + aS + aT + aB + bnd + aP0
    aPr = aP / bx.alpha_u
    b = src + (1.0 - bx.alpha_u) * aPr * x_star
    return [aPr, aE, aW, aN, aS, aT, aB], b, 1.0 / aPr


def form_u_cell(bx, st, k, j, i):
    """Row of the x-momentum system at u-face (k, j, i): (7 coefficients
    P,E,W,N,S,T,B, b, d) with d = A_x / a_P (the velocity change per unit
    pressure-correction difference)."""
    nx, ny, nz = bx.nx, bx.ny, bx.nz
    if i == 0 or i == nx:
        return _fixed_row(bx, 0.0)
    Ax, Ay, Az, V = _geometry(bx)
    u, v, w, p = st["u"], st["v"], st["w"], st["p"]
    r = bx.rho
    Fe = r * Ax * (u[k, j, i] + u[k, j, i + 1]) / 2
    Fw = r * Ax * (u[k, j, i - 1] + u[k, j, i]) / 2
    Fn = r * Ay * (v[k, j + 1, i - 1] + v[k, j + 1, i]) / 2
    Fs = r * Ay * (v[k, j, i - 1] + v[k, j, i]) / 2
    Ft = r * Az * (w[k + 1, j, i - 1] + w[k + 1, j, i]) / 2
    Fb = r * Az * (w[k, j, i - 1] + w[k, j, i]) / 2
    De, Dn, Dt = bx.mu * Ax / bx.hx, bx.mu * Ay / bx.hy, bx.mu * Az / bx.hz
    bnd = 0.0
    aE = De + max(-Fe, 0.0)
    aW = De + max(Fw, 0.0)
    aN = Dn + max(-Fn, 0.0) if j + 1 < ny else 0.0          # outlet: zero gradient
    if j > 0:
        aS = Dn + max(Fs, 0.0)
    else:                                                     # inlet plane: u = 0 at hy/2
        aS, bnd = 0.0, bnd + 2 * Dn + max(Fs, 0.0)
    if k + 1 < nz:
        aT = Dt + max(-Ft, 0.0)
    else:                                                     # wall z = Lz
        aT, bnd = 0.0, bnd + 2 * Dt + max(-Ft, 0.0)
    if k > 0:
        aB = Dt + max(Fb, 0.0)
    else:                                                     # wall z = 0
        aB, bnd = 0.0, bnd + 2 * Dt + max(Fb, 0.0)
    src = r * V / bx.dt * st["u0"][k, j, i] + (p[k, j, i - 1] - p[k, j, i]) * Ax
    row, b, dinv = _finish(bx, [aE, aW, aN, aS, aT, aB], bnd, src, u[k, j, i])
    return row, b, Ax * dinv


def form_v_cell(bx, st, k, j, i):
    """Row of the y-momentum system at v-face (k, j, i), j = 1..ny (j = 0 is
    the inlet row); the outlet face j = ny sees p = 0 above it."""
    nx, ny, nz = bx.nx, bx.ny, bx.nz
    if j == 0:
        return _fixed_row(bx, bx.v_in)
    Ax, Ay, Az, V = _geometry(bx)
    u, v, w, p = st["u"], st["v"], st["w"], st["p"]
    r = bx.rho
    jl, jh = j - 1, (j if j < ny else ny - 1)   # p rows below / above (zero gradient past the top)
    Fn = r * Ay * ((v[k, j, i] + v[k, j + 1, i]) / 2 if j < ny else v[k, j, i])
    Fs = r * Ay * (v[k, j - 1, i] + v[k, j, i]) / 2
    Fe = r * Ax * (u[k, jl, i + 1] + u[k, jh, i + 1]) / 2
    Fw = r * Ax * (u[k, jl, i] + u[k, jh, i]) / 2
    Ft = r * Az * (w[k + 1, jl, i] + w[k + 1, jh, i]) / 2
    Fb = r * Az * (w[k, jl, i] + w[k, jh, i]) / 2
    De, Dn, Dt = bx.mu * Ax / bx.hx, bx.mu * Ay / bx.hy, bx.mu * Az / bx.hz
    bnd = 0.0
    if i + 1 < nx:
        aE = De + max(-Fe, 0.0)
    else:
        aE, bnd = 0.0, bnd + 2 * De + max(-Fe, 0.0)
    if i > 0:
        aW = De + max(Fw, 0.0)
    else:
        aW, bnd = 0.0, bnd + 2 * De + max(Fw, 0.0)
    aN = Dn + max(-Fn, 0.0) if j < ny else 0.0
    aS = Dn + max(Fs, 0.0)
    if k + 1 < nz:
        aT = Dt + max(-Ft, 0.0)
    else:
        aT, bnd = 0.0, bnd + 2 * Dt + max(-Ft, 0.0)
    if k > 0:
        aB = Dt + max(Fb, 0.0)
    else:
        aB, bnd = 0.0, bnd + 2 * Dt + max(Fb, 0.0)
    p_above = p[k, j, i] if j < ny else 0.0
    src = r * V / bx.dt * st["v0"][k, j, i] + (p[k, j - 1, i] - p_above) * Ay + r * bx.gy * V
    row, b, dinv = _finish(bx, [aE, aW, aN, aS, aT, aB], bnd, src, v[k, j, i])
    return row, b, Ay * dinv


def form_w_cell(bx, st, k, j, i):
    """Row of the z-momentum system at w-face (k, j, i)."""
    nx, ny, nz = bx.nx, bx.ny, bx.nz
    if k == 0 or k == nz:
        return _fixed_row(bx, 0.0)
    Ax, Ay, Az, V = _geometry(bx)
    u, v, w, p = st["u"], st["v"], st["w"], st["p"]
    r = bx.rho
    Ft = r * Az * (w[k, j, i] + w[k + 1, j, i]) / 2
    Fb = r * Az * (w[k - 1, j, i] + w[k, j, i]) / 2
    Fe = r * Ax * (u[k - 1, j, i + 1] + u[k, j, i + 1]) / 2
    Fw = r * Ax * (u[k - 1, j, i] + u[k, j, i]) / 2
    Fn = r * Ay * (v[k - 1, j + 1, i] + v[k, j + 1, i]) / 2
    Fs = r * Ay * (v[k - 1, j, i] + v[k, j, i]) / 2
    De, Dn, Dt = bx.mu * Ax / bx.hx, bx.mu * Ay / bx.hy, bx.mu * Az / bx.hz
    bnd = 0.0
    if i + 1 < nx:
        aE = De + max(-Fe, 0.0)
    else:
        aE, bnd = 0.0, bnd + 2 * De + max(-Fe, 0.0)
    if i > 0:
        aW = De + max(Fw, 0.0)
    else:
        aW, bnd = 0.0, bnd + 2 * De + max(Fw, 0.0)
    aN = Dn + max(-Fn, 0.0) if j + 1 < ny else 0.0
    if j > 0:
        aS = Dn + max(Fs, 0.0)
    else:
        aS, bnd = 0.0, bnd + 2 * Dn + max(Fs, 0.0)
    aT = Dt + max(-Ft, 0.0)
    aB = Dt + max(Fb, 0.0)
    src = r * V / bx.dt * st["w0"][k, j, i] + (p[k - 1, j, i] - p[k, j, i]) * Az
    row, b, dinv = _finish(bx, [aE, aW, aN, aS, aT, aB], bnd, src, w[k, j, i])
    return row, b, Az * dinv


FORM = dict(u=form_u_cell, v=form_v_cell, w=form_w_cell)


def form_momentum(bx, st, comp):
    """Whole x-, y- or z-momentum system: (diags [7 arrays], b, d), each of
    the component's grid shape."""
    shape = bx.shapes()[comp]
    diags = [np.zeros(shape) for _ in range(7)]
    b = np.zeros(shape)
    d = np.zeros(shape)
    f = FORM[comp]
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                row, bb, dd = f(bx, st, k, j, i)
                for q in range(7):
                    diags[q][k, j, i] = row[q]
                b[k, j, i] = bb
                d[k, j, i] = dd
    return diags, b, d


def form_pressure_cell(bx, du, dv, dw, vel, k, j, i):
    """Row of the pressure-correction system at p-cell (k, j, i): the
    continuity balance of the cell with every face velocity written as its
    predicted value plus d times the p' difference across the face.  Faces
    with a fixed velocity have d = 0; the outlet face's outer p' is 0."""
    nx, ny, nz = bx.nx, bx.ny, bx.nz
    Ax, Ay, Az, _ = _geometry(bx)
    u, v, w = vel
    r = bx.rho
    aE = r * Ax * du[k, j, i + 1] if i + 1 < nx else 0.0
    aW = r * Ax * du[k, j, i] if i > 0 else 0.0
    aN = r * Ay * dv[k, j + 1, i] if j + 1 < ny else 0.0
    out = r * Ay * dv[k, j + 1, i] if j + 1 == ny else 0.0
    aS = r * Ay * dv[k, j, i] if j > 0 else 0.0
    aT = r * Az * dw[k + 1, j, i] if k + 1 < nz else 0.0
    aB = r * Az * dw[k, j, i] if k > 0 else 0.0
    aP = aE + aW + aN + aS + aT + aB + out
    b = r * ((u[k, j, i] - u[k, j, i + 1]) * Ax + (v[k, j, i] - v[k, j + 1, i]) * Ay
             + (w[k, j, i] - w[k + 1, j, i]) * Az)
    return [aP, aE, aW, aN, aS, aT, aB], b


def form_pressure(bx, du, dv, dw, vel):
    shape = bx.shapes()["p"]
    diags = [np.zeros(shape) for _ in range(7)]
    b = np.zeros(shape)
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                row, bb = form_pressure_cell(bx, du, dv, dw, vel, k, j, i)
                for q in range(7):
                    diags[q][k, j, i] = row[q]
                b[k, j, i] = bb
    return diags, b


def correct(bx, du, dv, dw, pp, vel, p):
    """Corrected (u, v, w, p): velocities take d times the p' difference
    across their face, pressure takes alpha_p p'."""
    nx, ny, nz = bx.nx, bx.ny, bx.nz
    u, v, w = (x.copy() for x in vel)
    for k in range(nz):
        for j in range(ny):
            for i in range(1, nx):
                u[k, j, i] += du[k, j, i] * (pp[k, j, i - 1] - pp[k, j, i])
    for k in range(nz):
        for j in range(1, ny + 1):
            for i in range(nx):
                above = pp[k, j, i] if j < ny else 0.0
                v[k, j, i] += dv[k, j, i] * (pp[k, j - 1, i] - above)
    for k in range(1, nz):
        for j in range(ny):
            for i in range(nx):
                w[k, j, i] += dw[k, j, i] * (pp[k - 1, j, i] - pp[k, j, i])
    return u, v, w, p + bx.alpha_p * pp


def continuity(bx, vel):
    """Mass inflow minus outflow of every p-cell, rho * sum(face velocity * area)."""
    Ax, Ay, Az, _ = _geometry(bx)
    u, v, w = vel
    return bx.rho * ((u[:, :, :-1] - u[:, :, 1:]) * Ax + (v[:, :-1, :] - v[:, 1:, :]) * Ay
                     + (w[:-1, :, :] - w[1:, :, :]) * Az)


# ---------------------------------------------------------------- linear algebra steps

def to_sparse(diags):
    """The matrix of 7 Patankar diagonals on a [k, j, i] grid (neighbours
    outside the grid dropped): A[c, c] = a_P, A[c, nb] = -a_nb."""
    nz, ny, nx = diags[0].shape
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def flat(k, j, i):
        return (k * ny + j) * nx + i

    rows, cols, vals = [flat(K, J, I).ravel()], [flat(K, J, I).ravel()], [diags[0].ravel()]
    for q, (dk, dj, di) in zip(range(1, 7), [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)]):
        k2, j2, i2 = K + dk, J + dj, I + di
        m = (k2 >= 0) & (k2 < nz) & (j2 >= 0) & (j2 < ny) & (i2 >= 0) & (i2 < nx)
        rows.append(flat(K, J, I)[m])
        cols.append(flat(k2, j2, i2)[m])
        vals.append(-diags[q][m])
    n = nx * ny * nz
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def solve_exact(diags, b):
    """x = A^-1 b by a sparse LU factorisation (SuperLU)."""
    A = to_sparse(diags)
    return spla.spsolve(A.tocsc(), b.ravel()).reshape(b.shape)


def residual(diags, b, x):
    return b - (to_sparse(diags) @ x.ravel()).reshape(b.shape)


def simple_iteration(bx, st, solve=solve_exact):
    """One SIMPLE iteration from state st (u, v, w, p, and the old-time u0,
    v0, w0).  Returns the new state and a dict of diagnostics: the momentum
    residual norms at the incoming iterate, the mass imbalance norm before the
    p' solve, the formed systems."""
    mom = {}
    new = dict(st)
    res = {}
    for c in ("u", "v", "w"):
        diags, b, d = form_momentum(bx, st, c)
        mom[c] = (diags, b, d)
        res[c] = float(np.linalg.norm(residual(diags, b, st[c])))
        new[c] = solve(diags, b)
    du, dv, dw = mom["u"][2], mom["v"][2], mom["w"][2]
    vel = (new["u"], new["v"], new["w"])
    pd, pb = form_pressure(bx, du, dv, dw, vel)
    pp = solve(pd, pb)
    u, v, w, p = correct(bx, du, dv, dw, pp, vel, st["p"])
    new.update(u=u, v=v, w=w, p=p)
    diag = dict(mom_residual=res, mass_residual=float(np.linalg.norm(pb)), momentum=mom,
                pressure=(pd, pb), pp=pp, predicted=vel)
    return new, diag
