"""Seeded synthetic inputs for the equation-set solve.

This module only draws inputs: coefficient diagonals, manufactured solutions
and loss weights.  It holds none of the solver's arithmetic (no stencil
product, no Krylov step), so both the HIP path and the CPU oracle may use it.

The paper's workloads (fluidized-bed and backward-facing-step matrices taken
from MFiX states, Sec. 3 and Sec. 4) are not available, so these generators
stand in for them at the paper's scale and shape: tall structured grids with
a long vertical axis (Sec. 3: 27x162x27 bed; Sec. 4: 150x150x450 PIC bed and
10M-30M cell BFS grids), four equation sets per time step on staggered grids
(Sec. 2.2.2: u, v, w momentum and pressure).

Two coefficient recipes, both in Patankar form a_P x_P - sum a_nb x_nb = b
with coefficients pointing out of the grid set to zero:

* ``cd`` (momentum-like convection-diffusion): for every interior face f
  between cell c and its +d neighbour, D_f ~ U[0.5, 1.5] and F_f ~ U[-1, 1];
  the upwind scheme gives the lower cell D_f + max(-F_f, 0) towards the face
  and the upper cell D_f + max(F_f, 0).  a_P = sum of the six a_nb + 0.1, so
  the matrix is nonsymmetric and strictly diagonally dominant by 0.1.
* ``sym`` (pressure-correction-like): a_f ~ U[0.5, 2] shared by both cells of
  a face; a_P = sum a_nb + 1e-3.  Symmetric positive definite and
  near-singular (a Neumann-like Laplacian with a 1e-3 shift).

Random draws: numpy PCG64 seeded by SeedSequence([2211, 15605, cfg, set]),
drawn in the order x-faces (all D, then all F, faces in flat order of their
lower cell), y-faces, z-faces, then x*, then the loss weights w.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SLOTS = ("P", "E", "W", "N", "S", "T", "B")


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def n(self):
        return self.nx * self.ny * self.nz


# The five workloads: name, recipe, grids (one per equation set).
CONFIGS = {
    0: dict(name="cd16", recipe="cd", grids=[Grid(16, 16, 16)], tol=1e-10, maxit=1000),
    1: dict(name="sym128x256x128", recipe="sym", grids=[Grid(128, 256, 128)], tol=1e-10, maxit=20000),
    2: dict(name="staggered4x96x384x96", recipe="cd",
            grids=[Grid(96, 384, 96), Grid(97, 384, 96), Grid(96, 385, 96), Grid(96, 384, 97)],
            tol=1e-10, maxit=1000),
    3: dict(name="adjoint64", recipe="cd", grids=[Grid(64, 64, 64)], tol=1e-10, maxit=1000),
    4: dict(name="tallbed4x192x768x192", recipe="cd", grids=[Grid(192, 768, 192)] * 4,
            tol=1e-10, maxit=2000),
}


def rng_for(cfg: int, set_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2211, 15605, int(cfg), int(set_id)])))


def _faces(rng, recipe, count):
    if recipe == "cd":
        D = rng.uniform(0.5, 1.5, count)
        F = rng.uniform(-1.0, 1.0, count)
        return D + np.maximum(-F, 0.0), D + np.maximum(F, 0.0)
    if recipe == "sym":
        a = rng.uniform(0.5, 2.0, count)
        return a, a
    raise ValueError(recipe)


def coefficients(grid: Grid, recipe: str, rng: np.random.Generator):
    """Seven FP64 arrays (P, E, W, N, S, T, B), each flat of length nx*ny*nz."""
    nx, ny, nz = grid.shape
    shp = (nz, ny, nx)
    E = np.zeros(shp); W = np.zeros(shp); N = np.zeros(shp); S = np.zeros(shp)
    T = np.zeros(shp); B = np.zeros(shp)
    # x-faces between (i, j, k) and (i+1, j, k): lower cell gets E, upper gets W
    lo, hi = _faces(rng, recipe, nz * ny * (nx - 1))
    E[:, :, :-1] = lo.reshape(nz, ny, nx - 1)
    W[:, :, 1:] = hi.reshape(nz, ny, nx - 1)
    lo, hi = _faces(rng, recipe, nz * (ny - 1) * nx)
    N[:, :-1, :] = lo.reshape(nz, ny - 1, nx)
    S[:, 1:, :] = hi.reshape(nz, ny - 1, nx)
    lo, hi = _faces(rng, recipe, (nz - 1) * ny * nx)
    T[:-1, :, :] = lo.reshape(nz - 1, ny, nx)
    B[1:, :, :] = hi.reshape(nz - 1, ny, nx)
    margin = 0.1 if recipe == "cd" else 1e-3
    P = E + W + N + S + T + B + margin
    return [a.ravel() for a in (P, E, W, N, S, T, B)]


def manufactured_solution(grid: Grid, rng: np.random.Generator):
    """x* ~ U[-1, 1] (drawn after the coefficients)."""
    return rng.uniform(-1.0, 1.0, grid.n)


def loss_weights(grid: Grid, rng: np.random.Generator):
    """w ~ N(0, 1) for L = sum(w * x) (drawn after x*)."""
    return rng.standard_normal(grid.n)


def make_set(cfg: int, set_id: int = 0, grid: Grid | None = None, recipe: str | None = None,
             with_weights: bool = False):
    """Coefficients and x* (and w) for one equation set of workload ``cfg``.

    ``grid``/``recipe`` override the workload's own for scaled-down cases
    (the seed still comes from cfg and set_id)."""
    c = CONFIGS[cfg]
    g = grid if grid is not None else c["grids"][set_id]
    rcp = recipe if recipe is not None else c["recipe"]
    rng = rng_for(cfg, set_id)
    diags = coefficients(g, rcp, rng)
    xs = manufactured_solution(g, rng)
    out = dict(grid=g, recipe=rcp, diags=diags, x_star=xs)
    if with_weights:
        out["w"] = loss_weights(g, rng)
    return out


def random_general(grid: Grid, seed: int, diag_shift: float = 0.5):
    """Coefficients with independent random values in every slot, including the
    outward-pointing ones (which the operator must ignore), for tests of
    indexing and boundaries.  a_P = sum of in-grid |a_nb| + diag_shift."""
    nx, ny, nz = grid.shape
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2211, 15605, 99, seed])))
    shp = (nz, ny, nx)
    nb = [rng.uniform(0.1, 1.0, shp) for _ in range(6)]
    inside = [np.ones(shp) for _ in range(6)]
    inside[0][:, :, -1] = 0; inside[1][:, :, 0] = 0
    inside[2][:, -1, :] = 0; inside[3][:, 0, :] = 0
    inside[4][-1, :, :] = 0; inside[5][0, :, :] = 0
    P = sum(a * m for a, m in zip(nb, inside)) + diag_shift
    return [P.ravel()] + [a.ravel() for a in nb]


# ---------------------------------------------------------------- SIMPLE box states
#
# The gas-only bed box: the verification case of Sec. 3 (gas properties,
# gravity along -y, inlet at the bottom, outlet at the top, vertical walls)
# on the pressure grid of the four-set time step above (p' 96x384x96; the
# u, v, w grids of that step are exactly its staggered faces), with cubic
# cells of 1.25 mm (a 12 cm x 48 cm x 12 cm column).  Small boxes of the same
# recipe serve the parity tests.

BED = dict(nx=96, ny=384, nz=96, hx=1.25e-3, hy=1.25e-3, hz=1.25e-3, rho=1.093, mu=1.9e-5, dt=1e-3,
           gy=-9.81, v_in=0.5, alpha_u=0.5, alpha_p=0.8)


def bed_box(nx=None, ny=None, nz=None, **kw):
    """The bed recipe, optionally with other cell counts (same cell size) or parameters."""
    b = dict(BED)
    for k, v in (("nx", nx), ("ny", ny), ("nz", nz)):
        if v is not None:
            b[k] = int(v)
    b.update(kw)
    return b


def box_state(box, seed: int, noise: float = 0.05, old: str = "same"):
    """Seeded initial fields, numpy FP64 [k, j, i] arrays: plug flow (v = v_in,
    u = w = 0) and a pressure that falls by rho |g| hy per row towards 0 above
    the top, each perturbed by uniform noise of relative size `noise` (velocity
    noise scaled by v_in, pressure noise by rho |g| hy).  old = "same": the
    old-time velocities equal these; "draw": drawn the same way, afterwards.
    Draw order: u, v, w, p, then u0, v0, w0."""
    nx, ny, nz = int(box["nx"]), int(box["ny"]), int(box["nz"])
    rng = np.random.default_rng(np.random.SeedSequence([2211, 15605, 1000, int(seed)]))
    vin = float(box["v_in"])
    dp = float(box["rho"]) * abs(float(box["gy"])) * float(box["hy"])
    shp = dict(u=(nz, ny, nx + 1), v=(nz, ny + 1, nx), w=(nz + 1, ny, nx), p=(nz, ny, nx))

    def velocities():
        u = noise * vin * rng.uniform(-1, 1, shp["u"])
        v = vin * (1.0 + noise * rng.uniform(-1, 1, shp["v"]))
        w = noise * vin * rng.uniform(-1, 1, shp["w"])
        return u, v, w

    u, v, w = velocities()
    j = np.arange(ny, dtype=np.float64)
    p = (ny - j)[None, :, None] * dp + noise * dp * rng.uniform(-1, 1, shp["p"])
    st = dict(u=u, v=v, w=w, p=p)
    if old == "same":
        st.update(u0=u.copy(), v0=v.copy(), w0=w.copy())
    else:
        u0, v0, w0 = velocities()
        st.update(u0=u0, v0=v0, w0=w0)
    return st
