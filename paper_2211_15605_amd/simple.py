"""Python API of the SIMPLE iteration on a gas-only bed box (include/eqsimple.h).

    box = dict(nx=96, ny=384, nz=96, hx=1.25e-3, hy=1.25e-3, hz=1.25e-3, rho=1.093, mu=1.9e-5,
               dt=1e-3, gy=-9.81, v_in=0.5, alpha_u=0.5, alpha_p=0.8)
    sb = SimpleBox(box)
    info = sb.iterate(vel, p, old, niter=10, tol=(1e-6, 1e-6), maxit=(50, 2000))

Fields are float64 CUDA tensors, contiguous, with the values of the grid
shapes of ``SimpleBox.shapes`` ([k, j, i] order, i fastest): p (nz, ny, nx),
u (nz, ny, nx+1), v (nz, ny+1, nx), w (nz+1, ny, nx).  Argument marshalling
only: formation, solves and correction run in the HIP library.
"""
from __future__ import annotations

import torch

from . import binding as B
from .solver import EqSolveError, _check_vec


def box_shapes(box):
    get = (lambda k: box[k]) if isinstance(box, dict) else (lambda k: getattr(box, k))
    nx, ny, nz = int(get("nx")), int(get("ny")), int(get("nz"))
    return dict(p=(nz, ny, nx), u=(nz, ny, nx + 1), v=(nz, ny + 1, nx), w=(nz + 1, ny, nx))


class SimpleBox:
    """One eqsimple_ctx: the work arrays and solvers of a box, bound to a stream."""

    def __init__(self, box, precision: str = "fp64", stream: torch.cuda.Stream | None = None, device=None):
        if precision not in B.PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(B.PRECISIONS))
        self.shapes = box_shapes(box)
        self.n = {k: v[0] * v[1] * v[2] for k, v in self.shapes.items()}
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            rc, h = B.eqsimple_create(box, B.PRECISIONS[precision], self.stream.cuda_stream)
        if rc != 0:
            raise EqSolveError(rc, "eqsimple_create")
        self._h = h

    # ------------------------------------------------------------ helpers
    def _ptrs(self, ts, names):
        return [_check_vec(t, self.n[c], "%s" % c, self.device) for t, c in zip(ts, names)]

    def zeros(self, comp):
        return torch.zeros(self.shapes[comp], dtype=torch.float64, device=self.device)

    def empty(self, comp):
        return torch.empty(self.shapes[comp], dtype=torch.float64, device=self.device)

    def momentum_outputs(self):
        """Output buffers of form_momentum (every value is written by the kernel)."""
        comps = ("u", "v", "w")
        return ([[self.empty(c) for _ in range(7)] for c in comps], [self.empty(c) for c in comps],
                [self.empty(c) for c in comps])

    def pressure_outputs(self):
        return [self.empty("p") for _ in range(7)], self.empty("p")

    def _call(self, rc, what):
        if rc < 0:
            raise EqSolveError(rc, what)
        return rc

    # ------------------------------------------------------------ stages
    def form_momentum(self, vel, p, old, out=None, norms=True):
        """(diags [3][7], b [3], d [3], res2 [3]) of the u, v, w systems.  out: buffers from
        momentum_outputs() to reuse; norms=False only enqueues the work (res2 is None)."""
        comps = ("u", "v", "w")
        vp = self._ptrs(vel, comps)
        pp = self._ptrs([p], ["p"])[0]
        op = self._ptrs(old, comps)
        diags, b, d = out if out is not None else self.momentum_outputs()
        dptr = [_check_vec(t, self.n[c], "diag", self.device) for s, c in zip(diags, comps) for t in s]
        bptr = self._ptrs(b, comps)
        ddptr = self._ptrs(d, comps)
        with torch.cuda.device(self.device):
            rc, res2 = B.eqsimple_form_momentum(self._h, vp, pp, op, dptr, bptr, ddptr, want_norms=norms)
        self._call(rc, "eqsimple_form_momentum")
        return diags, b, d, (res2 if norms else None)

    def form_pressure(self, d, vel, out=None, norms=True):
        """(diags [7], b, mass2) of the p' system (out, norms as for form_momentum)."""
        comps = ("u", "v", "w")
        dp = self._ptrs(d, comps)
        vp = self._ptrs(vel, comps)
        diags, b = out if out is not None else self.pressure_outputs()
        dptr = self._ptrs(diags, ["p"] * 7)
        bptr = self._ptrs([b], ["p"])[0]
        with torch.cuda.device(self.device):
            rc, m2 = B.eqsimple_form_pressure(self._h, dp, vp, dptr, bptr, want_norm=norms)
        self._call(rc, "eqsimple_form_pressure")
        return diags, b, (m2 if norms else None)

    def correct(self, d, pp, vel, p):
        """In place on vel (u, v, w) and p."""
        comps = ("u", "v", "w")
        dp = self._ptrs(d, comps)
        ppp = self._ptrs([pp], ["p"])[0]
        vp = self._ptrs(vel, comps)
        p_ = self._ptrs([p], ["p"])[0]
        with torch.cuda.device(self.device):
            rc = B.eqsimple_correct(self._h, dp, ppp, vp, p_)
        self._call(rc, "eqsimple_correct")

    def iterate(self, vel, p, old, niter=1, tol=(1e-6, 1e-6), maxit=(100, 5000)):
        """niter SIMPLE iterations in place on vel and p; returns the last one's info."""
        comps = ("u", "v", "w")
        vp = self._ptrs(vel, comps)
        p_ = self._ptrs([p], ["p"])[0]
        op = self._ptrs(old, comps)
        if int(niter) < 1:
            raise ValueError("niter must be >= 1")
        with torch.cuda.device(self.device):
            rc, info = B.eqsimple_iterate(self._h, vp, p_, op, niter, tol, maxit)
        self._call(rc, "eqsimple_iterate")
        return info.as_dict()

    def time_step(self, vel, p, max_iter=30, mass_tol=1e-3, tol=(1e-6, 1e-6), maxit=(100, 5000)):
        """One time step in place on vel and p: the current velocities become the old-time
        fields, then SIMPLE iterations until the mass imbalance falls to mass_tol times the
        first iteration's (at most max_iter); returns the info of the call."""
        comps = ("u", "v", "w")
        vp = self._ptrs(vel, comps)
        p_ = self._ptrs([p], ["p"])[0]
        if int(max_iter) < 1 or not (0.0 <= float(mass_tol) < 1.0):
            raise ValueError("max_iter must be >= 1 and mass_tol in [0, 1)")
        with torch.cuda.device(self.device):
            rc, info = B.eqsimple_step(self._h, vp, p_, max_iter, mass_tol, tol, maxit)
        self._call(rc, "eqsimple_step")
        return info.as_dict()

    def set_pressure_preconditioner(self, kind: str = "mg", **params):
        k = {"jacobi": B.EQS_PRECOND_JACOBI, "mg": B.EQS_PRECOND_MG}[kind]
        with torch.cuda.device(self.device):
            rc = B.eqsimple_set_pressure_preconditioner(self._h, k, params or None)
        self._call(rc, "eqsimple_set_pressure_preconditioner")

    def close(self):
        if getattr(self, "_h", None):
            B.eqsimple_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
