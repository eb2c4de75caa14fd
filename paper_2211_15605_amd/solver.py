"""Python API of the equation-set solver on torch tensors.

    ctx = Context([(nx, ny, nz)], precision="fp64")
    x, info = ctx.solve(diags, b, tol=1e-10, maxit=1000)

``diags`` is a sequence of 7 float64 CUDA tensors (P, E, W, N, S, T, B), each
holding nx*ny*nz values (flat, or shaped (nz, ny, nx)); ``b`` and ``x`` are
likewise.  Arguments are checked here (TypeError / ValueError) before the C
library is called; the library's own codes come back as ``info["status"]``
and, unless ``check=False``, as exceptions for status != 0.

Module-level calls: ``solve(diags, b, x0, tol, maxit, precision, grid)`` (a
one-off context per call) and ``solve_noalloc(...)`` (the FP64 solve on the
library's static workspace, no allocation at all).
"""
from __future__ import annotations

import torch

from . import binding as B


class EqSolveError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, B.strerror(code), code))


class EqSolveNotConverged(EqSolveError):
    def __init__(self, code, info, what="solve"):
        self.info = info
        super().__init__(code, what)


def _check_vec(t, n, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64, got %s" % (name, t.dtype))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError("%s must be on %s" % (name, device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != n:
        raise ValueError("%s has %d values, the grid has %d" % (name, t.numel(), n))
    return t.data_ptr()


class Context:
    """One eqs_ctx: the workspace for a fixed list of grids, bound to a stream."""

    def __init__(self, grids, precision: str = "fp64", stream: torch.cuda.Stream | None = None, device=None):
        if precision not in B.PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(B.PRECISIONS))
        grids = [tuple(int(v) for v in g) for g in grids]
        if not grids or any(len(g) != 3 or min(g) < 1 for g in grids):
            raise ValueError("grids must be (nx, ny, nz) triples of positive sizes")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            rc, h = B.eqsolve_create(grids, B.PRECISIONS[precision], self.stream.cuda_stream)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_create")
        self.h = h
        self.grids = grids
        self.precision = precision

    def close(self):
        if getattr(self, "h", None):
            B.eqsolve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def n(self, set_id=0):
        nx, ny, nz = self.grids[set_id]
        return nx * ny * nz

    def _diag_ptrs(self, diags, n):
        if len(diags) != 7:
            raise ValueError("need 7 coefficient tensors (P, E, W, N, S, T, B)")
        return [_check_vec(d, n, "diag[%d]" % k, self.device) for k, d in enumerate(diags)]

    def layout(self, set_id=0):
        rc, v = B.eqsolve_debug_layout(self.h, set_id)
        keys = ("cpt", "segments", "kc", "chunks", "tiles", "readbacks", "syncs", "flat_blocks", "fused_threads",
                "fused_segments", "fused_tiles", "fused_order")
        return dict(zip(keys, v))

    def set_preconditioner(self, kind="jacobi", **params):
        """'jacobi' (default) or 'mg' (aggregation multigrid V-cycle, FP64 contexts; params:
        omega, gamma, coarse_sweeps, coarse_cells).  See eqsolve_set_preconditioner."""
        k = {"jacobi": B.EQS_PRECOND_JACOBI, "mg": B.EQS_PRECOND_MG}.get(kind)
        if k is None:
            raise ValueError("preconditioner must be 'jacobi' or 'mg'")
        rc = B.eqsolve_set_preconditioner(self.h, k, params or None)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_set_preconditioner")

    def set_step_form(self, form="scaled"):
        """'scaled' (default: a per-solve pass writes the coefficients of A D^-1) or 'unscaled' (each
        step reads the caller's coefficients and 1/a_P; for solves of a few steps).  FP64 contexts;
        see eqsolve_set_step_form."""
        k = {"scaled": B.EQS_STEP_SCALED, "unscaled": B.EQS_STEP_UNSCALED}.get(form)
        if k is None:
            raise ValueError("form must be 'scaled' or 'unscaled'")
        rc = B.eqsolve_set_step_form(self.h, k)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_set_step_form")

    def precond_apply(self, diags, r, set_id=0, out=None):
        """z = B^-1 r, one V-cycle of the multigrid preconditioner (diagnostics); returns (z, levels)."""
        import torch
        n = self.n(set_id)
        dp = self._diag_ptrs(diags, n)
        rp = _check_vec(r, n, "r", self.device)
        z = out if out is not None else torch.empty_like(r)
        zp = _check_vec(z, n, "z", self.device)
        rc, levels = B.eqsolve_debug_precond(self.h, set_id, dp, rp, zp)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_debug_precond")
        return z, levels

    def autotune(self, cache_path=None, iters=6):
        """Choose every set's launch shape by timing candidates on synthetic systems of the
        same shapes (see eqsolve_autotune); returns the new layouts."""
        rc = B.eqsolve_autotune(self.h, cache_path, iters)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_autotune")
        return [self.layout(s) for s in range(len(self.grids))]

    def profile(self, kinds=("k1",), every=1):
        """Time every `every`-th launch of the given kernel kinds with HIP events on this
        context's stream (resets the totals); an empty list turns timing off."""
        mask = 0
        for k in kinds:
            mask |= 1 << (B.KERNEL_KINDS[k] if isinstance(k, str) else int(k))
        rc = B.eqsolve_debug_profile(self.h, mask, every)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_debug_profile")

    def kernel_stats(self, kind, fp32=False):
        """(launches, total ms) recorded for a kernel kind (see binding.KERNEL_KINDS)."""
        k = B.KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
        rc, cnt, ms = B.eqsolve_debug_kernel_stats(self.h, k, fp32)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_debug_kernel_stats")
        return cnt, ms

    def solve(self, diags, b, x=None, tol=1e-10, maxit=1000, set_id=0, check=True):
        n = self.n(set_id)
        dp = self._diag_ptrs(diags, n)
        bp = _check_vec(b, n, "b", self.device)
        if x is None:
            x = torch.zeros_like(b)
        xp = _check_vec(x, n, "x", self.device)
        if not (0.0 < tol < 1.0) or int(maxit) < 1:
            raise ValueError("tol must be in (0, 1) and maxit >= 1")
        rc, info = B.eqsolve_solve(self.h, set_id, dp, bp, xp, tol, maxit)
        d = info.as_dict()
        if rc < 0:
            raise EqSolveError(rc, "eqsolve_solve")
        if rc > 0 and check:
            raise EqSolveNotConverged(rc, d)
        return x, d

    def solve_batched(self, diags_list, b_list, x_list=None, tol=1e-10, maxit=1000, check=True):
        ns = len(self.grids)
        if len(diags_list) != ns or len(b_list) != ns:
            raise ValueError("need one system per set (%d)" % ns)
        if x_list is None:
            x_list = [torch.zeros_like(b) for b in b_list]
        tols = list(tol) if isinstance(tol, (list, tuple)) else [tol] * ns
        maxits = list(maxit) if isinstance(maxit, (list, tuple)) else [maxit] * ns
        dps, bps, xps = [], [], []
        for s in range(ns):
            n = self.n(s)
            dps.append(self._diag_ptrs(diags_list[s], n))
            bps.append(_check_vec(b_list[s], n, "b[%d]" % s, self.device))
            xps.append(_check_vec(x_list[s], n, "x[%d]" % s, self.device))
            if not (0.0 < tols[s] < 1.0) or int(maxits[s]) < 1:
                raise ValueError("tol must be in (0, 1) and maxit >= 1")
        rc, infos = B.eqsolve_solve_batched(self.h, dps, bps, xps, tols, maxits)
        ds = [i.as_dict() for i in infos]
        if rc < 0:
            raise EqSolveError(rc, "eqsolve_solve_batched")
        if rc > 0 and check:
            raise EqSolveNotConverged(rc, ds, "solve_batched")
        return x_list, ds

    def adjoint(self, diags, x, w, tol=1e-10, maxit=1000, set_id=0, want_diag=True, check=True):
        n = self.n(set_id)
        dp = self._diag_ptrs(diags, n)
        xp = _check_vec(x, n, "x", self.device)
        wp = _check_vec(w, n, "w", self.device)
        gb = torch.empty_like(w)
        gd = [torch.empty_like(w) for _ in range(7)] if want_diag else None
        rc, info = B.eqsolve_adjoint(self.h, set_id, dp, xp, wp, gb.data_ptr(),
                                     [g.data_ptr() for g in gd] if gd is not None else None, tol, maxit)
        d = info.as_dict()
        if rc < 0:
            raise EqSolveError(rc, "eqsolve_adjoint")
        if rc > 0 and check:
            raise EqSolveNotConverged(rc, d, "adjoint")
        return gb, gd, d

    def apply(self, diags, x, transpose=False, set_id=0, out=None):
        n = self.n(set_id)
        dp = self._diag_ptrs(diags, n)
        xp = _check_vec(x, n, "x", self.device)
        y = torch.empty_like(x) if out is None else out
        yp = _check_vec(y, n, "y", self.device)
        rc = B.eqsolve_apply(self.h, set_id, dp, xp, yp, transpose)
        if rc != 0:
            raise EqSolveError(rc, "eqsolve_apply")
        return y


def _grid_of(diags, grid):
    if grid is not None:
        g = tuple(int(v) for v in grid)
        if len(g) != 3 or min(g) < 1:
            raise ValueError("grid must be an (nx, ny, nz) triple of positive sizes")
        return g
    shp = tuple(diags[0].shape) if len(diags) else ()
    if len(shp) != 3:
        raise ValueError("pass grid=(nx, ny, nz), or diagonals shaped (nz, ny, nx)")
    return (shp[2], shp[1], shp[0])


def solve(diags, b, x0=None, tol=1e-10, maxit=1000, precision="fp64", grid=None, check=True):
    """Solve one system with a context made for it (workspace allocated, then released).
    grid: (nx, ny, nz), or taken from diagonals shaped (nz, ny, nx).  Returns (x, info)."""
    g = _grid_of(diags, grid)
    with Context([g], precision=precision, device=b.device if isinstance(b, torch.Tensor) else None) as ctx:
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        return ctx.solve(diags, b, x, tol=tol, maxit=maxit, check=check)


def solve_noalloc(diags, b, x, tol=1e-10, maxit=1000, grid=None, stream=None, check=True):
    """eqsolve_solve_noalloc: the FP64 solve on the library's static device workspace (no
    allocation by the library or here; x is written in place).  At most
    binding.NOALLOC_MAX_CELLS cells.  Returns (x, info)."""
    g = _grid_of(diags, grid)
    n = g[0] * g[1] * g[2]
    dev = b.device if isinstance(b, torch.Tensor) else None
    if len(diags) != 7:
        raise ValueError("need 7 coefficient tensors (P, E, W, N, S, T, B)")
    dp = [_check_vec(d, n, "diag[%d]" % k, dev) for k, d in enumerate(diags)]
    bp = _check_vec(b, n, "b", dev)
    xp = _check_vec(x, n, "x", dev)
    if not (0.0 < tol < 1.0) or int(maxit) < 1:
        raise ValueError("tol must be in (0, 1) and maxit >= 1")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc, info = B.eqsolve_solve_noalloc(g, dp, bp, xp, tol, maxit, st.cuda_stream)
    d = info.as_dict()
    if rc < 0:
        raise EqSolveError(rc, "eqsolve_solve_noalloc")
    if rc > 0 and check:
        raise EqSolveNotConverged(rc, d, "solve_noalloc")
    return x, d
