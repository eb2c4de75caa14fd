"""CPU oracle for the per-equation-set linear solve (arXiv 2211.15605).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It wraps the
plain C implementation in ``orc.c`` (FP64 right-Jacobi BiCGSTAB, the 7-point
stencil product and its transpose, the adjoint gradient formulas) and adds a
few NumPy helpers that are themselves defined in the plainest possible way.
It shares nothing with the HIP library.

Every function is pinned by ``tests/test_oracle_pins.py`` against facts that
do not come from this code: closed-form eigenpairs, the adjoint identity,
row-sum invariants, LAPACK dense and banded solves, exact finite termination
of Krylov methods, and central finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_default = None

# result codes of orc.c
OK, NOT_CONVERGED, BREAKDOWN, NONFINITE, BAD_ARG, NOMEM = 0, 1, 2, 3, -1, -2

SLOTS = ("P", "E", "W", "N", "S", "T", "B")


class OrcInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("half_exit", ctypes.c_int32),
        ("rel_res", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def compile_c(src: str, out: str) -> str:
    """gcc, OpenMP, IEEE arithmetic with no contraction and no fast-math."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile orc.c into liborc.so next to it."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    return compile_c(_SRC, _LIB)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _diag_ptrs(diags):
    arrs = [_f64(d).ravel() for d in diags]
    if len(arrs) != 7:
        raise ValueError("need 7 coefficient arrays (P, E, W, N, S, T, B)")
    ptrs = (ctypes.c_void_p * 7)(*[a.ctypes.data for a in arrs])
    return arrs, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p))


class OrcMgParams(ctypes.Structure):
    _fields_ = [
        ("omega", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("coarse_sweeps", ctypes.c_int32),
        ("coarse_cells", ctypes.c_int32),
    ]


def mg_params(omega=0.8, gamma=1.0, coarse_sweeps=30, coarse_cells=512):
    return OrcMgParams(float(omega), float(gamma), int(coarse_sweeps), int(coarse_cells))


class Oracle:
    """The oracle's functions bound to one compiled copy of orc.c."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        dpp = ctypes.POINTER(ctypes.c_void_p)
        L.orc_apply.argtypes = [ctypes.c_int] * 3 + [dpp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.orc_apply.restype = None
        L.orc_dot.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_dot.restype = ctypes.c_double
        L.orc_bicgstab.argtypes = [ctypes.c_int] * 3 + [dpp, ctypes.c_void_p, ctypes.c_void_p,
                                                        ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_int, ctypes.POINTER(OrcInfo),
                                                        ctypes.c_void_p]
        L.orc_bicgstab.restype = ctypes.c_int
        L.orc_bicgstab_mg.argtypes = [ctypes.c_int] * 3 + [dpp, ctypes.c_void_p, ctypes.c_void_p,
                                                           ctypes.c_double, ctypes.c_int,
                                                           ctypes.POINTER(OrcMgParams), ctypes.POINTER(OrcInfo),
                                                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        L.orc_bicgstab_mg.restype = ctypes.c_int
        L.orc_mg_coarsen.argtypes = [ctypes.c_int] * 3 + [dpp, ctypes.POINTER(ctypes.c_int), dpp]
        L.orc_mg_coarsen.restype = ctypes.c_int
        L.orc_mg_apply.argtypes = [ctypes.c_int] * 3 + [dpp, ctypes.POINTER(OrcMgParams), ctypes.c_void_p,
                                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
        L.orc_mg_apply.restype = ctypes.c_int
        L.orc_grad.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_void_p, dpp]
        L.orc_grad.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        self.L = L
        self.path = path

    def set_threads(self, n: int) -> None:
        self.L.orc_set_threads(int(n))

    def get_threads(self) -> int:
        return int(self.L.orc_get_threads())

    def apply(self, shape, diags, x, transpose: bool = False):
        """y = A x (or A^T x) for the 7-point operator on a grid shape = (nx, ny, nz)."""
        nx, ny, nz = shape
        keep, dp = _diag_ptrs(diags)
        x = _f64(x).ravel()
        y = np.empty(nx * ny * nz)
        assert x.size == y.size and all(a.size == y.size for a in keep)
        self.L.orc_apply(nx, ny, nz, dp, _ptr(x), _ptr(y), int(bool(transpose)))
        return y

    def dot(self, u, v) -> float:
        u = _f64(u).ravel()
        v = _f64(v).ravel()
        assert u.size == v.size
        return float(self.L.orc_dot(u.size, _ptr(u), _ptr(v)))

    def bicgstab(self, shape, diags, b, x0=None, tol=1e-10, maxit=1000, jacobi=True,
                 transpose=False, history=False):
        """Right-preconditioned BiCGSTAB on A (or A^T).  Returns (x, info[, history])."""
        nx, ny, nz = shape
        n = nx * ny * nz
        keep, dp = _diag_ptrs(diags)
        b = _f64(b).ravel()
        x = np.zeros(n) if x0 is None else _f64(x0).ravel().copy()
        assert b.size == n and x.size == n and all(a.size == n for a in keep)
        info = OrcInfo()
        hist = np.full(max(int(maxit), 1), np.nan) if history else None
        self.L.orc_bicgstab(nx, ny, nz, dp, _ptr(b), _ptr(x), float(tol), int(maxit),
                            int(bool(jacobi)), int(bool(transpose)), ctypes.byref(info),
                            _ptr(hist) if history else None)
        d = info.as_dict()
        if history:
            return x, d, hist[: max(d["iters"], 0)]
        return x, d

    def mg_coarsen(self, shape, diags):
        """Galerkin coarse operator (P^T A P, piecewise-constant P over 2x2x2 aggregates).
        Returns (coarse shape, 7 coarse diagonals)."""
        nx, ny, nz = shape
        keep, dp = _diag_ptrs(diags)
        cshape = ((nx + 1) // 2, (ny + 1) // 2, (nz + 1) // 2)
        nc = cshape[0] * cshape[1] * cshape[2]
        out = [np.empty(nc) for _ in range(7)]
        op = ctypes.cast((ctypes.c_void_p * 7)(*[o.ctypes.data for o in out]), ctypes.POINTER(ctypes.c_void_p))
        dims = (ctypes.c_int * 3)()
        rc = self.L.orc_mg_coarsen(nx, ny, nz, dp, dims, op)
        assert rc == 0 and tuple(dims) == cshape
        return cshape, out

    def mg_apply(self, shape, diags, r, params=None):
        """z = B^{-1} r, one V-cycle; returns (z, number of levels)."""
        nx, ny, nz = shape
        keep, dp = _diag_ptrs(diags)
        r = _f64(r).ravel()
        z = np.empty_like(r)
        prm = params if params is not None else mg_params()
        lv = ctypes.c_int(0)
        rc = self.L.orc_mg_apply(nx, ny, nz, dp, ctypes.byref(prm), _ptr(r), _ptr(z), ctypes.byref(lv))
        assert rc == 0, rc
        return z, lv.value

    def bicgstab_mg(self, shape, diags, b, x0=None, tol=1e-10, maxit=1000, params=None, history=False):
        """BiCGSTAB with the multigrid V-cycle as right preconditioner.
        Returns (x, info[, history]); info also carries the number of levels."""
        nx, ny, nz = shape
        n = nx * ny * nz
        keep, dp = _diag_ptrs(diags)
        b = _f64(b).ravel()
        x = np.zeros(n) if x0 is None else _f64(x0).ravel().copy()
        assert b.size == n and x.size == n and all(a.size == n for a in keep)
        info = OrcInfo()
        prm = params if params is not None else mg_params()
        hist = np.full(max(int(maxit), 1), np.nan) if history else None
        lv = ctypes.c_int(0)
        self.L.orc_bicgstab_mg(nx, ny, nz, dp, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(prm),
                               ctypes.byref(info), _ptr(hist) if history else None, ctypes.byref(lv))
        d = info.as_dict()
        d["levels"] = lv.value
        if history:
            return x, d, hist[: d["iters"]]
        return x, d

    def grad(self, shape, lam, x):
        """dL/da_k for the 7 coefficient arrays given lambda = A^{-T} dL/dx and x."""
        nx, ny, nz = shape
        n = nx * ny * nz
        lam = _f64(lam).ravel()
        x = _f64(x).ravel()
        g = [np.empty(n) for _ in range(7)]
        gp = (ctypes.c_void_p * 7)(*[a.ctypes.data for a in g])
        self.L.orc_grad(nx, ny, nz, _ptr(lam), _ptr(x), ctypes.cast(gp, ctypes.POINTER(ctypes.c_void_p)))
        return g

    # plain helpers built on the functions above
    def rel_residual(self, shape, diags, b, x, transpose=False) -> float:
        """||b - A x||_2 / ||b||_2 in FP64: the invariant every solve result must meet."""
        r = _f64(b).ravel() - self.apply(shape, diags, x, transpose)
        bb = self.dot(b, b)
        return float(np.sqrt(self.dot(r, r) / bb)) if bb > 0 else float(np.sqrt(self.dot(r, r)))

    def dense(self, shape, diags, transpose=False):
        """Dense matrix assembled column by column from A e_c (tiny grids only)."""
        nx, ny, nz = shape
        n = nx * ny * nz
        if n > 8192:
            raise ValueError("dense assembly is for tiny grids")
        M = np.empty((n, n))
        e = np.zeros(n)
        for c in range(n):
            e[c] = 1.0
            M[:, c] = self.apply(shape, diags, e, transpose)
            e[c] = 0.0
        return M

    def forward_error_certificate(self, shape, diags, b, x) -> float:
        """Varah (1975): ||x - x*||_inf <= ||b - A x||_inf / min_c(a_P - sum |a_nb|)."""
        m = diag_dominance_margin(shape, diags)
        if m <= 0:
            return float("inf")
        r = _f64(b).ravel() - self.apply(shape, diags, x)
        return float(np.max(np.abs(r)) / m)

    matching_digits = staticmethod(lambda ref, val: matching_digits(ref, val))


def default() -> Oracle:
    global _default
    with _lock:
        if _default is None:
            _default = Oracle(build())
    return _default


def set_threads(n):
    default().set_threads(n)


def get_threads():
    return default().get_threads()


def apply(shape, diags, x, transpose=False):
    return default().apply(shape, diags, x, transpose)


def dot(u, v):
    return default().dot(u, v)


def bicgstab(shape, diags, b, **kw):
    return default().bicgstab(shape, diags, b, **kw)


def grad(shape, lam, x):
    return default().grad(shape, lam, x)


def rel_residual(shape, diags, b, x, transpose=False):
    return default().rel_residual(shape, diags, b, x, transpose)


def dense(shape, diags, transpose=False):
    return default().dense(shape, diags, transpose)


def forward_error_certificate(shape, diags, b, x):
    return default().forward_error_certificate(shape, diags, b, x)


def diag_dominance_margin(shape, diags) -> float:
    """min_c (a_P - sum of in-grid |a_nb|): the Varah lower bound on sigma_min."""
    nx, ny, nz = shape
    a = [_f64(d).reshape(nz, ny, nx) for d in diags]
    s = np.abs(a[0]).copy()
    off = np.zeros_like(s)
    off[:, :, :-1] += np.abs(a[1][:, :, :-1])
    off[:, :, 1:] += np.abs(a[2][:, :, 1:])
    off[:, :-1, :] += np.abs(a[3][:, :-1, :])
    off[:, 1:, :] += np.abs(a[4][:, 1:, :])
    off[:-1, :, :] += np.abs(a[5][:-1, :, :])
    off[1:, :, :] += np.abs(a[6][1:, :, :])
    return float(np.min(s - off))


def matching_digits(ref, val):
    """Eq. (6) of the paper: -log10(|ref - val| / |ref|) per entry (non-zero ref only).

    Exact matches are reported as 17 digits (beyond FP64's resolution)."""
    ref = np.asarray(ref, dtype=np.float64).ravel()
    val = np.asarray(val, dtype=np.float64).ravel()
    nz = ref != 0
    rel = np.abs(ref[nz] - val[nz]) / np.abs(ref[nz])
    with np.errstate(divide="ignore"):
        d = -np.log10(rel)
    d[rel == 0] = 17.0
    return d
