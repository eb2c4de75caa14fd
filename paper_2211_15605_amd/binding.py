"""ctypes binding of libeqsolve.so (the C ABI in include/eqsolve.h).

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch provides device memory and the stream.  The library is loaded after
torch so that both share one HIP runtime; if it is missing this module raises
at load time, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libeqsolve.so")

EQS_FP64, EQS_FP32_REFINE, EQS_FP32 = 0, 1, 2
EQS_OK, EQS_NOT_CONVERGED, EQS_BREAKDOWN, EQS_NONFINITE = 0, 1, 2, 3
EQS_ERR_ARG, EQS_ERR_NOMEM, EQS_ERR_HIP, EQS_ERR_STATE, EQS_ERR_SIZE = -1, -2, -3, -4, -5
# the largest system eqsolve_solve_noalloc takes (EQS_NOALLOC_MAX_CELLS, EQS_NOALLOC_BYTES)
NOALLOC_MAX_CELLS, NOALLOC_BYTES = 262144, 40 << 20
EQS_INFO_SYMMETRIC, EQS_INFO_UNSCALED = 1, 2
EQS_STEP_SCALED, EQS_STEP_UNSCALED = 0, 1
PRECISIONS = {"fp64": EQS_FP64, "fp32_refine": EQS_FP32_REFINE, "fp32": EQS_FP32}

# symbols declared in include/eqsolve.h
SYMBOLS = ("eqsolve_create", "eqsolve_solve", "eqsolve_solve_batched", "eqsolve_adjoint", "eqsolve_apply",
           "eqsolve_destroy", "eqsolve_strerror", "eqsolve_autotune", "eqsolve_debug_layout",
           "eqsolve_debug_profile", "eqsolve_debug_kernel_stats", "eqsolve_set_preconditioner",
           "eqsolve_debug_precond", "eqsolve_solve_noalloc", "eqsolve_set_step_form", "eqsolve_debug_stream",
           "eqsimple_create", "eqsimple_form_momentum", "eqsimple_form_pressure", "eqsimple_correct",
           "eqsimple_iterate", "eqsimple_step", "eqsimple_set_pressure_preconditioner", "eqsimple_destroy")
KERNEL_KINDS = {"setup": 0, "recheck": 1, "report": 2, "k1": 3, "k2": 4, "k3": 5, "cast": 6, "outer": 7,
                "update": 8, "zero": 9, "grad": 10, "apply": 11, "scale": 12, "unscale": 13, "fused": 14,
                "fsetup": 15, "mat": 16}


class EqsGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


EQS_PRECOND_JACOBI, EQS_PRECOND_MG = 0, 1


class EqsMgParams(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("gamma", ctypes.c_double), ("coarse_sweeps", ctypes.c_int32),
                ("coarse_cells", ctypes.c_int32)]


BOX_FIELDS = ("nx", "ny", "nz", "hx", "hy", "hz", "rho", "mu", "dt", "gy", "v_in", "alpha_u", "alpha_p")


class EqsBox(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("pad", ctypes.c_int32)] + \
               [(f, ctypes.c_double) for f in BOX_FIELDS[3:]]


class EqsSimpleInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32 * 4), ("simple_iters", ctypes.c_int32),
                ("mom_residual", ctypes.c_double * 3), ("mass_residual", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": dict(zip(("p", "u", "v", "w"), list(self.iters))),
                "simple_iters": self.simple_iters, "mom_residual": list(self.mom_residual),
                "mass_residual": self.mass_residual}


class EqsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("rel_res", ctypes.c_double), ("sigma_restarts", ctypes.c_int32),
                ("sigma_reruns", ctypes.c_int32)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "outer": self.outer, "rel_res": self.rel_res,
                "symmetric": bool(self.flags & EQS_INFO_SYMMETRIC), "unscaled": bool(self.flags & EQS_INFO_UNSCALED),
                "sigma_restarts": self.sigma_restarts, "sigma_reruns": self.sigma_reruns}


_lock = threading.Lock()
_lib = None

VP = ctypes.c_void_p
VPP = ctypes.POINTER(ctypes.c_void_p)


def load(path: str | None = None):
    """Load libeqsolve.so (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError("libeqsolve.so is not built (%s); run `python -m paper_2211_15605_amd.build`" % p)
        L = ctypes.CDLL(p)
        L.eqsolve_create.argtypes = [ctypes.POINTER(VP), ctypes.POINTER(EqsGrid), ctypes.c_int32, ctypes.c_int32, VP]
        L.eqsolve_create.restype = ctypes.c_int
        L.eqsolve_solve.argtypes = [VP, ctypes.c_int32, VPP, VP, VP, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(EqsInfo)]
        L.eqsolve_solve.restype = ctypes.c_int
        L.eqsolve_solve_batched.argtypes = [VP, ctypes.POINTER(VPP), VPP, VPP, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(EqsInfo)]
        L.eqsolve_solve_batched.restype = ctypes.c_int
        L.eqsolve_adjoint.argtypes = [VP, ctypes.c_int32, VPP, VP, VP, VP, VPP, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(EqsInfo)]
        L.eqsolve_adjoint.restype = ctypes.c_int
        L.eqsolve_apply.argtypes = [VP, ctypes.c_int32, VPP, VP, VP, ctypes.c_int32]
        L.eqsolve_apply.restype = ctypes.c_int
        L.eqsolve_destroy.argtypes = [VP]
        L.eqsolve_destroy.restype = ctypes.c_int
        L.eqsolve_strerror.argtypes = [ctypes.c_int]
        L.eqsolve_strerror.restype = ctypes.c_char_p
        L.eqsolve_autotune.argtypes = [VP, ctypes.c_char_p, ctypes.c_int32]
        L.eqsolve_autotune.restype = ctypes.c_int
        L.eqsolve_debug_layout.argtypes = [VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.eqsolve_debug_layout.restype = ctypes.c_int
        L.eqsolve_debug_profile.argtypes = [VP, ctypes.c_int32, ctypes.c_int32]
        L.eqsolve_debug_profile.restype = ctypes.c_int
        L.eqsolve_debug_kernel_stats.argtypes = [VP, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        L.eqsolve_debug_kernel_stats.restype = ctypes.c_int
        L.eqsolve_set_preconditioner.argtypes = [VP, ctypes.c_int32, ctypes.POINTER(EqsMgParams)]
        L.eqsolve_set_preconditioner.restype = ctypes.c_int
        L.eqsolve_debug_precond.argtypes = [VP, ctypes.c_int32, VPP, VP, VP, ctypes.POINTER(ctypes.c_int32)]
        L.eqsolve_debug_precond.restype = ctypes.c_int
        L.eqsolve_solve_noalloc.argtypes = [ctypes.POINTER(EqsGrid), VPP, VP, VP, ctypes.c_double, ctypes.c_int32,
                                            ctypes.POINTER(EqsInfo), VP]
        L.eqsolve_solve_noalloc.restype = ctypes.c_int
        L.eqsolve_set_step_form.argtypes = [VP, ctypes.c_int32]
        L.eqsolve_set_step_form.restype = ctypes.c_int
        L.eqsolve_debug_stream.argtypes = [VPP, ctypes.c_int32, VPP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                           VP]
        L.eqsolve_debug_stream.restype = ctypes.c_int
        D3 = ctypes.POINTER(ctypes.c_double)
        L.eqsimple_create.argtypes = [ctypes.POINTER(VP), ctypes.POINTER(EqsBox), ctypes.c_int32, VP]
        L.eqsimple_form_momentum.argtypes = [VP, VPP, VP, VPP, VPP, VPP, VPP, D3]
        L.eqsimple_form_pressure.argtypes = [VP, VPP, VPP, VPP, VP, D3]
        L.eqsimple_correct.argtypes = [VP, VPP, VP, VPP, VP]
        L.eqsimple_iterate.argtypes = [VP, VPP, VP, VPP, ctypes.c_int32, D3, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(EqsSimpleInfo)]
        L.eqsimple_step.argtypes = [VP, VPP, VP, ctypes.c_int32, ctypes.c_double, D3, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(EqsSimpleInfo)]
        L.eqsimple_set_pressure_preconditioner.argtypes = [VP, ctypes.c_int32, ctypes.POINTER(EqsMgParams)]
        L.eqsimple_destroy.argtypes = [VP]
        for f in ("eqsimple_create", "eqsimple_form_momentum", "eqsimple_form_pressure", "eqsimple_correct",
                  "eqsimple_iterate", "eqsimple_step", "eqsimple_set_pressure_preconditioner", "eqsimple_destroy"):
            getattr(L, f).restype = ctypes.c_int
        if path is None:
            _lib = L
        return L


def strerror(code: int) -> str:
    return load().eqsolve_strerror(int(code)).decode()


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) if p else None for p in ptrs])
    return ctypes.cast(arr, VPP), arr


# ---------------------------------------------------------------- thin wrappers (same names as the C ABI)

def eqsolve_create(grids, precision: int, stream: int | None):
    L = load()
    g = (EqsGrid * len(grids))(*[EqsGrid(*map(int, gr)) for gr in grids])
    h = VP()
    rc = L.eqsolve_create(ctypes.byref(h), g, len(grids), int(precision), VP(stream or 0))
    return rc, h


def eqsolve_solve(h, set_id, diag_ptrs, b_ptr, x_ptr, tol, maxit):
    L = load()
    dp, keep = ptr_array(diag_ptrs)
    info = EqsInfo()
    rc = L.eqsolve_solve(h, int(set_id), dp, VP(b_ptr), VP(x_ptr), float(tol), int(maxit), ctypes.byref(info))
    return rc, info


def eqsolve_solve_batched(h, diag_ptrs_per_set, b_ptrs, x_ptrs, tols, maxits):
    L = load()
    n = len(b_ptrs)
    inner = [ptr_array(d) for d in diag_ptrs_per_set]
    outer = (VPP * n)(*[i[0] for i in inner])
    bp, kb = ptr_array(b_ptrs)
    xp, kx = ptr_array(x_ptrs)
    t = (ctypes.c_double * n)(*map(float, tols))
    m = (ctypes.c_int32 * n)(*map(int, maxits))
    infos = (EqsInfo * n)()
    rc = L.eqsolve_solve_batched(h, outer, bp, xp, t, m, infos)
    return rc, list(infos)


def eqsolve_solve_noalloc(grid, diag_ptrs, b_ptr, x_ptr, tol, maxit, stream):
    L = load()
    g = EqsGrid(*map(int, grid))
    dp, keep = ptr_array(diag_ptrs)
    info = EqsInfo()
    rc = L.eqsolve_solve_noalloc(ctypes.byref(g), dp, VP(b_ptr), VP(x_ptr), float(tol), int(maxit),
                                 ctypes.byref(info), VP(stream or 0))
    return rc, info


def eqsolve_adjoint(h, set_id, diag_ptrs, x_ptr, w_ptr, gb_ptr, gdiag_ptrs, tol, maxit):
    L = load()
    dp, k1 = ptr_array(diag_ptrs)
    gp, k2 = ptr_array(gdiag_ptrs) if gdiag_ptrs is not None else (None, None)
    info = EqsInfo()
    rc = L.eqsolve_adjoint(h, int(set_id), dp, VP(x_ptr), VP(w_ptr), VP(gb_ptr), gp, float(tol), int(maxit),
                           ctypes.byref(info))
    return rc, info


def eqsolve_apply(h, set_id, diag_ptrs, x_ptr, y_ptr, transpose):
    L = load()
    dp, keep = ptr_array(diag_ptrs)
    return L.eqsolve_apply(h, int(set_id), dp, VP(x_ptr), VP(y_ptr), int(bool(transpose)))


def eqsolve_destroy(h):
    return load().eqsolve_destroy(h)


def eqsolve_set_preconditioner(h, kind, params=None):
    """params: None (defaults) or a dict with omega, gamma, coarse_sweeps, coarse_cells."""
    prm = None
    if params is not None:
        prm = EqsMgParams(float(params.get("omega", 0.8)), float(params.get("gamma", 1.0)),
                          int(params.get("coarse_sweeps", 30)), int(params.get("coarse_cells", 512)))
    return load().eqsolve_set_preconditioner(h, int(kind), ctypes.byref(prm) if prm is not None else None)


def eqsolve_set_step_form(h, form):
    return load().eqsolve_set_step_form(h, int(form))


def eqsolve_debug_precond(h, set_id, diag_ptrs, r_ptr, z_ptr):
    dp, keep = ptr_array(diag_ptrs)
    lv = ctypes.c_int32(0)
    rc = load().eqsolve_debug_precond(h, int(set_id), dp, VP(r_ptr), VP(z_ptr), ctypes.byref(lv))
    return rc, lv.value


def eqsolve_debug_stream(in_ptrs, out_ptrs, n, nontemporal, stream):
    ip, keep_i = ptr_array(in_ptrs)
    op, keep_o = ptr_array(out_ptrs)
    return load().eqsolve_debug_stream(ip, len(in_ptrs), op, len(out_ptrs), int(n), int(bool(nontemporal)),
                                       VP(stream) if stream else None)


def eqsolve_debug_layout(h, set_id):
    out = (ctypes.c_int32 * 12)()
    rc = load().eqsolve_debug_layout(h, int(set_id), out)
    return rc, list(out)


def eqsolve_debug_profile(h, kind_mask, every=1):
    return load().eqsolve_debug_profile(h, int(kind_mask), int(every))


def eqsolve_debug_kernel_stats(h, kind, fp32):
    cnt = ctypes.c_int64()
    ms = ctypes.c_double()
    rc = load().eqsolve_debug_kernel_stats(h, int(kind), int(bool(fp32)), ctypes.byref(cnt), ctypes.byref(ms))
    return rc, int(cnt.value), float(ms.value)


def eqsolve_autotune(h, cache_path=None, iters=6):
    return load().eqsolve_autotune(h, cache_path.encode() if cache_path else None, int(iters))


# ---------------------------------------------------------------- SIMPLE box (include/eqsimple.h)

def make_box(box):
    """EqsBox from a mapping or an object with the BOX_FIELDS attributes."""
    get = (lambda k: box[k]) if isinstance(box, dict) else (lambda k: getattr(box, k))
    b = EqsBox()
    for f in BOX_FIELDS:
        setattr(b, f, int(get(f)) if f in ("nx", "ny", "nz") else float(get(f)))
    return b


def eqsimple_create(box, precision, stream):
    h = VP()
    b = make_box(box)
    rc = load().eqsimple_create(ctypes.byref(h), ctypes.byref(b), int(precision), VP(stream or 0))
    return rc, h


def eqsimple_form_momentum(h, vel, p, old, diag21, b3, d3, want_norms=True):
    vp, k1 = ptr_array(vel)
    op, k2 = ptr_array(old)
    dp, k3 = ptr_array(diag21)
    bp, k4 = ptr_array(b3)
    ddp, k5 = ptr_array(d3)
    res = (ctypes.c_double * 3)()
    rc = load().eqsimple_form_momentum(h, vp, VP(p), op, dp, bp, ddp, res if want_norms else None)
    return rc, list(res)


def eqsimple_form_pressure(h, d3, vel, diag7, b, want_norm=True):
    ddp, k1 = ptr_array(d3)
    vp, k2 = ptr_array(vel)
    dp, k3 = ptr_array(diag7)
    m = ctypes.c_double(0.0)
    rc = load().eqsimple_form_pressure(h, ddp, vp, dp, VP(b), ctypes.byref(m) if want_norm else None)
    return rc, m.value


def eqsimple_correct(h, d3, pp, vel, p):
    ddp, k1 = ptr_array(d3)
    vp, k2 = ptr_array(vel)
    return load().eqsimple_correct(h, ddp, VP(pp), vp, VP(p))


def eqsimple_iterate(h, vel, p, old, niter, tol2, maxit2):
    vp, k1 = ptr_array(vel)
    op, k2 = ptr_array(old)
    t = (ctypes.c_double * 2)(*map(float, tol2))
    m = (ctypes.c_int32 * 2)(*map(int, maxit2))
    info = EqsSimpleInfo()
    rc = load().eqsimple_iterate(h, vp, VP(p), op, int(niter), t, m, ctypes.byref(info))
    return rc, info


def eqsimple_step(h, vel, p, max_iter, mass_tol, tol2, maxit2):
    vp, k1 = ptr_array(vel)
    t = (ctypes.c_double * 2)(*map(float, tol2))
    m = (ctypes.c_int32 * 2)(*map(int, maxit2))
    info = EqsSimpleInfo()
    rc = load().eqsimple_step(h, vp, VP(p), int(max_iter), float(mass_tol), t, m, ctypes.byref(info))
    return rc, info


def eqsimple_set_pressure_preconditioner(h, kind, params=None):
    prm = None
    if params is not None:
        prm = EqsMgParams(float(params.get("omega", 0.8)), float(params.get("gamma", 1.0)),
                          int(params.get("coarse_sweeps", 30)), int(params.get("coarse_cells", 512)))
    return load().eqsimple_set_pressure_preconditioner(h, int(kind), ctypes.byref(prm) if prm is not None else None)


def eqsimple_destroy(h):
    return load().eqsimple_destroy(h)
