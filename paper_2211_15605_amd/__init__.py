"""MI355X-native equation-set solver (arXiv 2211.15605: equation decomposition).

The per-equation-set linear solve of a time step -- Jacobi-preconditioned
BiCGSTAB on the 7-point finite-volume system a_P x_P - sum a_nb x_nb = b --
runs in hand-written gfx950 HIP kernels behind the C ABI of
``include/eqsolve.h``; this package is its Python binding.

Submodules load lazily: ``workloads`` (seeded inputs) needs neither torch nor
the HIP library; ``solver``/``binding``/``autograd`` need both.
"""
import importlib

__all__ = ["Context", "EqSolveError", "EqSolveNotConverged", "EqSolveFn", "solve", "solve_noalloc", "workloads",
           "binding", "solver", "autograd"]


def __getattr__(name):
    if name in ("Context", "EqSolveError", "EqSolveNotConverged", "solve", "solve_noalloc"):
        return getattr(importlib.import_module(".solver", __name__), name)
    if name == "EqSolveFn":
        return importlib.import_module(".autograd", __name__).EqSolveFn
    if name in ("workloads", "binding", "solver", "autograd", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
