"""The C-ABI library loads and exports every function include/eqsolve.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("eqsolve.h", "eqsimple.h")]
LIB = os.path.join(ROOT, "paper_2211_15605_amd", "libeqsolve.so")


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(eqs(?:olve|imple)_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2211_15605_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    fns = declared_functions()
    for f in ("eqsolve_create", "eqsolve_solve", "eqsolve_solve_batched", "eqsolve_adjoint",
              "eqsolve_apply", "eqsolve_destroy", "eqsolve_strerror"):
        assert f in fns


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_symbol_list_matches_header():
    import importlib.util
    spec = importlib.util.spec_from_file_location("b", os.path.join(ROOT, "paper_2211_15605_amd", "binding.py"))
    src = open(spec.origin).read()
    m = re.search(r"SYMBOLS = \((.*?)\)", src, re.S)
    listed = sorted(re.findall(r'"(eqs(?:olve|imple)_\w+)"', m.group(1)))
    assert listed == declared_functions()


def test_library_is_built_for_gfx950_only(lib):
    # the offload bundle ids of the library built here name its device targets
    data = open(LIB, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx\w+)", data))
    assert targets == {b"gfx950"}, targets


def test_strerror_and_argument_errors_without_device(lib):
    lib.eqsolve_strerror.restype = ctypes.c_char_p
    assert b"converged" in lib.eqsolve_strerror(0)
    assert b"invalid argument" in lib.eqsolve_strerror(-1)
    # argument errors are found before any HIP call
    lib.eqsolve_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    assert lib.eqsolve_create(ctypes.byref(h), None, 1, 0, None) == -1
    lib.eqsolve_solve.restype = ctypes.c_int
    assert lib.eqsolve_solve(None, 0, None, None, None, ctypes.c_double(1e-10), 10, None) == -4
    assert lib.eqsolve_destroy(None) == 0


def test_noalloc_argument_and_size_errors_without_device(lib):
    # checked before any HIP call: bad arguments, and systems beyond the static workspace
    class G(ctypes.Structure):
        _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]
    f = lib.eqsolve_solve_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(G), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    fake = [ctypes.c_void_p(0x1000 * (k + 1)) for k in range(9)]
    diag = (ctypes.c_void_p * 7)(*fake[:7])
    g = G(64, 64, 64)
    assert f(None, diag, fake[7], fake[8], 1e-10, 10, None, None) == -1
    assert f(ctypes.byref(g), None, fake[7], fake[8], 1e-10, 10, None, None) == -1
    assert f(ctypes.byref(g), diag, fake[7], fake[7], 1e-10, 10, None, None) == -1   # x aliases b
    assert f(ctypes.byref(g), diag, fake[7], fake[8], 1.5, 10, None, None) == -1
    assert f(ctypes.byref(g), diag, fake[7], fake[8], 1e-10, 0, None, None) == -1
    big = G(64, 64, 65)   # 266,240 cells > EQS_NOALLOC_MAX_CELLS
    assert f(ctypes.byref(big), diag, fake[7], fake[8], 1e-10, 10, None, None) == -5
    lib.eqsolve_strerror.restype = ctypes.c_char_p
    assert b"static workspace" in lib.eqsolve_strerror(-5)


def test_stream_probe_argument_errors_without_device(lib):
    # checked before any HIP call: mixes other than 11 or 13 reads and 5 writes, null or aliased arrays
    f = lib.eqsolve_debug_stream
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                  ctypes.c_void_p]
    ins = (ctypes.c_void_p * 13)(*[0x1000 * (k + 1) for k in range(13)])
    outs = (ctypes.c_void_p * 5)(*[0x100000 * (k + 1) for k in range(5)])
    assert f(ins, 12, outs, 5, 100, 1, None) == -1
    assert f(ins, 13, outs, 4, 100, 1, None) == -1
    assert f(ins, 13, outs, 5, 0, 1, None) == -1
    assert f(None, 13, outs, 5, 100, 1, None) == -1
    aliased = (ctypes.c_void_p * 5)(*([0x1000] + [0x100000 * (k + 2) for k in range(4)]))
    assert f(ins, 13, aliased, 5, 100, 1, None) == -1
    holes = (ctypes.c_void_p * 13)(*([0x1000 * (k + 1) for k in range(12)] + [None]))
    assert f(holes, 13, outs, 5, 100, 1, None) == -1
