"""Host-side checks of the Python binding that need no GPU."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_missing_library_fails_loudly(tmp_path):
    from paper_2211_15605_amd import binding
    with pytest.raises(RuntimeError, match="not built"):
        binding.load(str(tmp_path / "libeqsolve.so"))


def test_symbol_table_is_loadable():
    from paper_2211_15605_amd import binding
    L = binding.load()
    for name in binding.SYMBOLS:
        assert hasattr(L, name)


def test_argument_checks_before_the_library():
    from paper_2211_15605_amd.solver import _check_vec
    with pytest.raises(TypeError):
        _check_vec(np.zeros(4), 4, "x", None)
    with pytest.raises(TypeError):
        _check_vec(torch.zeros(4, dtype=torch.float32), 4, "x", None)
    with pytest.raises(ValueError):
        _check_vec(torch.zeros(4, dtype=torch.float64), 4, "x", None)  # host tensor


def test_context_rejects_bad_precision_and_grids():
    from paper_2211_15605_amd.solver import Context
    with pytest.raises(ValueError):
        Context([(4, 4, 4)], precision="fp16")
    with pytest.raises(ValueError):
        Context([(4, 0, 4)])


def test_library_argument_errors_without_device():
    import ctypes

    from paper_2211_15605_amd import binding as B
    rc, h = B.eqsolve_create([(4, 4, 4)], 7, None)  # bad precision: rejected before any HIP call
    assert rc == B.EQS_ERR_ARG
    rc, h = B.eqsolve_create([(4, -1, 4)], 0, None)
    assert rc == B.EQS_ERR_ARG
    rc, h = B.eqsolve_create([(1025, 2, 2)], 0, None)  # rows wider than a stencil pass stages
    assert rc == B.EQS_ERR_ARG
    rc, h = B.eqsolve_create([(4, 4, 4)] * 9, 0, None)  # more sets than one launch table takes
    assert rc == B.EQS_ERR_ARG
    assert B.load().eqsolve_autotune(None, None, 4) == B.EQS_ERR_STATE
    assert B.eqsolve_debug_layout(None, 0)[0] == B.EQS_ERR_ARG
    assert B.strerror(B.EQS_BREAKDOWN).startswith("BiCGSTAB breakdown")


def test_simple_box_argument_errors_without_device():
    """eqsimple_create rejects bad boxes and precisions before any HIP call;
    the stage calls reject a missing context."""
    from paper_2211_15605_amd import binding as B
    from paper_2211_15605_amd import workloads as W
    for bad in (dict(nx=0), dict(nx=1024), dict(ny=0), dict(hx=0.0), dict(hz=float("inf")), dict(rho=-1.0),
                dict(mu=-1e-5), dict(mu=float("nan")), dict(dt=0.0), dict(alpha_u=0.0), dict(alpha_u=1.01),
                dict(alpha_p=2.0), dict(gy=float("nan")), dict(v_in=float("inf"))):
        box = W.bed_box(4, 4, 4)
        box.update(bad)
        rc, h = B.eqsimple_create(box, B.EQS_FP64, None)
        assert rc == B.EQS_ERR_ARG and not h.value, bad
    rc, h = B.eqsimple_create(W.bed_box(4, 4, 4), 7, None)
    assert rc == B.EQS_ERR_ARG
    L = B.load()
    assert L.eqsimple_form_momentum(None, None, None, None, None, None, None, None) == B.EQS_ERR_STATE
    assert L.eqsimple_iterate(None, None, None, None, 1, None, None, None) == B.EQS_ERR_STATE
    assert L.eqsimple_step(None, None, None, 1, 0.0, None, None, None) == B.EQS_ERR_STATE
    assert L.eqsimple_set_pressure_preconditioner(None, 1, None) == B.EQS_ERR_STATE
    assert L.eqsimple_destroy(None) == B.EQS_OK
