"""Plant plausible mistakes in a copy of the SIMPLE oracle and check the pins catch each.

Every mutant is a one-line textual change to the source of ``oracle/simple.py``,
loaded as a separate module; the pins of ``test_simple_pins.py`` then run
against it and at least one must fail.  Nothing here touches the real oracle.
"""
import sys
import types

import pytest

from oracle import simple as S_real
from tests import test_simple_pins as pins

SRC = open(S_real.__file__).read()

# (name, original text, planted text); each original occurs exactly once
MUTANTS = [
    ("u_east_flux_reads_west", "Fe = r * Ax * (u[k, j, i] + u[k, j, i + 1]) / 2",
     "Fe = r * Ax * (u[k, j, i] + u[k, j, i - 1]) / 2"),
    ("u_west_upwind_sign", "    aW = De + max(Fw, 0.0)\n    aN = Dn + max(-Fn, 0.0) if j + 1 < ny",
     "    aW = De + max(-Fw, 0.0)\n    aN = Dn + max(-Fn, 0.0) if j + 1 < ny"),
    ("u_inlet_conductance_not_doubled", "aS, bnd = 0.0, bnd + 2 * Dn + max(Fs, 0.0)\n    if k + 1 < nz:\n        aT = Dt + max(-Ft, 0.0)\n    else:                                                     # wall z = Lz",
     "aS, bnd = 0.0, bnd + Dn + max(Fs, 0.0)\n    if k + 1 < nz:\n        aT = Dt + max(-Ft, 0.0)\n    else:                                                     # wall z = Lz"),
    ("gravity_sign", "+ r * bx.gy * V", "- r * bx.gy * V"),
    ("outlet_ghost_pressure", "p_above = p[k, j, i] if j < ny else 0.0", "p_above = p[k, j, i] if j < ny else p[k, j - 1, i]"),
    ("relaxation_uses_unrelaxed_aP", "b = src + (1.0 - bx.alpha_u) * aPr * x_star", "b = src + (1.0 - bx.alpha_u) * aP * x_star"),
    ("d_from_unrelaxed_aP", "return [aPr, aE, aW, aN, aS, aT, aB], b, 1.0 / aPr",
     "return [aPr, aE, aW, aN, aS, aT, aB], b, 1.0 / aP"),
    ("pressure_outlet_term_dropped", "aP = aE + aW + aN + aS + aT + aB + out", "aP = aE + aW + aN + aS + aT + aB"),
    ("u_correction_sign", "u[k, j, i] += du[k, j, i] * (pp[k, j, i - 1] - pp[k, j, i])",
     "u[k, j, i] += du[k, j, i] * (pp[k, j, i] - pp[k, j, i - 1])"),
    ("w_north_flux_one_plane", "Fn = r * Ay * (v[k - 1, j + 1, i] + v[k, j + 1, i]) / 2",
     "Fn = r * Ay * (v[k, j + 1, i] + v[k, j + 1, i]) / 2"),
    ("v_cross_fluxes_one_row", "jl, jh = j - 1, (j if j < ny else ny - 1)", "jl, jh = j - 1, j - 1"),
    ("w_pressure_force_wrong_area", "src = r * V / bx.dt * st[\"w0\"][k, j, i] + (p[k - 1, j, i] - p[k, j, i]) * Az",
     "src = r * V / bx.dt * st[\"w0\"][k, j, i] + (p[k - 1, j, i] - p[k, j, i]) * Ax"),
    ("mass_imbalance_v_sign", "(v[k, j, i] - v[k, j + 1, i]) * Ay", "(v[k, j + 1, i] - v[k, j, i]) * Ay"),
    ("pressure_relaxation_dropped", "return u, v, w, p + bx.alpha_p * pp", "return u, v, w, p + pp"),
    ("v_wall_tangential_missing", "aE, bnd = 0.0, bnd + 2 * De + max(-Fe, 0.0)\n    if i > 0:\n        aW = De + max(Fw, 0.0)\n    else:\n        aW, bnd = 0.0, bnd + 2 * De + max(Fw, 0.0)\n    aN = Dn + max(-Fn, 0.0) if j < ny else 0.0",
     "aE, bnd = 0.0, bnd\n    if i > 0:\n        aW = De + max(Fw, 0.0)\n    else:\n        aW, bnd = 0.0, bnd + 2 * De + max(Fw, 0.0)\n    aN = Dn + max(-Fn, 0.0) if j < ny else 0.0"),
]


def load_mutant(orig, planted):
    assert SRC.count(orig) == 1, orig
    mod = types.ModuleType("simple_mutant")
    mod.__file__ = S_real.__file__
    sys.modules["simple_mutant"] = mod      # dataclasses look their module up here
    exec(compile(SRC.replace(orig, planted), "simple_mutant", "exec"), mod.__dict__)
    return mod


def battery():
    yield lambda: [pins.test_momentum_rows_equal_face_flux_balance(c, b) for c in "uvw" for b in range(len(pins.BOXES))]
    yield lambda: [pins.test_momentum_under_relaxation(c) for c in "uvw"]
    yield lambda: [pins.test_pressure_correction_restores_continuity(b) for b in range(len(pins.BOXES))]
    yield pins.test_pressure_relaxation_scales_only_the_pressure_update
    yield pins.test_hydrostatic_state_is_a_fixed_point
    yield pins.test_column_closed_form_is_a_fixed_point
    yield pins.test_column_iterations_reach_the_closed_form


def test_unmutated_oracle_passes_battery(monkeypatch):
    monkeypatch.setattr(pins, "S", S_real)
    for check in battery():
        check()


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(monkeypatch, name, orig, planted):
    monkeypatch.setattr(pins, "S", load_mutant(orig, planted))
    caught = []
    for check in battery():
        try:
            check()
        except (AssertionError, ValueError, IndexError, ZeroDivisionError, FloatingPointError):
            caught.append(check)
            break
    assert caught, "mutant %s survived every pin" % name
