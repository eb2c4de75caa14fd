"""Plant plausible mistakes in a copy of the oracle and check the pins catch each.

Every mutant is a one-line textual change to a temporary copy of ``orc.c``;
the pin tests of ``test_oracle_pins.py`` are then run against that copy and at
least one of them must fail.  Nothing here touches the real oracle.
"""
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as pins

ORC_SRC = os.path.join(os.path.dirname(O.__file__), "orc.c")

# (name, original text, planted text)
MUTANTS = [
    ("swap_E_W_coefficient", "acc -= a[SLOT_E][c] * x[c + sx];", "acc -= a[SLOT_W][c] * x[c + sx];"),
    ("N_uses_x_stride", "acc -= a[SLOT_N][c] * x[c + sy];", "acc -= a[SLOT_N][c] * x[c + sx];"),
    ("T_reads_wrong_plane", "acc -= a[SLOT_T][c] * x[c + sz];", "acc -= a[SLOT_T][c] * x[c + sy];"),
    ("transpose_E_unshifted", "acc -= a[SLOT_E][c - sx] * x[c - sx];", "acc -= a[SLOT_E][c] * x[c - sx];"),
    ("transpose_B_sign", "acc -= a[SLOT_B][c + sz] * x[c + sz];", "acc += a[SLOT_B][c + sz] * x[c + sz];"),
    ("dot_squares_u", "s += u[c] * v[c];", "s += u[c] * u[c];"),
    ("omega_sign_in_x", "x[c] += alpha * ph[c] + omega * sh[c];", "x[c] += alpha * ph[c] - omega * sh[c];"),
    ("beta_inverted", "(rho / rho_prev) * (alpha / omega)", "(rho / rho_prev) * (omega / alpha)"),
    ("precond_multiplies", "w[c] = pc->kind == 1 ? u[c] / pc->ap[c] : u[c];",
     "w[c] = pc->kind == 1 ? u[c] * pc->ap[c] : u[c];"),
    ("half_step_unpreconditioned", "for (long c = 0; c < n; c++) x[c] += alpha * ph[c];",
     "for (long c = 0; c < n; c++) x[c] += alpha * p[c];"),
    ("residual_sign", "r[c] = b[c] - r[c];", "r[c] = r[c] - b[c];"),
    ("grad_P_sign", "g[SLOT_P][c] = -l * x[c];", "g[SLOT_P][c] = l * x[c];"),
    ("grad_E_unshifted", "g[SLOT_E][c] = i + 1 < nx ? l * x[c + 1] : 0.0;",
     "g[SLOT_E][c] = i + 1 < nx ? l * x[c] : 0.0;"),
    ("grad_T_wrong_stride", "g[SLOT_T][c] = k + 1 < nz ? l * x[c + sz] : 0.0;",
     "g[SLOT_T][c] = k + 1 < nz ? l * x[c + sy] : 0.0;"),
    ("r_update_uses_plus", "r[c] = s[c] - omega * t[c];", "r[c] = s[c] + omega * t[c];"),
    ("sigma_uses_r", "double sigma = orc_dot(n, rh, v);", "double sigma = orc_dot(n, r, v);"),
    ("mg_internal_link_added", "ac[SLOT_P][C] -= coef;", "ac[SLOT_P][C] += coef;"),
    ("mg_link_to_opposite_slot", "ac[SLOT_E + d][C] += coef;", "ac[SLOT_E + (d ^ 1)][C] += coef;"),
    ("mg_restricts_r_not_residual", "rc[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))] += r[c] - q[c];",
     "rc[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))] += r[c];"),
    ("mg_post_smooth_sign", "z[c] = z1[c] + w * (r[c] - q[c]) / ap[c];", "z[c] = z1[c] - w * (r[c] - q[c]) / ap[c];"),
    ("mg_prolongs_to_wrong_aggregate", "z1[c] += m->prm.gamma * e[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))];",
     "z1[c] += m->prm.gamma * e[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 4))];"),
    ("mg_gamma_dropped", "z1[c] += m->prm.gamma * e[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))];",
     "z1[c] += e[i / 2 + (long)cx * (j / 2 + (long)cy * (k / 2))];"),
    ("mg_one_coarse_sweep_short", "for (int it = 0; it < m->prm.coarse_sweeps; it++) {",
     "for (int it = 1; it < m->prm.coarse_sweeps; it++) {"),
    ("mg_coarse_sweep_undamped", "z[c] += w * (r[c] - q[c]) / ap[c];", "z[c] += (r[c] - q[c]) / ap[c];"),
    ("mg_presmooth_undamped", "z1[c] = w * r[c] / ap[c];", "z1[c] = r[c] / ap[c];"),
]

# the pins run against each mutant (cheap ones; each returns normally or raises)
BATTERY = [
    lambda o: pins.test_apply_closed_form_eigenpairs(o, (5, 4, 3), False),
    lambda o: pins.test_apply_closed_form_eigenpairs(o, (5, 4, 3), True),
    lambda o: pins.test_apply_dirichlet_laplacian_eigenpair(o),
    lambda o: pins.test_apply_row_sums_ignore_outward_slots(o),
    lambda o: pins.test_apply_adjoint_identity(o, (6, 5, 4)),
    lambda o: pins.test_dot_against_exactly_rounded_sum(o),
    lambda o: pins.test_bicgstab_matches_dense_lu(o, 8),
    lambda o: pins.test_bicgstab_residual_invariant_and_certificate(o, 1e-10, 0),
    lambda o: pins.test_bicgstab_diagonal_system_exits_after_one_half_step(o),
    lambda o: pins.test_bicgstab_one_dimensional_matches_banded_lu(o),
    lambda o: pins.test_bicgstab_transpose_matches_dense_lu(o),
    lambda o: pins.test_grad_matches_finite_differences_of_dense_solve(o),
    lambda o: pins.test_mg_coarse_operator_is_galerkin_product(o, (5, 3, 4)),
    lambda o: pins.test_mg_vcycle_transpose_identity(o, "cd"),
    lambda o: pins.test_mg_vcycle_transpose_identity(o, "sym"),
    lambda o: pins.test_mg_bicgstab_matches_dense_lu(o),
    lambda o: pins.test_mg_vcycle_matches_dense_definition(o, "cd", (7, 6, 5), 8, 1.6, 3),
]


def test_mutant_table_applies_to_current_source():
    src = open(ORC_SRC).read()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, name


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(ORC_SRC).read()
    assert src.count(old) == 1
    mut = tmp_path / "orc_mut.c"
    mut.write_text(src.replace(old, new))
    so = O.compile_c(str(mut), str(tmp_path / "liborc_mut.so"))
    m = O.Oracle(so)
    caught = []
    for pin in BATTERY:
        try:
            pin(m)
        except Exception as e:  # AssertionError or a numerical failure
            caught.append(type(e).__name__)
    assert caught, "no pin caught mutant %s" % name


# Mistakes planted in the NumPy helper behind the forward-error certificate
# (diag_dominance_margin): each mutated copy of the function is run through the
# margin and certificate pins, and at least one must fail.
MARGIN_MUTANTS = [
    ("W_slot_unshifted", "off[:, :, 1:] += np.abs(a[2][:, :, 1:])", "off[:, :, 1:] += np.abs(a[2][:, :, :-1])"),
    ("T_slot_dropped", "off[:-1, :, :] += np.abs(a[5][:-1, :, :])", "pass"),
    ("N_slot_takes_outward_row", "off[:, :-1, :] += np.abs(a[3][:, :-1, :])", "off[:, :, :] += np.abs(a[3][:, :, :])"),
    ("max_instead_of_min", "return float(np.min(s - off))", "return float(np.max(s - off))"),
    ("sum_not_difference", "return float(np.min(s - off))", "return float(np.min(s + off))"),
]


def _margin_battery(fn):
    import types
    from oracle import oracle as O
    saved = O.diag_dominance_margin
    O.diag_dominance_margin = fn
    caught = []
    try:
        o = O.default()
        for pin in (lambda: pins.test_diag_dominance_margin_of_generated_systems(o, "cd", 0.1),
                    lambda: pins.test_diag_dominance_margin_of_generated_systems(o, "sym", 1e-3),
                    lambda: pins.test_diag_dominance_margin_ignores_outward_slots_and_finds_the_worst_row(o),
                    lambda: pins.test_forward_error_certificate_bounds_the_true_error(o)):
            try:
                pin()
            except Exception as e:
                caught.append(type(e).__name__)
    finally:
        O.diag_dominance_margin = saved
    return caught


def test_margin_mutant_table_applies_to_current_source():
    import inspect
    src = inspect.getsource(O.diag_dominance_margin)
    for name, old, new in MARGIN_MUTANTS:
        assert src.count(old) == 1, name
    assert not _margin_battery(O.diag_dominance_margin)   # the real helper passes


@pytest.mark.parametrize("name,old,new", MARGIN_MUTANTS, ids=[m[0] for m in MARGIN_MUTANTS])
def test_margin_pins_catch_planted_mistake(name, old, new):
    import inspect
    import textwrap
    import numpy as np
    src = textwrap.dedent(inspect.getsource(O.diag_dominance_margin))
    ns = {"np": np, "_f64": O._f64}
    exec(compile(src.replace(old, new), "<mutant %s>" % name, "exec"), ns)
    assert _margin_battery(ns["diag_dominance_margin"]), "no pin caught mutant %s" % name
