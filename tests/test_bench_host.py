"""Host-side logic of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_used_only_while_it_matches_the_kernel_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "fused_fp64_sym128x256x128_traffic.json")))
    got = bench.measured_traffic(1, "fused")
    if rec["kernel_source_sha256"] == bench.kernel_source_digest():
        assert got == rec["bytes_per_launch"]
        # counted traffic is the algorithmic bytes plus halo re-reads: within 20 % above
        assert rec["algorithmic_bytes_per_launch"] <= got <= 1.2 * rec["algorithmic_bytes_per_launch"]
    else:
        assert got is None
    assert bench.measured_traffic(2, "fused") is None
    assert bench.measured_traffic(1, "nonexistent") is None


def test_algorithmic_words_per_step():
    # single-sync step: reads s, t, p, v, y, r^, f and six coefficients, writes y, p, v, s, t
    assert bench.WORDS["fused"] == 13 + 5 == bench.STEP_WORDS[1]
    # three launches: K1 12, K2 9, K3 8
    assert bench.WORDS["k1"] + bench.WORDS["k2"] + bench.WORDS["k3"] == bench.STEP_WORDS[3] == 29


def test_symmetric_form_words_and_which_workloads_take_it():
    # the symmetric form reads s, t, p, v, y, r^, f, a_E, a_N, a_T and 1/a_P, writes y, p, v, s, t
    assert bench.WORDS["fused_sym"] == 11 + 5
    assert bench.step_words(1, True) == (16, 16) and bench.step_words(1, False) == (18, 18)
    assert bench.step_words(3, True) == (bench.WORDS["k1"], 29)  # the three-launch iteration has no such form
    # the device check wants a_W(c) == a_E(c-1), a_S(c) == a_N(c-nx), a_B(c) == a_T(c-nx*ny) bit for bit
    # wherever both cells are in the grid: the pressure-like recipe (config 1) meets it, the
    # convection-diffusion one (configs 0, 2-4) does not
    from paper_2211_15605_amd import workloads as W
    for recipe, want in (("sym", True), ("cd", False)):
        s = W.make_set(1, 0, grid=W.Grid(7, 5, 4), recipe=recipe)
        a = [d.reshape(4, 5, 7) for d in s["diags"]]
        same = (np.array_equal(a[2][:, :, 1:], a[1][:, :, :-1]) and np.array_equal(a[4][:, 1:, :], a[3][:, :-1, :])
                and np.array_equal(a[6][1:, :, :], a[5][:-1, :, :]))
        assert same is want, recipe


def test_multigrid_settings_per_recipe():
    assert bench.mg_params_for(1)["gamma"] == 1.6     # pressure-like, near-singular
    assert bench.mg_params_for(2)["gamma"] == 1.0     # convection-diffusion sets
