"""Host-side logic of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

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


def test_multigrid_settings_per_recipe():
    assert bench.mg_params_for(1)["gamma"] == 1.6     # pressure-like, near-singular
    assert bench.mg_params_for(2)["gamma"] == 1.0     # convection-diffusion sets
