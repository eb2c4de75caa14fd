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


def test_traffic_records_are_used_only_with_the_kernel_code_they_were_taken_with():
    import glob
    lib = os.path.join(ROOT, "paper_2211_15605_amd", "libeqsolve.so")
    if not os.path.exists(lib):
        from paper_2211_15605_amd import build
        build.build()
    recs = glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))
    assert recs
    for path in recs:
        rec = json.load(open(path))
        base = os.path.basename(path)[:-len("_traffic.json")]
        kern = "fused_sym" if base.startswith("fused_sym_") else base.split("_", 1)[0]
        workload = base[len(kern) + 1:]
        assert rec["workload"] == workload
        got = bench.measured_traffic(workload, kern)
        if rec["kernel_code_sha256"] == bench.kernel_code_digest(rec["symbol"]):
            assert got == rec["bytes_per_launch"]
            # counted traffic is the algorithmic bytes plus halo re-reads: within 20 % above
            assert 0.95 <= rec["traffic_over_algorithmic_full"] <= 1.2
        else:
            assert got is None
    assert bench.measured_traffic("nonexistent_workload", "fused") is None


def test_kernel_code_is_found_per_kernel_in_the_built_library():
    code = bench.kernel_code()
    fused = [k for k in code if "12fused_kernel" in k]
    # (FP64: scaled, symmetric, raw forms; FP32: scaled, symmetric) x 2 cells per thread x
    # (256 threads: 3 halo slot counts; 512: 2)
    assert len(fused) == (3 + 2) * 2 * (3 + 2), sorted(fused)
    assert all(len(code[k]) > 1000 for k in fused)
    sym = bench.mangled_kernel_name("void eqs::fused_kernel<double, 2, 1, 0, 512>(eqs::LaunchSets)")
    assert sym in code and bench.kernel_code_digest(sym) == bench.kernel_code_digest(sym)


def test_reduce_pmc_scales_by_the_copy_and_keeps_launches_that_did_work(tmp_path):
    # two synthetic counter files: three 1 GiB copies that read as 512 MiB fetched (scale 2),
    # 1 GiB written (scale 1), and four dispatches of the kernel, one of which did no work
    import csv
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    for counter, copy_kib, kvals in (("FETCH_SIZE", 512 * 1024, [100.0, 100.0, 80.0, 0.1]),
                                     ("WRITE_SIZE", 1024 * 1024, [50.0, 50.0, 40.0, 0.0])):
        d = tmp_path / counter
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(hdr)
            i = 0
            for v in kvals:
                w.writerow([i, "void eqs::fused_kernel<double, 2, 2, false>(eqs::LaunchSets)", 1024, counter, v])
                i += 1
            w.writerow([i, "other_kernel", 1024, counter, 1e6])
            for _ in range(3):
                i += 1
                w.writerow([i, "void at::native::copy_kernel_impl", 1 << 27, counter, copy_kib])
    out = tmp_path / "rec.json"
    ns = bench.argparse.Namespace(reduce_pmc=[str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE")],
                                  pmc_kernel="fused_kernel<double, 2, 2, false>", pmc_grid=1024, pmc_words=18,
                                  pmc_cells=1, pmc_workload="synthetic", pmc_out=str(out), pmc_commands=["a", "b"])
    real = bench.mangled_kernel_name
    bench.mangled_kernel_name = lambda name, lib=None: "_ZN3eqs12fused_kernelIdLi2ELi1ELb0ELi512EEEvNS_10LaunchSetsE"
    try:
        bench.reduce_pmc(ns)
    finally:
        bench.mangled_kernel_name = real
    rec = json.load(open(out))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["dispatches_with_work"] == 3 and rec["full_dispatches"] == 2
    assert abs(rec["bytes_per_launch"] - 1024 * (2 * (280 / 3) + (140 / 3))) < 1e-6
    assert rec["bytes_per_full_launch"] == 1024 * (2 * 100 + 50)


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


def _trace(tmp_path, rows):
    import csv
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"])
        for r in rows:
            w.writerow(r)
    return str(d)


def test_trace_gaps_groups_solves_and_splits_the_gaps(tmp_path, capsys):
    # two solves of three 200 us launches, 3 ms apart; in the first a copy sits between launches 2 and 3
    K = "void eqs::fused_kernel<double, 2, 1, 0, 512>(eqs::LaunchSets)"
    us = 1000
    rows = [(K, 0, 200 * us, 1024, 512), (K, 205 * us, 405 * us, 1024, 512),
            ("__amd_rocclr_copyBuffer", 410 * us, 412 * us, 128, 128), (K, 450 * us, 650 * us, 1024, 512),
            (K, 5000 * us, 5200 * us, 1024, 512), (K, 5200 * us, 5400 * us, 1024, 512),
            (K, 5400 * us, 5600 * us, 1024, 512), (K, 6000 * us, 6005 * us, 1024, 512)]
    ns = bench.argparse.Namespace(trace_gaps=_trace(tmp_path, rows), pmc_kernel="fused_kernel<double, 2, 1, 0, 512>",
                                  pmc_grid=1024)
    bench.trace_gaps(ns)
    out = [l for l in capsys.readouterr().out.splitlines() if l.startswith("| 0") or l.startswith("| 1")]
    assert out[0] == "| 0 | 3 | 0.60 | 0.65 | 7.69 % | 1, 5.00 | 1, 45.0 |"
    assert out[1] == "| 1 | 3 | 0.60 | 0.60 | 0.00 % | 2, 0.00 | 0, 0.0 |"


def test_simple_phases_of_one_iteration(tmp_path, capsys):
    # momentum formation 0-100, two momentum steps with work and one empty, p' formation, a multigrid
    # p' solve, correction, then the next iteration's formation at 1000 us
    us = 1000
    F = "void eqs::fused_kernel<double, 2, 1, 2, 256>(eqs::LaunchSets)"
    rows = [("form_momentum_kernel", 0, 100 * us, 1, 1), (F, 110 * us, 210 * us, 1, 1),
            (F, 210 * us, 310 * us, 1, 1), (F, 310 * us, 312 * us, 1, 1),
            ("form_pressure_kernel", 320 * us, 350 * us, 1, 1), ("eqs::mg_restrict_kernel", 360 * us, 370 * us, 1, 1),
            ("correct_kernel", 900 * us, 950 * us, 1, 1), ("form_momentum_kernel", 1000 * us, 1100 * us, 1, 1)]
    ns = bench.argparse.Namespace(simple_phases=_trace(tmp_path, rows))
    bench.simple_phases(ns)
    lines = capsys.readouterr().out.splitlines()
    assert "| multigrid, 2 | 1 | 100 | 220 | 30 | 550 | 50 | 1000 | 450 |" in lines
    assert any("fused_kernel<double, 2, 1, 2, 256>`: 202.0" in l for l in lines)


def test_summarize_counters_means_over_long_dispatches(tmp_path, capsys):
    import csv
    d = tmp_path / "pmc"
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        for i, (v, dur) in enumerate([(10.0, 600000), (30.0, 700000), (1000.0, 1000)]):
            w.writerow([i, "void eqs::fused_kernel<double, 2, 1, 0, 512>(eqs::LaunchSets)", 884736, "SQ_WAVES", v,
                        0, dur])
        w.writerow([9, "other_kernel(int)", 884736, "SQ_WAVES", 5.0, 0, 900000])
    ns = bench.argparse.Namespace(summarize_counters=str(d), trace_kernels="fused_kernel", pmc_grid=884736)
    bench.summarize_counters(ns)
    out = capsys.readouterr().out
    assert "`void eqs::fused_kernel<double, 2, 1, 0, 512>`: 2 dispatches; SQ_WAVES 20" in out
    assert "other_kernel" not in out
