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
