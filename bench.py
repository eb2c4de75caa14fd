#!/usr/bin/env python
"""Benchmark of the equation-set solve on one MI355X; prints one JSON line.

Workload (default): the large tall bed, four 7-point convection-diffusion
systems of 192 x 768 x 192 cells (113 M cells, the four equation sets of a
time step), b = A x* with x* ~ U[-1, 1], x0 = 0, relative tolerance 1e-10.
One step is the whole hot path on that batch: all four sets in one batched
FP64 Jacobi-BiCGSTAB call, then all four in one FP32-inner / FP64-refinement
call, each to ||b - A x|| <= 1e-10 ||b||.  The same four sets solved one after
another in plain FP64 are timed beside them (untimed by the step clock).

  value      FP64 BiCGSTAB cell-iterations per second of the batched call
             (sum over sets of cells x iterations / solve time, setup and exit
             recheck included), inputs resident in HBM
  roofline   the dominant kernel (the FP64 single-sync step, batched launch):
             algorithmic bytes per launch / mean launch time from HIP events on
             the solver's stream, against 8 TB/s; traffic from the committed
             rocprofv3 FETCH_SIZE / WRITE_SIZE record of the same code object;
             attainable: the rate of a plain streaming kernel with the same words
             per cell over the same cells (the practical ceiling), and the
             step's fraction of it
  cpu_baseline  the CPU oracle (plain C, OpenMP) solving the same systems; its
             solutions also give each GPU result's error and Eq. (6) digits

--config 1 selects the pressure-like 128 x 256 x 128 system (one set); the
default run also reports it as a section.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BiCGSTAB cell-iters/s & %HBM roofline; time to 1e-10 rel residual vs FP64"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM words per cell per launch of each iteration kernel (reads + writes) on the
# column-scaled operator: K1 r, p, v, 6 coefficients, r^ / p, v; K2 r, v, 6 coefficients / t;
# K3 y, p, r, v, t, r^ / y, r  (29 words per iteration)
WORDS = {"k1": 12, "k2": 9, "k3": 8}
# the single-sync step (one launch): reads s, t, p, v of the previous step, y, r^, f and six
# coefficients; writes y, p, v, s, t (18 words per cell and step)
WORDS["fused"] = 18
# its symmetric form (exactly symmetric matrices): a_E, a_N, a_T and 1/a_P in place of the six
# scaled coefficients (16 words)
WORDS["fused_sym"] = 16
# algorithmic HBM words per cell-iteration of each iteration scheme (reductions per step -> words)
STEP_WORDS = {1: 18, 3: 29}


def step_words(syncs, symmetric):
    """(dominant kernel's words per cell, words per cell-iteration) of the scheme that ran."""
    if syncs == 1:
        w = WORDS["fused_sym" if symmetric else "fused"]
        return w, w
    return WORDS["k1"], STEP_WORDS[syncs]


def _elf_sections(data):
    import struct
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize) for i in range(shnum)]
    stroff = secs[shstrndx][4]
    names = [data[stroff + s[0]: data.index(b"\0", stroff + s[0])].decode() for s in secs]
    return secs, names


def device_code_objects(lib=None):
    """The gfx950 code objects the library carries: its .hip_fatbin section holds one clang
    offload bundle per compiled source, each with a host entry and a device ELF."""
    import struct
    data = open(lib or os.path.join(ROOT, "paper_2211_15605_amd", "libeqsolve.so"), "rb").read()
    secs, names = _elf_sections(data)
    sec = secs[names.index(".hip_fatbin")]
    fb = data[sec[4]:sec[4] + sec[5]]
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    out, pos = [], 0
    while True:
        i = fb.find(magic, pos)
        if i < 0:
            return out
        n, = struct.unpack_from("<Q", fb, i + 24)
        p = i + 32
        for _ in range(n):
            eoff, esize, tlen = struct.unpack_from("<QQQ", fb, p)
            triple = fb[p + 24:p + 24 + tlen].decode()
            p += 24 + tlen
            if "amdgcn" in triple and esize:
                out.append(fb[i + eoff:i + eoff + esize])
        pos = i + 1


def kernel_code(lib=None):
    """{mangled kernel symbol: its machine code bytes} over the library's device code objects."""
    import struct
    out = {}
    for elf in device_code_objects(lib):
        secs, names = _elf_sections(elf)
        for si, sec in enumerate(secs):
            if sec[1] != 2:   # SHT_SYMTAB
                continue
            strsec = secs[sec[6]]
            for k in range(sec[5] // 24):
                st_name, st_info, _o, st_shndx, st_value, st_size = struct.unpack_from("<IBBHQQ", elf, sec[4] + 24 * k)
                if (st_info & 0xF) != 2 or st_size == 0 or st_shndx >= len(secs):   # STT_FUNC with code
                    continue
                nm = elf[strsec[4] + st_name: elf.index(b"\0", strsec[4] + st_name)].decode()
                tgt = secs[st_shndx]
                off = tgt[4] + (st_value - tgt[3])
                out[nm] = elf[off:off + st_size]
    return out


def kernel_code_digest(symbol, lib=None):
    """sha256 of one kernel's machine code in the built library (None if it has no such kernel)."""
    import hashlib
    code = kernel_code(lib).get(symbol)
    return hashlib.sha256(code).hexdigest() if code is not None else None


def mangled_kernel_name(demangled, lib=None):
    """The symbol of the kernel a profiler names `demangled` (as rocprofv3 prints it)."""
    import subprocess
    syms = sorted(kernel_code(lib))
    res = subprocess.run(["c++filt"], input="\n".join(syms), capture_output=True, text=True, check=True)
    for sym, dem in zip(syms, res.stdout.splitlines()):
        if dem.strip() == demangled.strip():
            return sym
    raise KeyError(demangled)


def traffic_record_path(workload, kern):
    return os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kern, workload))


def measured_traffic(workload, kern):
    """HBM bytes per launch of the FP64 iteration kernel `kern` on `workload` from the committed
    rocprofv3 counter record (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy), or None when the
    record is missing or the kernel's machine code has changed since the counters were taken."""
    path = traffic_record_path(workload, kern)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_code_sha256") != kernel_code_digest(rec.get("symbol", "")):
        return None
    return rec["bytes_per_launch"]


def stream_ceiling(cells, nreads, reps=10):
    """The rate (GB/s) of the library's plain streaming kernel with the step's byte mix (nreads FP64
    reads and 5 FP64 writes per cell, nontemporal stores) over `cells` cells: the practical ceiling
    against which the step's own rate is read.  Mean over `reps` back-to-back launches, timed with
    HIP events on torch's current stream (the stream the kernel is launched on)."""
    import torch
    from paper_2211_15605_amd import binding
    buf = torch.zeros((nreads + 5, cells), dtype=torch.float64, device="cuda")
    ins = [buf[k].data_ptr() for k in range(nreads)]
    outs = [buf[nreads + w].data_ptr() for w in range(5)]
    stream = torch.cuda.current_stream().cuda_stream

    def launch():
        rc = binding.eqsolve_debug_stream(ins, outs, cells, 1, stream)
        if rc != 0:
            raise RuntimeError("eqsolve_debug_stream: %s" % binding.strerror(rc))

    for _ in range(3):
        launch()
    torch.cuda.synchronize()
    # back-to-back launches between one event pair, as the step's launches follow each other
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del buf
    torch.cuda.empty_cache()
    return {"value": (nreads + 5) * 8 * cells / (ms * 1e-3) / 1e9, "unit": "GB/s", "mean_launch_ms": ms,
            "kernel": "plain streaming kernel, %d reads + 5 writes per cell (FP64, nontemporal stores, "
                      "256-thread blocks, one cell per thread)" % nreads,
            "cells": cells}


def mg_params_for(cfg):
    """Multigrid preconditioner settings per recipe: the pressure-like (sym) systems take an
    over-corrected coarse step, the convection-diffusion ones the plain Galerkin step."""
    from paper_2211_15605_amd import workloads as W
    # 15 coarsest-level sweeps: as few as keep the iteration count (config 1: 18 iterations with 15,
    # 20, 30 or 60 sweeps, 20 with 10)
    return dict(gamma=1.6 if W.CONFIGS[cfg]["recipe"] == "sym" else 1.0, coarse_cells=2048, coarse_sweeps=15)


def time_mg(Context, grids, solve, cfg, reps=3):
    """FP64 solves with the multigrid preconditioner (outside the timed steps)."""
    import numpy as np
    import torch
    cm = Context(grids, precision="fp64")
    prm = mg_params_for(cfg)
    cm.set_preconditioner("mg", **prm)
    ts, out = [], None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = solve(cm)
        torch.cuda.synchronize()
        if r:
            ts.append(time.perf_counter() - t0)
    cm.close()
    return float(np.min(ts)), out, prm


def time_simple(iters=8, warm=2):
    """SIMPLE iterations of one time step on the gas-only bed box (96 x 384 x 96 pressure cells:
    the p', u, v, w grids of the four-set time step), outside the timed steps: milliseconds per
    SIMPLE iteration with Jacobi and with multigrid p' solves, and the stage kernels' times."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.simple import SimpleBox

    dev = torch.device("cuda", 0)
    box = W.bed_box()
    st = W.box_state(box, seed=0, noise=0.05)
    comps = ("u", "v", "w")
    tol, maxit = (1e-5, 1e-6), (100, 2000)
    out = {"box": "%dx%dx%d pressure cells, h = %g m, dt = %g s, v_in = %g m/s" % (
        box["nx"], box["ny"], box["nz"], box["hx"], box["dt"], box["v_in"]),
        "tol": {"momentum": tol[0], "pressure": tol[1]}, "iterations_timed": iters}
    for kind in ("jacobi", "mg"):
        f = {k: torch.from_numpy(v).to(dev) for k, v in st.items()}
        vel, old = [f[c] for c in comps], [f[c + "0"] for c in comps]
        sb = SimpleBox(box)
        if kind == "mg":
            # the over-corrected coarse step: late in a time step the mass imbalance left is smooth
            # and the coarse correction carries the solve (measured over iterations 3-10: 24 p'
            # iterations per solve with gamma = 1.6, 34 with the plain Galerkin step)
            # (30 coarsest-level sweeps: with 15, 28 p' iterations per solve instead of 24)
            sb.set_pressure_preconditioner("mg", gamma=1.6, coarse_cells=2048, coarse_sweeps=30)
        first = sb.iterate(vel, f["p"], old, niter=1, tol=tol, maxit=maxit)
        if warm > 1:
            sb.iterate(vel, f["p"], old, niter=warm - 1, tol=tol, maxit=maxit)
        ts, infos = [], []
        for _ in range(iters):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos.append(sb.iterate(vel, f["p"], old, niter=1, tol=tol, maxit=maxit))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[kind] = {"ms_per_simple_iteration": 1e3 * float(np.mean(ts)),
                     "solver_iters_last": infos[-1]["iters"], "status_worst": max(i["status"] for i in infos),
                     "mass_residual_first_last": [first["mass_residual"], infos[-1]["mass_residual"]]}
        if kind == "mg":
            # stage kernels on the current state, `reps` calls each, every call between its own pair
            # of events on the library's stream (torch's current stream): the median, so host time
            # between calls does not count; outputs preallocated
            reps = 10
            mo = sb.momentum_outputs()
            po = sb.pressure_outputs()
            d = mo[2]
            pp = torch.zeros_like(f["p"])
            vc = [v.clone() for v in vel]
            pc = f["p"].clone()
            sb.form_momentum(vel, f["p"], old, out=mo)
            sb.form_pressure(d, vel, out=po)
            calls = {"form_momentum": lambda: sb.form_momentum(vel, f["p"], old, out=mo, norms=False),
                     "form_pressure": lambda: sb.form_pressure(d, vel, out=po, norms=False),
                     "correct": lambda: sb.correct(d, pp, vc, pc)}
            nu, nv, nw, npc = (int(np.prod(sb.shapes[c])) for c in ("u", "v", "w", "p"))
            # algorithmic bytes: every input field read once, every output written once
            by = {"form_momentum": 8 * (2 * (nu + nv + nw) + npc + 9 * (nu + nv + nw)),
                  "form_pressure": 8 * (2 * (nu + nv + nw) + 8 * npc),
                  "correct": 8 * (3 * (nu + nv + nw) + 3 * npc)}
            for name, fn in calls.items():
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
                torch.cuda.synchronize()
                for e0, e1 in ev:
                    e0.record()
                    fn()
                    e1.record()
                torch.cuda.synchronize()
                ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
                out["stage_" + name] = {"ms": ms, "algorithmic_MB": by[name] / 1e6,
                                        "GBps": by[name] / (ms * 1e-3) / 1e9}
            del mo, po
            del d, pp, vc, pc
            # whole time steps (one call each): from the initial fields, SIMPLE iterations until the
            # mass imbalance has fallen by 1e-4, at most 50
            g = {k: torch.from_numpy(v).to(dev) for k, v in st.items()}
            vg = [g[c] for c in comps]
            steps = []
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                si = sb.time_step(vg, g["p"], max_iter=50, mass_tol=1e-4, tol=tol, maxit=maxit)
                torch.cuda.synchronize()
                steps.append({"ms": 1e3 * (time.perf_counter() - t0), "simple_iters": si["simple_iters"],
                              "status": si["status"], "mass_residual_last": si["mass_residual"]})
            out["time_steps_mg"] = steps
            del g, vg
        sb.close()
        del f, vel, old
    out["mg_speedup_per_iteration"] = out["jacobi"]["ms_per_simple_iteration"] / out["mg"]["ms_per_simple_iteration"]
    return out


def time_batching(runs=5, warm=2):
    """The four staggered grids of a time step at reduced scales (the grids of the 96 x 384 x 96
    step divided by 4 and by 8 along each axis, as the pressure grid divides), convection-diffusion,
    tol 1e-10: one batched call against the four sets solved one after another, FP64 and FP32 +
    refinement (median milliseconds; outside the timed steps)."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.solver import Context

    dev = torch.device("cuda", 0)
    out = []
    for div in (4, 8):
        nx, ny, nz = 96 // div, 384 // div, 96 // div
        grids = [W.Grid(nx, ny, nz), W.Grid(nx + 1, ny, nz), W.Grid(nx, ny + 1, nz), W.Grid(nx, ny, nz + 1)]
        sets = [W.make_set(2, i, grid=g) for i, g in enumerate(grids)]
        Ds = [[torch.from_numpy(d).to(dev) for d in s_["diags"]] for s_ in sets]
        row = {"grids": ["%dx%dx%d" % g.shape for g in grids], "cells": int(sum(g.n for g in grids))}
        for prec in ("fp64", "fp32_refine"):
            ctx = Context([g.shape for g in grids], precision=prec)
            c64 = Context([g.shape for g in grids], precision="fp64")
            bs = [c64.apply(D, torch.from_numpy(s_["x_star"]).to(dev), set_id=i) for i, (D, s_) in
                  enumerate(zip(Ds, sets))]
            c64.close()
            tb, tq, st = [], [], []
            for r in range(warm + runs):
                xs = [torch.zeros_like(b) for b in bs]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, infos = ctx.solve_batched(Ds, bs, xs, tol=1e-10, maxit=1000, check=False)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for i in range(4):
                    x = torch.zeros_like(bs[i])
                    ctx.solve(Ds[i], bs[i], x, tol=1e-10, maxit=1000, set_id=i, check=False)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if r >= warm:
                    tb.append(t1 - t0)
                    tq.append(t2 - t1)
                    st.append(max(i["status"] for i in infos))
            ctx.close()
            row[prec] = {"batched_ms": 1e3 * float(np.median(tb)), "sequential_ms": 1e3 * float(np.median(tq)),
                         "speedup": float(np.median(tq) / np.median(tb)), "status_worst": max(st)}
        out.append(row)
    return out


def time_adjoint(runs=5, warm=2):
    """The adjoint workload (64^3 convection-diffusion, loss sum(w x), tol 1e-10, FP64): median
    milliseconds of the forward solve and of the adjoint call (A^T solve + the 7 coefficient
    gradients), outside the timed steps."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.solver import Context

    dev = torch.device("cuda", 0)
    s = W.make_set(3, 0, with_weights=True)
    g = s["grid"]
    D = [torch.from_numpy(d).to(dev) for d in s["diags"]]
    w = torch.from_numpy(s["w"]).to(dev)
    ctx = Context([g.shape], precision="fp64")
    b = ctx.apply(D, torch.from_numpy(s["x_star"]).to(dev))
    tf, ta = [], []
    for r in range(warm + runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, fi = ctx.solve(D, b, torch.zeros_like(b), tol=1e-10, maxit=1000, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gb, gd, ai = ctx.adjoint(D, x, w, tol=1e-10, maxit=1000, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r >= warm:
            tf.append(t1 - t0)
            ta.append(t2 - t1)
    # the same pair with the multigrid preconditioner (the adjoint then runs the V-cycle of A^T)
    ctx.set_preconditioner("mg", **mg_params_for(3))
    tfm, tam = [], []
    for r in range(warm + runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, fim = ctx.solve(D, b, torch.zeros_like(b), tol=1e-10, maxit=1000, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gb, gd, aim = ctx.adjoint(D, x, w, tol=1e-10, maxit=1000, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r >= warm:
            tfm.append(t1 - t0)
            tam.append(t2 - t1)
    ctx.close()
    return {"workload": "adjoint64: 64x64x64 convection-diffusion, L = sum(w x), tol 1e-10, FP64",
            "forward_ms": 1e3 * float(np.median(tf)), "forward_iters": fi["iters"],
            "adjoint_ms": 1e3 * float(np.median(ta)), "adjoint_iters": ai["iters"],
            "multigrid": {"forward_ms": 1e3 * float(np.median(tfm)), "forward_iters": fim["iters"],
                          "adjoint_ms": 1e3 * float(np.median(tam)), "adjoint_iters": aim["iters"]},
            "status": max(fi["status"], ai["status"], fim["status"], aim["status"])}


def time_latency(runs=10, warm=3):
    """The small convection-diffusion system (16^3 cells, tol 1e-10), latency-bound: median
    microseconds per FP64 solve from x0 = 0 (outside the timed steps)."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.solver import Context

    dev = torch.device("cuda", 0)
    cfg = W.CONFIGS[0]
    s = W.make_set(0, 0)
    g = s["grid"]
    D = [torch.from_numpy(d).to(dev) for d in s["diags"]]
    ctx = Context([g.shape], precision="fp64")
    b = ctx.apply(D, torch.from_numpy(s["x_star"]).to(dev))
    ts, info = [], None
    for r in range(warm + runs):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = ctx.solve(D, b, x, tol=cfg["tol"], maxit=cfg["maxit"], check=False)
        torch.cuda.synchronize()
        if r >= warm:
            ts.append(time.perf_counter() - t0)
    ctx.close()
    us = 1e6 * float(np.median(ts))
    return {"workload": "cd16: 16x16x16 convection-diffusion, tol 1e-10, FP64", "us_per_solve": us,
            "iters": info["iters"], "us_per_iteration": us / max(info["iters"], 1), "status": info["status"]}


def copy_calibration(res, dev):
    """A plain copy of known size, for scaling the HBM byte counters of a profiled run."""
    import torch
    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    res["copy_calibration_bytes"] = {"read": nb, "write": nb}
    del src, dst


def gpu_leg(args, cfg_id, steps=None, warmup=None, with_mg=True):
    """One set (the pressure-like 128 x 256 x 128 system): FP64 and FP32 + refinement solves per step.
    Returns (result dict, host solutions {"fp64": [x], "fp32_refine": [x]})."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.solver import Context

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda", 0)
    cfg = W.CONFIGS[cfg_id]
    g = cfg["grids"][0]
    s = W.make_set(cfg_id, 0)
    D = [torch.from_numpy(d).to(dev) for d in s["diags"]]
    xs = torch.from_numpy(s["x_star"]).to(dev)
    del s
    c64 = Context([g.shape], precision="fp64")
    c32 = Context([g.shape], precision="fp32_refine")
    if not args.no_tune:
        # launch shapes by measurement on synthetic systems of this shape (untimed)
        c64.autotune(os.environ.get("EQS_TUNE_CACHE"))
        c32.autotune(os.environ.get("EQS_TUNE_CACHE"))
    b = c64.apply(D, xs)  # b = A x* on the device
    tol, maxit = cfg["tol"], cfg["maxit"]

    def step(rec):
        x64 = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x64, i64 = c64.solve(D, b, x64, tol=tol, maxit=maxit, check=False)
        t1 = time.perf_counter()
        x32 = torch.zeros_like(b)
        x32, i32 = c32.solve(D, b, x32, tol=tol, maxit=maxit, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rec is not None:
            rec.append((t1 - t0, t2 - t1, i64, i32))
        return x64, x32

    for _ in range(warmup):
        step(None)
    # the dominant kernel: the fused step (single-sync iteration) or K1 (three launches per step)
    syncs = c64.layout()["syncs"]
    kern = "fused" if syncs == 1 else "k1"
    # the kernel's own start and end stamps on every 8th launch of the timed FP64 solves
    # (sampling keeps the timing's own cost out of the measured solve time)
    c64.profile([kern], every=8)
    rec = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        x64, x32 = step(rec)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start

    n = g.n
    t64 = float(np.mean([r[0] for r in rec]))
    t32 = float(np.mean([r[1] for r in rec]))
    it64 = float(np.mean([r[2]["iters"] for r in rec]))
    it32 = float(np.mean([r[3]["iters"] for r in rec]))
    # the library counts only launches that did work (not the few enqueued past convergence)
    k1_cnt, k1_ms = c64.kernel_stats(kern)
    c64.profile([])
    k1_avg_ms = k1_ms / k1_cnt
    form_sym = bool(rec[-1][2]["symmetric"])
    kw, sw = step_words(syncs, form_sym)
    k1_bytes = kw * 8 * n
    achieved = k1_bytes / (k1_avg_ms * 1e-3) / 1e9
    err64 = float(torch.max(torch.abs(x64 - xs)))
    err32 = float(torch.max(torch.abs(x32 - xs)))
    res = {
        "workload": cfg["name"],
        "value": n * it64 / t64,
        "ms_per_step": 1e3 * t_total / steps,
        "fp64": {"time_to_tol_ms": 1e3 * t64, "iters": it64, "status": rec[-1][2]["status"], "rel_res": rec[-1][2]["rel_res"],
                 "cell_iters_per_s": n * it64 / t64, "model_GBps": n * it64 * sw * 8 / t64 / 1e9,
                 "max_abs_err_vs_xstar": err64},
        "fp32_refine": {"time_to_tol_ms": 1e3 * t32, "inner_iters": it32, "outer": rec[-1][3]["outer"],
                        "sigma_restarts": rec[-1][3]["sigma_restarts"], "status": rec[-1][3]["status"],
                        "rel_res": rec[-1][3]["rel_res"], "cell_iters_per_s": n * it32 / t32,
                        "model_GBps": n * it32 * sw * 4 / t32 / 1e9, "max_abs_err_vs_xstar": err32,
                        "speedup_vs_fp64": t64 / t32},
        "roofline": {"bound": "hbm", "kernel": kern + ("_sym" if form_sym and syncs == 1 else "") + "_fp64",
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(cfg["name"], kern + ("_sym" if form_sym and syncs == 1 else "")),
                     "bytes_per_launch": k1_bytes, "words_per_cell": kw, "mean_launch_ms": k1_avg_ms,
                     "launches": k1_cnt},
        "syncs_per_iteration": syncs,
        "symmetric_form": {"fp64": form_sym, "fp32_refine": bool(rec[-1][3]["symmetric"])},
        "kernels_fp64_ms": {kern: {"launches": k1_cnt, "mean_ms": k1_avg_ms}},
        "layout": c64.layout(),
        "layout_fp32_refine": c32.layout(),
        "cells": n,
    }
    # what a plain kernel streaming the same words per cell reaches over the same cells
    att = stream_ceiling(n, kw - 5)
    att["frac"] = achieved / att["value"]
    res["roofline"]["attainable"] = att
    if with_mg:
        tmg, (xmg, img), mgp = time_mg(Context, [g.shape], lambda cm: cm.solve(D, b, torch.zeros_like(b), tol=tol,
                                                                               maxit=maxit, check=False), cfg_id)
        res["fp64_multigrid"] = {"time_to_tol_ms": 1e3 * tmg, "iters": img["iters"], "status": img["status"],
                                 "rel_res": img["rel_res"], "max_abs_err_vs_xstar": float(torch.max(torch.abs(xmg - xs))),
                                 "speedup_vs_fp64_jacobi": t64 / tmg, "params": mgp}
    if args.calibrate_copy:
        copy_calibration(res, dev)
    sols = {"fp64": [x64.cpu().numpy()], "fp32_refine": [x32.cpu().numpy()]}
    c64.close()
    c32.close()
    return res, sols


def gpu_leg_batched(args):
    """All equation sets of the workload in one call (the four-set time step, the large tall bed).
    Returns (result dict, host solutions {"fp64": [x per set], "fp32_refine": [...]})."""
    import numpy as np
    import torch

    from paper_2211_15605_amd import workloads as W
    from paper_2211_15605_amd.solver import Context

    dev = torch.device("cuda", 0)
    cfg = W.CONFIGS[args.config]
    grids = [g.shape for g in cfg["grids"]]
    Ds, bs, xss = [], [], []
    c64 = Context(grids, precision="fp64")
    c32 = Context(grids, precision="fp32_refine")
    if not args.no_tune:
        c64.autotune(os.environ.get("EQS_TUNE_CACHE"))
        c32.autotune(os.environ.get("EQS_TUNE_CACHE"))
    for i in range(len(grids)):
        s = W.make_set(args.config, i)
        D = [torch.from_numpy(d).to(dev) for d in s["diags"]]
        xs = torch.from_numpy(s["x_star"]).to(dev)
        del s
        Ds.append(D)
        xss.append(xs)
        bs.append(c64.apply(D, xs, set_id=i))
        print("bench: set %d of %s on the device" % (i, cfg["name"]), file=sys.stderr, flush=True)
    tol, maxit = cfg["tol"], cfg["maxit"]
    n_all = [int(np.prod(g)) for g in grids]

    def step(rec):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x64, i64 = c64.solve_batched(Ds, bs, tol=tol, maxit=maxit, check=False)
        t1 = time.perf_counter()
        x32, i32 = c32.solve_batched(Ds, bs, tol=tol, maxit=maxit, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rec is not None:
            rec.append((t1 - t0, t2 - t1, i64, i32))
        return x64, x32

    for _ in range(args.warmup):
        step(None)
    syncs = c64.layout()["syncs"]
    kern = "fused" if syncs == 1 else "k1"
    # the kernel's own start and end stamps on every launch of the timed FP64 solves
    c64.profile([kern], every=1)
    rec = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        x64, x32 = step(rec)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    print("bench: %d timed steps done" % args.steps, file=sys.stderr, flush=True)
    k1_cnt, k1_ms = c64.kernel_stats(kern)
    c64.profile([])
    # the same sets one after another (plain FP64, the comparison the batched forms are measured
    # against), each in a context of its own with the launch shape tuned for it alone
    singles = [Context([g], precision="fp64") for g in grids]
    if not args.no_tune:
        for cs in singles:
            cs.autotune(None)
    for i, cs in enumerate(singles):
        cs.solve(Ds[i], bs[i], tol=tol, maxit=maxit, check=False)  # warm-up (graph capture)
    seq = []
    for _ in range(max(1, args.steps // 2)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, cs in enumerate(singles):
            cs.solve(Ds[i], bs[i], tol=tol, maxit=maxit, check=False)
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
    for cs in singles:
        cs.close()
    del singles
    print("bench: sequential FP64 solves done", file=sys.stderr, flush=True)
    t64 = float(np.mean([r[0] for r in rec]))
    t32 = float(np.mean([r[1] for r in rec]))
    ci64 = sum(n * inf["iters"] for n, inf in zip(n_all, rec[-1][2]))
    ci32 = sum(n * inf["iters"] for n, inf in zip(n_all, rec[-1][3]))
    # a batched launch takes the symmetric form only when every set does
    form_sym = all(i["symmetric"] for i in rec[-1][2])
    kw, sw = step_words(syncs, form_sym)
    # algorithmic bytes of the timed launches: kw words per cell of every set still iterating
    # (a launch past a set's last iteration does nothing for it)
    k1_bytes_total = sum(kw * 8 * n * inf["iters"] for n, inf in zip(n_all, rec[-1][2])) * len(rec)
    achieved = k1_bytes_total / (k1_ms * 1e-3) / 1e9
    err64 = max(float(torch.max(torch.abs(x - xs))) for x, xs in zip(x64, xss))
    err32 = max(float(torch.max(torch.abs(x - xs))) for x, xs in zip(x32, xss))
    kname = kern + ("_sym" if form_sym and syncs == 1 else "")
    res = {
        "workload": cfg["name"],
        "value": ci64 / t64,
        "ms_per_step": 1e3 * t_total / args.steps,
        "fp64": {"time_to_tol_ms": 1e3 * t64, "iters": [i["iters"] for i in rec[-1][2]],
                 "status": [i["status"] for i in rec[-1][2]],
                 "rel_res": [i["rel_res"] for i in rec[-1][2]], "cell_iters_per_s": ci64 / t64,
                 "model_GBps": ci64 * sw * 8 / t64 / 1e9, "max_abs_err_vs_xstar": err64,
                 "sequential_time_to_tol_ms": 1e3 * float(np.mean(seq)),
                 "batched_speedup_vs_sequential": float(np.mean(seq)) / t64},
        "fp32_refine": {"time_to_tol_ms": 1e3 * t32, "inner_iters": [i["iters"] for i in rec[-1][3]],
                        "status": [i["status"] for i in rec[-1][3]],
                        "outer": [i["outer"] for i in rec[-1][3]],
                        "sigma_restarts": [i["sigma_restarts"] for i in rec[-1][3]],
                        "rel_res": [i["rel_res"] for i in rec[-1][3]],
                        "cell_iters_per_s": ci32 / t32, "model_GBps": ci32 * sw * 4 / t32 / 1e9,
                        "max_abs_err_vs_xstar": err32,
                        "speedup_vs_fp64_batched": t64 / t32,
                        "speedup_vs_fp64_sequential": float(np.mean(seq)) / t32},
        "roofline": {"bound": "hbm", "kernel": kname + "_fp64 (batched launch)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(cfg["name"], kname),
                     "bytes_per_launch": k1_bytes_total / max(k1_cnt, 1),
                     "bytes": "%d words x 8 B per cell of every set still iterating, averaged over the timed "
                              "launches" % kw,
                     "words_per_cell": kw, "launches": k1_cnt, "mean_launch_ms": k1_ms / max(k1_cnt, 1)},
        "syncs_per_iteration": syncs,
        "symmetric_form": {"fp64": form_sym, "fp32_refine": all(i["symmetric"] for i in rec[-1][3])},
        "kernels_fp64_ms": {kern: {"launches": k1_cnt, "mean_ms": k1_ms / max(k1_cnt, 1)}},
        "layout": [c64.layout(i) for i in range(len(grids))],
        "layout_fp32_refine": [c32.layout(i) for i in range(len(grids))],
        "cells": sum(n_all),
    }
    sols = {"fp64": [x.cpu().numpy() for x in x64], "fp32_refine": [x.cpu().numpy() for x in x32]}
    del x64, x32
    c32.close()
    # what a plain kernel streaming the same words per cell reaches over the launch's cells
    att = stream_ceiling(sum(n_all), kw - 5)
    att["frac"] = achieved / att["value"]
    res["roofline"]["attainable"] = att
    if not args.no_mg:
        tmg, (xmg, img), mgp = time_mg(Context, grids,
                                       lambda cm: cm.solve_batched(Ds, bs, tol=tol, maxit=maxit, check=False),
                                       args.config, reps=2)
        res["fp64_multigrid"] = {"time_to_tol_ms": 1e3 * tmg, "iters": [i["iters"] for i in img],
                                 "status": [i["status"] for i in img],
                                 "rel_res": [i["rel_res"] for i in img],
                                 "max_abs_err_vs_xstar": max(float(torch.max(torch.abs(x - xs)))
                                                             for x, xs in zip(xmg, xss)),
                                 "speedup_vs_fp64_jacobi_batched": t64 / tmg, "params": mgp}
        del xmg
    if args.calibrate_copy:
        copy_calibration(res, dev)
    c64.close()
    return res, sols


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(args, gpu_sols):
    """The CPU oracle on the same systems: it solves every set to the workload's tolerance (the
    cpu_baseline rate is taken on set 0's solve, with the thread count it used, and a tenth of its
    iterations on one thread), and its solutions give each GPU result's error and the matching
    digits of Eq. (6) (min / 1st percentile / median over the cells)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2211_15605_amd import workloads as W

    o = O.default()
    cfg = W.CONFIGS[args.config]
    out, t0_rate = {}, None
    digits = {k: [] for k in gpu_sols}
    for i, g in enumerate(cfg["grids"]):
        s = W.make_set(args.config, i)
        b = o.apply(g.shape, s["diags"], s["x_star"])
        t0 = time.perf_counter()
        xo, info = o.bicgstab(g.shape, s["diags"], b, tol=cfg["tol"], maxit=cfg["maxit"])
        t = time.perf_counter() - t0
        print("bench: oracle solved set %d (%d iterations, %.1f s)" % (i, info["iters"], t), file=sys.stderr,
              flush=True)
        if i == 0:
            t0_rate = (g.n * info["iters"] / t, info["iters"], t)
        ref = np.max(np.abs(xo))
        for prec, xs in gpu_sols.items():
            d = O.matching_digits(xo, xs[i])
            digits[prec].append({"set": i, "max_abs_err_vs_oracle": float(np.max(np.abs(xs[i] - xo))),
                                 "max_rel_err_vs_oracle": float(np.max(np.abs(xs[i] - xo)) / ref),
                                 "digits_min": float(np.min(d)), "digits_p1": float(np.percentile(d, 1)),
                                 "digits_median": float(np.median(d)),
                                 "oracle_rel_res": float(o.rel_residual(g.shape, s["diags"], b, xs[i]))})
        if i == 0:
            # the same oracle on one thread, over a tenth of the iterations
            cores = o.get_threads()
            o.set_threads(1)
            try:
                t1s = time.perf_counter()
                _, info1 = o.bicgstab(g.shape, s["diags"], b, tol=cfg["tol"], maxit=max(4, info["iters"] // 10))
                t1 = time.perf_counter() - t1s
            finally:
                o.set_threads(cores)
            single = {"value": g.n * info1["iters"] / t1, "cores": 1,
                      "sample": "%d iterations, %.1f s" % (info1["iters"], t1)}
        del s, b, xo
    out["cpu_baseline"] = {
        "value": t0_rate[0], "unit": "cell-iters/s", "cores": o.get_threads(), "kind": "oracle",
        "cpu": cpu_model(), "host_cpus": os.cpu_count(),
        "sample": "the full FP64 BiCGSTAB solve of set 0 (%dx%dx%d, %d iterations to %g, %.1f s)" % (
            cfg["grids"][0].nx, cfg["grids"][0].ny, cfg["grids"][0].nz, t0_rate[1], cfg["tol"], t0_rate[2]),
        "single_thread": single}
    out["vs_oracle"] = {"equation_6": "digits = -log10(|x_oracle - x_gpu| / |x_oracle|) per cell", **digits}
    return out


def reduce_pmc(args):
    """Write the traffic record of one kernel from two rocprofv3 --pmc runs of the same bench
    command (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what the counter
    reads for the 1 GiB copies of --calibrate-copy.  The kernel's dispatches are those with its
    name and grid size; only dispatches that did work (above 1 % of the largest) count."""
    import csv
    import glob

    def rows(d, counter):
        f = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
        assert f, "no counter_collection.csv under %s" % d
        out = []
        for r in csv.DictReader(open(f[0])):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
        out.sort()
        return out

    res = {}
    for counter, d in (("FETCH_SIZE", args.reduce_pmc[0]), ("WRITE_SIZE", args.reduce_pmc[1])):
        rs = rows(d, counter)
        copies = [v for _, name, _, v in rs if "copy" in name.lower()
                  and v * 1024 > 0.25 * (1 << 30)]
        assert len(copies) >= 3, "no 1 GiB copy dispatches found (run with --calibrate-copy)"
        scale = (1 << 30) / (1024.0 * sorted(copies[-3:])[1])
        ks = [v for _, name, grid, v in rs if args.pmc_kernel in name and grid == args.pmc_grid]
        assert ks, "no dispatch of %s with grid %d" % (args.pmc_kernel, args.pmc_grid)
        work = [v for v in ks if v > 0.01 * max(ks)]
        full = [v for v in work if v > 0.9 * max(ks)]
        res[counter] = dict(scale=scale, dispatches=len(work), mean_kib=sum(work) / len(work),
                            full_dispatches=len(full), full_mean_kib=sum(full) / len(full))
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    per = 1024.0 * (f["mean_kib"] * f["scale"] + w["mean_kib"] * w["scale"])
    per_full = 1024.0 * (f["full_mean_kib"] * f["scale"] + w["full_mean_kib"] * w["scale"])
    alg_full = args.pmc_words * 8 * args.pmc_cells
    rec = {"kernel": args.pmc_kernel, "grid_work_items": args.pmc_grid, "workload": args.pmc_workload,
           "command_fetch": args.pmc_commands[0], "command_write": args.pmc_commands[1],
           "fetch_scale": f["scale"], "write_scale": w["scale"],
           "dispatches_with_work": f["dispatches"], "fetch_kib_mean": f["mean_kib"], "write_kib_mean": w["mean_kib"],
           "bytes_per_launch": per,
           "full_dispatches": f["full_dispatches"], "bytes_per_full_launch": per_full,
           "algorithmic_bytes_per_full_launch": alg_full, "traffic_over_algorithmic_full": per_full / alg_full}
    kname = [name for _, name, grid, _v in rows(args.reduce_pmc[0], "FETCH_SIZE")
             if args.pmc_kernel in name and grid == args.pmc_grid][0]
    rec["symbol"] = mangled_kernel_name(kname)
    rec["kernel_code_sha256"] = kernel_code_digest(rec["symbol"])
    json.dump(rec, open(args.pmc_out, "w"), indent=1)
    print(json.dumps(rec))


def summarize_trace(args):
    """Markdown summary of a rocprofv3 --kernel-trace run (kernel_trace.csv): per kernel and grid
    size, the launches that did work (a launch past its sets' convergence returns in < 10 us) and
    their mean and median durations."""
    import csv
    import glob
    import collections
    f = sorted(glob.glob(os.path.join(args.summarize_trace, "**", "*kernel_trace.csv"), recursive=True))
    assert f, "no kernel_trace.csv under %s" % args.summarize_trace
    g = collections.defaultdict(list)
    for r in csv.DictReader(open(f[0])):
        g[(r["Kernel_Name"], int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]))].append(
            int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    lines = ["| kernel | blocks per launch | launches | with work (> 10 us) | mean us (with work) | median us (with work) "
             "| total ms |", "|---|---|---|---|---|---|---|"]
    tot = sum(sum(v) for v in g.values())
    for (name, blocks), v in sorted(g.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) < args.trace_min_share * tot:
            continue
        w = [x for x in v if x > 10000]
        short = name[:name.rindex("(")] if name.endswith(")") and "(" in name else name
        if args.trace_kernels and not any(k in short for k in args.trace_kernels.split(",")):
            continue
        med = sorted(w)[len(w) // 2] / 1e3 if w else 0.0
        lines.append("| `%s` | %d | %d | %d | %.1f | %.1f | %.2f |" % (short, blocks, len(v), len(w),
                                                                   (sum(w) / len(w) / 1e3) if w else 0.0, med,
                                                                   sum(v) / 1e6))
    print("\n".join(lines))


def trace_gaps(args):
    """Launch boundaries of one kernel in a kernel trace: its launches of `--pmc-grid` work-items that
    did work (> 100 us), grouped into solves (a pause of more than 3 ms starts a new one); per solve,
    the launches' summed durations against their span, and the gaps between launches that follow
    each other directly in the stream and between those with other work (a host readback, another
    kernel) between them."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(args.trace_gaps, "**", "*kernel_trace.csv"), recursive=True))
    assert f, "no kernel_trace.csv under %s" % args.trace_gaps
    rows = sorted(csv.DictReader(open(f[0])), key=lambda r: int(r["Start_Timestamp"]))
    t = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    sel = [i for i, r in enumerate(rows) if args.pmc_kernel in r["Kernel_Name"]
           and (not args.pmc_grid or int(r["Grid_Size_X"]) == args.pmc_grid) and t[i][1] - t[i][0] > 100000]
    groups = [[sel[0]]] if sel else []
    for a, b in zip(sel, sel[1:]):
        if t[b][0] - t[a][1] > 3000000:
            groups.append([])
        groups[-1].append(b)
    print("| solve | launches | summed ms | span ms | idle share | back-to-back gaps: n, mean us | other gaps: n, total us |")
    print("|---|---|---|---|---|---|---|")
    for n, g in enumerate(groups):
        busy = sum(t[i][1] - t[i][0] for i in g)
        span = t[g[-1]][1] - t[g[0]][0]
        adj = [t[b][0] - t[a][1] for a, b in zip(g, g[1:]) if b == a + 1]
        oth = [t[b][0] - t[a][1] for a, b in zip(g, g[1:]) if b != a + 1]
        print("| %d | %d | %.2f | %.2f | %.2f %% | %d, %.2f | %d, %.1f |" % (
            n, len(g), busy / 1e6, span / 1e6, 100.0 * (span - busy) / span, len(adj),
            (sum(adj) / len(adj) / 1e3) if adj else 0.0, len(oth), sum(oth) / 1e3))


def simple_phases(args):
    """Per SIMPLE iteration of a kernel trace of the SIMPLE section (from one momentum formation to the
    next): the phases' means in us (momentum formation, momentum solve phase, p' formation, p' solve
    phase, correction, the whole iteration, everything but the p' solve), grouped by the p' solver
    (multigrid or Jacobi) and the number of momentum steps that did work, and the kernels of the
    momentum solve phase summed per iteration."""
    import csv
    import glob
    import collections
    f = sorted(glob.glob(os.path.join(args.simple_phases, "**", "*kernel_trace.csv"), recursive=True))
    assert f, "no kernel_trace.csv under %s" % args.simple_phases
    rows = sorted(csv.DictReader(open(f[0])), key=lambda r: int(r["Start_Timestamp"]))
    t0 = [int(r["Start_Timestamp"]) / 1e3 for r in rows]
    t1 = [int(r["End_Timestamp"]) / 1e3 for r in rows]
    name = [r["Kernel_Name"] for r in rows]
    fm = [i for i, n in enumerate(name) if "form_momentum_kernel" in n]
    groups = collections.defaultdict(list)
    kern = collections.defaultdict(lambda: collections.defaultdict(float))
    for a, b in zip(fm, fm[1:]):
        try:
            ip = next(i for i in range(a, b) if "form_pressure_kernel" in name[i])
            ic = next(i for i in range(ip, b) if "correct_kernel" in name[i])
        except StopIteration:
            continue
        mg = any("mg_" in name[i] for i in range(ip, ic))
        steps = sum(1 for i in range(a + 1, ip) if "fused_kernel" in name[i] and t1[i] - t0[i] > 10)
        key = ("multigrid" if mg else "Jacobi", steps)
        ph = (t1[a] - t0[a], t0[ip] - t1[a], t1[ip] - t0[ip], t0[ic] - t1[ip], t1[ic] - t0[ic], t0[b] - t0[a])
        groups[key].append(ph)
        for i in range(a + 1, ip):
            n = name[i]
            kern[key][n[:n.rindex("(")] if n.endswith(")") and "(" in n else n] += t1[i] - t0[i]
    print("| p' solver, momentum steps | iterations | momentum formation | momentum solve phase | p' formation | "
          "p' solve phase | correction | iteration | everything but the p' solve |")
    print("|---|---|---|---|---|---|---|---|---|")
    for key in sorted(groups):
        v = groups[key]
        m = [sum(x[j] for x in v) / len(v) for j in range(6)]
        print("| %s, %d | %d | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f |" % (
            key[0], key[1], len(v), m[0], m[1], m[2], m[3], m[4], m[5], m[5] - m[3]))
    for key in sorted(groups):
        n = len(groups[key])
        print("\n%s p' solves, %d momentum steps: kernels of the momentum solve phase, us per iteration" % key)
        for k, t in sorted(kern[key].items(), key=lambda kv: -kv[1]):
            if t / n >= 1.0:
                print("  `%s`: %.1f" % (k, t / n))


def summarize_counters(args):
    """Mean of every counter of a rocprofv3 --pmc run (counter_collection.csv) per kernel, over its
    dispatches of `--pmc-grid` work-items (all, if 0) that ran longer than 500 us."""
    import csv
    import glob
    import collections
    f = sorted(glob.glob(os.path.join(args.summarize_counters, "**", "*counter_collection.csv"), recursive=True))
    assert f, "no counter_collection.csv under %s" % args.summarize_counters
    disp = collections.defaultdict(dict)
    for r in csv.DictReader(open(f[0])):
        name = r["Kernel_Name"]
        short = name[:name.rindex("(")] if name.endswith(")") and "(" in name else name
        if args.trace_kernels and not any(k in short for k in args.trace_kernels.split(",")):
            continue
        if args.pmc_grid and int(r["Grid_Size"]) != args.pmc_grid:
            continue
        if int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) <= 500000:
            continue
        disp[(short, r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
    per = collections.defaultdict(list)
    for (short, _), d in disp.items():
        per[short].append(d)
    for short, ds in sorted(per.items()):
        names = sorted(ds[0])
        print("`%s`: %d dispatches; " % (short, len(ds)) + ", ".join(
            "%s %.4g" % (c, sum(d.get(c, 0.0) for d in ds) / len(ds)) for c in names))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes (no autotuning)")
    ap.add_argument("--no-mg", action="store_true", help="skip the multigrid-preconditioned solves")
    ap.add_argument("--no-simple", action="store_true",
                    help="skip the sections beside the workload (SIMPLE iteration, 16^3 latency, small batches, "
                         "adjoint, the pressure-like system)")
    ap.add_argument("--only-simple", action="store_true",
                    help="run only the SIMPLE-iteration section and print it as the JSON line (for profiling)")
    ap.add_argument("--only-latency", action="store_true",
                    help="run only the 16^3 latency section and print it as the JSON line (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB three times (reference for HBM byte counters)")
    ap.add_argument("--reduce-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write a traffic record from two rocprofv3 --pmc runs (no GPU needed)")
    ap.add_argument("--pmc-kernel", default="fused_kernel<double, 2, 1, 0, 512>")
    ap.add_argument("--pmc-grid", type=int, default=0, help="work-items of the kernel's launch")
    ap.add_argument("--pmc-words", type=int, default=18)
    ap.add_argument("--pmc-cells", type=int, default=0)
    ap.add_argument("--pmc-workload", default="")
    ap.add_argument("--pmc-out", default="")
    ap.add_argument("--pmc-commands", nargs=2, default=["", ""])
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR", help="print a markdown summary of a kernel trace")
    ap.add_argument("--trace-min-share", type=float, default=0.01)
    ap.add_argument("--trace-kernels", default="", help="comma-separated name parts: only those kernels")
    ap.add_argument("--trace-gaps", metavar="TRACE_DIR",
                    help="launch boundaries of --pmc-kernel (launches of --pmc-grid work-items) per solve")
    ap.add_argument("--simple-phases", metavar="TRACE_DIR",
                    help="per-iteration phases of a kernel trace of the SIMPLE section")
    ap.add_argument("--summarize-counters", metavar="PMC_DIR",
                    help="per-kernel means of every counter of a --pmc run (dispatches of --pmc-grid work-items)")
    args = ap.parse_args()
    if args.trace_gaps:
        trace_gaps(args)
        return
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.simple_phases:
        simple_phases(args)
        return
    if args.reduce_pmc:
        reduce_pmc(args)
        return
    if args.summarize_trace:
        summarize_trace(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the equation sets of a time step are solved on a single "
              "device here; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2211_15605_amd import workloads as W

    if args.only_simple:
        out = {"simple_bed": time_simple()}
        if args.calibrate_copy:
            import torch
            copy_calibration(out, torch.device("cuda", 0))
        print(json.dumps(out))
        return
    if args.only_latency:
        print(json.dumps({"latency_cd16": time_latency()}))
        return
    cfg = W.CONFIGS[args.config]
    batched = len(cfg["grids"]) > 1
    r, sols = gpu_leg_batched(args) if batched else gpu_leg(args, args.config, with_mg=not args.no_mg)
    sections = {}
    if not args.no_simple:
        if args.config != 1:
            c1, _ = gpu_leg(args, 1, steps=3, warmup=1, with_mg=not args.no_mg)
            sections["pressure_like_128x256x128"] = c1
        sections["simple_bed"] = time_simple()
        sections["latency_cd16"] = time_latency()
        sections["batching_small"] = time_batching()
        sections["adjoint64"] = time_adjoint()
        print("bench: sections done", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu_baseline else cpu_leg(args, sols)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "cell-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %s%s 7-point system%s on %s cells, b = A x*, x0 = 0, tol %g; step = "
                               "FP64 solve + FP32-inner/FP64-refinement solve%s" % (
                                   cfg["name"], "%d " % len(cfg["grids"]) if batched else "",
                                   "symmetric near-singular" if cfg["recipe"] == "sym" else "convection-diffusion",
                                   "s" if batched else "", " + ".join("%dx%dx%d" % gg.shape for gg in cfg["grids"]),
                                   cfg["tol"], " (all sets in one call)" if batched else ""),
                   "cells": r["cells"], "layout": r["layout"], "layout_fp32_refine": r["layout_fp32_refine"]},
        "roofline": r["roofline"],
        "cpu_baseline": cpu["cpu_baseline"] if cpu else None,
        "vs_oracle": cpu["vs_oracle"] if cpu else None,
        "fp64": r["fp64"],
        "fp32_refine": r["fp32_refine"],
        "fp64_multigrid": r.get("fp64_multigrid"),
        "kernels_fp64_ms": r["kernels_fp64_ms"],
        "symmetric_form": r.get("symmetric_form"),
        "copy_calibration_bytes": r.get("copy_calibration_bytes"),
    }
    line.update(sections)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
