"""Build the HIP library libeqsolve.so in-tree for gfx950.

    python -m paper_2211_15605_amd.build

Compiles every HIP source of the package with hipcc (no JIT, no torch
extension machinery): the result is a plain shared library whose C ABI is
declared in include/eqsolve.h.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libeqsolve.so")
SOURCES = ["eqs_kernels.hip", "eqs_host.cpp", "eqs_noalloc.hip", "eqs_probe.hip", "simple_kernels.hip", "simple_host.cpp"]
ARCH = os.environ.get("EQS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def flags(shared: bool = True):
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC"] + (["-shared"] if shared else []) + [
        "-Wall", "-Wno-unused-function",
        # no packed-FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel, each with a fixed compilation-unit id, so
    the same sources always give the same device code object), then link the library."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        stem = os.path.splitext(src)[0]
        obj = os.path.join(objdir, stem + ".o")
        cmd = [hipcc()] + flags(shared=False) + ["-cuid=" + stem, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    errors = []
    for src, p in procs:
        out = p.communicate()[0]
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and "warning generated" not in l)
        if p.returncode != 0:
            errors.append("%s:\n%s" % (src, out))
        elif verbose and out.strip():
            print(out)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
