"""Build the HIP shared library libkatsevich.so in-tree (gfx950).

Usage: ``python -m paper_2201_02309_amd.build`` (or ``__graft_entry__.build()``).
Every object is recompiled on each call.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "katsevich")
LIB = os.path.join(PKG, "libkatsevich.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
# device code: no packed-FP32 instructions; hardware float atomics
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
SOURCES = [("plan.cpp", False), ("capi.cpp", False), ("filter.hip", True), ("bp.hip", True),
           ("bp_adjoint.hip", True), ("plan_gpu.hip", True), ("data.hip", True),
           ("hilbert_mfma.hip", True)]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src, device in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if device:
            cmd = [HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE
        else:   # host-only C++ (HIP runtime API calls, no device code)
            cmd = [HIPCC, "-x", "c++", "-c", os.path.join(CSRC, src), "-o", obj, "-pthread",
                   "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + COMMON
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        logs = list(ex.map(lambda j: _run(j[0]), jobs))
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-o", tmp] + [o for _, o in jobs] + [f"--offload-arch={ARCH}",
                                                                    "-pthread", "-fPIC"]
    logs.append(_run(link))
    os.replace(tmp, LIB)
    if verbose:
        for l in logs:
            if l.strip():
                sys.stderr.write(l)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
