"""Builds libazint.so in the package directory for gfx950.

Host plan builder: g++ without floating-point contraction (its integer
results must be reproducible); the device plan builder likewise.  Kernels
and the C ABI: hipcc for gfx950 with packed-fp32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libazint.so")
ARCH = os.environ.get("AZINT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
HIP_SOURCES = ("kernels.hip", "azint_api.hip", "plan_device.hip", "fused.hip")
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
              "-Wall", "-Wextra"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    host = os.path.join(BUILD, "plan_builder.o")
    steps = [(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "plan_builder.cpp"), "-o", host],
              host)]
    for name in HIP_SOURCES:
        obj = os.path.join(BUILD, name.replace(".hip", ".o"))
        # the device plan builder and the matrix-free kernel decide bin
        # indices: no contraction, as on the host
        extra = (["-ffp-contract=off", "-fno-fast-math"]
                 if name in ("plan_device.hip", "fused.hip") else [])
        steps.append(([hipcc, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, name), "-o", obj],
                      obj))
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(steps), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda st: _run(st[0], verbose), steps))
    objs = [obj for _, obj in steps]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
