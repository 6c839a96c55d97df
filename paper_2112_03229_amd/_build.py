"""Builds the package's native libraries in-tree.

* ``_lib/libsearchsorted.so``: the HIP library behind ``include/searchsorted.h``
  (hipcc, gfx950 only).
* ``_lib/libssinputs.so``: the host-only seeded input generators (gcc).

Every call recompiles.  Flags: -O3; no fast-math (the search is exact IEEE
comparison work); packed FP32 instructions disabled for device code.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
REPO = os.path.dirname(HERE)
ARCH = os.environ.get("SS_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["ss_runtime.hip", "ss_single.hip", "ss_plan.hip", "ss_tuner.hip", "ss_noalloc.hip",
               "ss_learned.hip"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_inputs(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    out = os.path.join(LIBDIR, "libssinputs.so")
    tmp = out + ".tmp"
    _run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-shared", "-fPIC", "-pthread", "-o", tmp,
          os.path.join(CSRC, "inputs.c"), "-lm"], verbose)
    os.replace(tmp, out)
    return out


def hip_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
        "-Wno-unused-result",
        # packed FP32 ops are kept out of every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fno-gpu-rdc", "-fvisibility=hidden",
        f"-I{os.path.join(REPO, 'include')}",
    ]


def build_hip(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    objs, procs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *hip_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s}")
    for p, s in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    out = os.path.join(LIBDIR, "libsearchsorted.so")
    tmp = out + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = False) -> None:
    build_inputs(verbose)
    build_hip(verbose)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
