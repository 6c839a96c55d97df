"""Builds the package's native libraries in-tree.

* ``_lib/libsearchsorted.so``: the HIP library behind ``include/searchsorted.h``
  (hipcc, gfx950 only).
* ``_lib/libssinputs.so``: the host-only seeded input generators (gcc).
* ``build_sanitized(dir)``: both again with the host code instrumented by
  AddressSanitizer and UndefinedBehaviorSanitizer (clang), for the CPU suite.

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


def build_hip(verbose: bool = False, jobs: int = 4, libdir: str = LIBDIR,
              extra: tuple = ()) -> str:
    os.makedirs(libdir, exist_ok=True)
    objdir = os.path.join(libdir, "obj")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    objs, procs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *hip_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
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
    out = os.path.join(libdir, "libsearchsorted.so")
    tmp = out + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


# The device-checked variant: every search routine's LDS index and every
# full tile's target range is tested in the kernels, violations are counted
# (ss_debug_violations) and clamped instead of faulting.  Slower; for tests.
CHECKED_LIBDIR = os.path.join(LIBDIR, "checked")


def build_checked(verbose: bool = False) -> str:
    return build_hip(verbose, libdir=CHECKED_LIBDIR, extra=("-DSS_DEVICE_CHECKS=1",))


CLANG = "/opt/rocm/llvm/bin/clang"
# host-side AddressSanitizer + UndefinedBehaviorSanitizer (device code is not
# instrumented; on a hipcc line each flag goes to the host pass only)
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


def asan_runtime() -> str:
    """The sanitizer runtime the instrumented libraries need preloaded."""
    return subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                   text=True).strip()


def build_sanitized(outdir: str, verbose: bool = False) -> dict:
    """Builds the library (host code instrumented) and the input generators
    with AddressSanitizer and UndefinedBehaviorSanitizer into outdir; returns
    the environment that makes the package load them (SS_LIBRARY,
    SS_INPUTS_LIB) plus the preload of the sanitizer runtime."""
    os.makedirs(outdir, exist_ok=True)
    inputs = os.path.join(outdir, "libssinputs.so")
    _run([CLANG, "-O1", *SANITIZE, "-std=c11", "-D_GNU_SOURCE", "-shared", "-fPIC", "-pthread",
          "-o", inputs, os.path.join(CSRC, "inputs.c"), "-lm"], verbose)
    host_san = []
    for f in SANITIZE:
        host_san += ["-Xarch_host", f]
    hipcc = _hipcc()
    objs, procs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *hip_flags(), *host_san, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    for p, s in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    lib = os.path.join(outdir, "libsearchsorted.so")
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host",
          "-fsanitize=address,undefined", "-o", lib, *objs], verbose)
    return {"SS_LIBRARY": lib, "SS_INPUTS_LIB": inputs, "LD_PRELOAD": asan_runtime(),
            "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def build_all(verbose: bool = False) -> None:
    build_inputs(verbose)
    build_hip(verbose)
    build_checked(verbose)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
