"""Compile libewald.so in-tree: the host set-up with g++, the kernels with
hipcc for gfx950 (one translation unit per group of fused-kernel
instantiations, compiled in parallel), linked by hipcc.  Always recompiles."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libewald.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are switched off for every HIP translation unit
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wextra", "-Werror",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Werror"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 4
    return max(1, min(n, int(os.environ.get("MAX_JOBS", "16"))))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    host_o = os.path.join(BUILD, "ewald_host.o")
    cxx = shutil.which("g++") or "g++"
    compiles = [[cxx, *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, "ewald_host.cpp"), "-o", host_o]]
    objs = [host_o]
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
        compiles.append([HIPCC, *HIP_FLAGS, *inc, "-c", src, "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(_run, compiles))
    r = _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs])
    if verbose:
        for x in results + [r]:
            if x.stdout or x.stderr:
                print(x.stdout + x.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
