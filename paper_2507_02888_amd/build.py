"""Compile libewald.so in-tree: the host set-up with g++, the kernels with
hipcc for gfx950, linked by hipcc.  Always recompiles."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libewald.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are switched off for every HIP translation unit
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    host_o = os.path.join(BUILD, "ewald_host.o")
    dev_o = os.path.join(BUILD, "ewald_device.o")
    cxx = shutil.which("g++") or "g++"
    steps = [
        [cxx, *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, "ewald_host.cpp"), "-o", host_o],
        [HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, "ewald_device.hip"), "-o", dev_o],
        [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", host_o, dev_o],
    ]
    for cmd in steps:
        r = _run(cmd)
        if verbose and (r.stdout or r.stderr):
            print(r.stdout + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
