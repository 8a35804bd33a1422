"""The C caller example of the ABI (madelung_sc.c): compiled with the C
compiler against include/ewald.h and libewald.so, run by the GPU tests."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "madelung_sc.c")
EXE = os.path.join(HERE, "madelung_sc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out: str = EXE) -> str:
    cc = shutil.which("gcc") or "gcc"
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", out,
           "-L", os.path.join(ROOT, "paper_2507_02888_amd"), "-lewald", "-L", os.path.join(ROCM, "lib"),
           "-lamdhip64", "-lm", "-Wl,-rpath," + os.path.join(ROOT, "paper_2507_02888_amd"),
           "-Wl,-rpath,$ORIGIN/../../paper_2507_02888_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C example build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return out
