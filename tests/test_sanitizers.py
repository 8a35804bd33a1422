"""The FP64 oracle and the library's host set-up built with the address and
undefined-behaviour sanitizers (g++ on the CPU, no device code) and run by a
small driver over cells of every shape the workloads use: any out-of-bounds
access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2507_02888_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc/g++")
def test_oracle_and_host_setup_under_sanitizers(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    objs = []
    oracle_o = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", *san, "-fopenmp", "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", oracle_o],
                   check=True)
    objs.append(oracle_o)
    for src in (os.path.join(CSRC, "ewald_host.cpp"), os.path.join(HERE, "device_stubs.cpp"),
                os.path.join(HERE, "driver.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", *san, "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src,
                        "-o", o], check=True)
        objs.append(o)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", *san, "-fopenmp", *objs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
