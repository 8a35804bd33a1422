"""The ABI from C: include/ewald.h compiles as C99 and a C program links
against libewald.so (CPU); the program runs on the GPU and reproduces the
simple-cubic Wigner-lattice Madelung energy and zero move deltas for a lone
charge (tests/c_api/madelung_sc.c)."""
import os
import subprocess

import pytest

from tests import c_api


def test_c_example_compiles_and_links(tmp_path):
    if not os.path.exists(os.path.join(c_api.ROOT, "paper_2507_02888_amd", "libewald.so")):
        pytest.skip("libewald.so not built")
    exe = c_api.build(str(tmp_path / "madelung_sc"))
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_example_runs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = c_api.EXE if os.path.exists(c_api.EXE) else c_api.build(c_api.EXE)
    print(f"[c example] {exe}", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert ": ok" in r.stdout
