"""Host-side logic of bench.py that needs no GPU: the oracle baseline and its
in-run parity check, the thread count, and the one-GPU restriction."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2507_02888_amd import workloads as wl  # noqa: E402


def test_cpu_baseline_and_parity_bounds(oracle_lib):
    cfg = wl.config(1)
    cpu = bench.cpu_baseline(cfg, 1, 6, 2)
    assert cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["kind"] == "oracle"
    ref = cpu["ref"]
    exact = dict(energy=ref["e0"][:1, 4].copy(), jastrow=ref["j0"][:1].copy(), delta=ref["delta"][:, :1].copy(),
                 djas=ref["djas"][:, :1].copy())
    sysm = cfg.systems[0]
    assert bench.parity("fp64", exact, ref, sysm)["ok"]
    assert bench.parity("mixed", exact, ref, sysm)["ok"]
    off = dict(exact, delta=exact["delta"] + 1e-8)
    p64, pmx = bench.parity("fp64", off, ref, sysm), bench.parity("mixed", off, ref, sysm)
    assert not p64["ok"] and pmx["ok"]
    assert abs(p64["max_abs_delta_err"] - 1e-8) < 1e-12
    far = dict(exact, energy=exact["energy"] * (1 + 1e-5))
    assert not bench.parity("mixed", far, ref, sysm)["ok"]
    assert np.isfinite(p64["max_rel_energy_err"])


def test_host_threads_and_model():
    assert bench.host_threads() >= 1
    assert isinstance(bench.cpu_model(), str)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
