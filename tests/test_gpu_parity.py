"""GPU parity of libewald against the FP64 oracle, called through the C ABI.

Tolerances (relative to E_ref = max(|E_oracle|, (alpha/sqrt(pi)) sum q^2)):
  FP64 form   energies and move deltas within 1e-10 E_ref;
  FP32-mixed  energies within 1e-6 E_ref, each move delta within 1e-5 Ha.
"""
import copy
import dataclasses
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2507_02888_amd import ewald as ew
from paper_2507_02888_amd import workloads as wl

pytestmark = pytest.mark.gpu

FP64, MIXED = ew.EWALD_FP64, ew.EWALD_FP32_MIXED


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ew.load()


def djas_bound(case, w):
    """FP32-mixed bound on a Jastrow delta (see bench.mixed_djastrow_bound)."""
    import bench
    return bench.mixed_djastrow_bound(case.system(w), case.ja, case.systems[int(case.b.walker_sys[w])].info["n_g"])


def e_scale(system):
    q = np.concatenate([system.mobile_q, system.fixed_q])
    return system.alpha / math.sqrt(math.pi) * float(np.sum(q * q))


class Case:
    """Seeded inputs of a workload subset, uploaded, with a library batch."""

    def __init__(self, cfg_id, walkers, moves, precision, walker_start=0, refresh_every=None, jastrow=True,
                 u_term=False, cfg=None):
        self.cfg = wl.config(cfg_id) if cfg is None else cfg
        if u_term:  # the same workload with the Jastrow two-body polynomial term
            self.cfg.systems = [wl.with_u_term(s, cfg_id) for s in self.cfg.systems]
        self.b = wl.make_batch(self.cfg, walkers=walkers, moves=moves, walker_start=walker_start)
        K = self.cfg.refresh_every if refresh_every is None else refresh_every
        self.ja = self.b.jastrow_a if jastrow else None
        if self.ja is None and jastrow and cfg_id != 5:
            self.ja = np.random.default_rng([7, cfg_id]).uniform(-0.01, 0.01, 64)
        self.systems = [ew.System(s, precision=precision, refresh_every=K if precision == MIXED else 0,
                                  jastrow_a=self.ja) for s in self.cfg.systems]
        self.batch = ew.Batch(self.systems, self.b.walker_sys)
        W, S, d = self.b.walkers, self.b.steps, self.cfg.systems[0].dim
        self.W, self.S, self.dim = W, S, d
        dev = "cuda"
        self.pos = torch.tensor(self.b.pos, dtype=torch.float64, device=dev)
        self.k = torch.tensor(self.b.k, dtype=torch.int32, device=dev)
        self.new_pos = torch.tensor(self.b.new_pos, dtype=torch.float64, device=dev)
        self.accept = torch.tensor(self.b.accept, dtype=torch.uint8, device=dev)
        self.energy = torch.zeros(W, dtype=torch.float64, device=dev)
        self.jastrow = torch.zeros(W, dtype=torch.float64, device=dev)

    def system(self, w):
        return self.cfg.systems[int(self.b.walker_sys[w])]

    def run_energy(self):
        self.batch.energy(self.pos, self.energy, self.jastrow)
        torch.cuda.synchronize()
        return self.energy.cpu().numpy().copy(), self.jastrow.cpu().numpy().copy()

    def per_step(self):
        d = torch.zeros((self.S, self.W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        for m in range(self.S):
            self.batch.move_delta(self.k[m], self.new_pos[m], d[m], dj[m])
            self.batch.accept(self.accept[m])
        torch.cuda.synchronize()
        return d.cpu().numpy(), dj.cpu().numpy()

    def stepped(self):
        """The same sequence through the step call: each move's accept folded
        into the next move's delta, the last one through the accept call."""
        d = torch.zeros((self.S, self.W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        for m in range(self.S):
            self.batch.step(self.accept[m - 1] if m else None, self.k[m], self.new_pos[m], d[m], dj[m])
        self.batch.accept(self.accept[self.S - 1])
        torch.cuda.synchronize()
        return d.cpu().numpy(), dj.cpu().numpy()

    def fused(self, steps=None):
        S = self.S if steps is None else steps
        d = torch.zeros((S, self.W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        self.batch.run_moves(self.k[:S].contiguous(), self.new_pos[:S].contiguous(), self.accept[:S].contiguous(), d, dj)
        torch.cuda.synchronize()
        return d.cpu().numpy(), dj.cpu().numpy()

    def oracle(self, oracle_lib, w, steps=None):
        S = self.S if steps is None else steps
        return oracle_lib.run(self.system(w), self.b.walker_pos(w), self.b.k[:S, w], self.b.new_pos[:S, w],
                              self.b.accept[:S, w], jastrow_a=self.ja)

    def final_cartesian(self):
        """Positions currently in the state, as a Cartesian packed array."""
        out = np.zeros_like(self.b.pos)
        for w in range(self.W):
            s = self.batch.walker_positions(w)
            lat = self.system(w).lattice[: self.dim, : self.dim]
            out[self.b.pos_offsets[w]: self.b.pos_offsets[w + 1]] = s @ lat
        return out


SUBSETS = {1: (1, 54, 0), 2: (3, 24, 0), 3: (3, 24, 0), 4: (6, 12, 0), 5: (2, 6, 0)}


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 4, 5])
def test_energy_parity(oracle_lib, cfg_id, precision):
    W, S, w0 = SUBSETS[cfg_id]
    say(f"[energy] cfg={cfg_id} precision={precision} walkers={W}")
    c = Case(cfg_id, W, 0, precision, walker_start=w0)
    e, j = c.run_energy()
    tol = 1e-10 if precision == FP64 else 1e-6
    for w in range(W):
        sysw = c.system(w)
        ref = oracle_lib.energy(sysw, *oracle_lib.particles(sysw, c.b.walker_pos(w)), jastrow_a=c.ja)
        scale = max(abs(ref["total"]), e_scale(sysw))
        assert abs(e[w] - ref["total"]) <= tol * scale, (w, e[w], ref["total"])
        assert abs(j[w] - ref["jastrow"]) <= tol * max(1.0, abs(ref["jastrow"]))


@pytest.mark.parametrize("cfg_id", [2, 3, 4])
def test_rho_elementwise(oracle_lib, cfg_id):
    say(f"[rho] cfg={cfg_id}")
    c = Case(cfg_id, 2, 0, FP64)
    c.run_energy()
    for w in range(2):
        sysw = c.system(w)
        t = c.systems[int(c.b.walker_sys[w])].tables()
        valid = t["shell"] >= 0
        d = sysw.dim
        B = 2 * math.pi * np.linalg.inv(sysw.lattice[:d, :d]).T
        g = np.zeros((int(valid.sum()), 3))
        g[:, :d] = t["n"][valid][:, :d] @ B
        ref = oracle_lib.rho_at(sysw, *oracle_lib.particles(sysw, c.b.walker_pos(w)), g)
        got = c.batch.walker_rho(w)[valid]
        assert np.max(np.abs(got - ref)) <= 1e-9 * math.sqrt(sysw.n_mobile + sysw.n_fixed)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 4, 5])
def test_moves_per_step(oracle_lib, cfg_id, precision):
    W, S, w0 = SUBSETS[cfg_id]
    say(f"[moves per-step] cfg={cfg_id} precision={precision} walkers={W} steps={S}")
    c = Case(cfg_id, W, S, precision, walker_start=w0)
    e0, j0 = c.run_energy()
    d, dj = c.per_step()
    for w in range(W):
        sysw = c.system(w)
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(sysw))
        if precision == FP64:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"]))
        else:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w)
    # telescoping: E0 + sum of accepted deltas equals a fresh energy of the final state
    acc = c.b.accept.astype(bool)
    final = torch.tensor(c.final_cartesian(), dtype=torch.float64, device="cuda")
    e_tel = e0 + np.sum(np.where(acc, d, 0.0), axis=0)
    c2 = Case(cfg_id, W, 0, precision, walker_start=w0)
    c2.pos = final
    e_fin, _ = c2.run_energy()
    for w in range(W):
        scale = max(abs(e_fin[w]), e_scale(c.system(w)))
        tol = 1e-10 * scale if precision == FP64 else 1e-6 * scale + 1e-5 * S
        assert abs(e_tel[w] - e_fin[w]) <= tol


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [2, 3])
def test_degree32_pair_polynomial(oracle_lib, cfg_id, precision):
    """alpha r_c = 3.5 (above 2.83): the pair potential's fit of erf(sqrt y)/sqrt y
    takes the degree-32 FP64 (degree-22 FP32) polynomial in the energy,
    per-step and fused kernels; energies and every delta and Jastrow delta of
    both paths against the oracle (the mixed form at K = 3)."""
    cfg = wl.config(cfg_id)
    s0 = cfg.systems[0]
    L = s0.length
    cfg.systems = [dataclasses.replace(s0, alpha=7.0 / L, r_cut=0.5 * L, g_cut=s0.g_cut * 1.4)]
    assert cfg.systems[0].alpha * cfg.systems[0].r_cut > 2.83
    W, S = 2, 16
    say(f"[degree-32 polynomial] cfg={cfg_id} precision={precision}")
    for path in ("per-step", "fused"):
        c = Case(cfg_id, W, S, precision, refresh_every=3, cfg=copy.deepcopy(cfg))
        e0, _ = c.run_energy()
        d, dj = c.per_step() if path == "per-step" else c.fused()
        for w in range(W):
            sysw = c.system(w)
            r = c.oracle(oracle_lib, w)
            scale = max(abs(r["energy0"]), e_scale(sysw))
            if precision == FP64:
                assert abs(e0[w] - r["energy0"]) <= 1e-10 * scale, path
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"])), path
            else:
                assert abs(e0[w] - r["energy0"]) <= 1e-6 * scale, path
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w), path


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [2, 3, 4, 5])
def test_fused_matches_per_step(cfg_id, precision):
    W, S, w0 = SUBSETS[cfg_id]
    say(f"[fused vs per-step] cfg={cfg_id} precision={precision}")
    a = Case(cfg_id, W, S, precision, walker_start=w0, refresh_every=5)
    a.run_energy()
    d1, j1 = a.per_step()
    b = Case(cfg_id, W, S, precision, walker_start=w0, refresh_every=5)
    b.run_energy()
    d2, j2 = b.fused()
    tol = 1e-12 if precision == FP64 else 1e-7
    scale = max(abs(x) for x in a.energy.cpu().numpy())
    assert np.max(np.abs(d1 - d2)) <= tol * max(1.0, scale)
    assert np.max(np.abs(j1 - j2)) <= tol * max(1.0, scale)
    for w in range(W):
        ha, hb = a.batch.walker_header(w), b.batch.walker_header(w)
        assert ha["n_accepts"] == hb["n_accepts"] == int(a.b.accept[:, w].sum())
        assert np.array_equal(a.batch.walker_positions(w), b.batch.walker_positions(w))
        ra, rb = a.batch.walker_rho(w), b.batch.walker_rho(w)
        assert np.max(np.abs(ra - rb)) <= (1e-12 if precision == FP64 else 1e-9) * math.sqrt(a.system(w).n_mobile)


def test_mixed_refresh(oracle_lib):
    """FP32-mixed: rho is rebuilt in FP64 every K accepted moves; the running
    rho stays within the drift bound and matches a fresh FP64 rho."""
    K = 4
    say("[refresh] cfg=2 K=4")
    c = Case(2, 2, 40, MIXED, refresh_every=K)
    c.run_energy()
    c.per_step()
    f = Case(2, 2, 40, MIXED, refresh_every=K)
    f.run_energy()
    f.fused()
    for case in (c, f):
        for w in range(2):
            h = case.batch.walker_header(w)
            acc = int(c.b.accept[:, w].sum())
            assert h["n_accepts"] == acc
            assert h["n_refresh"] == acc // K
            assert 0.0 < h["drift_max"] < 1e-5
            # running rho vs an FP64 rebuild of the final positions
            sysw = case.system(w)
            t = case.systems[0].tables()
            valid = t["shell"] >= 0
            B = 2 * math.pi * np.linalg.inv(sysw.lattice).T
            g = t["n"][valid] @ B
            pos = case.batch.walker_positions(w) @ sysw.lattice
            ref = oracle_lib.rho_at(sysw, pos, sysw.mobile_q, g)
            assert np.max(np.abs(case.batch.walker_rho(w)[valid] - ref)) < 1e-5


@pytest.mark.parametrize("name", ["sc", "bcc", "fcc"])
def test_single_charge_madelung(name):
    """One charge per cell with alpha large enough that no image lies within
    the (inscribed) cutoff: the library's energy is the converged Madelung
    energy of the Wigner lattice (golden values, tests/golden/madelung.txt)."""
    from tests.test_oracle_pins import golden, CELLS_3D
    _, ref, tol = golden()[name]
    lat = CELLS_3D[name](4.0 / 3.0 * math.pi)
    s = wl.System(name, 3, lat, 1, -np.ones(1), np.zeros((0, 3)), np.zeros(0), 1, 1, 1)
    L = s.length
    a = 7.0 / L
    r_ins = ew.System(s, alpha=a, g_cut=12.5 * a, r_cut=0.1).info["r_inscribed"]
    say(f"[madelung] {name}")
    sysh = ew.System(s, alpha=a, g_cut=12.5 * a, r_cut=r_ins)
    batch = ew.Batch([sysh], np.zeros(1, dtype=np.int32))
    pos = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    batch.energy(pos, e)
    torch.cuda.synchronize()
    assert abs(e.item() - ref) <= tol * abs(ref)


def test_determinism():
    say("[determinism] cfg=3 mixed")
    out = []
    for _ in range(2):
        c = Case(3, 3, 16, MIXED, refresh_every=3)
        e, _ = c.run_energy()
        d, _ = c.per_step()
        d2, _ = c.fused(8)
        out.append((e, d, d2, c.batch.walker_rho(1)))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_invalid_k_gives_nan_and_no_move():
    say("[invalid k]")
    c = Case(2, 3, 1, FP64)
    c.run_energy()
    rho0 = c.batch.walker_rho(1)
    k = torch.tensor([0, -1, 250], dtype=torch.int32, device="cuda")
    d = torch.zeros(3, dtype=torch.float64, device="cuda")
    c.batch.move_delta(k, c.new_pos[0], d)
    c.batch.accept(torch.ones(3, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    dn = d.cpu().numpy()
    assert np.isfinite(dn[0]) and np.isnan(dn[1]) and np.isnan(dn[2])
    assert np.array_equal(c.batch.walker_rho(1), rho0)
    assert c.batch.walker_header(1)["n_accepts"] == 0
    assert c.batch.walker_header(0)["n_accepts"] == 1


def test_call_order_errors():
    say("[call order]")
    c = Case(1, 1, 2, FP64)
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(ew.EwaldError) as e:
        c.batch.move_delta(c.k[0], c.new_pos[0], d)
    assert e.value.status == ew.EWALD_E_STATE
    c.run_energy()
    with pytest.raises(ew.EwaldError) as e:
        c.batch.accept(c.accept[0])
    assert e.value.status == ew.EWALD_E_STATE
    c.batch.move_delta(c.k[0], c.new_pos[0], d)
    with pytest.raises(ew.EwaldError) as e:
        c.fused(1)
    assert e.value.status == ew.EWALD_E_STATE
    c.batch.accept(c.accept[0])
    c.fused(1)


def test_two_particles_and_ions(oracle_lib):
    """Smallest even system plus fixed ions (the pair bookkeeping's edge cases)."""
    lat = np.array([[6.0, 0.3, 0.0], [0.5, 5.5, 0.2], [0.1, -0.4, 6.2]])
    ions = np.array([[1.0, 1.0, 1.0], [3.0, 2.0, 4.0], [4.5, 4.0, 0.5]])
    s = wl.System("tiny", 3, lat, 2, np.array([-1.0, -2.0]), ions, np.array([1.0, 1.0, 1.0]),
                  1.1, 2.6, 8 * 2 * math.pi / 6.0)
    say("[tiny]")
    for prec in (FP64, MIXED):
        sysh = ew.System(s, precision=prec, refresh_every=2 if prec == MIXED else 0)
        batch = ew.Batch([sysh], np.zeros(1, dtype=np.int32))
        p0 = np.array([[0.2, 0.3, 0.1], [5.0, 1.0, 3.0]])
        pos = torch.tensor(p0, device="cuda")
        e = torch.zeros(1, dtype=torch.float64, device="cuda")
        batch.energy(pos, e)
        ks = np.array([1, 0, 1, 1], dtype=np.int32)
        newp = np.array([[2.0, 2.5, 3.0], [1.1, 1.2, 1.0], [-3.0, 7.0, 2.0], [3.2, 2.1, 4.1]])
        acc = np.array([1, 1, 0, 1], dtype=np.uint8)
        d = torch.zeros(4, dtype=torch.float64, device="cuda")
        for m in range(4):
            batch.move_delta(torch.tensor(ks[m:m + 1], device="cuda"),
                             torch.tensor(newp[m:m + 1], device="cuda"), d[m:m + 1])
            batch.accept(torch.tensor(acc[m:m + 1], device="cuda"))
        torch.cuda.synchronize()
        r = oracle_lib.run(s, p0, ks, newp, acc)
        scale = max(abs(r["energy0"]), e_scale(s))
        tol = 1e-10 * scale if prec == FP64 else 1e-5
        assert abs(e.item() - r["energy0"]) <= (1e-10 if prec == FP64 else 1e-6) * scale
        assert np.max(np.abs(d.cpu().numpy() - r["delta"])) <= tol
        # the fused sweep on this triclinic cell (general minimum-image reduction)
        assert ew.ewald_sys_geometry(sysh.handle)[0] == 0
        batch.energy(pos, e)
        df = torch.zeros((4, 1), dtype=torch.float64, device="cuda")
        batch.run_moves(torch.tensor(ks.reshape(4, 1), device="cuda"), torch.tensor(newp.reshape(4, 1, 3), device="cuda"),
                        torch.tensor(acc.reshape(4, 1), device="cuda"), df)
        torch.cuda.synchronize()
        assert np.max(np.abs(df.cpu().numpy()[:, 0] - r["delta"])) <= tol


@pytest.mark.parametrize("n", [7, 65])
def test_odd_particle_counts(oracle_lib, n):
    """An odd number of particles leaves one particle alone in the last rho
    rebuild tile (the tiles take particles in pairs): energy, per-step and
    fused moves, with rebuilds every 2 accepts in the mixed form."""
    rng = np.random.default_rng([11, n])
    lat = np.array([[6.0, 0.3, 0.0], [0.5, 5.5, 0.2], [0.1, -0.4, 6.2]])
    ions = rng.uniform(0, 6, (3, 3))
    q = np.where(np.arange(n) % 3 == 0, -0.5, -1.0)
    s = wl.System("odd%d" % n, 3, lat, n, q, ions, np.array([1.0, 2.0, 1.5]), 1.1, 2.6, 8 * 2 * math.pi / 6.0)
    p0 = rng.uniform(0, 6, (n, 3))
    M = 12
    ks = rng.integers(0, n, M).astype(np.int32)
    newp = rng.uniform(-1, 7, (M, 3))
    acc = (rng.uniform(size=M) < 0.6).astype(np.uint8)
    r = oracle_lib.run(s, p0, ks, newp, acc)
    scale = max(abs(r["energy0"]), e_scale(s))
    for prec in (FP64, MIXED):
        say(f"[odd n={n} prec={prec}]")
        sysh = ew.System(s, precision=prec, refresh_every=2 if prec == MIXED else 0)
        batch = ew.Batch([sysh], np.zeros(1, dtype=np.int32))
        pos = torch.tensor(p0, device="cuda")
        e = torch.zeros(1, dtype=torch.float64, device="cuda")
        batch.energy(pos, e)
        torch.cuda.synchronize()
        assert abs(e.item() - r["energy0"]) <= (1e-10 if prec == FP64 else 1e-6) * scale
        tol = 1e-10 * scale if prec == FP64 else 1e-5
        d = torch.zeros(M, dtype=torch.float64, device="cuda")
        for m in range(M):
            batch.move_delta(torch.tensor(ks[m:m + 1], device="cuda"),
                             torch.tensor(newp[m:m + 1], device="cuda"), d[m:m + 1])
            batch.accept(torch.tensor(acc[m:m + 1], device="cuda"))
        torch.cuda.synchronize()
        assert np.max(np.abs(d.cpu().numpy() - r["delta"])) <= tol
        batch.energy(pos, e)
        df = torch.zeros((M, 1), dtype=torch.float64, device="cuda")
        batch.run_moves(torch.tensor(ks.reshape(M, 1), device="cuda"), torch.tensor(newp.reshape(M, 1, 3), device="cuda"),
                        torch.tensor(acc.reshape(M, 1), device="cuda"), df)
        torch.cuda.synchronize()
        assert np.max(np.abs(df.cpu().numpy()[:, 0] - r["delta"])) <= tol
        if prec == MIXED:
            assert batch.walker_header(0)["n_refresh"] == int(acc.sum()) // 2


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [2, 3, 5])
def test_general_frame_matches_ortho(cfg_id, precision):
    """The fused sweep with the general minimum-image reduction (forced)
    equals the one in the orthogonal-sublattice frame on the same cell."""
    W, S, w0 = SUBSETS[cfg_id]
    say(f"[general vs ortho frame] cfg={cfg_id} precision={precision}")
    a = Case(cfg_id, W, S, precision, walker_start=w0)
    assert ew.ewald_sys_geometry(a.systems[0].handle)[0] > 0
    assert a.batch.tuning()["general_frame"] == 0
    a.run_energy()
    d1, j1 = a.fused()
    b = Case(cfg_id, W, S, precision, walker_start=w0)
    b.batch.set_tuning(general_frame=1)
    assert b.batch.tuning()["general_frame"] == 1
    b.run_energy()
    d2, j2 = b.fused()
    tol = 1e-12 if precision == FP64 else 1e-9
    scale = max(abs(x) for x in a.energy.cpu().numpy())
    assert np.max(np.abs(d1 - d2)) <= tol * max(1.0, scale)
    assert np.max(np.abs(j1 - j2)) <= tol * max(1.0, scale)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_full_size_sampled(oracle_lib, precision):
    """The N=1024 workload at its full 8192 walkers, in the launch shape the
    benchmark uses: sampled walkers against the oracle."""
    cfg = wl.config(5)
    say(f"[full size] precision={precision}")
    c = Case(5, cfg.walkers, 4, precision)
    e, j = c.run_energy()
    d, dj = c.fused()
    assert np.all(np.isfinite(e)) and np.all(np.isfinite(d))
    tol_e = 1e-10 if precision == FP64 else 1e-6
    for w in (0, 4097, cfg.walkers - 1):
        sysw = c.system(w)
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(sysw))
        assert abs(e[w] - r["energy0"]) <= tol_e * scale
        if precision == FP64:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale
        else:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_graph_replay_matches_eager(precision):
    """move_delta + accept captured once in a HIP graph and replayed move by
    move (inputs copied in eagerly between replays) give the eager results."""
    say(f"[graph] cfg=2 precision={precision}")
    S = 12
    eager = Case(2, 4, S, precision, refresh_every=3)
    eager.run_energy()
    d_ref, dj_ref = eager.per_step()

    c = Case(2, 4, S, precision, refresh_every=3)
    c.run_energy()
    k_buf = torch.zeros_like(c.k[0])
    np_buf = torch.zeros_like(c.new_pos[0])
    acc_buf = torch.zeros_like(c.accept[0])
    d_buf = torch.zeros(c.W, dtype=torch.float64, device="cuda")
    dj_buf = torch.zeros_like(d_buf)
    k_buf.copy_(c.k[0])
    np_buf.copy_(c.new_pos[0])
    acc_buf.copy_(c.accept[0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c.batch.move_delta(k_buf, np_buf, d_buf, dj_buf)
        c.batch.accept(acc_buf)
    torch.cuda.synchronize()
    # capture recorded the kernels without running them: replay every move
    for m in range(S):
        k_buf.copy_(c.k[m])
        np_buf.copy_(c.new_pos[m])
        acc_buf.copy_(c.accept[m])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d_buf.cpu().numpy(), d_ref[m]), m
        assert np.array_equal(dj_buf.cpu().numpy(), dj_ref[m]), m
    for w in range(c.W):
        assert np.array_equal(c.batch.walker_rho(w), eager.batch.walker_rho(w))
        assert np.array_equal(c.batch.walker_positions(w), eager.batch.walker_positions(w))


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_tuning_shapes_agree(precision):
    """Every fused-kernel launch shape (workgroup size, chunk length, frame)
    gives the same sweep up to rounding order."""
    W, S, w0 = SUBSETS[5]
    say(f"[tuning shapes] precision={precision}")
    ref = Case(5, W, S, precision, walker_start=w0, refresh_every=3)
    t = ref.batch.tuning()
    assert t["fused"] == 1 and t["threads"] == 1024 and 1 <= t["chunk"] <= 64
    ref.run_energy()
    d0, j0 = ref.fused()
    # FP64: rounding order only.  FP32-mixed: the FP32 partial sums run over
    # segment groups that differ with the shape (9e-8 Ha on deltas and 3e-7
    # on Jastrow deltas between the 1024- and 512-thread layouts here); the
    # bounds sit ten times above that, well inside the form's 1e-5 budget,
    # so a shape-specific error shows
    scale = max(1.0, max(abs(x) for x in ref.energy.cpu().numpy()))
    tol = 1e-12 * scale if precision == FP64 else 1e-6
    tol_j = 1e-12 * scale if precision == FP64 else 3e-6
    for threads, chunk, general, waves in ((512, 0, 0, 0), (1024, 5, 0, 0), (512, 1, 1, 0), (0, 64, 1, 0),
                                           (512, 0, 0, 4), (512, 3, 1, 4)):
        c = Case(5, W, S, precision, walker_start=w0, refresh_every=3)
        c.batch.set_tuning(threads, chunk, general, waves)
        t = c.batch.tuning()
        assert t["threads"] == (threads or 1024) and t["general_frame"] == general
        assert t["waves"] == (waves or (2 if t["threads"] <= 512 else 0))
        if chunk:  # an upper bound: fewer moves per chunk when LDS does not hold them
            assert t["chunk"] == chunk if chunk <= 8 else 8 <= t["chunk"] <= chunk
        c.run_energy()
        d, j = c.fused()
        say(f"  shape {threads, chunk, general, waves}: max |d - d0| = {np.max(np.abs(d - d0)):.3e}, "
            f"max |j - j0| = {np.max(np.abs(j - j0)):.3e}")
        assert np.max(np.abs(d - d0)) <= tol, (threads, chunk, general)
        assert np.max(np.abs(j - j0)) <= tol_j
        for w in range(W):
            assert np.max(np.abs(c.batch.walker_rho(w) - ref.batch.walker_rho(w))) <= 1e-9
    with pytest.raises(ew.EwaldError):
        ref.batch.set_tuning(threads=256)  # not a shape for 990 segments
    with pytest.raises(ew.EwaldError):
        ref.batch.set_tuning(chunk=65)
    with pytest.raises(ew.EwaldError):
        ref.batch.set_tuning(threads=512, waves=3)  # 512 x 2 comes at two and four waves per SIMD
    with pytest.raises(ew.EwaldError):
        ref.batch.set_tuning(threads=1024, waves=4)  # 1024 threads: four waves per SIMD by construction


def two_d_systems():
    """A 2D hexagonal gas of 1000 electrons with 643 G segments (the
    1024-thread and 512 x 2 fused shapes) and a 64-electron oblique cell,
    which has no orthogonal-sublattice frame (general minimum image)."""
    n = 1000
    area = math.pi * n
    L = math.sqrt(area)
    big = wl.System("hex1000", 2, wl.hex_cell(area), n, -np.ones(n), np.zeros((0, 2)), np.zeros(0), 5.0 / L,
                    0.5 * L, 40 * 2 * math.pi / L)
    n = 64
    L = math.sqrt(math.pi * n)
    ob = np.zeros((3, 3))
    ob[0, 0], ob[1, 0], ob[1, 1], ob[2, 2] = L, 0.31 * L, 0.93 * L, 1.0
    obl = wl.System("oblique64", 2, ob, n, -np.ones(n), np.zeros((0, 2)), np.zeros(0), 5.0 / L, 0.42 * L,
                    12 * 2 * math.pi / L)
    return big, obl


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_two_d_larger_shapes_and_oblique_cell(oracle_lib, precision):
    """2D cells beyond the workloads' shapes: energies and every delta of the
    per-step calls and of the fused sweep at each available workgroup size,
    against the oracle (the mixed form at K = 3)."""
    W, S = 2, 12
    for sy, shapes in zip(two_d_systems(), ((1024, 512), (0, 1024))):
        rng = np.random.default_rng([2, sy.n_mobile])
        lat = sy.lattice[:2, :2]
        pos = rng.random((W, sy.n_mobile, 2)) @ lat
        k = rng.integers(0, sy.n_mobile, (S, W)).astype(np.int32)
        newp = np.stack([pos[w][k[:, w]] + rng.normal(0, 0.6, (S, 2)) for w in range(W)], axis=1)
        acc = (rng.uniform(size=(S, W)) < 0.6).astype(np.uint8)
        say(f"[2d shapes] {sy.name} oracle")
        refs = [oracle_lib.run(sy, pos[w], k[:, w], newp[:, w], acc[:, w]) for w in range(W)]
        packed = torch.tensor(pos.reshape(W * sy.n_mobile, 2), device="cuda")
        kt, nt, at = (torch.tensor(x, device="cuda") for x in (k, newp, acc))
        for path in ("per-step",) + shapes:
            say(f"[2d shapes] {sy.name} precision={precision} path={path}")
            h = ew.System(sy, precision=precision, refresh_every=3 if precision == MIXED else 0)
            if sy.name.startswith("oblique"):
                assert ew.ewald_sys_geometry(h.handle)[0] == 0
            b = ew.Batch([h], np.zeros(W, dtype=np.int32))
            e = torch.zeros(W, dtype=torch.float64, device="cuda")
            b.energy(packed, e)
            d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
            if path == "per-step":
                for m in range(S):
                    b.move_delta(kt[m], nt[m], d[m])
                    b.accept(at[m])
            else:
                b.set_tuning(threads=path)
                t = b.tuning()
                assert t["fused"] == 1 and (path == 0 or t["threads"] == path)
                b.run_moves(kt, nt, at, d)
            torch.cuda.synchronize()
            en, dn = e.cpu().numpy(), d.cpu().numpy()
            for w in range(W):
                r = refs[w]
                scale = max(abs(r["energy0"]), e_scale(sy))
                assert b.walker_header(w)["n_accepts"] == int(acc[:, w].sum())
                if precision == MIXED:
                    assert abs(en[w] - r["energy0"]) <= 1e-6 * scale
                    assert np.max(np.abs(dn[:, w] - r["delta"])) <= 1e-5, (path, w)
                else:
                    assert abs(en[w] - r["energy0"]) <= 1e-10 * scale
                    assert np.max(np.abs(dn[:, w] - r["delta"])) <= 1e-10 * scale, (path, w)
            b.close()
            h.close()


def test_largest_sizes(oracle_lib):
    """Near the library's limits: 2040 electrons (EWALD_MAX_PARTICLES is
    2048) and 1960 G segments (EWALD_MAX_SEGMENTS is 2048), which only the
    512-thread four-segment fused kernel and the eight-segment energy kernel
    take.  Energies and every delta of a fused sweep and of the per-step calls
    against the oracle, in both forms (the mixed form at K = 3, so that it
    rebuilds rho between chunks and after accepts)."""
    n, W, S = 2040, 2, 8
    L = (4 * math.pi * n / 3) ** (1 / 3)
    sy = wl.System("max2040", 3, np.eye(3) * L, n, -np.ones(n), np.zeros((0, 3)), np.zeros(0), 5.0 / L, 0.5 * L,
                   15.0 * 2 * math.pi / L)
    rng = np.random.default_rng(2040)
    pos = rng.uniform(0, L, (W, n, 3))
    k = rng.integers(0, n, (S, W)).astype(np.int32)
    newp = np.stack([pos[w][k[:, w]] + rng.normal(0, 0.5, (S, 3)) for w in range(W)], axis=1)
    acc = (rng.uniform(size=(S, W)) < 0.6).astype(np.uint8)
    say("[largest sizes] oracle")
    refs = [oracle_lib.run(sy, pos[w], k[:, w], newp[:, w], acc[:, w]) for w in range(W)]
    packed = torch.tensor(pos.reshape(W * n, 3), device="cuda")
    kt, nt, at = (torch.tensor(x, device="cuda") for x in (k, newp, acc))
    for precision in (FP64, MIXED):
        for path in ("fused", "per-step"):
            say(f"[largest sizes] precision={precision} path={path}")
            h = ew.System(sy, precision=precision, refresh_every=3 if precision == MIXED else 0)
            assert 1024 < ew.ewald_sys_query(h.handle)["n_slots"] // 4 <= 2048
            b = ew.Batch([h], np.zeros(W, dtype=np.int32))
            e = torch.zeros(W, dtype=torch.float64, device="cuda")
            b.energy(packed, e)
            d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
            if path == "fused":
                t = b.tuning()
                assert t["fused"] == 1 and t["threads"] == 512
                b.run_moves(kt, nt, at, d)
            else:
                for m in range(S):
                    b.move_delta(kt[m], nt[m], d[m])
                    b.accept(at[m])
            torch.cuda.synchronize()
            en, dn = e.cpu().numpy(), d.cpu().numpy()
            for w in range(W):
                r = refs[w]
                scale = max(1.0, abs(r["energy0"]))
                h_w = b.walker_header(w)
                assert h_w["n_accepts"] == int(acc[:, w].sum())
                if precision == MIXED:
                    assert h_w["n_refresh"] >= 1
                    assert abs(en[w] - r["energy0"]) <= 1e-6 * scale
                    assert np.max(np.abs(dn[:, w] - r["delta"])) <= 1e-5, (path, w)
                else:
                    assert abs(en[w] - r["energy0"]) <= 1e-10 * scale
                    assert np.max(np.abs(dn[:, w] - r["delta"])) <= 1e-10 * scale, (path, w)
            b.close()
            h.close()


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_extra_particles_and_ions_at_large_shapes(precision):
    """The 512- and 1024-thread fused kernels built with their loops over
    particles beyond the registers' share and over fixed ions: a walker of
    1100 electrons (more than a 1024-thread workgroup holds in registers)
    beside a small walker with ions, both with ~1000 G segments, against the
    per-step kernels."""
    rng = np.random.default_rng([13, precision])
    systems = []
    for n, nion in ((1100, 0), (40, 3)):
        L = (4 * math.pi * n / 3) ** (1 / 3) if n > 100 else 8.0
        lat = np.eye(3) * L
        ions = rng.uniform(0, L, (nion, 3))
        qf = np.full(nion, 2.0)
        systems.append(wl.System("x%d" % n, 3, lat, n, -np.ones(n), ions, qf, 5.0 / L, 0.5 * L,
                                 12 * 2 * math.pi / L))
    walker_sys = np.array([0, 1], dtype=np.int32)
    M = 8
    pos = [rng.uniform(0, systems[i].lattice[0, 0], (systems[i].n_mobile, 3)) for i in walker_sys]
    packed = torch.tensor(np.concatenate(pos), device="cuda")
    k = np.stack([rng.integers(0, systems[i].n_mobile, M) for i in walker_sys], axis=1).astype(np.int32)
    newp = np.stack([rng.uniform(0, systems[i].lattice[0, 0], (M, 3)) for i in walker_sys], axis=1)
    acc = (rng.uniform(size=(M, 2)) < 0.6).astype(np.uint8)
    kt, nt, at = (torch.tensor(x, device="cuda") for x in (k, newp, acc))

    def batch():
        hs = [ew.System(sy, precision=precision, refresh_every=2 if precision == MIXED else 0) for sy in systems]
        b = ew.Batch(hs, walker_sys)
        e = torch.zeros(2, dtype=torch.float64, device="cuda")
        b.energy(packed, e)
        return hs, b, e

    hs, ref, e = batch()
    assert min(ew.ewald_sys_query(h.handle)["n_slots"] for h in hs) > 4 * 512
    say(f"[extra loops] precision={precision} per-step")
    d0 = torch.zeros((M, 2), dtype=torch.float64, device="cuda")
    for m in range(M):
        ref.move_delta(kt[m], nt[m], d0[m])
        ref.accept(at[m])
    torch.cuda.synchronize()
    scale = max(1.0, float(e.abs().max()))
    tol = 1e-12 * scale if precision == FP64 else 1e-5
    for threads in (1024, 512):
        say(f"[extra loops] precision={precision} threads={threads}")
        _, b, _ = batch()
        b.set_tuning(threads=threads)
        t = b.tuning()
        assert t["fused"] == 1 and t["threads"] == threads
        d = torch.zeros((M, 2), dtype=torch.float64, device="cuda")
        b.run_moves(kt, nt, at, d)
        torch.cuda.synchronize()
        assert np.max(np.abs(d.cpu().numpy() - d0.cpu().numpy())) <= tol, threads
        for w in range(2):
            assert np.array_equal(b.walker_positions(w), ref.walker_positions(w))
            assert np.max(np.abs(b.walker_rho(w) - ref.walker_rho(w))) <= 1e-9 * math.sqrt(systems[w].n_mobile)
            assert b.walker_header(w)["n_accepts"] == int(acc[:, w].sum())


def test_autotune_keeps_state_and_caches(tmp_path, oracle_lib):
    """The autotuner probes on a copy of the state (the walkers' state is
    unchanged), stores its choice in the cache file and re-applies it from there; the tuned sweep
    still matches the oracle."""
    W, S, w0 = SUBSETS[2]
    say("[autotune] cfg=2")
    c = Case(2, W, S, FP64, walker_start=w0)
    c.run_energy()
    before = [c.batch.walker_rho(w) for w in range(W)]
    pos_before = [c.batch.walker_positions(w) for w in range(W)]
    cache = tmp_path / "tune.txt"
    c.batch.autotune(n_moves=8, cache_path=str(cache))
    t1 = c.batch.tuning()
    assert t1["fused"] == 1
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and "threads=" in lines[0]
    for w in range(W):
        assert np.array_equal(c.batch.walker_rho(w), before[w])
        assert np.array_equal(c.batch.walker_positions(w), pos_before[w])
        assert c.batch.walker_header(w)["n_accepts"] == 0
    c2 = Case(2, W, S, FP64, walker_start=w0)
    c2.run_energy()
    c2.batch.set_tuning(256, 7, 1)
    c2.batch.autotune(n_moves=8, cache_path=str(cache))  # from the cache: no new line
    assert c2.batch.tuning() == t1
    assert len(cache.read_text().strip().splitlines()) == 1
    # a cached line the library rejects (no such workgroup size) is measured
    # afresh and the new choice appended
    key = lines[0].split("|")[0]
    cache.write_text(key + "|threads=999 chunk=0 general_frame=0 waves=2 walkers_per_block=0\n")
    c2.batch.autotune(n_moves=8, cache_path=str(cache))
    assert c2.batch.tuning()["fused"] == 1
    lines2 = cache.read_text().strip().splitlines()
    assert len(lines2) == 2 and lines2[1].startswith(key + "|threads=") and "threads=999" not in lines2[1]
    d, _ = c.fused()
    for w in range(W):
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(c.system(w)))
        assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_uneven_batch_fused_graph(precision):
    """The uneven batch (walkers of 64/216/512 electrons plus ions in one
    launch): the fused sweep, autotuned, captured once in a HIP graph and
    replayed three times, equals three eager sweeps over the same proposals."""
    W, S = 24, 12
    say(f"[uneven graph] cfg=4 precision={precision}")
    eager = Case(4, W, S, precision, refresh_every=3)
    assert len(set(int(x) for x in eager.b.walker_sys)) == 3
    eager.run_energy()
    eager.batch.autotune(n_moves=8)
    ref = [eager.fused() for _ in range(3)]
    g_case = Case(4, W, S, precision, refresh_every=3)
    g_case.run_energy()
    g_case.batch.set_tuning(**{k: v for k, v in eager.batch.tuning().items() if k != "fused"})
    d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    dj = torch.zeros_like(d)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        g_case.batch.run_moves(g_case.k, g_case.new_pos, g_case.accept, d, dj)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == FP64 else 1e-9
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        scale = max(1.0, float(np.max(np.abs(ref[r][0]))))
        assert np.max(np.abs(d.cpu().numpy() - ref[r][0])) <= tol * scale, r
        assert np.max(np.abs(dj.cpu().numpy() - ref[r][1])) <= tol * scale, r
    for w in range(W):
        assert np.array_equal(g_case.batch.walker_positions(w), eager.batch.walker_positions(w))
        assert g_case.batch.walker_header(w)["n_accepts"] == eager.batch.walker_header(w)["n_accepts"]


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_uneven_batch_fused_vs_oracle(oracle_lib, precision):
    """The uneven batch in one fused launch (walkers of 64, 216 and 512
    electrons with their +4 ions, launched most expensive first), autotuned,
    against the oracle walker by walker: every delta and Jastrow delta, the
    accept counts, the mixed form's rebuild counts at K=4, and the final
    positions."""
    W, S, K = 6, 24, 4
    say(f"[uneven fused vs oracle] cfg=4 precision={precision}")
    c = Case(4, W, S, precision, refresh_every=K)
    assert len(set(int(x) for x in c.b.walker_sys)) == 3
    e0, _ = c.run_energy()
    c.batch.autotune(n_moves=8)
    assert c.batch.tuning()["fused"] == 1
    d, dj = c.fused()
    fin = c.final_cartesian()
    for w in range(W):
        r, sysw = c.oracle(oracle_lib, w), c.system(w)
        scale = max(abs(r["energy0"]), e_scale(sysw))
        acc = int(c.b.accept[:, w].sum())
        h = c.batch.walker_header(w)
        assert h["n_accepts"] == acc
        if precision == FP64:
            assert abs(e0[w] - r["energy0"]) <= 1e-10 * scale
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, w
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"])), w
        else:
            assert h["n_refresh"] == acc // K
            assert abs(e0[w] - r["energy0"]) <= 1e-6 * scale
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, w
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w), w
        # final positions (wrapped by the library) equal the oracle's modulo the lattice
        lat = sysw.lattice[: c.dim, : c.dim]
        got = fin[c.b.pos_offsets[w]: c.b.pos_offsets[w + 1]]
        diff = (got - r["pos_final"][: sysw.n_mobile]) @ np.linalg.inv(lat)
        assert np.max(np.abs(diff - np.rint(diff))) <= 1e-12


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [2, 3, 4])
def test_small_walker_shapes_vs_oracle(oracle_lib, cfg_id, precision):
    """Every launch shape available to the smaller workloads (308 or 28
    segments; 250, 300 or 64/216/512 particles plus ions): 256 threads (two
    particles per lane where needed, plus the ion loop) compiled for 2, 3 and
    4 waves per SIMD, and 1024 threads (most lanes idle), through the fused
    sweep against the oracle: deltas, Jastrow deltas and the mixed form's
    rebuild counts at K=4."""
    W = 6 if cfg_id == 4 else 3
    S, K = 16, 4
    refs = None
    for threads, waves in ((256, 2), (256, 3), (256, 4), (1024, 0)):
        say(f"[small shapes] cfg={cfg_id} precision={precision} threads={threads} waves={waves}")
        c = Case(cfg_id, W, S, precision, refresh_every=K)
        if refs is None:
            refs = [c.oracle(oracle_lib, w) for w in range(W)]
        c.batch.set_tuning(threads=threads, waves=waves)
        t = c.batch.tuning()
        assert t["fused"] == 1 and t["threads"] == threads and t["waves"] == waves
        e0, _ = c.run_energy()
        d, dj = c.fused()
        for w in range(W):
            r, sysw = refs[w], c.system(w)
            scale = max(abs(r["energy0"]), e_scale(sysw))
            acc = int(c.b.accept[:, w].sum())
            h = c.batch.walker_header(w)
            assert h["n_accepts"] == acc
            if precision == FP64:
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, (threads, w)
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"])), (threads, w)
            else:
                assert h["n_refresh"] == acc // K
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, (threads, w)
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w), (threads, w)


@pytest.mark.parametrize("precision", [MIXED, FP64], ids=["mixed", "fp64"])
def test_n1024_long_sweep_with_rebuilds(oracle_lib, precision):
    """The N=1024 workload (bcc cell, 3577 G, Jastrow) at its refresh interval
    K=64: 2 walkers x 280 moves, so that the FP32-mixed form rebuilds rho in
    FP64 twice per walker mid-sequence.  The per-step kernels (accept plus the
    rebuild kernel) and the fused sweep at 1024 threads (running rho kept in
    LDS during its rebuild) and at 512 threads (two and four waves per SIMD)
    are each compared with the oracle on every delta and Jastrow delta, and
    the final rho element by element."""
    W, S = 2, 280
    refs = None
    for path in ("per-step", "step", 1024, 512, "512w4"):
        say(f"[n1024 long] precision={precision} path={path}")
        c = Case(5, W, S, precision)
        if refs is None:
            refs = [c.oracle(oracle_lib, w) for w in range(W)]
        e0, j0 = c.run_energy()
        if path == "per-step":
            d, dj = c.per_step()
        elif path == "step":
            d, dj = c.stepped()
        else:
            threads, waves = (512, 4) if path == "512w4" else (path, 0)
            c.batch.set_tuning(threads=threads, waves=waves)
            tn = c.batch.tuning()
            assert tn["threads"] == threads and tn["fused"] == 1 and tn["waves"] == (waves or tn["waves"])
            d, dj = c.fused()
        for w in range(W):
            r, sysw = refs[w], c.system(w)
            scale = max(abs(r["energy0"]), e_scale(sysw))
            acc = int(c.b.accept[:, w].sum())
            h = c.batch.walker_header(w)
            assert h["n_accepts"] == acc
            if precision == MIXED:
                assert acc // 64 == 2 and h["n_refresh"] == 2
                assert 0.0 < h["drift_max"] < 1e-5
                assert abs(e0[w] - r["energy0"]) <= 1e-6 * scale
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w), path
            else:
                assert abs(e0[w] - r["energy0"]) <= 1e-10 * scale
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"])), path
            # running rho against the oracle's rho of the final positions
            t = c.systems[0].tables()
            valid = t["shell"] >= 0
            B = 2 * math.pi * np.linalg.inv(sysw.lattice).T
            g = t["n"][valid] @ B
            ref_rho = oracle_lib.rho_at(sysw, r["pos_final"], sysw.mobile_q, g)
            tol_rho = 1e-5 if precision == MIXED else 1e-9
            assert np.max(np.abs(c.batch.walker_rho(w)[valid] - ref_rho)) <= tol_rho, path


# Jastrow derivatives (gradient and Laplacian of J with respect to the moved
# particle at the proposed configuration) against the oracle's pair form.
# Bounds: FP64 1e-9, FP32-mixed 1e-5, relative to the largest |value| of the
# walker's sequence (at least 1): z = conj(rho') exp(iG.r') is formed in FP32
# in the mixed form, with an error of a few units of FP32 rounding times
# |rho'| per G, summed over the half set.
DERIV_SUBSETS = {1: (1, 24), 2: (2, 12), 3: (2, 16), 5: (2, 5)}


def deriv_case(cfg_id, precision):
    W, S = DERIV_SUBSETS[cfg_id]
    c = Case(cfg_id, W, S, precision)
    return c, W, S


def check_derivs(c, oracle_lib, g, l, precision, what):
    tol = 1e-9 if precision == FP64 else 1e-5
    for w in range(c.W):
        r = oracle_lib.run(c.system(w), c.b.walker_pos(w), c.b.k[:, w], c.b.new_pos[:, w], c.b.accept[:, w],
                           jastrow_a=c.ja, derivs=True)
        sg = max(1.0, float(np.max(np.abs(r["jgrad"]))))
        sl = max(1.0, float(np.max(np.abs(r["jlap"]))))
        assert np.max(np.abs(g[:, w] - r["jgrad"])) <= tol * sg, (what, w)
        assert np.max(np.abs(l[:, w] - r["jlap"])) <= tol * sl, (what, w)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 5])
def test_jastrow_derivs_per_step(oracle_lib, cfg_id, precision):
    """move_delta with derivatives, move by move, against the oracle; the
    energy and Jastrow deltas equal those of the plain call."""
    c, W, S = deriv_case(cfg_id, precision)
    say(f"[jastrow derivs per-step] cfg={cfg_id} precision={precision}")
    c.run_energy()
    d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    dj = torch.zeros_like(d)
    g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
    l = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    for m in range(S):
        c.batch.move_delta_grad(c.k[m], c.new_pos[m], d[m], dj[m], g[m], l[m])
        c.batch.accept(c.accept[m])
    torch.cuda.synchronize()
    ref = Case(cfg_id, W, S, precision)
    ref.run_energy()
    d0, j0 = ref.per_step()
    scale = max(1.0, float(np.max(np.abs(c.energy.cpu().numpy()))))
    assert np.max(np.abs(d.cpu().numpy() - d0)) <= 1e-12 * scale
    assert np.max(np.abs(dj.cpu().numpy() - j0)) <= 1e-12 * scale
    check_derivs(c, oracle_lib, g.cpu().numpy(), l.cpu().numpy(), precision, "per-step")


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 5])
def test_jastrow_derivs_fused(oracle_lib, cfg_id, precision):
    """run_moves with derivatives against the oracle; the deltas equal the
    plain fused sweep's, and the state after the sweep equals it too."""
    c, W, S = deriv_case(cfg_id, precision)
    say(f"[jastrow derivs fused] cfg={cfg_id} precision={precision}")
    c.run_energy()
    d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    dj = torch.zeros_like(d)
    g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
    l = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    c.batch.run_moves_grad(c.k, c.new_pos, c.accept, d, dj, g, l)
    torch.cuda.synchronize()
    ref = Case(cfg_id, W, S, precision)
    ref.run_energy()
    d0, j0 = ref.fused()
    scale = max(1.0, float(np.max(np.abs(c.energy.cpu().numpy()))))
    assert np.max(np.abs(d.cpu().numpy() - d0)) <= 1e-12 * scale
    assert np.max(np.abs(dj.cpu().numpy() - j0)) <= 1e-12 * scale
    for w in range(W):
        assert np.array_equal(c.batch.walker_positions(w), ref.batch.walker_positions(w))
        assert np.max(np.abs(c.batch.walker_rho(w) - ref.batch.walker_rho(w))) <= 1e-12 * math.sqrt(c.system(w).n_mobile)
    check_derivs(c, oracle_lib, g.cpu().numpy(), l.cpu().numpy(), precision, "fused")


# FP32-mixed form at a refresh interval of 3 accepts: the fused sweep rebuilds
# rho between chunks several times, reusing the chunk's LDS for the rebuild
# tiles and the running-rho copy; the per-shell tables the moves read must
# survive it.  (cfg, tuning, u term): each workload's default shape and
# another one, and the p term with the two-body u term.
DERIV_REBUILD_CASES = [(2, dict(), False), (2, dict(threads=256, waves=3), False), (2, dict(threads=1024), False),
                       (3, dict(), False), (3, dict(threads=1024), False), (5, dict(), False),
                       (5, dict(threads=512), False), (2, dict(), True), (5, dict(), True)]


@pytest.mark.parametrize("cfg_id,tuning,u_term", DERIV_REBUILD_CASES,
                         ids=[f"cfg{c}-" + ("-".join(f"{k}{v}" for k, v in t.items()) or "default") + ("-u" if u else "")
                              for c, t, u in DERIV_REBUILD_CASES])
def test_jastrow_derivs_with_rebuilds(oracle_lib, cfg_id, tuning, u_term):
    """Gradient and Laplacian of every proposed move through several rebuilds
    (fused sweep and per-step calls) against the oracle; the fused deltas and
    final state equal those of the plain fused sweep at the same shape."""
    W, S, K = 2, (12 if cfg_id == 5 else 24), 3
    c = Case(cfg_id, W, S, MIXED, refresh_every=K, u_term=u_term)
    say(f"[jastrow derivs with rebuilds] cfg={cfg_id} K={K} tuning={tuning} u_term={u_term}")
    if tuning:
        c.batch.set_tuning(**tuning)
    c.run_energy()
    d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    dj = torch.zeros_like(d)
    g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
    l = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    c.batch.run_moves_grad(c.k, c.new_pos, c.accept, d, dj, g, l)
    torch.cuda.synchronize()
    assert all(c.batch.walker_header(w)["n_refresh"] >= 2 for w in range(W))
    ref = Case(cfg_id, W, S, MIXED, refresh_every=K, u_term=u_term)
    if tuning:
        ref.batch.set_tuning(**tuning)
    ref.run_energy()
    d0, j0 = ref.fused()
    scale = max(1.0, float(np.max(np.abs(c.energy.cpu().numpy()))))
    assert np.max(np.abs(d.cpu().numpy() - d0)) <= 1e-12 * scale
    assert np.max(np.abs(dj.cpu().numpy() - j0)) <= 1e-12 * scale
    for w in range(W):
        assert np.max(np.abs(c.batch.walker_rho(w) - ref.batch.walker_rho(w))) <= 1e-12 * math.sqrt(c.system(w).n_mobile)
    check_derivs(c, oracle_lib, g.cpu().numpy(), l.cpu().numpy(), MIXED, "fused, rebuilds")
    p = Case(cfg_id, W, S, MIXED, refresh_every=K, u_term=u_term)
    p.run_energy()
    for m in range(S):
        p.batch.move_delta_grad(p.k[m], p.new_pos[m], d[m], dj[m], g[m], l[m])
        p.batch.accept(p.accept[m])
    torch.cuda.synchronize()
    check_derivs(p, oracle_lib, g.cpu().numpy(), l.cpu().numpy(), MIXED, "per-step, rebuilds")


def test_jastrow_derivs_argument_errors():
    say("[jastrow derivs errors]")
    c = Case(2, 1, 1, FP64, jastrow=False)
    c.run_energy()
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ew.EwaldError) as e:  # no Jastrow coefficients in this batch
        c.batch.move_delta_grad(c.k[0], c.new_pos[0], d, None, g, d)
    assert e.value.status == ew.EWALD_E_ARG
    with pytest.raises(ew.EwaldError) as e:  # only one of the two outputs
        ew.ewald_move_delta_grad_batch(c.batch.handle, c.batch.state.data_ptr(), c.k[0].data_ptr(),
                                       c.new_pos[0].data_ptr(), d.data_ptr(), 0, g.data_ptr(), 0)
    assert e.value.status == ew.EWALD_E_ARG


# Jastrow two-body polynomial term u (Eq. (8)) added to the Jastrow outputs:
# value, move deltas (per-step and fused) and derivatives against the oracle.
# The u term is FP64 in both forms, so the mixed form keeps its bounds.
U_SUBSETS = {1: (1, 20), 2: (2, 12), 3: (2, 16), 5: (2, 6)}


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 5])
def test_u_term_energy_and_moves(oracle_lib, cfg_id, precision):
    W, S = U_SUBSETS[cfg_id]
    say(f"[u term] cfg={cfg_id} precision={precision}")
    results = {}
    for path in ("per-step", "fused"):
        c = Case(cfg_id, W, S, precision, refresh_every=4, u_term=True)
        e0, j0 = c.run_energy()
        results[path] = (e0, j0) + (c.per_step() if path == "per-step" else c.fused())
    for w in range(W):
        sysw = c.system(w)
        assert sysw.u_alpha is not None
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(sysw))
        jscale = max(1.0, abs(r["j0"]))
        for path, (e0, j0, d, dj) in results.items():
            if precision == FP64:
                assert abs(e0[w] - r["energy0"]) <= 1e-10 * scale
                assert abs(j0[w] - r["j0"]) <= 1e-10 * jscale, (path, j0[w], r["j0"])
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * jscale, path
            else:
                assert abs(j0[w] - r["j0"]) <= 1e-6 * jscale, (path, j0[w], r["j0"])
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, path
                assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w), path


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 3, 5])
def test_u_term_derivs(oracle_lib, cfg_id, precision):
    """Jastrow gradient and Laplacian with the u term, per-step and fused
    (orthogonal-sublattice and general frames), against the oracle."""
    W, S = U_SUBSETS[cfg_id]
    for path in ("per-step", "fused", "fused-general"):
        say(f"[u term derivs] cfg={cfg_id} precision={precision} path={path}")
        c = Case(cfg_id, W, S, precision, u_term=True)
        if path == "fused-general":
            c.batch.set_tuning(general_frame=1)
        c.run_energy()
        d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
        l = torch.zeros((S, W), dtype=torch.float64, device="cuda")
        if path == "per-step":
            for m in range(S):
                c.batch.move_delta_grad(c.k[m], c.new_pos[m], d[m], dj[m], g[m], l[m])
                c.batch.accept(c.accept[m])
        else:
            c.batch.run_moves_grad(c.k, c.new_pos, c.accept, d, dj, g, l)
        torch.cuda.synchronize()
        check_derivs(c, oracle_lib, g.cpu().numpy(), l.cpu().numpy(), precision, path)


# Blip orbitals (Sec. 2.4) against the oracle's plain sum over the grid.
SKEW = np.array([[6.0, 0.4, 0.1], [0.7, 5.5, -0.3], [0.2, -0.5, 6.4]])


@pytest.mark.parametrize("n_orb", [6, 5, 130])
def test_blips_small_grid(oracle_lib, n_orb):
    """A skewed cell, an 8 x 9 x 10 grid, even (paired loads), odd and
    more-than-one-chunk orbital counts; points inside, outside and on the
    cell's faces; values, gradients and Laplacians within 1e-12 relative."""
    say(f"[blips small] n_orb={n_orb}")
    grid = (8, 9, 10)
    rng = np.random.default_rng([17, n_orb])
    coef = rng.uniform(-1, 1, grid + (n_orb,))
    s = rng.uniform(-1.5, 2.5, (37, 3))
    s[:4] = [[0, 0, 0], [1, 0.5, 0.25], [0.125, 1.0 / 9, 0.1], [0.999999999, 0, 1]]
    pts = s @ SKEW
    b = ew.Blips(SKEW, grid, n_orb)
    dev = "cuda"
    c_t = torch.tensor(coef, device=dev)
    p_t = torch.tensor(pts, device=dev)
    val = torch.zeros((len(pts), n_orb), dtype=torch.float64, device=dev)
    grad = torch.zeros((len(pts), 3, n_orb), dtype=torch.float64, device=dev)
    lap = torch.zeros_like(val)
    b.eval(c_t, p_t, val, grad, lap)
    v_only = torch.zeros_like(val)
    b.eval(c_t, p_t, v_only)
    torch.cuda.synchronize()
    rv, rg, rl = oracle_lib.blip_eval(SKEW, grid, coef, pts)
    sv = max(1.0, float(np.max(np.abs(rv))))
    sg = max(1.0, float(np.max(np.abs(rg))))
    sl = max(1.0, float(np.max(np.abs(rl))))
    assert np.max(np.abs(val.cpu().numpy() - rv)) <= 1e-12 * sv
    assert np.array_equal(v_only.cpu().numpy(), val.cpu().numpy())
    assert np.max(np.abs(grad.cpu().numpy() - rg)) <= 1e-12 * sg
    assert np.max(np.abs(lap.cpu().numpy() - rl)) <= 1e-12 * sl
    with pytest.raises(ew.EwaldError):
        ew.ewald_blip_eval_batch(b.handle, c_t.data_ptr(), len(pts), p_t.data_ptr(), val.data_ptr(),
                                 grad.data_ptr(), 0)
    with pytest.raises(ew.EwaldError):
        ew.Blips(SKEW, (3, 9, 10), 4)


def test_blips_full_size_sampled(oracle_lib):
    """The benchmarked blip workload (bcc N=1024 cell, 40^3 grid, 512
    orbitals, 65536 proposal points in one call): sampled points against the
    oracle."""
    say("[blips full size]")
    cfg = wl.config(5)
    lat = cfg.systems[0].lattice
    coef = wl.blip_coefficients()
    pts = wl.blip_points(8192, 8)
    dev = "cuda"
    c_t = torch.tensor(coef, device=dev)
    p_t = torch.tensor(pts, device=dev)
    P, M = pts.shape[0], wl.BLIP_ORBITALS
    val = torch.zeros((P, M), dtype=torch.float64, device=dev)
    grad = torch.zeros((P, 3, M), dtype=torch.float64, device=dev)
    lap = torch.zeros_like(val)
    b = ew.Blips(lat, wl.BLIP_GRID, M)
    b.eval(c_t, p_t, val, grad, lap)
    torch.cuda.synchronize()
    sample = np.array([0, 1, 4097, 32768, 65535, 12345])
    rv, rg, rl = oracle_lib.blip_eval(lat, wl.BLIP_GRID, coef, pts[sample])
    assert np.max(np.abs(val[sample].cpu().numpy() - rv)) <= 1e-12 * max(1.0, float(np.max(np.abs(rv))))
    assert np.max(np.abs(grad[sample].cpu().numpy() - rg)) <= 1e-12 * max(1.0, float(np.max(np.abs(rg))))
    assert np.max(np.abs(lap[sample].cpu().numpy() - rl)) <= 1e-12 * max(1.0, float(np.max(np.abs(rl))))
    assert bool(torch.isfinite(val).all()) and bool(torch.isfinite(lap).all())



# Layered two-dimensional systems (Eq. (5) with z != 0): the electron-hole
# bilayer against the oracle's pair-by-pair energy, through the per-step
# kernels and the fused kernels with a second plane.
@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_bilayer_energy_and_moves(oracle_lib, precision):
    W, S, K = 3, 24, 4
    say(f"[bilayer] precision={precision}")
    out = {}
    for path in ("per-step", "run_moves", "run_moves_1024"):
        c = Case(3, W, S, precision, refresh_every=K, jastrow=False, cfg=wl.bilayer_config())
        e0, _ = c.run_energy()
        if path == "run_moves_1024":
            c.batch.set_tuning(threads=1024)
            assert c.batch.tuning()["threads"] == 1024
        if path != "per-step":
            assert c.batch.tuning()["fused"] == 1
        out[path] = (e0,) + (c.per_step() if path == "per-step" else c.fused())
        for w in range(W):
            h = c.batch.walker_header(w)
            acc = int(c.b.accept[:, w].sum())
            assert h["n_accepts"] == acc
            if precision == MIXED:
                assert h["n_refresh"] == acc // K
    for w in range(W):
        sysw = c.system(w)
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(sysw))
        for path, (e0, d, _) in out.items():
            if precision == FP64:
                assert abs(e0[w] - r["energy0"]) <= 1e-10 * scale, (path, e0[w], r["energy0"])
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale, path
            else:
                assert abs(e0[w] - r["energy0"]) <= 1e-6 * scale, path
                assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5, path


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_layers_with_ions_and_telescoping(oracle_lib, precision):
    """Two planes with fixed ions in the second one and unequal plane
    populations (different plane charges, so the cross-plane background
    term counts): energies, deltas, and E0 + accepted deltas against a fresh
    energy of the final positions."""
    say(f"[layers ions] precision={precision}")
    base = wl.bilayer(6, 2.2)
    ions = np.array([[3.0, 4.0], [40.0, 17.0], [20.0, 60.0]])
    sysm = dataclasses.replace(base, n_mobile=9, mobile_q=np.array([-1.0] * 5 + [1.0] * 4),
                               mobile_layer=np.array([0] * 5 + [1] * 4, dtype=np.int32),
                               fixed_pos=ions, fixed_q=np.array([1.0, -0.5, 2.0]),
                               fixed_layer=np.array([1, 1, 0], dtype=np.int32))
    rng = np.random.default_rng(77)
    lat = sysm.lattice[:2, :2]
    W, S = 2, 16
    pos = [rng.random((9, 2)) @ lat for _ in range(W)]
    k = rng.integers(0, 9, (S, W)).astype(np.int32)
    newp = np.stack([[pos[w][k[m, w]] + rng.normal(0, 4.0, 2) for w in range(W)] for m in range(S)])
    acc = (rng.random((S, W)) < 0.6).astype(np.uint8)
    h = ew.System(sysm, precision=precision, refresh_every=3 if precision == MIXED else 0)
    b = ew.Batch([h], np.zeros(W, dtype=np.int32))
    dev = "cuda"
    e = torch.zeros(W, dtype=torch.float64, device=dev)
    b.energy(torch.tensor(np.concatenate(pos), device=dev), e)
    kt, nt, at = (torch.tensor(x, device=dev) for x in (k, newp, acc))
    d = torch.zeros((S, W), dtype=torch.float64, device=dev)
    for m in range(S):
        b.move_delta(kt[m], nt[m], d[m])
        b.accept(at[m])
    # the same sequence through the fused kernel (second plane in registers)
    bf = ew.Batch([h], np.zeros(W, dtype=np.int32))
    ef = torch.zeros(W, dtype=torch.float64, device=dev)
    bf.energy(torch.tensor(np.concatenate(pos), device=dev), ef)
    assert bf.tuning()["fused"] == 1
    df = torch.zeros((S, W), dtype=torch.float64, device=dev)
    bf.run_moves(kt, nt, at, df)
    torch.cuda.synchronize()
    e0, dd = e.cpu().numpy(), d.cpu().numpy()
    tol_f = 1e-12 * max(1.0, float(np.max(np.abs(e0)))) if precision == FP64 else 1e-7
    assert np.max(np.abs(df.cpu().numpy() - dd)) <= tol_f
    for w in range(W):
        assert np.array_equal(bf.walker_positions(w), b.walker_positions(w))
        assert bf.walker_header(w)["n_refresh"] == b.walker_header(w)["n_refresh"]
    for w in range(W):
        r = oracle_lib.run(sysm, pos[w], k[:, w], newp[:, w], acc[:, w])
        scale = max(abs(r["energy0"]), e_scale(sysm))
        tol_e = 1e-10 * scale if precision == FP64 else 1e-6 * scale
        tol_d = 1e-10 * scale if precision == FP64 else 1e-5
        assert abs(e0[w] - r["energy0"]) <= tol_e, (e0[w], r["energy0"])
        assert np.max(np.abs(dd[:, w] - r["delta"])) <= tol_d
        # telescoping against a fresh energy of the final positions
        fin = b.walker_positions(w) @ lat
        e_fin = oracle_lib.energy(sysm, *oracle_lib.particles(sysm, fin))["total"]
        tel = e0[w] + float(np.sum(dd[acc[:, w].astype(bool), w]))
        assert abs(tel - e_fin) <= (1e-10 * scale if precision == FP64 else 1e-6 * scale + 1e-5 * S)


# The step call (the previous move's accept folded into the next delta)
# against the two-call sequence move_delta + accept: the same arithmetic in
# the same order, so every output and the whole final state agree bit for bit.
def same_state(a, b, W):
    for w in range(W):
        ha, hb = a.batch.walker_header(w), b.batch.walker_header(w)
        for key in ("counter", "pending_k", "n_accepts", "n_refresh", "drift_max"):
            assert ha[key] == hb[key], (w, key, ha[key], hb[key])
        assert np.array_equal(a.batch.walker_positions(w), b.batch.walker_positions(w)), w
        assert np.array_equal(a.batch.walker_rho(w), b.batch.walker_rho(w)), w


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 2, 3, 4, 5])
def test_step_matches_two_calls(cfg_id, precision):
    W, S, w0 = SUBSETS[cfg_id]
    S = max(S, 12)
    say(f"[step vs two calls] cfg={cfg_id} precision={precision} walkers={W} steps={S}")
    # K = 3: the mixed form rebuilds rho (and recomputes the folded deltas) often
    a = Case(cfg_id, W, S, precision, walker_start=w0, refresh_every=3)
    a.run_energy()
    d1, j1 = a.per_step()
    b = Case(cfg_id, W, S, precision, walker_start=w0, refresh_every=3)
    b.run_energy()
    d2, j2 = b.stepped()
    assert np.array_equal(d1, d2) and np.array_equal(j1, j2)
    same_state(a, b, W)
    if precision == MIXED:
        assert any(a.batch.walker_header(w)["n_refresh"] > 0 for w in range(W))


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [1, 5])
def test_step_vs_oracle(oracle_lib, cfg_id, precision):
    """Step-call deltas and Jastrow deltas against the oracle, telescoped
    energy against a fresh energy of the final positions."""
    W, S, w0 = SUBSETS[cfg_id]
    say(f"[step vs oracle] cfg={cfg_id} precision={precision}")
    c = Case(cfg_id, W, S, precision, walker_start=w0)
    e0, _ = c.run_energy()
    d, dj = c.stepped()
    for w in range(W):
        r = c.oracle(oracle_lib, w)
        scale = max(abs(r["energy0"]), e_scale(c.system(w)))
        if precision == FP64:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-10 * scale
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= 1e-10 * max(1.0, abs(r["j0"]))
        else:
            assert np.max(np.abs(d[:, w] - r["delta"])) <= 1e-5
            assert np.max(np.abs(dj[:, w] - r["djas"])) <= djas_bound(c, w)
        fin = c.batch.walker_positions(w) @ c.system(w).lattice[: c.dim, : c.dim]
        e_fin = oracle_lib.energy(c.system(w), *oracle_lib.particles(c.system(w), fin))["total"]
        tel = e0[w] + float(np.sum(d[c.b.accept[:, w].astype(bool), w]))
        assert abs(tel - e_fin) <= (1e-10 * scale if precision == FP64 else 1e-6 * scale + 1e-5 * S)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("u_term", [False, True], ids=["p", "p+u"])
def test_step_grad_matches_two_calls(precision, u_term):
    """Jastrow gradient and Laplacian outputs of the step call against
    move_delta_grad + accept (and the u term's pair loop with the accepted
    particle taken from the pending record)."""
    cfg_id = 2
    W, S = 2, 12
    say(f"[step grad] precision={precision} u_term={u_term}")
    outs = []
    for path in ("two calls", "step"):
        c = Case(cfg_id, W, S, precision, refresh_every=3, u_term=u_term)
        c.run_energy()
        d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
        lp = torch.zeros_like(d)
        for m in range(S):
            if path == "two calls":
                c.batch.move_delta_grad(c.k[m], c.new_pos[m], d[m], dj[m], g[m], lp[m])
                c.batch.accept(c.accept[m])
            else:
                c.batch.step(c.accept[m - 1] if m else None, c.k[m], c.new_pos[m], d[m], dj[m], g[m], lp[m])
        if path == "step":
            c.batch.accept(c.accept[S - 1])
        torch.cuda.synchronize()
        outs.append((c, [x.cpu().numpy() for x in (d, dj, g, lp)]))
    (a, ra), (b, rb) = outs
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)
    same_state(a, b, W)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_step_bilayer_matches_two_calls(precision):
    """Layered system: an accepted move in either plane folded into a delta
    of a particle in the same or the other plane."""
    say(f"[step bilayer] precision={precision}")
    base = wl.bilayer(6, 2.2)
    sysm = dataclasses.replace(base, n_mobile=9, mobile_q=np.array([-1.0] * 5 + [1.0] * 4),
                               mobile_layer=np.array([0] * 5 + [1] * 4, dtype=np.int32),
                               fixed_pos=np.array([[3.0, 4.0], [40.0, 17.0]]), fixed_q=np.array([1.0, -0.5]),
                               fixed_layer=np.array([1, 0], dtype=np.int32))
    rng = np.random.default_rng(78)
    lat = sysm.lattice[:2, :2]
    W, S = 3, 24
    pos = np.concatenate([rng.random((9, 2)) @ lat for _ in range(W)])
    k = rng.integers(0, 9, (S, W)).astype(np.int32)
    newp = rng.random((S, W, 2)) @ lat
    acc = (rng.random((S, W)) < 0.6).astype(np.uint8)
    dev = "cuda"
    kt, nt, at = (torch.tensor(x, device=dev) for x in (k, newp, acc))
    h = ew.System(sysm, precision=precision, refresh_every=2 if precision == MIXED else 0)
    res = []
    for path in ("two calls", "step"):
        b = ew.Batch([h], np.zeros(W, dtype=np.int32))
        b.energy(torch.tensor(pos, device=dev), torch.zeros(W, dtype=torch.float64, device=dev))
        d = torch.zeros((S, W), dtype=torch.float64, device=dev)
        for m in range(S):
            if path == "two calls":
                b.move_delta(kt[m], nt[m], d[m])
                b.accept(at[m])
            else:
                b.step(at[m - 1] if m else None, kt[m], nt[m], d[m])
        if path == "step":
            b.accept(at[S - 1])
        torch.cuda.synchronize()
        res.append((b, d.cpu().numpy()))
    (ba, da), (bb, db) = res
    assert np.array_equal(da, db)
    for w in range(W):
        assert np.array_equal(ba.walker_positions(w), bb.walker_positions(w))
        for plane in (0, 1):
            assert np.array_equal(ba.walker_rho(w, plane), bb.walker_rho(w, plane))
        ha, hb = ba.walker_header(w), bb.walker_header(w)
        assert all(np.array_equal(ha[x], hb[x]) for x in ha), (ha, hb)


def test_step_invalid_k_still_applies_accept():
    """A step whose new move has an invalid particle index gives NaN for it
    but still applies the previous move's accept (as accept + move_delta)."""
    say("[step invalid k]")
    res = []
    for path in ("two calls", "step"):
        c = Case(2, 3, 2, FP64)
        c.run_energy()
        d = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
        ones = torch.ones(3, dtype=torch.uint8, device="cuda")
        bad = torch.tensor([-1, 1, 250], dtype=torch.int32, device="cuda")
        if path == "two calls":
            c.batch.move_delta(c.k[0], c.new_pos[0], d[0])
            c.batch.accept(ones)
            c.batch.move_delta(bad, c.new_pos[1], d[1])
        else:
            c.batch.step(None, c.k[0], c.new_pos[0], d[0])
            c.batch.step(ones, bad, c.new_pos[1], d[1])
        c.batch.accept(ones)
        torch.cuda.synchronize()
        res.append((c, d.cpu().numpy()))
    (a, da), (b, db) = res
    assert np.isnan(db[1, 0]) and np.isfinite(db[1, 1]) and np.isnan(db[1, 2])
    assert np.array_equal(da, db, equal_nan=True)
    same_state(a, b, 3)
    assert b.batch.walker_header(0)["n_accepts"] == 1 and b.batch.walker_header(1)["n_accepts"] == 2


def test_step_call_order():
    say("[step call order]")
    c = Case(1, 1, 3, FP64)
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(ew.EwaldError) as e:
        c.batch.step(None, c.k[0], c.new_pos[0], d)
    assert e.value.status == ew.EWALD_E_STATE
    c.run_energy()
    with pytest.raises(ew.EwaldError) as e:  # nothing pending to accept
        c.batch.step(c.accept[0], c.k[0], c.new_pos[0], d)
    assert e.value.status == ew.EWALD_E_STATE
    c.batch.step(None, c.k[0], c.new_pos[0], d)
    c.batch.step(c.accept[0], c.k[1], c.new_pos[1], d)
    with pytest.raises(ew.EwaldError) as e:  # a move is pending
        c.fused(1)
    assert e.value.status == ew.EWALD_E_STATE
    c.batch.accept(c.accept[1])
    c.fused(1)


def test_empty_inputs():
    """Degenerate sizes through the C ABI: a sweep of zero moves is a no-op
    (state byte for byte as before, outputs untouched), so is a blip
    evaluation at zero points; a negative move or point count and a batch of
    no walkers are rejected with E_ARG."""
    say("[empty inputs]")
    c = Case(2, 3, 2, FP64)
    c.run_energy()
    before = c.batch.state.clone()
    d = torch.full((1, 3), 7.0, dtype=torch.float64, device="cuda")
    args = (c.k.data_ptr(), c.new_pos.data_ptr(), c.accept.data_ptr(), d.data_ptr())
    ew.ewald_run_moves_batch(c.batch.handle, c.batch.state.data_ptr(), 0, *args)
    torch.cuda.synchronize()
    assert torch.equal(c.batch.state, before) and bool((d == 7.0).all())
    with pytest.raises(ew.EwaldError) as e:
        ew.ewald_run_moves_batch(c.batch.handle, c.batch.state.data_ptr(), -1, *args)
    assert e.value.status == ew.EWALD_E_ARG
    with pytest.raises(ew.EwaldError) as e:
        ew.ewald_batch_create([c.systems[0].handle], np.zeros(0, dtype=np.int32))
    assert e.value.status == ew.EWALD_E_ARG
    bl = ew.Blips(SKEW, (4, 4, 4), 2)
    coef = torch.ones((4, 4, 4, 2), dtype=torch.float64, device="cuda")
    pos = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    val = torch.full((1, 2), 7.0, dtype=torch.float64, device="cuda")
    ew.ewald_blip_eval_batch(bl.handle, coef.data_ptr(), 0, pos.data_ptr(), val.data_ptr())
    torch.cuda.synchronize()
    assert bool((val == 7.0).all())
    with pytest.raises(ew.EwaldError) as e:
        ew.ewald_blip_eval_batch(bl.handle, coef.data_ptr(), -1, pos.data_ptr(), val.data_ptr())
    assert e.value.status == ew.EWALD_E_ARG
    bl.close()


def test_call_timers():
    """Per-call timers: invocation counts per call name, GPU times from event
    pairs around the enqueued work (positive, and within the wall time of the
    calls), nothing recorded on the GPU for a call made during graph capture,
    and reset."""
    say("[timers]")
    ew.ewald_timing_report(reset=True)
    ew.ewald_timing_enable(True)
    try:
        c = Case(2, 4, 6, FP64)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        c.run_energy()
        d = torch.zeros((6, 4), dtype=torch.float64, device="cuda")
        for m in range(2):
            c.batch.move_delta(c.k[m], c.new_pos[m], d[m])
            c.batch.accept(c.accept[m])
        for m in range(2, 5):
            c.batch.step(c.accept[m - 1] if m > 2 else None, c.k[m], c.new_pos[m], d[m])
        c.batch.accept(c.accept[4])
        t1.record()
        torch.cuda.synchronize()
        wall = t0.elapsed_time(t1)
        rep = ew.ewald_timing_report()
        assert rep["ewald_energy_batch"]["calls"] == 1
        assert rep["ewald_move_delta_batch"]["calls"] == 2
        assert rep["ewald_accept_batch"]["calls"] == 3
        assert rep["ewald_step_batch"]["calls"] == 3
        for name, r in rep.items():
            assert r["gpu_calls"] == r["calls"], name
            assert r["gpu_ms_total"] > 0.0 and r["host_ms_total"] >= 0.0, name
        assert sum(r["gpu_ms_total"] for r in rep.values()) <= wall * 1.01 + 0.05
        # a call captured into a graph is counted without GPU events
        k_buf, np_buf, d_buf = c.k[5].clone(), c.new_pos[5].clone(), torch.zeros(4, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            c.batch.move_delta(k_buf, np_buf, d_buf)
        torch.cuda.synchronize()
        rep = ew.ewald_timing_report(reset=True)
        assert rep["ewald_move_delta_batch"]["calls"] == 3 and rep["ewald_move_delta_batch"]["gpu_calls"] == 2
        assert ew.ewald_timing_report() == {}
    finally:
        ew.ewald_timing_enable(False)
        ew.ewald_timing_report(reset=True)


# Queue mode of the fused sweep (walkers_per_block > 0: fewer workgroups than
# walkers, each taking the next walker from a work counter): every walker is
# computed as with one workgroup per walker, so outputs and states agree bit
# for bit.
@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("cfg_id", [2, 4, 5])
def test_queue_mode_matches_one_walker_per_workgroup(cfg_id, precision):
    W, S = {2: (9, 12), 4: (12, 12), 5: (3, 8)}[cfg_id]
    say(f"[queue] cfg={cfg_id} precision={precision} walkers={W}")
    ref = Case(cfg_id, W, S, precision, refresh_every=3)
    ref.run_energy()
    d0, j0 = ref.fused()
    for wpb in (1, 4, W):
        c = Case(cfg_id, W, S, precision, refresh_every=3)
        c.run_energy()
        c.batch.set_tuning(walkers_per_block=wpb)
        t = c.batch.tuning()
        assert t["walkers_per_block"] == wpb and t["fused"] == 1
        d, j = c.fused()
        assert np.array_equal(d, d0) and np.array_equal(j, j0), wpb
        same_state(ref, c, W)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_queue_mode_graph_replay(precision):
    """The counter reset is a kernel, so a captured queue-mode sweep replays
    correctly: three replays equal three eager sweeps."""
    W, S = 10, 8
    say(f"[queue graph] cfg=4 precision={precision}")
    eager = Case(4, W, S, precision, refresh_every=3)
    eager.run_energy()
    eager.batch.set_tuning(walkers_per_block=3)
    ref = [eager.fused() for _ in range(3)]
    g_case = Case(4, W, S, precision, refresh_every=3)
    g_case.run_energy()
    g_case.batch.set_tuning(walkers_per_block=3)
    d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
    dj = torch.zeros_like(d)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        g_case.batch.run_moves(g_case.k, g_case.new_pos, g_case.accept, d, dj)
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), ref[r][0]), r
        assert np.array_equal(dj.cpu().numpy(), ref[r][1]), r
    same_state(eager, g_case, W)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_queue_mode_derivs_u_term(precision):
    """Queue mode with the Jastrow derivative outputs and the u term."""
    W, S = 5, 8
    say(f"[queue derivs] cfg=2 precision={precision}")
    outs = []
    for wpb in (0, 2):
        c = Case(2, W, S, precision, refresh_every=3, u_term=True)
        c.run_energy()
        c.batch.set_tuning(walkers_per_block=wpb)
        d = torch.zeros((S, W), dtype=torch.float64, device="cuda")
        dj = torch.zeros_like(d)
        g = torch.zeros((S, W, c.dim), dtype=torch.float64, device="cuda")
        lp = torch.zeros_like(d)
        c.batch.run_moves_grad(c.k, c.new_pos, c.accept, d, dj, g, lp)
        torch.cuda.synchronize()
        outs.append((c, [x.cpu().numpy() for x in (d, dj, g, lp)]))
    for x, y in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(x, y)
    same_state(outs[0][0], outs[1][0], W)


def test_queue_mode_arguments_and_autotune():
    """walkers_per_block < 0 is an argument error; with more walkers than
    workgroups fit at once the autotuner times the queue mode too, and the
    tuned sweep equals one workgroup per walker."""
    say("[queue autotune] cfg=3 fp64")
    c = Case(3, 1100, 6, FP64)
    with pytest.raises(ew.EwaldError) as e:
        c.batch.set_tuning(walkers_per_block=-1)
    assert e.value.status == ew.EWALD_E_ARG
    with pytest.raises(ew.EwaldError) as e:  # the queue kernels are compiled for two waves per SIMD
        c.batch.set_tuning(threads=256, waves=4, walkers_per_block=2)
    assert e.value.status == ew.EWALD_E_ARG
    c.run_energy()
    c.batch.autotune(n_moves=6)
    t = c.batch.tuning()
    assert t["fused"] == 1 and t["walkers_per_block"] >= 0
    d1, j1 = c.fused()
    ref = Case(3, 1100, 6, FP64)
    ref.run_energy()
    ref.batch.set_tuning(**{k: v for k, v in t.items() if k not in ("fused", "walkers_per_block")})
    d0, j0 = ref.fused()
    assert np.array_equal(d0, d1) and np.array_equal(j0, j1)
