"""Pins of the FP64 oracle against what the mathematics fixes.

Every check here is independent of the oracle's own formulas: literature
Madelung energies, the exact independence of the converged energy from the
Ewald split parameter, invariances of the periodic energy (translation,
permutation, lattice-basis choice, scaling), and exact identities of the
single-particle move (incremental delta versus a full recompute, telescoping).
tests/test_oracle_mutations.py shows that plausible mistakes planted in a copy
of the oracle make these checks fail.
"""
import math
import os

import numpy as np
import pytest

from paper_2507_02888_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "madelung.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, dim, val, tol = line.split()
        out[name] = (int(dim), float(val), float(tol))
    return out


def converged(system, alpha_times_l=5.0):
    """Cutoffs at which both truncations are far below 1e-15."""
    L = system.length
    a = alpha_times_l / L
    return dict(alpha=a, r_cut=7.0 / a, g_cut=14.0 * a)


def one_charge(lattice, dim):
    return wl.System("w", dim, lattice, 1, -np.ones(1), np.zeros((0, dim)), np.zeros(0), 1, 1, 1)


CELLS_3D = {
    "sc": lambda v: wl.sc_cell(v),
    "fcc": lambda v: wl.fcc_cell(v),
    "bcc": lambda v: wl.bcc_cell(v),
}


def square_cell(area):
    m = np.eye(3)
    m[0, 0] = m[1, 1] = math.sqrt(area)
    return m


CELLS_2D = {"triangular": wl.hex_cell, "square": square_cell}


@pytest.mark.parametrize("name", ["sc", "fcc", "bcc"])
@pytest.mark.parametrize("rs", [1.0, 2.5])
def test_wigner_3d(oracle_lib, name, rs):
    dim, ref, tol = golden()[name]
    s = one_charge(CELLS_3D[name](4.0 / 3.0 * math.pi * rs ** 3), 3)
    for f in (4.0, 5.5):
        e = oracle_lib.energy(s, np.zeros((1, 3)), -np.ones(1), **converged(s, f))
        assert abs(e["total"] * rs - ref) <= tol * abs(ref)


@pytest.mark.parametrize("name", ["triangular", "square"])
def test_wigner_2d(oracle_lib, name):
    dim, ref, tol = golden()[name]
    rs = 1.7
    s = one_charge(CELLS_2D[name](math.pi * rs ** 2), 2)
    for f in (4.0, 5.5):
        e = oracle_lib.energy(s, np.zeros((1, 2)), -np.ones(1), **converged(s, f))
        assert abs(e["total"] * rs - ref) <= tol * abs(ref)


def nacl(r0=1.3):
    a = 2.0 * r0
    na = np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float) * a / 2
    cl = na + np.array([a / 2, 0, 0])
    pos = np.concatenate([na, cl])
    q = np.array([1.0] * 4 + [-1.0] * 4)
    s = wl.System("nacl", 3, a * np.eye(3), 8, q, np.zeros((0, 3)), np.zeros(0), 1, 1, 1)
    return s, pos, q


def test_nacl_madelung(oracle_lib):
    _, ref, tol = golden()["nacl"]
    r0 = 1.3
    s, pos, q = nacl(r0)
    e = oracle_lib.energy(s, pos, q, **converged(s))
    # four formula units: E = -4 M / r0
    m = -e["total"] * r0 / 4.0
    assert abs(m - ref) <= tol * ref
    # the reciprocal and real parts individually depend on alpha; the sum must not
    e2 = oracle_lib.energy(s, pos, q, **converged(s, 3.5))
    assert abs(e2["recip"] - e["recip"]) > 1e-3
    assert abs(e2["total"] - e["total"]) <= 1e-12 * abs(e["total"])


def random_system(dim, skew, n, seed, neutral):
    if dim == 3:
        lat = np.array([[5.0, 0.3, -0.2], [1.1, 4.6, 0.4], [-0.7, 0.9, 5.3]]) if skew else 5.0 * np.eye(3)
    else:
        lat = np.array([[5.0, 0.0, 0.0], [1.7, 4.4, 0.0], [0.0, 0.0, 1.0]]) if skew else square_cell(25.0)
    g = np.random.default_rng(seed)
    q = g.choice([-1.0, 1.0, 2.0], size=n)
    if neutral:
        q[-1] -= q.sum()
    pos = g.random((n, dim)) @ lat[:dim, :dim]
    s = wl.System("r", dim, lat, n, q, np.zeros((0, dim)), np.zeros(0), 1, 1, 1)
    return s, pos, q


@pytest.mark.parametrize("dim,skew,neutral", [(3, False, True), (3, True, True), (3, True, False),
                                               (2, False, True), (2, True, False)])
def test_alpha_independence(oracle_lib, dim, skew, neutral):
    s, pos, q = random_system(dim, skew, 12, 7, neutral)
    es = [oracle_lib.energy(s, pos, q, **converged(s, f))["total"] for f in (3.5, 5.0, 7.0)]
    scale = max(abs(es[0]), (np.sum(q * q)) / s.length)
    for e in es[1:]:
        assert abs(e - es[0]) <= 1e-10 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_translation_and_lattice_shift(oracle_lib, dim):
    s, pos, q = random_system(dim, True, 10, 3, True)
    kw = converged(s)
    e0 = oracle_lib.energy(s, pos, q, **kw)["total"]
    g = np.random.default_rng(5)
    shifted = pos + g.normal(size=dim) * 3.0
    assert abs(oracle_lib.energy(s, shifted, q, **kw)["total"] - e0) <= 1e-12 * abs(e0) * 10
    # moving single particles by lattice vectors changes nothing
    lat = s.lattice[:dim, :dim]
    moved = pos.copy()
    moved[0] += lat[0] - 2 * lat[dim - 1]
    moved[3] -= lat[1]
    assert abs(oracle_lib.energy(s, moved, q, **kw)["total"] - e0) <= 1e-12 * abs(e0) * 10
    # the truncated model (r_cut below the inscribed radius) is invariant too
    kt = dict(alpha=5.0 / s.length, r_cut=0.45 * s.length, g_cut=8 * 2 * math.pi / s.length)
    et = oracle_lib.energy(s, pos, q, **kt)["total"]
    assert abs(oracle_lib.energy(s, moved + lat[0] * 0.0 + (shifted - pos), q, **kt)["total"] - et) <= 1e-11 * abs(et)


def test_permutation_invariance(oracle_lib):
    s, pos, q = random_system(3, True, 11, 4, False)
    kw = converged(s)
    e0 = oracle_lib.energy(s, pos, q, **kw)["total"]
    p = np.random.default_rng(1).permutation(11)
    assert abs(oracle_lib.energy(s, pos[p], q[p], **kw)["total"] - e0) <= 1e-12 * abs(e0) * 10


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_basis_invariance(oracle_lib, dim):
    """The same lattice described by another basis gives the same energy."""
    s, pos, q = random_system(dim, True, 9, 8, True)
    kw = converged(s)
    e0 = oracle_lib.energy(s, pos, q, **kw)["total"]
    # a unimodular integer change of basis
    m = np.array([[1, 2, 0], [1, 3, 0], [1, 0, 1]], dtype=float) if dim == 3 else \
        np.array([[1, 2, 0], [1, 3, 0], [0, 0, 1]], dtype=float)
    lat2 = m @ s.lattice
    s2 = wl.System("b", dim, lat2, 9, q, np.zeros((0, dim)), np.zeros(0), 1, 1, 1)
    assert abs(abs(np.linalg.det(lat2[:dim, :dim])) - s.measure) < 1e-9
    e2 = oracle_lib.energy(s2, pos, q, **kw)["total"]
    assert abs(e2 - e0) <= 1e-11 * abs(e0)


@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneity(oracle_lib, dim):
    s, pos, q = random_system(dim, True, 8, 2, True)
    kw = converged(s)
    e0 = oracle_lib.energy(s, pos, q, **kw)["total"]
    lam = 1.7
    s2 = wl.System("h", dim, s.lattice * lam, 8, q, np.zeros((0, dim)), np.zeros(0), 1, 1, 1)
    kw2 = dict(alpha=kw["alpha"] / lam, r_cut=kw["r_cut"] * lam, g_cut=kw["g_cut"] / lam)
    if dim == 2:
        s2.lattice[2, 2] = 1.0
    e2 = oracle_lib.energy(s2, pos * lam, q, **kw2)["total"]
    assert abs(e2 - e0 / lam) <= 1e-11 * abs(e0)


@pytest.mark.parametrize("cfg_id", [1, 3, 4])
def test_incremental_moves_match_recompute(oracle_lib, cfg_id):
    """dE from the incremental update equals E(R') - E(R), and the accepted
    deltas telescope to the final energy (truncated-model cutoffs)."""
    cfg = wl.config(cfg_id)
    # the smallest system of the workload (for the uneven batch: the 2x2x2 cell)
    first = 0
    if len(cfg.systems) > 1:
        wsys = wl.make_batch(cfg, walkers=64, moves=0).walker_sys
        first = int(np.nonzero(wsys == 0)[0][0])
    b = wl.make_batch(cfg, walkers=1, moves=12, walker_start=first)
    sysm = cfg.systems[int(b.walker_sys[0])]
    ja = np.random.default_rng(3).uniform(-0.01, 0.01, 40)
    r = oracle_lib.run(sysm, b.walker_pos(0), b.k[:, 0], b.new_pos[:, 0], b.accept[:, 0], jastrow_a=ja)
    cur = b.walker_pos(0).copy()
    e_cur = oracle_lib.energy(sysm, *oracle_lib.particles(sysm, cur), jastrow_a=ja)
    scale = max(abs(e_cur["total"]), sysm.alpha / math.sqrt(math.pi) * float(np.sum(oracle_lib.particles(sysm, cur)[1] ** 2)))
    assert abs(e_cur["total"] - r["energy0"]) <= 1e-12 * scale
    for m in range(b.steps):
        k = int(b.k[m, 0])
        prop = cur.copy()
        prop[k] = b.new_pos[m, 0]
        e_new = oracle_lib.energy(sysm, *oracle_lib.particles(sysm, prop), jastrow_a=ja)
        assert abs((e_new["total"] - e_cur["total"]) - r["delta"][m]) <= 1e-10 * scale
        assert abs((e_new["jastrow"] - e_cur["jastrow"]) - r["djas"][m]) <= 1e-10 * max(1.0, abs(e_cur["jastrow"]))
        if b.accept[m, 0]:
            cur, e_cur = prop, e_new
    acc = b.accept[:, 0].astype(bool)
    assert abs(r["energy0"] + r["delta"][acc].sum() - e_cur["total"]) <= 1e-10 * scale
    assert np.allclose(r["pos_final"], cur, atol=0, rtol=0)


def test_jastrow_structure_factor_equals_pair_form(oracle_lib):
    """sum_H a_s |rho|^2 = N sum_H a_s + 2 sum_{i<j} p(r_ij) with the paper's
    plane-wave pair function p(r) = sum_s a_s sum_{G in star s, half} cos(G.r)
    for unit charges; p is evaluated here by direct pair sums."""
    cfg = wl.config(1)
    s = cfg.systems[0]
    pos = wl.random_positions(s, 15, 0)
    q = -np.ones(15)
    ja = np.random.default_rng(9).uniform(-0.01, 0.01, 60)
    j = oracle_lib.energy(s, pos, q, jastrow_a=ja)["jastrow"]
    g, g2, shell = oracle_lib.gvectors(s)
    a = np.where(shell < len(ja), ja[np.minimum(shell, len(ja) - 1)], 0.0)
    pair = 0.0
    for i in range(15):
        for k in range(i + 1, 15):
            pair += 0.5 * np.sum(a * np.cos(g @ (pos[i] - pos[k])))  # full set: half of it
    n_sum_half = 0.5 * np.sum(a) * 15
    assert abs(j - (n_sum_half + 2 * pair)) <= 1e-10 * max(1.0, abs(j))


@pytest.mark.parametrize("cfg_id,n_full,n_shells", [(1, 2108, 54), (2, 2108, 54), (3, 198, 21), (5, 7154, 106)])
def test_g_counts(oracle_lib, cfg_id, n_full, n_shells):
    """Counts of the reciprocal lattice points of the five workloads, checked
    against the continuum estimate (4/3 pi G_c^3)/(2pi)^3 * Omega (2D: area)."""
    s = wl.config(cfg_id).systems[0]
    n, sh = oracle_lib.count_g(s)
    assert (n, sh) == (n_full, n_shells)
    if s.dim == 3:
        est = 4.0 / 3.0 * math.pi * s.g_cut ** 3 * s.measure / (2 * math.pi) ** 3
    else:
        est = math.pi * s.g_cut ** 2 * s.measure / (2 * math.pi) ** 2
    assert abs(n - est) < 0.05 * est
    g, g2, shell = oracle_lib.gvectors(s)
    assert np.all(g2 <= s.g_cut ** 2 * (1 + 1e-12))
    # closed under G -> -G
    keys = {tuple(np.round(v, 9)) for v in g}
    assert all(tuple(np.round(-v, 9)) in keys for v in g)


def test_cutoff_shells(oracle_lib):
    """Moving r_cut across one shell of images of a simple-cubic Wigner lattice
    removes exactly that shell: 12 second neighbours at sqrt(2) L and 8 third
    neighbours at sqrt(3) L, each weighted 1/2 erfc(alpha R)/R."""
    L = 3.0
    s = one_charge(wl.sc_cell(L ** 3), 3)
    a = 1.1 / L
    kw = dict(alpha=a, g_cut=14.0 * a)
    e = {rc: oracle_lib.energy(s, np.zeros((1, 3)), -np.ones(1), r_cut=rc * L, **kw)["total"]
         for rc in (1.2, 1.5, 1.8)}
    r2, r3 = math.sqrt(2.0) * L, math.sqrt(3.0) * L
    assert abs((e[1.5] - e[1.2]) - 6.0 * math.erfc(a * r2) / r2) <= 1e-13
    assert abs((e[1.8] - e[1.5]) - 4.0 * math.erfc(a * r3) / r3) <= 1e-13


SHELLS = os.path.join(os.path.dirname(__file__), "golden", "lattice_shells.txt")


def shell_table(dim):
    out = []
    for line in open(SHELLS):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        d, m, r = (int(x) for x in line.split())
        if d == dim:
            out.append((m, r))
    return out


def count_sums_of_squares(m, dim):
    """Brute force: integer vectors of `dim` components with squared norm m."""
    n = int(math.isqrt(m)) + 1
    rng_ = range(-n, n + 1)
    if dim == 2:
        return sum(1 for a in rng_ for b in rng_ if a * a + b * b == m)
    return sum(1 for a in rng_ for b in rng_ for c in rng_ if a * a + b * b + c * c == m)


def test_shell_golden_values_are_sums_of_squares():
    """The golden shell populations equal a direct count of lattice vectors."""
    for dim in (2, 3):
        for m, r in shell_table(dim):
            assert count_sums_of_squares(m, dim) == r


@pytest.mark.parametrize("dim", [3, 2])
def test_jastrow_shells_cubic(oracle_lib, dim):
    """Shell index s(G) behind J = sum_H a_s(G) |rho(G)|^2 (Sec. 2.3, Eq. (9)):
    one unit charge in a simple-cubic (square) cell has |rho(G)|^2 = 1 for every
    G, so J with a = e_s (one shell switched on) counts the half set of shell s,
    which holds r_dim(m_s)/2 vectors with |G|^2 = (2 pi/L)^2 m_s; m_s runs over
    the representable norms in ascending order (tests/golden/lattice_shells.txt)."""
    L = 6.0
    lat = L * np.eye(3) if dim == 3 else square_cell(L * L)
    s = one_charge(lat, dim)
    kw = dict(alpha=5.0 / L, r_cut=0.5 * L, g_cut=8.0 * 2 * math.pi / L)
    pos = np.full((1, dim), 0.37)
    table = shell_table(dim)
    for idx, (m, r) in enumerate(table):
        a = np.zeros(len(table) + 5)
        a[idx] = 1.0
        j = oracle_lib.energy(s, pos, -np.ones(1), jastrow_a=a, **kw)["jastrow"]
        assert abs(j - r / 2.0) <= 1e-9, (dim, idx, m, j, r / 2.0)
    # and the shells carry exactly those norms
    g, g2, shell = oracle_lib.gvectors(s, **kw)
    unit = (2 * math.pi / L) ** 2
    for idx, (m, r) in enumerate(table):
        sel = shell == idx
        assert int(sel.sum()) == r
        assert np.allclose(g2[sel] / unit, m, rtol=1e-12, atol=0)


@pytest.mark.parametrize("cfg_id", [1, 3, 5])
def test_shell_index_order(oracle_lib, cfg_id):
    """s(G) is nondecreasing in |G|^2, equal exactly when |G|^2 is equal (to the
    1e-9 relative tolerance that defines a shell), and starts at 0."""
    s = wl.config(cfg_id).systems[0]
    g, g2, shell = oracle_lib.gvectors(s)
    o = np.argsort(g2, kind="stable")
    g2s, shs = g2[o], shell[o]
    assert shs[0] == 0
    steps = np.diff(shs)
    assert np.all((steps == 0) | (steps == 1))
    same = np.abs(np.diff(g2s)) <= 1e-9 * g2s[1:]
    assert np.array_equal(steps == 0, same)


@pytest.mark.parametrize("cfg_id", [2, 3])
def test_run_batch_matches_run(oracle_lib, cfg_id):
    """The OpenMP batch driver gives, walker by walker, exactly the single-walker
    results: it only regroups the [S][W] inputs and outputs."""
    cfg = wl.config(cfg_id)
    b = wl.make_batch(cfg, walkers=3, moves=5)
    s = cfg.systems[0]
    ja = np.random.default_rng(4).uniform(-0.01, 0.01, 40)
    pos = b.pos.reshape(3, s.n_mobile, s.dim)
    r = oracle_lib.run_batch(s, pos, b.k, b.new_pos, b.accept, jastrow_a=ja, n_threads=2)
    for w in range(3):
        one = oracle_lib.run(s, b.walker_pos(w), b.k[:, w], b.new_pos[:, w], b.accept[:, w], jastrow_a=ja)
        assert np.array_equal(r["e0"][w], one["e0"])
        assert r["j0"][w] == one["j0"]
        assert np.array_equal(r["delta"][:, w], one["delta"])
        assert np.array_equal(r["djas"][:, w], one["djas"])


def jastrow_system(dim, n, seed):
    """A small cell (the 54-electron cubic cell of the workloads, or the 2D
    hexagonal one) with mixed charges and seeded Jastrow coefficients."""
    s = wl.config(1 if dim == 3 else 3).systems[0]
    g = np.random.default_rng([31, dim, seed])
    pos = wl.random_positions(s, n, seed)
    q = np.where(np.arange(n) % 4 == 3, 2.0, -1.0)
    ja = g.uniform(-0.01, 0.01, 60)
    return s, pos, q, ja


@pytest.mark.parametrize("dim", [3, 2])
def test_jastrow_derivs_finite_differences(oracle_lib, dim):
    """grad_k J and lap_k J (pair form) against central differences of the
    oracle's J value (itself pinned by the pair-form identity and the shell
    populations): fourth-order stencils, h = 1e-3 bohr."""
    s, pos, q, ja = jastrow_system(dim, 10, 1)
    h = 1e-3

    def J(p):
        return oracle_lib.energy(s, p, q, jastrow_a=ja)["jastrow"]

    for k in (0, 3, 7):
        grad, lap = oracle_lib.jastrow_derivs(s, pos, q, k, ja)
        j0 = J(pos)
        fd_grad = np.zeros(dim)
        fd_lap = 0.0
        for d in range(dim):
            f = {}
            for m in (-2, -1, 1, 2):
                p = pos.copy()
                p[k, d] += m * h
                f[m] = J(p)
            fd_grad[d] = (f[-2] - 8 * f[-1] + 8 * f[1] - f[2]) / (12 * h)
            fd_lap += (-f[-2] + 16 * f[-1] - 30 * j0 + 16 * f[1] - f[2]) / (12 * h * h)
        scale = max(1.0, float(np.max(np.abs(grad))), abs(lap))
        assert np.max(np.abs(grad - fd_grad)) <= 1e-8 * scale, (k, grad, fd_grad)
        assert abs(lap - fd_lap) <= 1e-6 * scale, (k, lap, fd_lap)


@pytest.mark.parametrize("dim", [3, 2])
def test_jastrow_derivs_structure_factor_form(oracle_lib, dim):
    """The pair-form derivatives equal the structure-factor form
    grad_k J = -q_k sum_G a G Im(conj(rho) e_k), lap_k J = -q_k sum_G a |G|^2
    (Re(conj(rho) e_k) - q_k) over the full G set, e_k = exp(i G.r_k), and the
    gradients of all particles sum to zero (translation invariance)."""
    s, pos, q, ja = jastrow_system(dim, 9, 2)
    g, g2, shell = oracle_lib.gvectors(s)
    a = np.where(shell < len(ja), ja[np.minimum(shell, len(ja) - 1)], 0.0)
    pos3 = np.zeros((pos.shape[0], 3))
    pos3[:, :dim] = pos
    rho = oracle_lib.rho_at(s, pos, q, g)
    total = np.zeros(dim)
    for k in range(pos.shape[0]):
        grad, lap = oracle_lib.jastrow_derivs(s, pos, q, k, ja)
        ek = np.exp(1j * (g @ pos3[k]))
        z = np.conj(rho) * ek
        sf_grad = -q[k] * (a * z.imag) @ g[:, :dim]
        sf_lap = -q[k] * np.sum(a * g2 * (z.real - q[k]))
        scale = max(1.0, float(np.max(np.abs(sf_grad))), abs(sf_lap))
        assert np.max(np.abs(grad - sf_grad)) <= 1e-11 * scale
        assert abs(lap - sf_lap) <= 1e-11 * scale
        total += grad
    assert np.max(np.abs(total)) <= 1e-11 * max(1.0, scale)


def test_run_derivs_at_proposed_configuration(oracle_lib):
    """The move driver's derivative outputs are those of the proposed
    configuration (moved particle at its proposal), accepted or not."""
    cfg = wl.config(1)
    b = wl.make_batch(cfg, walkers=1, moves=6)
    s = cfg.systems[0]
    acc = np.array([1, 0, 1, 0, 0, 1], dtype=np.uint8)
    ja = np.random.default_rng(12).uniform(-0.01, 0.01, 50)
    r = oracle_lib.run(s, b.walker_pos(0), b.k[:, 0], b.new_pos[:, 0], acc, jastrow_a=ja, derivs=True)
    cur = b.walker_pos(0).copy()
    for m in range(6):
        k = int(b.k[m, 0])
        prop = cur.copy()
        prop[k] = b.new_pos[m, 0]
        grad, lap = oracle_lib.jastrow_derivs(s, *oracle_lib.particles(s, prop), k, ja)
        assert np.array_equal(r["jgrad"][m], grad) and r["jlap"][m] == lap
        if acc[m]:
            cur = prop
