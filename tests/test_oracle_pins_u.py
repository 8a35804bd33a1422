"""Pins of the oracle's Jastrow two-body polynomial term u (Sec. 2.3, Eq. (8)):

  u_c(r) = sum_l alpha_{c,l} r^l (r - L_u)^C for r < L_u,   U = sum_{i<j} u_c(r_ij),

checked against what the mathematics fixes rather than against the oracle's
own formula: hand-evaluated values at simple distances (sign convention of
(r - L_u)^C, the power index l, the spin channel, ions taking no part), the
Kato cusp the seeded coefficients are built to satisfy (an independent
relation between alpha_0, alpha_1, C and L_u), the order-C zero at the cutoff,
fourth-order finite differences for the gradient and Laplacian, minimum-image
and translation invariance, and incremental move deltas against recomputes.
tests/test_oracle_mutations.py plants mistakes in the u code and checks that
these catch them.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2507_02888_amd import workloads as wl


def big_cube(n_mobile, L=10.0, fixed_pos=None, fixed_q=None):
    """A simple-cubic cell of edge L (inscribed radius L/2) whose Ewald
    cutoffs are irrelevant here (only the Jastrow value is read)."""
    fp = np.zeros((0, 3)) if fixed_pos is None else np.asarray(fixed_pos, dtype=float)
    fq = np.zeros(0) if fixed_q is None else np.asarray(fixed_q, dtype=float)
    return wl.System("cube", 3, L * np.eye(3), n_mobile, -np.ones(n_mobile), fp, fq, 5.0 / L, 0.5 * L,
                     4 * 2 * math.pi / L)


def with_u(system, alpha, C, Lu, spin):
    return dataclasses.replace(system, u_alpha=np.asarray(alpha, dtype=float).reshape(2, -1), u_C=C, u_cut=Lu,
                               mobile_spin=np.asarray(spin, dtype=np.int32))


def U(oracle_lib, s, pos):
    p, q = oracle_lib.particles(s, pos)
    return oracle_lib.energy(s, p, q)["jastrow"]


def test_u_closed_form_values(oracle_lib):
    """Hand-evaluated values: (r - L_u)^C with C = 3 is negative inside the
    cutoff; alpha_l multiplies r^l; channel 0 serves equal spin labels and
    channel 1 unequal ones; nothing beyond L_u."""
    base = big_cube(2)
    two = lambda r: np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]])
    z = np.zeros(5)
    # alpha_{0,0} = 1, L_u = 2, C = 3: u(1) = (1 - 2)^3 = -1, u(0.5) = -3.375
    s = with_u(base, np.concatenate([[1.0, 0, 0, 0, 0], z]), 3, 2.0, [0, 0])
    assert U(oracle_lib, s, two(1.0)) == pytest.approx(-1.0, abs=1e-14)
    assert U(oracle_lib, s, two(0.5)) == pytest.approx(-3.375, abs=1e-14)
    assert U(oracle_lib, s, two(2.5)) == 0.0
    # alpha_{0,2} = 1: u(0.5) = 0.25 (0.5 - 2)^3 = -0.84375
    s = with_u(base, np.concatenate([[0, 0, 1.0, 0, 0], z]), 3, 2.0, [0, 0])
    assert U(oracle_lib, s, two(0.5)) == pytest.approx(-0.84375, abs=1e-14)
    # C = 2, alpha_{0,1} = 2: u(1.5) = 2 * 1.5 * (1.5 - 3)^2 = 6.75 with L_u = 3
    s = with_u(base, np.concatenate([[0, 2.0, 0, 0, 0], z]), 2, 3.0, [1, 1])
    assert U(oracle_lib, s, two(1.5)) == pytest.approx(6.75, abs=1e-13)
    # unequal labels use channel 1 only: alpha_{1,0} = 2 -> u(1) = 2 (1 - 2)^3 = -2
    s = with_u(base, np.concatenate([[5.0, 0, 0, 0, 0], [2.0, 0, 0, 0, 0]]), 3, 2.0, [0, 1])
    assert U(oracle_lib, s, two(1.0)) == pytest.approx(-2.0, abs=1e-14)
    # a fixed ion near both electrons adds nothing
    ion = big_cube(2, fixed_pos=[[1.5, 1.2, 1.0]], fixed_q=[1.0])
    s = with_u(ion, np.concatenate([[1.0, 0, 0, 0, 0], [1.0, 0, 0, 0, 0]]), 3, 2.0, [0, 0])
    assert U(oracle_lib, s, two(1.0)) == pytest.approx(-1.0, abs=1e-14)


def test_u_minimum_image(oracle_lib):
    """A pair across the cell boundary counts at its nearest-image distance:
    equal to the same separation inside the cell, in a skewed (fcc) cell too,
    and unchanged by lattice translations of either particle."""
    for cell in (10.0 * np.eye(3), wl.fcc_cell(250.0)):
        base = wl.System("c", 3, cell, 2, -np.ones(2), np.zeros((0, 3)), np.zeros(0), 1.0, 1.0, 1.0)
        Lu = 0.5 * min(np.linalg.norm(cell, axis=1))
        rng = np.random.default_rng(4)
        s = with_u(base, rng.uniform(-1, 1, 10) / Lu ** 4, 3, Lu, [0, 1])
        inside = np.array([[0.2, 0.3, 0.1], [0.2 + 0.4 * Lu, 0.3 + 0.3 * Lu, 0.1]])
        ref = U(oracle_lib, s, inside)
        assert ref != 0.0
        for shift in ([1, 0, 0], [0, -1, 2], [-1, 1, 1]):
            moved = inside.copy()
            moved[1] += np.asarray(shift, dtype=float) @ cell
            assert U(oracle_lib, s, moved) == pytest.approx(ref, rel=1e-12, abs=1e-14)
        # the same pair placed on either side of a cell face
        across = inside - inside[0] + 0.02 * cell[0]
        across[1] -= cell[0]
        assert U(oracle_lib, s, across) == pytest.approx(ref, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("cfg_id", [1, 3, 5])
@pytest.mark.parametrize("parallel", [True, False])
def test_u_cusp(oracle_lib, cfg_id, parallel):
    """The seeded coefficients satisfy the Kato cusp u'(0) = 1/(d+1)
    (parallel) or 1/(d-1) (antiparallel): the slope of U at zero separation,
    from a cubic fit to four small separations, equals it.  The relation used
    to set alpha_1 is independent of the oracle's evaluation of u."""
    cfg = wl.config(cfg_id)
    full = wl.with_u_term(cfg.systems[0], cfg_id)
    d = full.dim
    base = wl.System("pair", d, full.lattice, 2, -np.ones(2), np.zeros((0, d)), np.zeros(0), full.alpha,
                     full.r_cut, full.g_cut)
    s = dataclasses.replace(base, u_alpha=full.u_alpha, u_C=full.u_C, u_cut=full.u_cut,
                            mobile_spin=np.array([0, 0] if parallel else [0, 1], dtype=np.int32))
    h = 1e-3
    xs = h * np.arange(1, 5)
    direction = np.ones(d) / math.sqrt(d)
    vals = []
    for x in xs:
        pos = np.zeros((2, d)) + 0.25 * full.lattice[0, :d]
        pos[1] += x * direction
        vals.append(U(oracle_lib, s, pos))
    slope = np.polyfit(xs, vals, 3)[-2]
    assert slope == pytest.approx(wl.cusp_slope(d, parallel), rel=1e-6)


def test_u_order_c_zero_at_cutoff(oracle_lib):
    """u vanishes at L_u to order C: U(L_u - 2h)/U(L_u - h) -> 2^C, and U is
    exactly zero beyond L_u (seeded coefficients of the N=54 system, whose
    cell is simple cubic with L_u = L/2)."""
    cfg = wl.config(1)
    full = wl.with_u_term(cfg.systems[0], 1)
    base = wl.System("pair", 3, full.lattice, 2, -np.ones(2), np.zeros((0, 3)), np.zeros(0), 1.0, 1.0, 1.0)
    for C in (2, 3):
        s = dataclasses.replace(base, u_alpha=full.u_alpha, u_C=C, u_cut=full.u_cut,
                                mobile_spin=np.array([0, 1], dtype=np.int32))

        def at(r):  # along a face diagonal, where r slightly beyond L_u (= L/2) has no nearer image
            pos = np.zeros((2, 3)) + 0.1
            pos[1, :2] += r / math.sqrt(2.0)
            return U(oracle_lib, s, pos)

        h = 1e-4 * full.u_cut
        assert at(full.u_cut - 2 * h) / at(full.u_cut - h) == pytest.approx(2.0 ** C, rel=1e-3)
        assert at(full.u_cut + h) == 0.0


def u_system(dim, n, seed):
    cfg_id = 1 if dim == 3 else 3
    full = wl.with_u_term(wl.config(cfg_id).systems[0], cfg_id)
    s = wl.System("u", dim, full.lattice, n, -np.ones(n), np.zeros((0, dim)), np.zeros(0), full.alpha,
                  full.r_cut, full.g_cut)
    spin = (np.arange(n) % 2).astype(np.int32)
    s = dataclasses.replace(s, u_alpha=full.u_alpha, u_C=full.u_C, u_cut=full.u_cut, mobile_spin=spin)
    # particles clustered so that many pairs fall inside L_u
    g = np.random.default_rng([31, dim, seed])
    pos = g.uniform(0.0, 0.6 * full.u_cut, (n, dim)) + 0.1 * full.lattice[0, :dim]
    return s, pos


@pytest.mark.parametrize("dim", [3, 2])
def test_u_derivs_finite_differences(oracle_lib, dim):
    """Gradient and Laplacian of U with respect to one particle against
    fourth-order central differences of U (h = 1e-4 L_u)."""
    s, pos = u_system(dim, 8, 1)
    q = -np.ones(8)
    h = 1e-4 * s.u_cut

    def J(p):
        return oracle_lib.energy(s, p, q)["jastrow"]

    for k in (0, 3, 6):
        grad, lap = oracle_lib.jastrow_derivs(s, pos, q, k, None)
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
        scale = max(1e-3, float(np.max(np.abs(grad))), abs(lap))
        assert np.max(np.abs(grad - fd_grad)) <= 1e-8 * scale, (k, grad, fd_grad)
        assert abs(lap - fd_lap) <= 1e-5 * scale, (k, lap, fd_lap)


@pytest.mark.parametrize("cfg_id", [1, 3])
def test_u_incremental_moves_and_invariance(oracle_lib, cfg_id):
    """With the u term (and the plane-wave term) the move driver's Jastrow
    deltas equal J(R') - J(R) from recomputes, and J is invariant under a
    permutation of equal-spin particles and a common translation."""
    cfg = wl.config(cfg_id)
    s = wl.with_u_term(cfg.systems[0], cfg_id)
    b = wl.make_batch(cfg, walkers=1, moves=10)
    ja = np.random.default_rng(5).uniform(-0.01, 0.01, 30)
    r = oracle_lib.run(s, b.walker_pos(0), b.k[:, 0], b.new_pos[:, 0], b.accept[:, 0], jastrow_a=ja)
    cur = b.walker_pos(0).copy()
    j_cur = oracle_lib.energy(s, *oracle_lib.particles(s, cur), jastrow_a=ja)["jastrow"]
    assert j_cur == pytest.approx(r["j0"], rel=1e-13)
    for m in range(b.steps):
        k = int(b.k[m, 0])
        prop = cur.copy()
        prop[k] = b.new_pos[m, 0]
        j_new = oracle_lib.energy(s, *oracle_lib.particles(s, prop), jastrow_a=ja)["jastrow"]
        assert abs((j_new - j_cur) - r["djas"][m]) <= 1e-11 * max(1.0, abs(j_cur))
        if b.accept[m, 0]:
            cur, j_cur = prop, j_new
    n = s.n_mobile
    perm = np.arange(n)
    perm[[0, 2]] = perm[[2, 0]]  # particles 0 and 2 carry the same label
    assert s.mobile_spin[0] == s.mobile_spin[2]
    j_perm = oracle_lib.energy(s, *oracle_lib.particles(s, cur[perm]), jastrow_a=ja)["jastrow"]
    assert j_perm == pytest.approx(j_cur, rel=1e-12)
    shift = np.full(s.dim, 0.37)
    j_shift = oracle_lib.energy(s, *oracle_lib.particles(s, cur + shift), jastrow_a=ja)["jastrow"]
    assert j_shift == pytest.approx(j_cur, rel=1e-11)
