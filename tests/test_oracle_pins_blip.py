"""Pins of the oracle's blip-orbital evaluation (Sec. 2.4): orbitals on a
periodic grid of cubic B-spline blip functions Th (Th(0) = 1), evaluated at
arbitrary points with their gradient and Laplacian.

Checked against what the mathematics fixes: the B-spline's partition of
unity (sum_i Th(x - i) = 3/2, so constant coefficients give a constant
orbital with zero derivatives), its reproduction of linear functions away
from the periodic seam (sum_i i Th(x - i) = 3/2 x), plane-wave coefficients
at grid nodes (sum_i e^{i t i} Th(j - i) = e^{i t j} (1 + cos t / 2)),
lattice periodicity, and fourth-order finite differences for the gradient
and Laplacian in a skewed cell (where the Laplacian needs the mixed second
derivatives).  tests/test_oracle_mutations.py plants mistakes and checks
that these catch them.
"""
import math

import numpy as np
import pytest


SKEW = np.array([[6.0, 0.4, 0.1], [0.7, 5.5, -0.3], [0.2, -0.5, 6.4]])
GRID = (8, 9, 10)


def frac_to_cart(s, lat):
    return np.asarray(s) @ lat


def test_blip_partition_of_unity(oracle_lib):
    coef = np.full(GRID + (2,), 1.0)
    coef[..., 1] = -2.5
    pts = frac_to_cart(np.random.default_rng(1).random((7, 3)), SKEW)
    val, grad, lap = oracle_lib.blip_eval(SKEW, GRID, coef, pts)
    assert np.allclose(val[:, 0], 1.5 ** 3, rtol=0, atol=1e-13)
    assert np.allclose(val[:, 1], -2.5 * 1.5 ** 3, rtol=0, atol=1e-13)
    assert np.max(np.abs(grad)) <= 1e-12 and np.max(np.abs(lap)) <= 1e-11


def test_blip_linear_reproduction(oracle_lib):
    """Coefficients a = i (the first grid index) reproduce 3/2 x_1 wherever
    the four supporting grid points do not wrap; the gradient is
    3/2 n_1 Ainv[:, 0] and the Laplacian zero."""
    n1 = GRID[0]
    coef = np.zeros(GRID + (1,))
    coef[..., 0] = np.arange(n1, dtype=float)[:, None, None]
    rng = np.random.default_rng(2)
    s = rng.random((6, 3))
    s[:, 0] = rng.uniform(2.0 / n1, (n1 - 3.0) / n1, 6)  # x_1 in [2, n1 - 3]
    pts = frac_to_cart(s, SKEW)
    val, grad, lap = oracle_lib.blip_eval(SKEW, GRID, coef, pts)
    ainv = np.linalg.inv(SKEW)
    assert np.allclose(val[:, 0], 1.5 ** 3 * n1 * s[:, 0], rtol=1e-13, atol=1e-12)
    want = 1.5 ** 3 * n1 * ainv[:, 0]
    assert np.allclose(grad[:, :, 0], want[None, :], rtol=1e-12, atol=1e-12)
    assert np.max(np.abs(lap)) <= 1e-10


@pytest.mark.parametrize("m", [(1, 0, 0), (2, -3, 1), (0, 4, 5)])
def test_blip_plane_wave_at_nodes(oracle_lib, m):
    """a[i,j,k] = cos(2 pi (m1 i/n1 + m2 j/n2 + m3 k/n3)) and the sine: at a
    grid node the orbitals equal the plane wave times prod_d (1 + cos t_d / 2),
    t_d = 2 pi m_d / n_d."""
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in GRID], indexing="ij"), axis=-1)
    ph = 2 * math.pi * sum(m[d] * idx[..., d] / GRID[d] for d in range(3))
    coef = np.stack([np.cos(ph), np.sin(ph)], axis=-1)
    nodes = np.array([[0, 0, 0], [3, 5, 7], [7, 8, 9], [4, 1, 2]])
    pts = frac_to_cart(nodes / np.array(GRID, dtype=float), SKEW)
    val, _, _ = oracle_lib.blip_eval(SKEW, GRID, coef, pts, derivs=False)
    fac = np.prod([1.0 + 0.5 * math.cos(2 * math.pi * m[d] / GRID[d]) for d in range(3)])
    phn = 2 * math.pi * (nodes @ (np.array(m) / np.array(GRID, dtype=float)))
    assert np.allclose(val[:, 0], fac * np.cos(phn), rtol=0, atol=1e-13)
    assert np.allclose(val[:, 1], fac * np.sin(phn), rtol=0, atol=1e-13)


def test_blip_lattice_periodicity(oracle_lib):
    coef = np.random.default_rng(3).uniform(-1, 1, GRID + (4,))
    base = frac_to_cart(np.random.default_rng(4).random((5, 3)), SKEW)
    v0, g0, l0 = oracle_lib.blip_eval(SKEW, GRID, coef, base)
    for shift in ([1, 0, 0], [0, -2, 1], [-1, 1, 3]):
        v, g, l = oracle_lib.blip_eval(SKEW, GRID, coef, base + np.asarray(shift, dtype=float) @ SKEW)
        assert np.allclose(v, v0, rtol=0, atol=1e-12)
        assert np.allclose(g, g0, rtol=0, atol=1e-10)
        assert np.allclose(l, l0, rtol=0, atol=1e-9)


def test_blip_derivs_finite_differences(oracle_lib):
    """Gradient and Laplacian against fourth-order central differences of the
    values in a skewed cell (h = 1e-3 bohr)."""
    coef = np.random.default_rng(5).uniform(-1, 1, GRID + (3,))
    pts = frac_to_cart(np.random.default_rng(6).random((4, 3)), SKEW)
    val, grad, lap = oracle_lib.blip_eval(SKEW, GRID, coef, pts)
    h = 1e-3
    fd_g = np.zeros_like(grad)
    fd_l = np.zeros_like(lap)
    for e in range(3):
        f = {}
        for m in (-2, -1, 1, 2):
            q = pts.copy()
            q[:, e] += m * h
            f[m] = oracle_lib.blip_eval(SKEW, GRID, coef, q, derivs=False)[0]
        fd_g[:, e] = (f[-2] - 8 * f[-1] + 8 * f[1] - f[2]) / (12 * h)
        fd_l += (-f[-2] + 16 * f[-1] - 30 * val + 16 * f[1] - f[2]) / (12 * h * h)
    scale = max(1.0, float(np.max(np.abs(grad))))
    assert np.max(np.abs(grad - fd_g)) <= 1e-8 * scale
    assert np.max(np.abs(lap - fd_l)) <= 1e-5 * max(1.0, float(np.max(np.abs(lap))))


def test_blip_function_values(oracle_lib):
    """Hand-evaluated values of the blip function through the oracle's
    orbital at points on the first grid axis with one nonzero coefficient:
    Th(0) = 1, Th(1/2) = 23/32, Th(1) = 1/4, Th(3/2) = 1/32, Th(2) = 0."""
    grid = (8, 8, 8)
    coef = np.zeros(grid + (1,))
    coef[4, 0, 0, 0] = 1.0
    lat = 8.0 * np.eye(3)
    xs = np.array([4.0, 4.5, 5.0, 5.5, 6.0, 3.5])
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1)  # grid spacing 1 bohr
    val, _, _ = oracle_lib.blip_eval(lat, grid, coef, pts, derivs=False)
    assert np.allclose(val[:, 0], [1.0, 23 / 32, 0.25, 1 / 32, 0.0, 23 / 32], rtol=0, atol=1e-15)
