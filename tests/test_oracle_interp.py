"""Pins of the oracle's periodic cubic Lagrange interpolation."""
import numpy as np
import pytest
from scipy.interpolate import lagrange

from oracle.interp import interpolate, lagrange_weights


def test_weights_match_textbook_lagrange_polynomials():
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])
    rng = np.random.default_rng(0)
    for t in rng.uniform(0, 1, 7):
        w = lagrange_weights(np.array(t))
        for i in range(4):
            e = np.zeros(4)
            e[i] = 1.0
            assert float(w[i]) == pytest.approx(lagrange(nodes, e)(t), abs=1e-13)
    # partition of unity and exact node values at t = 0
    t = rng.uniform(0, 1, 50)
    assert np.allclose(sum(lagrange_weights(t)), 1.0, atol=1e-14)
    assert [float(x) for x in lagrange_weights(np.array(0.0))] == [0.0, 1.0, 0.0, 0.0]


def test_reproduces_tensor_cubics_away_from_the_wrap():
    n = (14, 11)
    l1, l2 = np.meshgrid(np.arange(n[0], dtype=float), np.arange(n[1], dtype=float),
                         indexing="ij")
    p = lambda s: 0.3 * s ** 3 - s ** 2 + 2 * s - 1
    q = lambda s: -0.1 * s ** 3 + 0.5 * s + 4
    u = p(l1) * q(l2)
    rng = np.random.default_rng(1)
    xi = np.stack([rng.uniform(1.0, n[0] - 3.0, 40), rng.uniform(1.0, n[1] - 3.0, 40)])
    np.testing.assert_allclose(interpolate(u, xi), p(xi[0]) * q(xi[1]), rtol=1e-12)


def test_periodic_wrap_and_nodes():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((6, 8, 5))
    xi = np.stack([rng.uniform(-3, 9, 30), rng.uniform(-3, 11, 30), rng.uniform(-2, 7, 30)])
    shift = np.array([6.0, -16.0, 10.0])[:, None]
    np.testing.assert_allclose(interpolate(u, xi), interpolate(u, xi + shift), atol=1e-12)
    nodes = np.stack(np.meshgrid(*[np.arange(s, dtype=float) for s in u.shape],
                                 indexing="ij")).reshape(3, -1)
    np.testing.assert_array_equal(interpolate(u, nodes), u.reshape(-1))


def test_brute_force_single_point_3d():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((7, 9, 6))
    pt = np.array([5.3, 0.25, -0.8])
    f = np.floor(pt).astype(int)
    t = pt - f
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])
    acc = 0.0
    for a in range(4):
        for b in range(4):
            for c in range(4):
                wa = lagrange(nodes, np.eye(4)[a])(t[0])
                wb = lagrange(nodes, np.eye(4)[b])(t[1])
                wc = lagrange(nodes, np.eye(4)[c])(t[2])
                acc += wa * wb * wc * u[(f[0] + a - 1) % 7, (f[1] + b - 1) % 9, (f[2] + c - 1) % 6]
    assert float(interpolate(u, pt[:, None])[0]) == pytest.approx(acc, abs=1e-12)
