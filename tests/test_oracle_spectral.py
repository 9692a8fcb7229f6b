"""Pins of the oracle's spectral calculus (Sec. 2.2) against closed forms.

Every check uses trigonometric polynomials whose derivatives, Laplacian
powers and integrals are known exactly, or operator identities that a sign,
index or Nyquist mistake breaks.
"""
import math

import numpy as np
import pytest

from oracle import spectral as sp

PI = math.pi


def coords(grid):
    return np.meshgrid(*[2 * PI * np.arange(n) / n for n in grid.shape], indexing="ij")


@pytest.mark.parametrize("shape", [(16, 24), (12, 18, 8)])
def test_derivative_of_trig_polynomial(shape):
    g = sp.Grid(shape)
    x = coords(g)
    if g.d == 2:
        u = np.sin(2 * x[0]) * np.cos(3 * x[1]) + 0.5 * np.cos(x[0] - 5 * x[1])
        du = [2 * np.cos(2 * x[0]) * np.cos(3 * x[1]) - 0.5 * np.sin(x[0] - 5 * x[1]),
              -3 * np.sin(2 * x[0]) * np.sin(3 * x[1]) + 2.5 * np.sin(x[0] - 5 * x[1])]
    else:
        u = np.sin(x[0] + 2 * x[1]) * np.cos(3 * x[2])
        du = [np.cos(x[0] + 2 * x[1]) * np.cos(3 * x[2]),
              2 * np.cos(x[0] + 2 * x[1]) * np.cos(3 * x[2]),
              -3 * np.sin(x[0] + 2 * x[1]) * np.sin(3 * x[2])]
    for j in range(g.d):
        np.testing.assert_allclose(sp.deriv(g, u, j), du[j], atol=1e-12)


def test_nyquist_mode_has_zero_first_derivative():
    g = sp.Grid((16, 8))
    x = coords(g)
    u = np.cos(8 * x[0]) + np.cos(4 * x[1])       # both at their Nyquist index
    for j in range(2):
        assert np.max(np.abs(sp.deriv(g, u, j))) < 1e-12
    # but the even-order operator keeps it: -Lap cos(8 x1) = 64 cos(8 x1)
    lap = sp.apply_reg(g, np.stack([np.cos(8 * x[0]), np.zeros(g.shape)]), 1)
    np.testing.assert_allclose(lap[0], 64 * np.cos(8 * x[0]), atol=1e-10)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_regularisation_operator_powers(p):
    g = sp.Grid((20, 16))
    x = coords(g)
    k = (3, 2)
    ksq = k[0] ** 2 + k[1] ** 2
    v = np.stack([np.sin(k[0] * x[0] + k[1] * x[1]), np.cos(5 * x[1])])
    Lv = sp.apply_reg(g, v, p, alpha=0.7)
    np.testing.assert_allclose(Lv[0], 0.7 * ksq ** p * v[0], atol=1e-9 * ksq ** p)
    np.testing.assert_allclose(Lv[1], 0.7 * 25 ** p * v[1], atol=1e-9 * 25 ** p)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reg_value_closed_form(p):
    # v = (sin(a x1), cos(b x2)): R = (a^2p + b^2p) * 2 pi^2 on [0,2pi)^2
    g = sp.Grid((24, 16))
    x = coords(g)
    a, b = 3, 5
    v = np.stack([np.sin(a * x[0]), np.cos(b * x[1])])
    expect = (a ** (2 * p) + b ** (2 * p)) * 2 * PI ** 2
    assert sp.reg_value(g, v, p) == pytest.approx(expect, rel=1e-12)
    # p = 1 is the H1 seminorm ||grad v||^2, p = 2 is ||Lap v||^2
    if p == 1:
        gv = sum(g.inner(sp.deriv(g, v[c], j), sp.deriv(g, v[c], j))
                 for c in range(2) for j in range(2))
        assert gv == pytest.approx(expect, rel=1e-12)
    if p == 2:
        lap = [sum(sp.deriv(g, sp.deriv(g, v[c], j), j) for j in range(2)) for c in range(2)]
        assert sum(g.inner(l, l) for l in lap) == pytest.approx(expect, rel=1e-12)


def test_inverse_with_zero_mode_rule():
    g = sp.Grid((16, 12))
    rng = np.random.default_rng(0)
    u = rng.standard_normal((2,) + g.shape)
    alpha = 3e-2
    w = sp.apply_reg_inverse(g, u, 2, alpha)
    back = sp.apply_reg(g, w, 2, alpha)
    # identity on the zero-mean part, the zero mode is annihilated by L
    np.testing.assert_allclose(back, u - u.mean(axis=(1, 2), keepdims=True), atol=1e-10)
    # the zero mode itself: (alpha L)^-1 c = c / alpha
    c = np.full((2,) + g.shape, 2.5)
    np.testing.assert_allclose(sp.apply_reg_inverse(g, c, 2, alpha), c / alpha, rtol=1e-13)
    # closed form on a single mode
    x = coords(g)
    s = np.stack([np.sin(2 * x[0] + x[1]), np.zeros(g.shape)])
    np.testing.assert_allclose(sp.apply_reg_inverse(g, s, 1, alpha)[0],
                               s[0] / (alpha * 5), atol=1e-12)


def test_derivative_is_skew_adjoint_and_inner_product_is_quadrature():
    g = sp.Grid((12, 20, 8))
    rng = np.random.default_rng(1)
    a = rng.standard_normal(g.shape)
    b = rng.standard_normal(g.shape)
    for j in range(3):
        lhs = g.inner(sp.deriv(g, a, j), b)
        rhs = -g.inner(a, sp.deriv(g, b, j))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    x = coords(g)
    # int sin^2(x1) over [0,2pi)^3 = pi (2 pi)^2
    assert g.inner(np.sin(x[0]), np.sin(x[0])) == pytest.approx(PI * (2 * PI) ** 2, rel=1e-13)


@pytest.mark.parametrize("shape", [(16, 16), (12, 8, 10)])
def test_leray_projection(shape):
    g = sp.Grid(shape)
    rng = np.random.default_rng(2)
    v = rng.standard_normal((g.d,) + g.shape)
    w = rng.standard_normal((g.d,) + g.shape)
    Pv = sp.leray(g, v)
    # divergence-free, idempotent, symmetric
    assert np.max(np.abs(sp.divergence(g, Pv))) <= 1e-12 * np.max(np.abs(v))
    np.testing.assert_allclose(sp.leray(g, Pv), Pv, atol=1e-12)
    assert g.inner(Pv, w) == pytest.approx(g.inner(v, sp.leray(g, w)), rel=1e-12)
    # kills gradients of smooth potentials (no Nyquist content), keeps curls
    x = coords(g)
    phi = np.sin(x[0]) * np.cos(2 * x[1])
    assert np.max(np.abs(sp.leray(g, sp.gradient(g, phi)))) < 1e-12
    if g.d == 2:
        curl = np.stack([sp.deriv(g, phi, 1), -sp.deriv(g, phi, 0)])
        np.testing.assert_allclose(sp.leray(g, curl), curl, atol=1e-12)
    # the mean flow is divergence-free and untouched
    const = np.ones((g.d,) + g.shape)
    np.testing.assert_allclose(sp.leray(g, const), const, atol=1e-13)
