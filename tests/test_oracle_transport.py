"""Pins of the oracle's transport solves, objective and reduced gradient.

Closed forms: constant velocities (exact shifts) and the shear-free flow
v = (c sin x1, 0), whose flow map is known exactly:
    tan(phi_t(x)/2) = tan(x/2) e^{c t}   (along x1),
so the advection state, the continuity state and both adjoints have exact
solutions in terms of phi and its Jacobian.
"""
import math

import numpy as np
import pytest

import synth
from oracle import spectral as sp
from oracle.transport import TransportProblem

PI = math.pi


def grid_x(shape):
    return np.meshgrid(*[2 * PI * np.arange(n) / n for n in shape], indexing="ij")


def smooth_image(x):
    return np.exp(np.cos(x[0])) * (1.0 + 0.3 * np.sin(x[1] + 0.4))


def flow(x1, c):
    """phi_1 along x1 for v = (c sin x1, 0) and its derivative."""
    s, co = np.sin(x1 / 2), np.cos(x1 / 2)
    y = 2 * np.arctan2(np.exp(c) * s, co)
    jac = np.exp(c) / (co ** 2 + np.exp(2 * c) * s ** 2)
    return y, jac


def sine_problem(n, nt, c, model="advection", m0=None, m1=None):
    shape = (n, n)
    x = grid_x(shape)
    m0 = smooth_image(x) if m0 is None else m0(x)
    m1 = np.zeros(shape) if m1 is None else m1(x)
    P = TransportProblem(m0, m1, nt, 1e-2, 1, model=model)
    v = np.stack([c * np.sin(x[0]), np.zeros(shape)])
    return P, v, x


# -- exact shifts ------------------------------------------------------------
def test_integer_shift_is_exact_roll():
    rng = np.random.default_rng(0)
    shape = (16, 12)
    m0 = rng.standard_normal(shape)
    nt = 4
    u = np.array([2, -1])                       # cells per step
    v = np.stack([np.full(shape, u[j] * (2 * PI / shape[j]) * nt) for j in range(2)])
    P = TransportProblem(m0, m0, nt, 1.0, 1)
    X, _ = P.characteristics(v)
    np.testing.assert_allclose(X, P.nodes - u[:, None, None], atol=1e-13)
    m = P.forward(v)
    np.testing.assert_allclose(m[-1], np.roll(m0, tuple(nt * u), axis=(0, 1)), atol=1e-13)


def test_fractional_shift_converges_at_interpolation_order():
    errs = []
    for n in (32, 64, 128):
        shape = (n, n)
        x = grid_x(shape)
        m0f = lambda a, b: np.sin(a) * np.cos(2 * b) + 0.5 * np.cos(3 * a + b)
        vel = np.array([0.37, -0.21])
        v = np.stack([np.full(shape, vel[j]) for j in range(2)])
        P = TransportProblem(m0f(x[0], x[1]), m0f(x[0], x[1]), 4, 1.0, 1)
        m = P.forward(v)
        exact = m0f(x[0] - vel[0], x[1] - vel[1])
        errs.append(np.max(np.abs(m[-1] - exact)))
    # orientation: transporting by +v moves the profile towards +v
    assert errs[0] < 1e-2
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8


# -- closed-form nonlinear flow ----------------------------------------------
def _order(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_characteristics_are_second_order():
    errs = []
    c = 0.8
    for nt in (4, 8, 16):
        P, v, x = sine_problem(128, nt, c)
        X, Y = P.characteristics(v)
        h = P.grid.h[0]
        # one step of the exact flow backwards / forwards
        back, _ = flow(x[0], -c / nt)
        fwd, _ = flow(x[0], c / nt)
        dx = (X[0] * h - back + PI) % (2 * PI) - PI
        dy = (Y[0] * h - fwd + PI) % (2 * PI) - PI
        errs.append(max(np.max(np.abs(dx)), np.max(np.abs(dy))))
        np.testing.assert_allclose(X[1], P.nodes[1], atol=1e-13)
    # local truncation error of Heun: third order per step
    assert min(_order(errs)) > 2.7


@pytest.mark.parametrize("case", ["adv_state", "cont_state", "adv_adjoint", "cont_adjoint"])
def test_transport_matches_exact_flow(case):
    c = 0.5
    errs = []
    for n, nt in ((32, 4), (64, 8), (128, 16)):
        model = "advection" if case.startswith("adv") else "continuity"
        P, v, x = sine_problem(n, nt, c, model=model)
        X, Y = P.characteristics(v)
        cf, cb = P.source_factors(v, X, Y)
        if case.endswith("state"):
            got = P.forward(v, X, cf)[-1]
            y, jac = flow(x[0], -c)
            exact = smooth_image([y, x[1]])
            if model == "continuity":
                exact = exact * jac
        else:
            lam1 = smooth_image(x)
            got = P.adjoint(-lam1, Y, cb)[0]          # lam^nt = m1 - m^nt = lam1
            y, jac = flow(x[0], c)
            exact = smooth_image([y, x[1]])
            if model == "advection":
                exact = exact * jac
        errs.append(np.max(np.abs(got - exact)) / np.max(np.abs(exact)))
    assert errs[-1] < 2e-3
    assert min(_order(errs)) > 1.8


def test_continuity_mass_drift_shrinks():
    drift = []
    for n, nt in ((32, 4), (64, 8), (128, 16)):
        P, v, x = sine_problem(n, nt, 0.5, model="continuity")
        m = P.forward(v)
        drift.append(abs(m[-1].sum() - m[0].sum()) / m[0].sum())
    assert drift[-1] < 1e-4 and drift[0] > drift[-1]


# -- objective and gradient ----------------------------------------------------
def test_objective_closed_form_at_zero_velocity():
    shape = (32, 24)
    x = grid_x(shape)
    P = TransportProblem(np.sin(x[0]), np.zeros(shape), 4, 0.3, 2)
    # 1/2 int sin^2 = 1/2 * pi * 2 pi ; regulariser is zero at v = 0
    assert P.objective(np.zeros((2,) + shape)) == pytest.approx(PI ** 2, rel=1e-13)
    # with v a single mode: R(v) = |k|^4 * 2 pi^2 for v1 = sin(3 x2)
    v = np.stack([1e-9 * np.sin(3 * x[1]), np.zeros(shape)])
    _, mis, reg = P.objective(v, return_parts=True)
    assert reg == pytest.approx(0.5 * 0.3 * 81 * 2 * PI ** 2 * 1e-18, rel=1e-10)


def _c0_small(shape=(32, 32), seed=0):
    wl = synth.workload("c0", shape=shape, seed=seed)
    m1 = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order).forward(wl.vstar)[-1]
    return wl, m1


def test_inverse_crime_and_zero_data():
    wl, m1 = _c0_small()
    P = TransportProblem(wl.m0, m1, wl.nt, wl.alpha, wl.reg_order)
    J, g, st = P.gradient(wl.vstar, return_states=True)
    assert J == pytest.approx(0.5 * wl.alpha * P.reg_value(wl.vstar), rel=1e-14)
    assert max(np.max(np.abs(l)) for l in st["lam"]) == 0.0
    np.testing.assert_allclose(g, sp.apply_reg(P.grid, wl.vstar, 1, wl.alpha), atol=1e-15)
    Z = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order)
    J0, g0 = Z.gradient(np.zeros_like(wl.vstar))
    assert J0 == 0.0 and np.max(np.abs(g0)) == 0.0


@pytest.mark.parametrize("model", ["advection", "continuity"])
def test_gradient_matches_finite_differences_under_refinement(model):
    """The discretised continuous gradient agrees with central differences of
    the discrete objective up to a discretisation gap that must shrink when n
    and n_t are refined together; the sign of the adjoint final condition is
    pinned by the agreement itself."""
    gaps = []
    for n, nt in ((16, 2), (32, 4), (64, 8)):
        x = grid_x((n, n))
        m0 = smooth_image(x)
        vstar = np.stack([0.4 * np.sin(x[0] + x[1]), 0.3 * np.cos(2 * x[0] - x[1])])
        base = TransportProblem(m0, m0, nt, 1e-2, 1, model=model)
        m1 = base.forward(vstar)[-1]
        P = TransportProblem(m0, m1, nt, 1e-2, 1, model=model)
        v = 0.5 * vstar
        _, g = P.gradient(v)
        dirs = [np.stack([np.cos(x[0] - 2 * x[1]), np.sin(x[1])]), vstar]
        worst = 0.0
        for dvec in dirs:
            hh = 1e-4
            fd = (P.objective(v + hh * dvec) - P.objective(v - hh * dvec)) / (2 * hh)
            an = P.grid.inner(g, dvec)
            assert np.sign(fd) == np.sign(an)
            worst = max(worst, abs(fd - an) / abs(an))
        gaps.append(worst)
    assert gaps[-1] < 2e-3
    assert gaps[0] > gaps[1] > gaps[2]


def test_brute_force_fd_gradient_16x16():
    """Every entry of |h| g against a central difference of J (16^2, nt=4)."""
    n, nt = 16, 4
    x = grid_x((n, n))
    m0 = smooth_image(x)
    vstar = np.stack([0.4 * np.sin(x[0] + x[1]), 0.3 * np.cos(2 * x[0] - x[1])])
    m1 = TransportProblem(m0, m0, nt, 1e-2, 1).forward(vstar)[-1]
    P = TransportProblem(m0, m1, nt, 1e-2, 1)
    v = 0.5 * vstar
    _, g = P.gradient(v)
    fd = np.zeros_like(v)
    hh = 1e-5
    for idx in np.ndindex(v.shape):
        e = np.zeros_like(v)
        e[idx] = hh
        fd[idx] = (P.objective(v + e) - P.objective(v - e)) / (2 * hh)
    an = P.grid.cell * g
    rel = np.linalg.norm(fd - an) / np.linalg.norm(fd)
    cos = np.sum(fd * an) / (np.linalg.norm(fd) * np.linalg.norm(an))
    assert rel < 0.15 and cos > 0.99


def test_incompressible_gradient_is_divergence_free():
    wl = synth.workload("c2", shape=(16, 16, 16))
    m1 = TransportProblem(wl.m0, wl.m0, 2, wl.alpha, wl.reg_order,
                          incompressible=True).forward(wl.vstar)[-1]
    P = TransportProblem(wl.m0, m1, 2, wl.alpha, wl.reg_order, incompressible=True)
    assert np.max(np.abs(sp.divergence(P.grid, wl.vstar))) < 1e-12 * np.max(np.abs(wl.vstar))
    _, g = P.gradient(0.3 * wl.vstar)
    assert np.max(np.abs(sp.divergence(P.grid, g))) < 1e-11 * np.max(np.abs(g))
