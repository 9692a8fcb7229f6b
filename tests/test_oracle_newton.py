"""Pins of the oracle's Gauss--Newton--Krylov baseline.

PCG against a dense solve; the Gauss--Newton matvec against finite
differences of the reduced gradient at a zero-residual point (where the
Gauss--Newton and the full Hessian coincide), its symmetry and positivity up
to the optimize-then-discretize gap (shrinking under refinement), and the
exact reduction to alpha L when the image has no gradient.
"""
import math

import numpy as np
import pytest

import synth
from oracle import newton as nk
from oracle import spectral as sp
from oracle.transport import TransportProblem

PI = math.pi


def grid_x(shape):
    return np.meshgrid(*[2 * PI * np.arange(n) / n for n in shape], indexing="ij")


def test_pcg_solves_spd_systems():
    rng = np.random.default_rng(3)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(0.5, 40.0, n)) @ Q.T
    Mi = np.diag(1.0 / np.diag(A))
    b = rng.standard_normal(n)
    inner = lambda a, c: float(a @ c)
    x, its = nk.pcg(lambda p: A @ p, lambda r: Mi @ r, inner, b, 1e-12, maxit=200)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    # loose tolerance: the residual bound is met at exit
    x, its = nk.pcg(lambda p: A @ p, lambda r: Mi @ r, inner, b, 1e-2, maxit=200)
    assert np.linalg.norm(b - A @ x) <= 1e-2 * np.linalg.norm(b)
    assert its < n


def smooth_case(n, nt):
    shape = (n, n)
    x = grid_x(shape)
    m0 = np.exp(np.cos(x[0])) * (1.0 + 0.3 * np.sin(x[1] + 0.4))
    vstar = np.stack([0.4 * np.sin(x[0] + x[1]), 0.3 * np.cos(2 * x[0] - x[1])])
    gen = TransportProblem(m0, m0, nt, 1e-3, 1)
    m1 = gen.forward(vstar)[-1]
    P = TransportProblem(m0, m1, nt, 1e-3, 1)
    d = np.stack([np.cos(x[0] - 2 * x[1]), np.sin(x[1])])
    e = np.stack([np.sin(2 * x[0]), np.cos(x[0] + x[1])])
    return P, vstar, d, e


def test_gn_matvec_is_the_derivative_of_the_gradient_at_zero_residual():
    gaps = []
    for n, nt in ((32, 4), (64, 8)):
        P, vstar, d, _ = smooth_case(n, nt)
        Hd = nk.gn_matvec(P, vstar, d)
        eps = 1e-4
        fd = (P.gradient(vstar + eps * d)[1] - P.gradient(vstar - eps * d)[1]) / (2 * eps)
        gaps.append(np.linalg.norm(fd - Hd) / np.linalg.norm(Hd))
    # second order in the joint refinement (the OTD gap of this scheme)
    assert gaps[-1] < 5e-3
    assert gaps[-1] < 0.3 * gaps[0]


def test_gn_matvec_symmetric_and_positive_up_to_discretisation():
    asym = []
    for n, nt in ((32, 4), (64, 8)):
        P, vstar, d, e = smooth_case(n, nt)
        v = 0.5 * vstar
        _, _, states = P.gradient(v, return_states=True)
        Hd = nk.gn_matvec(P, v, d, states)
        He = nk.gn_matvec(P, v, e, states)
        a, b = P.grid.inner(e, Hd), P.grid.inner(d, He)
        asym.append(abs(a - b) / max(abs(a), abs(b)))
        assert P.grid.inner(d, Hd) > 0 and P.grid.inner(e, He) > 0
    assert asym[-1] < 1e-4 and asym[-1] < 0.25 * asym[0]


def test_gn_matvec_reduces_to_regulariser_without_image_gradient():
    shape, nt = (24, 36), 3
    P = TransportProblem(np.full(shape, 2.0), np.full(shape, 1.0), nt, 3e-2, 2)
    x = grid_x(shape)
    v = np.stack([0.3 * np.sin(x[1]), 0.2 * np.cos(x[0])])
    vt = np.stack([np.cos(2 * x[0] + x[1]), np.sin(x[0] - 3 * x[1])])
    np.testing.assert_allclose(nk.gn_matvec(P, v, vt), sp.apply_reg(P.grid, vt, 2, 3e-2),
                               rtol=0, atol=1e-10)


def test_forcing_sequence():
    assert nk.forcing(1.0, 1.0) == 0.5
    assert nk.forcing(1e-4, 1.0) == pytest.approx(1e-2)


def test_nk_reduces_the_gradient_in_few_iterations():
    wl = synth.workload("c0", shape=(32, 32))
    gen = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order)
    P = TransportProblem(wl.m0, gen.forward(wl.vstar)[-1], wl.nt, wl.alpha, wl.reg_order)
    res = nk.nk_solve(P, eps_rel=1e-3, n_iter=20)
    assert res.records[-1].ginf <= 1e-3 * res.g0inf
    assert len(res.records) <= 8
    assert [r.rho for r in res.records] == [1.0] * len(res.records)   # full Newton steps
    Js = [r.J for r in res.records]
    assert all(Js[i + 1] < Js[i] for i in range(len(Js) - 1))


# ---- preconditioners of the Newton step (h0rpc, 2lrpcsym) ---------------------
def test_gmres_solves_dense_nonsymmetric_systems():
    rng = np.random.default_rng(5)
    n = 30
    A = 3.0 * np.eye(n) + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    inner = lambda a, c: float(a @ c)
    x, its = nk.gmres(lambda p: A @ p, b, inner, 1e-13, 60)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12)
    x, its = nk.gmres(lambda p: A @ p, b, inner, 1e-2, 60)
    assert np.linalg.norm(b - A @ x) <= 1e-2 * np.linalg.norm(b) and its < n


def test_h0_matvec_is_the_gauss_newton_hessian_at_zero_velocity():
    P, _, d, e = smooth_case(32, 4)
    for x in (d, e):
        H0 = nk.h0_matvec(P, x)
        np.testing.assert_allclose(H0, nk.gn_matvec(P, np.zeros_like(x), x), rtol=0,
                                   atol=1e-12 * np.abs(H0).max())


def test_h0_preconditioner_inverts_h0():
    P, _, d, _ = smooth_case(16, 2)
    z = nk.h0_precond_apply(P, d, tol=1e-12, maxit=400)
    np.testing.assert_allclose(nk.h0_matvec(P, z), d, rtol=0, atol=1e-9 * np.abs(d).max())


def test_restriction_and_prolongation_are_spectral():
    fine, coarse = (24, 32), (12, 16)
    xf, xc = grid_x(fine), grid_x(coarse)
    f = lambda x: np.cos(2 * x[0] - 3 * x[1]) + 0.5 * np.sin(5 * x[0]) + 0.2 * np.cos(7 * x[1] + 1)
    np.testing.assert_allclose(nk.restrict(f(xf), coarse), f(xc), atol=1e-13)
    np.testing.assert_allclose(nk.prolong(f(xc), fine), f(xf), atol=1e-13)
    # modes the coarse grid drops (its Nyquist and beyond) are removed
    g = lambda x: np.cos(6 * x[0]) + np.sin(11 * x[1])
    np.testing.assert_allclose(nk.restrict(g(xf), coarse), 0.0, atol=1e-13)


@pytest.mark.parametrize("incompressible", [False, True])
def test_two_level_reduces_to_ireg_without_image_gradient(incompressible):
    shape, nt = (16, 24), 2
    P = TransportProblem(np.full(shape, 2.0), np.full(shape, 1.0), nt, 3e-2, 2,
                         incompressible=incompressible)
    x = grid_x(shape)
    v = np.stack([0.3 * np.sin(x[1]), 0.2 * np.cos(x[0])])
    r = np.stack([np.cos(2 * x[0] + x[1]) + 0.3 * np.sin(7 * x[1]), np.sin(x[0] - 3 * x[1]) + 1.0])
    z = nk.TwoLevel(P, v).apply(r)
    np.testing.assert_allclose(z, nk.precond_apply(P, r), rtol=0, atol=1e-12)
    if incompressible:
        assert np.abs(sp.divergence(P.grid, z)).max() < 1e-12


@pytest.fixture(scope="module")
def newton_system_64():
    wl = synth.workload("c0", shape=(64, 64))
    gen = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order)
    P = TransportProblem(wl.m0, gen.forward(wl.vstar)[-1], wl.nt, 1e-3, wl.reg_order)
    v = 0.5 * wl.vstar
    _, g, st = P.gradient(v, return_states=True)
    return P, v, g, st


def test_preconditioners_cut_the_cg_iterations(newton_system_64):
    """A tight solve of one Newton system (64^2, alpha = 1e-3): the zero-velocity
    Hessian and the two-level preconditioner need a fraction of the iterations
    of the regulariser preconditioner (a wrong sign or a broken operator in
    either makes it useless or divergent)."""
    P, v, g, st = newton_system_64
    H = lambda x: nk.gn_matvec(P, v, x, st)
    its = {}
    for name, Minv, flex in (("ireg", lambda r: nk.precond_apply(P, r), False),
                             ("h0rpc", lambda r: nk.h0_precond_apply(P, r), True),
                             ("2lrpcsym", nk.TwoLevel(P, v).apply, True)):
        x, its[name] = nk.pcg(H, Minv, P.grid.inner, -g, 1e-6, 300, flexible=flex)
        res = H(x) + g
        assert np.sqrt(P.grid.inner(res, res) / P.grid.inner(g, g)) <= 1e-6
    assert its["h0rpc"] <= its["ireg"] / 3 and its["2lrpcsym"] <= its["ireg"] / 2, its


def test_nk_converges_with_every_preconditioner():
    wl = synth.workload("c0", shape=(32, 32))
    gen = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order)
    P = TransportProblem(wl.m0, gen.forward(wl.vstar)[-1], wl.nt, 1e-3, wl.reg_order)
    for pc in nk.PRECONDITIONERS:
        res = nk.nk_solve(P, eps_rel=1e-2, n_iter=20, precond=pc)
        assert res.records[-1].ginf <= 1e-2 * res.g0inf, pc
        Js = [r.J for r in res.records]
        assert all(Js[i + 1] < Js[i] for i in range(len(Js) - 1)), pc
