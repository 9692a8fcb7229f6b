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
