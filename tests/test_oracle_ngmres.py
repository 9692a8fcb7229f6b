"""Pins of the oracle's line search, least squares and GA-NGMRES loop.

Linear-case equivalences (Sec. 2.3): with g(v) = A v - b and the Richardson
map q(v) = v - g(v), NGMRES with an untruncated window reproduces GMRES, and
GA-NGMRES(w; 1, w) reproduces restarted GMRES(w+1) after every NGMRES step.
Both are checked against a brute-force GMRES (explicit Krylov basis and a
dense least-squares solve).  The special cases listed after Alg. 3 and the
window semantics min(k, w) are checked on the transport problem itself.
"""
import numpy as np
import pytest

import synth
from oracle import ngmres as ng
from oracle.transport import TransportProblem


def linear_backend(n=30, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(0.3, 1.6, n)) @ Q.T
    b = rng.standard_normal(n)

    def grad(v):
        r = A @ v - b
        return 0.5 * v @ A @ v - b @ v, r

    def qmap(v, J, g):
        return v - g, {}

    return A, b, grad, qmap


def gmres_bruteforce(A, b, x0, k):
    """argmin ||A x - b|| over x0 + K_k(A, r0) with an orthonormal Krylov basis."""
    r0 = A @ x0 - b
    K = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], axis=1)
    Qk, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(A @ Qk, -r0, rcond=None)[0]
    return x0 + Qk @ c


def test_ngmres_infinite_window_is_gmres():
    A, b, grad, qmap = linear_backend()
    x0 = np.zeros_like(b)
    res = ng.ga_ngmres(grad, qmap, x0, w=100, sigma=1, tau=0, eps_rel=1e-14,
                       n_iter=10, keep_iterates=True)
    for k in range(1, 11):
        xk = gmres_bruteforce(A, b, x0, k)
        np.testing.assert_allclose(res.iterates[k], xk, rtol=0, atol=1e-10 * np.abs(xk).max())
    # and the residual norms are monotone
    norms = [np.linalg.norm(A @ x - b) for x in res.iterates]
    assert all(norms[i + 1] <= norms[i] for i in range(len(norms) - 1))


@pytest.mark.parametrize("w", [1, 2, 3])
def test_ga_ngmres_w_1_w_is_restarted_gmres(w):
    A, b, grad, qmap = linear_backend(seed=w)
    x0 = np.zeros_like(b)
    cycles = 3
    res = ng.ga_ngmres(grad, qmap, x0, w=w, sigma=1, tau=w, eps_rel=1e-14,
                       n_iter=(w + 1) * cycles + 1, keep_iterates=True)
    kinds = [r.kind for r in res.records]
    assert kinds[0] == "ngmres" and kinds[1:w + 1] == ["fp"] * w
    for j in range(1, cycles + 1):
        start = res.iterates[(w + 1) * (j - 1) + 1]
        expect = gmres_bruteforce(A, b, start, w + 1)
        np.testing.assert_allclose(res.iterates[(w + 1) * j + 1], expect,
                                   atol=1e-10 * np.abs(expect).max())


def test_lsq_gram_matches_lstsq_and_handles_rank_deficiency():
    rng = np.random.default_rng(4)
    r = rng.standard_normal(200)
    gs = [rng.standard_normal(200) for _ in range(4)]
    beta = ng.lsq_from_gram(ng.gram([r] + gs))
    np.testing.assert_allclose(beta, ng.lsq_direct(r, gs), rtol=1e-10)
    # duplicated history vector: fallback to the pseudo-inverse; the residual
    # equals the least-squares optimum and the solution is minimum-norm
    gs2 = gs[:2] + [gs[1].copy()] + gs[2:]
    b2 = ng.lsq_from_gram(ng.gram([r] + gs2))
    D = np.stack([r - g for g in gs2], axis=1)
    assert np.linalg.norm(r + D @ b2) == pytest.approx(np.linalg.norm(r + D @ ng.lsq_direct(r, gs2)),
                                                       rel=1e-10)
    assert b2[1] == pytest.approx(b2[2], rel=1e-10)


def test_armijo_backtracking_and_rho_memory():
    # J(v) = 1/2 a v^2 along s = -1 from v = 1: J(1 + rho s) < J(1) + c rho <g,s>
    a = 4.0
    J = lambda x: 0.5 * a * x * x
    v, g = 1.0, a
    s, gs = -1.0, -a
    calls = []

    def obj(x):
        calls.append(x)
        return J(x)

    # from rho = 1: trial 1 - 1 = 0 gives J = 0 < 2 - 4e-4: accepted at once,
    # stored step doubles
    q, Jq, rho, bar, t = ng.armijo(obj, v, J(v), s, gs, 1.0)
    assert (q, rho, bar, t) == (0.0, 1.0, 2.0, 1)
    # from rho = 4: trials 4 (J=18), 2 (J=2, not < 2 - 8e-4), 1 -> accepted
    calls.clear()
    q, Jq, rho, bar, t = ng.armijo(obj, v, J(v), s, gs, 4.0)
    assert calls == [-3.0, -1.0, 0.0] and (rho, bar, t) == (1.0, 1.0, 3)
    with pytest.raises(ng.LineSearchError):
        ng.armijo(obj, v, J(v), 1.0, 1.0, 1.0, max_backtracks=3)   # ascent direction


def _small_problem(shape=(24, 24)):
    wl = synth.workload("c0", shape=shape)
    m1 = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order).forward(wl.vstar)[-1]
    return TransportProblem(wl.m0, m1, wl.nt, wl.alpha, wl.reg_order)


def test_precond_direction_is_descent():
    P = _small_problem()
    _, g = P.gradient(0.3 * np.ones((2,) + P.grid.shape))
    s, gs = ng.precond(P, g)
    assert gs < 0
    np.testing.assert_allclose(P.grid.inner(g, s), gs)


def _run(P, **kw):
    res = ng.solve(P, eps_rel=1e-12, **kw)
    return np.stack([r.J for r in res.records]), res.v


def test_tau_zero_identity_and_variants():
    P = _small_problem()
    base = _run(P, w=3, sigma=1, tau=0, n_iter=6)
    for sigma in (2, 5):
        other = _run(P, w=3, sigma=sigma, tau=0, n_iter=6)
        np.testing.assert_array_equal(base[0], other[0])
        np.testing.assert_array_equal(base[1], other[1])
    alt = _run(P, w=3, sigma=1, tau=0, n_iter=6, variant="ALT")
    np.testing.assert_array_equal(base[1], alt[1])


def test_window_independence_when_n_iter_le_w():
    P = _small_problem()
    a = _run(P, w=5, sigma=2, tau=1, n_iter=5)
    b = _run(P, w=50, sigma=2, tau=1, n_iter=5)
    np.testing.assert_array_equal(a[1], b[1])
    # and a window that truncates does change the result
    c = _run(P, w=1, sigma=2, tau=1, n_iter=5)
    assert np.max(np.abs(a[1] - c[1])) > 0


def test_switch_semantics():
    P = _small_problem()
    res = ng.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=7)
    assert [r.kind for r in res.records] == ["ngmres", "ngmres", "fp"] * 2 + ["ngmres"]
    res = ng.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=7, variant="ALT")
    assert [r.kind for r in res.records] == ["fp", "ngmres", "ngmres"] * 2 + ["fp"]
    # sigma = 0 is the plain line-searched fixed-point iteration (RPGD)
    res = ng.solve(P, w=5, sigma=0, tau=1, eps_rel=1e-12, n_iter=3)
    assert [r.kind for r in res.records] == ["fp"] * 3


def test_determinism_and_descent():
    P = _small_problem()
    a = ng.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=8)
    b = ng.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=8)
    np.testing.assert_array_equal(a.v, b.v)
    assert a.records[-1].ginf < 0.2 * a.g0inf
    assert a.records[-1].J < P.objective(np.zeros_like(a.v))


# -- Anderson acceleration (Alg. 2) and GA-AA -----------------------------------
def test_aa_infinite_window_is_q_of_gmres():
    """Linear case: the AA iterate v^{k+1} equals q applied to the k-step GMRES
    iterate (Sec. 2.3)."""
    A, b, grad, qmap = linear_backend(seed=7)
    x0 = np.zeros_like(b)
    res = ng.ga_aa(grad, qmap, x0, w=100, sigma=1, tau=0, eps_rel=1e-14, n_iter=10,
                   keep_iterates=True)
    for k in range(1, 10):
        xk = gmres_bruteforce(A, b, x0, k)
        qx = xk - (A @ xk - b)
        np.testing.assert_allclose(res.iterates[k + 1], qx, atol=1e-10 * np.abs(qx).max())


def test_aa_switch_and_window_semantics():
    P = _small_problem()
    res = ng.solve(P, w=3, sigma=2, tau=1, eps_rel=1e-12, n_iter=7, accel="aa")
    # k = 0 has an empty window: a plain fixed-point step
    assert [r.kind for r in res.records] == ["fp", "aa", "fp", "aa", "aa", "fp", "aa"]
    a = ng.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=5, accel="aa")
    b = ng.solve(P, w=40, sigma=2, tau=1, eps_rel=1e-12, n_iter=5, accel="aa")
    np.testing.assert_array_equal(a.v, b.v)
    # w = 0: every step is the line-searched fixed-point step (RPGD)
    c = ng.solve(P, w=0, sigma=1, tau=0, eps_rel=1e-12, n_iter=4, accel="aa")
    d = ng.solve(P, w=0, sigma=0, tau=1, eps_rel=1e-12, n_iter=4)
    np.testing.assert_array_equal(c.v, d.v)
