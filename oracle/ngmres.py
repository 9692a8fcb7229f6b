"""Preconditioned fixed-point map, least-squares mixing and GA-NGMRES.

Paper, Sec. 2.3:
  * search direction s = -(alpha L)^-1 g(v)                 (eqs. e:searchdir, e:rpgd)
  * Armijo backtracking: accept rho when
        J(v + rho s) < J(v) + c rho <g, s>,   c = 1e-4      (eqs. e:linesearch, e:armijo)
    halving rho until it holds; rho is kept between iterations and doubled
    for the next iteration when the first trial is accepted;
  * fixed-point map q(v) = v + rho s                         (eq. e:fixedpoint)
  * AA(w) (Alg. 2) and its alternating form GA-AA(w; sigma, tau), driven by
    ga_aa below;
  * NGMRES(w) (Alg. 1) and GA-NGMRES(w; sigma, tau) (Alg. 3): with
    w_k = min(k, w) and r = g(q(v^k)),
        beta = argmin || r + sum_{i=0}^{w_k} beta_i (r - g(v^{k-i})) ||_2
        v^{k+1} = q + sum_i beta_i (q - v^{k-i});
    an iteration is a plain fixed-point step v^{k+1} = q when
    mod(k, sigma + tau) >= sigma (variant 1) or mod(k, sigma + tau) < tau
    (variant 2, aNGMRES(w)[sigma]-FP[tau]).
  * stop when ||g(v^{k+1})||_inf <= eps_rel ||g(v^0)||_inf or after n_iter
    updates.

Readings (the paper leaves these open):
  * at most 30 backtracking halvings, no cap on the stored rho; failure stops
    the solver with an error;
  * the Armijo test is strict and uses the grid inner product <.,.>_h;
  * the least-squares problem is unweighted l2 over all d*N entries, solved
    through its FP64 Gram matrix: M_ij = (r - g_i).(r - g_j),
    y_i = -(r - g_i).r, Cholesky; if Cholesky fails or the squared ratio of
    the smallest to the largest Cholesky pivot is below 1e-12, the solution
    is the eigen pseudo-inverse with cutoff 1e-12 * lambda_max;
  * the window holds the last w+1 pairs (v, g), i = 0..w_k (w_k+1 columns);
  * after a fixed-point step the stop test reuses g(q) = g(v^{k+1}).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import spectral as sp

ARMIJO_C = 1e-4
MAX_BACKTRACKS = 30
LSQ_CUTOFF = 1e-12


class LineSearchError(RuntimeError):
    pass


# -- preconditioner --------------------------------------------------------
def precond(problem, g):
    """s = -(alpha L_p)^-1 g (Leray-projected when incompressible), <g,s>_h."""
    s = -sp.apply_reg_inverse(problem.grid, g, problem.p, problem.alpha)
    if problem.incompressible:
        s = sp.leray(problem.grid, s)
    return s, problem.grid.inner(g, s)


# -- line search -----------------------------------------------------------
def armijo(objective, v, J, s, gs, rho_bar, c=ARMIJO_C, max_backtracks=MAX_BACKTRACKS):
    """Backtracking from the stored step rho_bar.

    Returns (q, J(q), rho, new rho_bar, number of trials)."""
    rho = rho_bar
    for t in range(max_backtracks + 1):
        trial = v + rho * s
        Jt = objective(trial)
        if Jt < J + c * rho * gs:
            new_bar = 2.0 * rho if t == 0 else rho
            return trial, Jt, rho, new_bar, t + 1
        rho *= 0.5
    raise LineSearchError("Armijo condition not met")


# -- least squares ---------------------------------------------------------
def gram(vectors):
    """G_ab = <u_a, u_b> (plain l2 over all entries)."""
    k = len(vectors)
    G = np.zeros((k, k))
    for a in range(k):
        for b in range(a, k):
            G[a, b] = G[b, a] = float(np.sum(vectors[a] * vectors[b]))
    return G


def lsq_from_gram(G):
    """beta from the Gram matrix of u = [r, g_0, ..., g_w]."""
    Grr = G[0, 0]
    Gr = G[0, 1:]
    M = Grr - Gr[:, None] - Gr[None, :] + G[1:, 1:]
    y = -(Grr - Gr)
    try:
        L = np.linalg.cholesky(M)
        piv = np.diag(L) ** 2
        if piv.min() >= LSQ_CUTOFF * piv.max():
            z = np.linalg.solve(L, y)
            return np.linalg.solve(L.T, z)
    except np.linalg.LinAlgError:
        pass
    lam, Q = np.linalg.eigh(M)
    lmax = lam.max()
    keep = lam > LSQ_CUTOFF * lmax
    return Q[:, keep] @ ((Q[:, keep].T @ y) / lam[keep])


def lsq_direct(r, gs):
    """Cross-check: numpy lstsq on the explicit difference matrix."""
    D = np.stack([(r - g).ravel() for g in gs], axis=1)
    return np.linalg.lstsq(D, -r.ravel(), rcond=None)[0]


def is_fp_step(k, sigma, tau, variant="GA"):
    if variant == "GA":
        return (k % (sigma + tau)) >= sigma
    if variant == "ALT":
        return (k % (sigma + tau)) < tau
    raise ValueError(variant)


@dataclass
class Record:
    k: int
    kind: str
    J: float
    ginf: float
    beta: np.ndarray | None = None
    rho: float | None = None
    trials: int = 0


@dataclass
class Result:
    v: np.ndarray
    J: float
    g: np.ndarray
    iterations: int
    g0inf: float
    records: list = field(default_factory=list)
    iterates: list = field(default_factory=list)
    n_grad: int = 0
    n_obj: int = 0


def ga_ngmres(grad, qmap, v0, w, sigma, tau, eps_rel, n_iter, variant="GA",
              lsq=lsq_from_gram, keep_iterates=False):
    """Generic GA-NGMRES(w; sigma, tau) (Alg. 3; tau = 0 gives Alg. 1).

    grad(v) -> (J, g);  qmap(v, J, g) -> (q, info dict).  sigma = 0 gives the
    plain fixed-point iteration (RPGD when qmap is the line-searched map)."""
    v = np.array(v0, dtype=np.float64)
    J, g = grad(v)
    n_grad = 1
    g0 = float(np.max(np.abs(g)))
    hist = [(v, g)]                      # most recent last, at most w+1 pairs
    res = Result(v=v, J=J, g=g, iterations=0, g0inf=g0)
    if keep_iterates:
        res.iterates.append(v.copy())
    k = 0
    while True:
        wk = min(k, w)
        q, info = qmap(v, J, g)
        Jq, gq = grad(q)
        n_grad += 1
        fp = sigma == 0 or is_fp_step(k, sigma, tau, variant)
        beta = None
        if fp:
            v, J, g = q, Jq, gq
        else:
            window = hist[::-1][: wk + 1]        # i = 0..w_k : v^{k-i}
            beta = lsq(gq, [gp for _, gp in window]) if lsq is lsq_direct \
                else lsq(gram([gq] + [gp for _, gp in window]))
            vn = q.copy()
            for b, (vp, _) in zip(beta, window):
                vn = vn + b * (q - vp)
            v = vn
            J, g = grad(v)
            n_grad += 1
        hist.append((v, g))
        if len(hist) > w + 1:
            hist.pop(0)
        k += 1
        ginf = float(np.max(np.abs(g)))
        res.records.append(Record(k, "fp" if fp else "ngmres", J, ginf, beta,
                                  info.get("rho"), info.get("trials", 0)))
        if keep_iterates:
            res.iterates.append(v.copy())
        if ginf <= eps_rel * g0 or k >= n_iter:
            break
    res.v, res.J, res.g, res.iterations = v, J, g, k
    res.n_grad = n_grad
    return res


def ga_aa(grad, qmap, v0, w, sigma, tau, eps_rel, n_iter, variant="GA",
          lsq=lsq_from_gram, keep_iterates=False):
    """Generic GA-AA(w; sigma, tau): Alg. 2 (Anderson acceleration) with the
    alternation of Alg. 3.  With r^k = v^k - q(v^k) and w_k = min(k, w),
        xi = argmin || r^k + sum_{i=1}^{w_k} xi_i (r^k - r^{k-i}) ||_2
        v^{k+1} = q(v^k) + sum_i xi_i (q(v^k) - q(v^{k-i}));
    an iteration is a plain fixed-point step v^{k+1} = q(v^k) when the switch
    of Alg. 3 says so, and when w_k = 0.  The pairs (r, q) of the last w
    iterations are kept."""
    v = np.array(v0, dtype=np.float64)
    J, g = grad(v)
    n_grad = 1
    g0 = float(np.max(np.abs(g)))
    hist = []                            # (r, q), most recent last, at most w
    res = Result(v=v, J=J, g=g, iterations=0, g0inf=g0)
    if keep_iterates:
        res.iterates.append(v.copy())
    k = 0
    while True:
        wk = min(k, w)
        q, info = qmap(v, J, g)
        r = v - q
        fp = sigma == 0 or is_fp_step(k, sigma, tau, variant) or wk == 0
        xi = None
        if fp:
            vn = q
            J, g = grad(vn)
            n_grad += 1
        else:
            window = hist[::-1][:wk]          # i = 1..w_k : (r^{k-i}, q^{k-i})
            xi = lsq(gram([r] + [rp for rp, _ in window]))
            vn = q.copy()
            for c, (_, qp) in zip(xi, window):
                vn = vn + c * (q - qp)
            J, g = grad(vn)
            n_grad += 1
        hist.append((r, q))
        if len(hist) > w:
            hist.pop(0)
        v = vn
        k += 1
        ginf = float(np.max(np.abs(g)))
        res.records.append(Record(k, "fp" if fp else "aa", J, ginf, xi,
                                  info.get("rho"), info.get("trials", 0)))
        if keep_iterates:
            res.iterates.append(v.copy())
        if ginf <= eps_rel * g0 or k >= n_iter:
            break
    res.v, res.J, res.g, res.iterations = v, J, g, k
    res.n_grad = n_grad
    return res


class LineSearchMap:
    """q(v) = v - rho (alpha L)^-1 g(v) with Armijo backtracking and rho memory."""

    def __init__(self, problem, rho0=1.0):
        self.problem = problem
        self.rho_bar = rho0
        self.n_obj = 0

    def __call__(self, v, J, g):
        s, gs = precond(self.problem, g)

        def obj(x):
            self.n_obj += 1
            return self.problem.objective(x)

        q, Jq, rho, self.rho_bar, trials = armijo(obj, v, J, s, gs, self.rho_bar)
        return q, dict(rho=rho, trials=trials, Jq=Jq)


def solve(problem, w=5, sigma=2, tau=1, eps_rel=1e-2, n_iter=200, variant="GA",
          v0=None, keep_iterates=False, accel="ngmres"):
    """GA-NGMRES (accel="ngmres") or GA-AA (accel="aa") on the transport
    problem starting from v0 (default 0)."""
    v0 = np.zeros((problem.grid.d,) + problem.grid.shape) if v0 is None else v0
    qmap = LineSearchMap(problem)
    driver = {"ngmres": ga_ngmres, "aa": ga_aa}[accel]
    res = driver(problem.gradient, qmap, v0, w, sigma, tau, eps_rel, n_iter,
                 variant=variant, keep_iterates=keep_iterates)
    res.n_obj = qmap.n_obj
    return res
