"""Inexact Gauss--Newton--Krylov baseline (the paper's NK comparison).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Appendix A (eqs. e:hessian-matvec, e:incremental-state,
e:incremental-adjoint, e:newton-step): Newton steps H s = -g(v) solved
matrix-free by preconditioned CG, with a Gauss--Newton approximation of the
Hessian (the terms carrying the adjoint lam are dropped, so H_gn >= 0), a
superlinear forcing sequence for the CG tolerance, and the inverse of the
regularisation operator as preconditioner ("ireg").

  incremental state    d_t mt + grad mt . v = -grad m . vt,   mt(0) = 0
  GN incremental adj.  -d_t lt - div(lt v) = 0,   lt(1) = -mt(1)
  GN Hessian matvec    H vt = alpha L vt + int lt grad m dt  (Leray-projected
                       body force when incompressible)

Readings (the paper points to its earlier work for these):
  * lt(1) = -mt(1): the increment of lam(1) = m1 - m(1) under this build's sign
    reading of the adjoint final value (the printed mt(1) belongs to the
    opposite sign convention);
  * the incremental state is integrated along the state's characteristics with
    the trapezoidal rule for the source f = -vt . grad m:
        mt^{j+1} = I[mt^j](X) + h_t/2 (I[f^j](X) + f^{j+1});
    the GN adjoint takes the adjoint's scheme with final value -mt^{nt};
  * forcing eta_k = min(1/2, sqrt(||g_k|| / ||g_0||)) (superlinear), CG stops
    when ||r|| <= eta_k ||g_k|| or after 50 iterations; norms are <.,.>_h;
  * outer step v + rho s with Armijo backtracking from rho = 1 (c = 1e-4,
    at most 30 halvings), stop when ||g||_inf <= eps ||g_0||_inf;
  * the advection model (compressible or incompressible).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import spectral as sp
from .interp import interpolate
from .ngmres import ARMIJO_C, MAX_BACKTRACKS, LineSearchError

CG_MAXIT = 50


def gn_matvec(problem, v, vt, states=None):
    """H_gn[v] vt.  states: the dict returned by problem.gradient(v,
    return_states=True) (recomputed when None)."""
    if problem.model != "advection":
        raise ValueError("the Gauss-Newton matvec is written for the advection model")
    if states is None:
        _, _, states = problem.gradient(v, return_states=True)
    m, X, Y, cb = states["m"], states["X"], states["Y"], states["cb"]
    grid, nt, ht = problem.grid, problem.nt, problem.ht
    # source of the incremental state at every time level
    f = [-np.sum(vt * sp.gradient(grid, m[j]), axis=0) for j in range(nt + 1)]
    mt = np.zeros_like(m[0])
    for j in range(nt):
        mt = interpolate(mt, X) + 0.5 * ht * (interpolate(f[j], X) + f[j + 1])
    # Gauss-Newton incremental adjoint
    lt = [None] * (nt + 1)
    lt[nt] = -mt
    for j in range(nt - 1, -1, -1):
        nxt = interpolate(lt[j + 1], Y)
        lt[j] = cb * nxt if cb is not None else nxt
    w = problem.trapezoid_weights()
    b = np.zeros_like(v)
    for j in range(nt + 1):
        b += w[j] * lt[j] * sp.gradient(grid, m[j])
    if problem.incompressible:
        b = sp.leray(grid, b)
    return sp.apply_reg(grid, vt, problem.p, problem.alpha) + b


def precond_apply(problem, r):
    """M^-1 r = (alpha L)^-1 r (zero-mode rule; Leray-projected when incompressible)."""
    z = sp.apply_reg_inverse(problem.grid, r, problem.p, problem.alpha)
    return sp.leray(problem.grid, z) if problem.incompressible else z


def pcg(apply_H, apply_Minv, inner, b, tol, maxit=CG_MAXIT):
    """Preconditioned CG from x = 0 for H x = b; stops when ||r|| <= tol ||b||
    (norms from `inner`) or after maxit iterations, or on non-positive
    curvature (returns the iterate so far).  Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.sqrt(inner(b, b))
    if bn == 0.0:
        return x, 0
    z = apply_Minv(r)
    p = z.copy()
    rz = inner(r, z)
    for it in range(1, maxit + 1):
        Hp = apply_H(p)
        pHp = inner(p, Hp)
        if pHp <= 0.0:
            return x, it - 1
        a = rz / pHp
        x = x + a * p
        r = r - a * Hp
        if np.sqrt(inner(r, r)) <= tol * bn:
            return x, it
        z = apply_Minv(r)
        rz_new = inner(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


@dataclass
class NKRecord:
    k: int
    J: float
    ginf: float
    cg_iters: int
    rho: float
    trials: int


@dataclass
class NKResult:
    v: np.ndarray
    J: float
    g0inf: float
    records: list = field(default_factory=list)
    iterates: list = field(default_factory=list)


def forcing(gnorm, g0norm):
    return min(0.5, np.sqrt(gnorm / g0norm))


def nk_solve(problem, eps_rel=1e-2, n_iter=50, v0=None, keep_iterates=False,
             maxit=CG_MAXIT, c=ARMIJO_C, max_backtracks=MAX_BACKTRACKS):
    """Inexact GN-Krylov from v0 (default 0) until ||g||_inf <= eps_rel ||g0||_inf."""
    grid = problem.grid
    v = np.zeros((grid.d,) + grid.shape) if v0 is None else np.array(v0, dtype=np.float64)
    J, g, states = problem.gradient(v, return_states=True)
    g0inf = float(np.max(np.abs(g)))
    g0n = np.sqrt(grid.inner(g, g))
    res = NKResult(v=v, J=J, g0inf=g0inf)
    if keep_iterates:
        res.iterates.append(v.copy())
    for k in range(1, n_iter + 1):
        gn = np.sqrt(grid.inner(g, g))
        s, its = pcg(lambda x: gn_matvec(problem, v, x, states),
                     lambda r: precond_apply(problem, r), grid.inner, -g, forcing(gn, g0n), maxit)
        gs = grid.inner(g, s)
        rho, trials = 1.0, 0
        while True:
            trials += 1
            Jt = problem.objective(v + rho * s)
            if Jt < J + c * rho * gs:
                break
            if trials > max_backtracks:
                raise LineSearchError("Armijo condition not met")
            rho *= 0.5
        v = v + rho * s
        J, g, states = problem.gradient(v, return_states=True)
        ginf = float(np.max(np.abs(g)))
        res.records.append(NKRecord(k, J, ginf, its, rho, trials))
        if keep_iterates:
            res.iterates.append(v.copy())
        if ginf <= eps_rel * g0inf:
            break
    res.v, res.J = v, J
    return res
