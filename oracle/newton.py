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
  * lt(1) = -mt(1): the increment of lam(1) = m1 - m(1) under this implementation's sign
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

Preconditioners of the Newton step (Appendix A): "ireg" is (alpha L)^-1; the
two below replace it by an inexact inverse of an approximate Hessian, solved
by an inner Krylov method, so the outer PCG takes the flexible
(Polak-Ribiere) update beta = <r_new - r_old, z_new> / <r_old, z_old>, which
equals the usual one for a fixed preconditioner.

  * "h0rpc" (zero-velocity approximation): H0 vt = alpha L vt + [P] grad m0
    (grad m0 . vt), the Gauss-Newton Hessian at v = 0 (no PDE solves),
    inverted by GMRES on the left regularisation-preconditioned system
    (alpha L)^-1 H0 z = (alpha L)^-1 r (not symmetric, hence GMRES);
  * "2lrpcsym" (two-level): the low-frequency part of the Hessian in the
    symmetric regularisation-preconditioned form
    H_pc = I + Hreg^-1/2 H_data Hreg^-1/2, Hreg = alpha L, inverted by CG on
    a grid with half the cells per axis, where H_data is the Gauss-Newton data
    term of the same problem discretised there (images and velocity
    restricted spectrally); the high frequencies take Hreg^-1:
        M^-1 r = prolong(Hreg^-1/2 y) + P_hf Hreg^-1 r,
        (I + Hreg^-1/2 H_data,c Hreg^-1/2) y = Hreg^-1/2 restrict(r).
    The coarse grid keeps the wavenumbers |k_i| <= n_i/4 - 1 (its Nyquist
    modes dropped, so restriction and prolongation are exact inverses there);
    P_hf removes exactly those modes.

Readings for both (the paper gives neither tolerance): the inner solve stops
at a relative residual of PC_TOL or after PC_MAXIT iterations; the coarse
grid halves every axis (all even).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import spectral as sp
from .interp import interpolate
from .ngmres import ARMIJO_C, MAX_BACKTRACKS, LineSearchError

CG_MAXIT = 50
PC_TOL = 1e-1
PC_MAXIT = 10
PRECONDITIONERS = ("ireg", "h0rpc", "2lrpcsym")


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


def pcg(apply_H, apply_Minv, inner, b, tol, maxit=CG_MAXIT, flexible=False):
    """Preconditioned CG from x = 0 for H x = b; stops when ||r|| <= tol ||b||
    (norms from `inner`) or after maxit iterations, or on non-positive
    curvature (returns the iterate so far).  flexible: Polak-Ribiere beta (for
    a preconditioner that is itself an inexact iterative solve).  Returns
    (x, iterations)."""
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
        r_old = r
        r = r - a * Hp
        if np.sqrt(inner(r, r)) <= tol * bn:
            return x, it
        z = apply_Minv(r)
        rz_new = inner(r, z)
        beta = ((rz_new - inner(r_old, z)) if flexible else rz_new) / rz
        p = z + beta * p
        rz = rz_new
    return x, maxit


def gmres(apply_A, b, inner, tol, maxit):
    """GMRES from x = 0 (no restart) for A x = b: x minimises ||b - A x|| over
    the Krylov space (Arnoldi with modified Gram-Schmidt, Givens rotations on
    the Hessenberg matrix; norms from `inner`).  Stops when the residual norm
    is <= tol ||b|| or after maxit iterations.  Returns (x, iterations)."""
    bn = np.sqrt(inner(b, b))
    x = np.zeros_like(b)
    if bn == 0.0:
        return x, 0
    V = [b / bn]
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    e = np.zeros(maxit + 1)
    e[0] = bn
    its = 0
    for j in range(maxit):
        w = apply_A(V[j])
        for i in range(j + 1):
            H[i, j] = inner(w, V[i])
            w = w - H[i, j] * V[i]
        hn = np.sqrt(inner(w, w))
        H[j + 1, j] = hn
        for i in range(j):   # previous rotations on the new column
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j], H[j + 1, j] = den, 0.0
        e[j + 1] = -sn[j] * e[j]
        e[j] = cs[j] * e[j]
        its = j + 1
        if abs(e[j + 1]) <= tol * bn or hn == 0.0:   # converged, or the space is invariant
            break
        V.append(w / hn)
    y = np.linalg.solve(np.triu(H[:its, :its]), e[:its])
    for i in range(its):
        x = x + y[i] * V[i]
    return x, its


def h0_matvec(problem, vt, grad_m0=None):
    """H0 vt = alpha L vt + [P] grad m0 (grad m0 . vt): the Gauss-Newton
    Hessian at v = 0."""
    grid = problem.grid
    gm = sp.gradient(grid, problem.m0) if grad_m0 is None else grad_m0
    data = np.sum(gm * vt, axis=0) * gm
    if problem.incompressible:
        data = sp.leray(grid, data)
    return sp.apply_reg(grid, vt, problem.p, problem.alpha) + data


def h0_precond_apply(problem, r, grad_m0=None, tol=PC_TOL, maxit=PC_MAXIT):
    """z ~ H0^-1 r by GMRES on (alpha L)^-1 H0 z = (alpha L)^-1 r."""
    grid = problem.grid
    gm = sp.gradient(grid, problem.m0) if grad_m0 is None else grad_m0
    z, _ = gmres(lambda x: precond_apply(problem, h0_matvec(problem, x, gm)),
                 precond_apply(problem, r), grid.inner, tol, maxit)
    return z


# ---- two-level preconditioner ---------------------------------------------
def _kept_modes(n_f, n_c):
    """Fine and coarse FFT indices of the wavenumbers |k| <= n_c/2 - 1."""
    m = n_c // 2 - 1
    ks = np.arange(-m, m + 1)
    return ks % n_f, ks % n_c


def restrict(f, shape_c):
    """Spectral restriction of a scalar field to the coarse grid (the kept
    wavenumbers, values of the band-limited interpolant)."""
    F = np.fft.fftn(f)
    idx = [_kept_modes(nf, nc) for nf, nc in zip(f.shape, shape_c)]
    G = np.zeros(shape_c, dtype=complex)
    G[np.ix_(*[c for _, c in idx])] = F[np.ix_(*[fi for fi, _ in idx])] * (
        np.prod(shape_c) / np.prod(f.shape))
    return np.real(np.fft.ifftn(G))


def prolong(fc, shape_f):
    """Spectral prolongation of a coarse scalar field (zero padding)."""
    G = np.fft.fftn(fc)
    idx = [_kept_modes(nf, nc) for nf, nc in zip(shape_f, fc.shape)]
    F = np.zeros(shape_f, dtype=complex)
    F[np.ix_(*[fi for fi, _ in idx])] = G[np.ix_(*[c for _, c in idx])] * (
        np.prod(shape_f) / np.prod(fc.shape))
    return np.real(np.fft.ifftn(F))


def _vec(op, v, shape):
    return np.stack([op(v[c], shape) for c in range(v.shape[0])])


def reg_inverse_sqrt(grid, v, p, alpha, incompressible):
    """Hreg^-1/2 v = (alpha L_p)^-1/2 v (zero symbol entry set to one), Leray-projected
    when incompressible."""
    lp = sp.symbol(grid, p).astype(np.float64)
    lp = np.where(lp == 0.0, 1.0, lp)
    out = np.stack([sp.ifft(sp.fft(v[c]) / np.sqrt(alpha * lp)) for c in range(v.shape[0])])
    return sp.leray(grid, out) if incompressible else out


class TwoLevel:
    """The 2lrpcsym preconditioner at the velocity v (the coarse problem's
    state history is computed once per v)."""

    def __init__(self, problem, v, tol=PC_TOL, maxit=PC_MAXIT):
        from .transport import TransportProblem
        if any(n % 2 for n in problem.grid.shape):
            raise ValueError("the two-level preconditioner halves every axis: sizes must be even")
        self.P = problem
        self.tol, self.maxit = tol, maxit
        self.shape_c = tuple(n // 2 for n in problem.grid.shape)
        self.Pc = TransportProblem(restrict(problem.m0, self.shape_c),
                                   restrict(problem.m1, self.shape_c), problem.nt, problem.alpha,
                                   problem.p, model=problem.model,
                                   incompressible=problem.incompressible)
        self.vc = _vec(restrict, v, self.shape_c)
        _, _, self.states = self.Pc.gradient(self.vc, return_states=True)

    def coarse_operator(self, y):
        """(I + Hreg^-1/2 H_data,c Hreg^-1/2) y on the kept wavenumbers."""
        Pc, g = self.Pc, self.Pc.grid
        R = lambda x: reg_inverse_sqrt(g, x, Pc.p, Pc.alpha, Pc.incompressible)
        x = R(y)
        data = gn_matvec(Pc, self.vc, x, self.states) - sp.apply_reg(g, x, Pc.p, Pc.alpha)
        out = y + R(data)
        return _vec(restrict, _vec(prolong, out, self.P.grid.shape), self.shape_c)

    def apply(self, r):
        P, Pc = self.P, self.Pc
        g = Pc.grid
        R = lambda x: reg_inverse_sqrt(g, x, Pc.p, Pc.alpha, Pc.incompressible)
        rc = _vec(restrict, r, self.shape_c)
        y, _ = pcg(self.coarse_operator, lambda x: x, g.inner, R(rc), self.tol, self.maxit)
        low = _vec(prolong, R(y), P.grid.shape)
        high = precond_apply(P, r - _vec(prolong, rc, P.grid.shape))
        return low + high


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
             maxit=CG_MAXIT, c=ARMIJO_C, max_backtracks=MAX_BACKTRACKS, precond="ireg"):
    """Inexact GN-Krylov from v0 (default 0) until ||g||_inf <= eps_rel ||g0||_inf,
    with the preconditioner "ireg", "h0rpc" or "2lrpcsym"."""
    if precond not in PRECONDITIONERS:
        raise ValueError(f"unknown preconditioner {precond!r}")
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
        if precond == "ireg":
            Minv = lambda r: precond_apply(problem, r)
        elif precond == "h0rpc":
            gm0 = sp.gradient(grid, problem.m0)
            Minv = lambda r: h0_precond_apply(problem, r, gm0)
        else:
            Minv = TwoLevel(problem, v).apply
        s, its = pcg(lambda x: gn_matvec(problem, v, x, states), Minv, grid.inner, -g,
                     forcing(gn, g0n), maxit, flexible=precond != "ireg")
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
