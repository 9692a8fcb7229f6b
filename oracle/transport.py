"""State, adjoint, objective and reduced gradient (optimize-then-discretize).

Paper, Sec. 2.1 and 2.2:
  * objective  J(v) = 1/2 ||m(1) - m1||^2 + alpha/2 R(v)          (eq. e:varopt)
  * state      d_t m + grad m . v = 0,  m(0) = m0                 (eq. e:varopt)
               or, for mass-preserving transport (Sec. 3.6, eq.
               e:varopt-optimal-transport), d_t pi + div(pi v) = 0
  * adjoint    -d_t lam - div(lam v) = 0, final value at t = 1    (eq. e:adjoint)
  * gradient   g(v) = alpha L v + int_0^1 lam grad m dt           (eq. e:reduced-gradient)
  * time       n_t steps of size h_t = 1/n_t, trapezoidal rule for int dt;
               semi-Lagrangian scheme with an explicit RK2 (Heun) backtrace.

Readings (the paper is silent or garbled here):
  * adjoint final value lam(1) = m1 - m(1): the sign that makes the gradient
    above the derivative of J for the Lagrangian of eq. e:lagrangian (the
    printed final condition has the opposite sign);
  * continuity model: adjoint -d_t lam - v . grad lam = 0, lam(1) = pi1 - pi(1),
    gradient g = alpha L v - int pi grad lam dt (same Lagrangian calculus);
  * incompressible model (Sec. 3.5): Leray-projected body force,
    g = alpha L v + P int lam grad m dt;
  * the divergence source terms of the continuity state and of the advection
    adjoint are integrated with Heun's rule along the characteristic, with the
    divergence interpolated at the departure point, which gives one stationary
    multiplicative factor per grid point;
  * <a, b>_h = |h| sum a b is the spatial quadrature; g is the L2 Riesz
    representer (a grid function), so dJ(v)[d] ~ <g, d>_h.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp
from .interp import index_grid, interpolate


class TransportProblem:
    def __init__(self, m0, m1, nt: int, alpha: float, reg_order: int,
                 model: str = "advection", incompressible: bool = False):
        self.m0 = np.asarray(m0, dtype=np.float64)
        self.m1 = np.asarray(m1, dtype=np.float64)
        self.grid = sp.Grid(self.m0.shape)
        self.nt = int(nt)
        self.ht = 1.0 / self.nt
        self.alpha = float(alpha)
        self.p = int(reg_order)
        if model not in ("advection", "continuity"):
            raise ValueError(model)
        self.model = model
        self.incompressible = bool(incompressible)
        self.nodes = index_grid(self.grid.shape)

    # -- characteristics (once per stationary v) -------------------------
    def cells_per_step(self, v):
        """u_j = v_j h_t / h_j: velocity in cells per time step."""
        return np.stack([v[j] * self.ht / self.grid.h[j] for j in range(self.grid.d)])

    def characteristics(self, v):
        """RK2 departure points in index units.

        State (velocity +v):   xi* = i - u(i),  X = i - (u(i) + I[u](xi*)) / 2
        Adjoint (velocity -v): xi' = i + u(i),  Y = i + (u(i) + I[u](xi')) / 2
        """
        u = self.cells_per_step(v)
        i = self.nodes
        d = self.grid.d
        pred_x = i - u
        pred_y = i + u
        X = np.stack([i[j] - 0.5 * (u[j] + interpolate(u[j], pred_x)) for j in range(d)])
        Y = np.stack([i[j] + 0.5 * (u[j] + interpolate(u[j], pred_y)) for j in range(d)])
        return X, Y

    def source_factors(self, v, X, Y):
        """Heun factors for the divergence source terms (None if not needed).

        continuity state, d pi/dt = -delta pi along +v:
            c_f = 1 - h_t/2 (delta(X) + delta) + h_t^2/2 delta delta(X)
        advection adjoint, d lam/dtau = +delta lam along -v:
            c_b = 1 + h_t/2 (delta(Y) + delta) + h_t^2/2 delta delta(Y)
        """
        if self.incompressible:
            return None, None
        delta = sp.divergence(self.grid, v)
        ht = self.ht
        if self.model == "continuity":
            dX = interpolate(delta, X)
            cf = 1.0 - 0.5 * ht * (dX + delta) + 0.5 * ht * ht * delta * dX
            return cf, None
        dY = interpolate(delta, Y)
        cb = 1.0 + 0.5 * ht * (dY + delta) + 0.5 * ht * ht * delta * dY
        return None, cb

    # -- solves ----------------------------------------------------------
    def forward(self, v, X=None, cf=None):
        """m^0..m^nt with m^{j+1} = c_f * I[m^j](X)  (c_f = 1 for advection)."""
        if X is None:
            X, Y = self.characteristics(v)
            cf, _ = self.source_factors(v, X, Y)
        m = [self.m0.copy()]
        for _ in range(self.nt):
            nxt = interpolate(m[-1], X)
            if cf is not None:
                nxt = cf * nxt
            m.append(nxt)
        return m

    def adjoint(self, mT, Y, cb=None):
        """lam^nt = m1 - m^nt, then lam^j = c_b * I[lam^{j+1}](Y), j = nt-1..0.
        Returns the list lam^0..lam^nt."""
        lam = [None] * (self.nt + 1)
        lam[self.nt] = self.m1 - mT
        for j in range(self.nt - 1, -1, -1):
            nxt = interpolate(lam[j + 1], Y)
            if cb is not None:
                nxt = cb * nxt
            lam[j] = nxt
        return lam

    # -- objective and gradient ------------------------------------------
    def reg_value(self, v):
        return sp.reg_value(self.grid, v, self.p)

    def objective(self, v, return_parts=False):
        """J(v) = 1/2 <m(1)-m1, m(1)-m1>_h + alpha/2 R(v)."""
        m = self.forward(v)
        r = m[-1] - self.m1
        mis = 0.5 * self.grid.inner(r, r)
        reg = 0.5 * self.alpha * self.reg_value(v)
        if return_parts:
            return mis + reg, mis, reg
        return mis + reg

    def trapezoid_weights(self):
        w = np.ones(self.nt + 1)
        w[0] = w[-1] = 0.5
        return w * self.ht

    def gradient(self, v, return_states=False):
        """Returns (J(v), g(v)); g = alpha L_p v + b (b Leray-projected when
        incompressible), b = h_t sum_j w_j lam^j grad m^j (advection) or
        -h_t sum_j w_j pi^j grad lam^j (continuity)."""
        X, Y = self.characteristics(v)
        cf, cb = self.source_factors(v, X, Y)
        m = self.forward(v, X, cf)
        r = m[-1] - self.m1
        J = 0.5 * self.grid.inner(r, r) + 0.5 * self.alpha * self.reg_value(v)
        lam = self.adjoint(m[-1], Y, cb)
        wts = self.trapezoid_weights()
        b = np.zeros_like(v)
        for j in range(self.nt + 1):
            if self.model == "advection":
                b += wts[j] * lam[j] * sp.gradient(self.grid, m[j])
            else:
                b -= wts[j] * m[j] * sp.gradient(self.grid, lam[j])
        if self.incompressible:
            b = sp.leray(self.grid, b)
        g = sp.apply_reg(self.grid, v, self.p, self.alpha) + b
        if return_states:
            return J, g, dict(m=m, lam=lam, X=X, Y=Y, cf=cf, cb=cb, b=b)
        return J, g

    def relative_mismatch(self, v):
        """||m(1) - m1||_h^2 / ||m0 - m1||_h^2 (the tables' "dist")."""
        m = self.forward(v)
        r = m[-1] - self.m1
        r0 = self.m0 - self.m1
        return self.grid.inner(r, r) / self.grid.inner(r0, r0)
