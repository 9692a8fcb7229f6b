"""Deformation map y and the determinant of its gradient (diagnostics).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Sec. 3 (the result figures of the baseline and of the incompressible
model, Sec. 3.5): the computed transport map y, with m(1) = m0 o y, is shown
together with det grad y; all values positive means y is a diffeomorphism,
and for incompressible flows det grad y = 1 (min, mean, max and standard
deviation are reported).

Reading (the paper does not spell out how y is computed): y(x) is the foot at
t = 0 of the characteristic through x at t = 1, built with the same
semi-Lagrangian steps as the state.  Written as y(x) = x + h D(x) with a
periodic displacement D in cells,
    D^0 = 0,   D^{j+1}(i) = (X_i - i) + I[D^j](X_i),    j = 0..nt-1,
with X the state's RK2 departure points and I the periodic cubic Lagrange
interpolation; then
    grad y = Id + (h_a d D_a / d x_b)_{ab}   (spectral derivatives),
and det grad y pointwise.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp
from .interp import interpolate


def deformation_map(problem, v, X=None):
    """D^{nt} (shape (d, n...), cells) of the transport problem's velocity v."""
    if X is None:
        X, _ = problem.characteristics(v)
    disp = X - problem.nodes
    d = problem.grid.d
    D = np.zeros_like(disp)
    for _ in range(problem.nt):
        D = np.stack([disp[a] + interpolate(D[a], X) for a in range(d)])
    return D


def jacobian(grid, D):
    """grad y: J[a][b] = delta_ab + h_a dD_a/dx_b."""
    d = grid.d
    return [[(1.0 if a == b else 0.0) + grid.h[a] * sp.deriv(grid, D[a], b) for b in range(d)]
            for a in range(d)]


def determinant(J):
    """Pointwise determinant of a 2x2 or 3x3 field of matrices (list of lists)."""
    if len(J) == 2:
        return J[0][0] * J[1][1] - J[0][1] * J[1][0]
    return (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
            - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
            + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))


def det_grad_y(problem, v):
    """(D, det grad y) for velocity v."""
    D = deformation_map(problem, v)
    return D, determinant(jacobian(problem.grid, D))


def det_stats(det):
    """(min, mean, max, std) as the paper reports them."""
    det = np.asarray(det, dtype=np.float64)
    return float(det.min()), float(det.mean()), float(det.max()), float(det.std())
