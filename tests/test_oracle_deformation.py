"""Pins of the oracle's deformation map y and det grad y.

Closed forms: a constant velocity of whole cells per step (exact shift, det 1);
a shear v = (c sin x2, 0), whose map y = x - t v is reproduced by the RK2
scheme to rounding (det 1); the flow v = (c sin x1, 0), whose map is known in
closed form (tan(y/2) = tan(x/2) e^{-c}), approached at second order under
joint refinement.  Invariants: in 2-D the mean of det grad y over a periodic
grid is exactly 1 (the quadratic terms cancel by Parseval), and an
incompressible flow gives det grad y -> 1 under refinement.
"""
import math

import numpy as np

import synth
from oracle import deformation as dfm
from oracle.transport import TransportProblem

PI = math.pi


def grid_x(shape):
    return np.meshgrid(*[2 * PI * np.arange(n) / n for n in shape], indexing="ij")


def problem(shape, nt, incompressible=False):
    z = np.zeros(shape)
    return TransportProblem(z, z, nt, 1e-2, 1, incompressible=incompressible)


def test_integer_shift_is_exact():
    shape, nt = (16, 24), 4
    P = problem(shape, nt)
    h = P.grid.h
    u = np.array([2.0, -1.0])                 # cells per step
    v = np.stack([np.full(shape, u[j] * h[j] / P.ht) for j in range(2)])
    D, det = dfm.det_grad_y(P, v)
    for j in range(2):
        np.testing.assert_allclose(D[j], -nt * u[j], rtol=0, atol=1e-12)
    np.testing.assert_allclose(det, 1.0, rtol=0, atol=1e-13)


def test_shear_map_is_reproduced():
    shape, nt, c = (32, 32), 4, 0.7
    P = problem(shape, nt)
    x = grid_x(shape)
    v = np.stack([c * np.sin(x[1]), np.zeros(shape)])
    D, det = dfm.det_grad_y(P, v)
    np.testing.assert_allclose(D[0] * P.grid.h[0], -v[0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(D[1], 0.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(det, 1.0, rtol=0, atol=1e-12)


def flow_map(x1, c):
    """Foot at t = 0 of the characteristic of v = (c sin x1, 0) through x1 at
    t = 1, and its derivative."""
    s, co = np.sin(x1 / 2), np.cos(x1 / 2)
    y = 2 * np.arctan2(np.exp(-c) * s, co)
    jac = np.exp(-c) / (co ** 2 + np.exp(-2 * c) * s ** 2)
    return y, jac


def test_sine_flow_converges_at_second_order():
    c = 0.5
    errs_y, errs_det = [], []
    for n, nt in ((32, 4), (64, 8), (128, 16)):
        P = problem((n, n), nt)
        x = grid_x((n, n))
        v = np.stack([c * np.sin(x[0]), np.zeros((n, n))])
        D, det = dfm.det_grad_y(P, v)
        y, jac = flow_map(x[0], c)
        dy = np.angle(np.exp(1j * (y - x[0])))            # periodic difference
        errs_y.append(np.max(np.abs(D[0] * P.grid.h[0] - dy)))
        errs_det.append(np.max(np.abs(det - jac)))
        np.testing.assert_allclose(D[1], 0.0, atol=1e-14)
    order = lambda e: [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    assert errs_y[-1] < 1e-4 and errs_det[-1] < 1e-3
    assert min(order(errs_y)) > 1.8 and min(order(errs_det)) > 1.8


def test_mean_determinant_is_one_in_2d():
    wl = synth.workload("c0", shape=(48, 36))
    P = problem(wl.shape, wl.nt)
    D, det = dfm.det_grad_y(P, 3.0 * wl.vstar)
    assert abs(det.mean() - 1.0) < 1e-13
    assert det.std() > 1e-3                  # a genuinely compressible map
    lo, mean, hi, std = dfm.det_stats(det)
    assert lo <= mean <= hi and std == det.std()


def test_incompressible_flow_preserves_volume_under_refinement():
    devs = []
    for n, nt in ((16, 2), (32, 4), (64, 8)):
        wl = synth.workload("c2", shape=(n, n, n))
        P = problem(wl.shape, nt, incompressible=True)
        D, det = dfm.det_grad_y(P, wl.vstar)
        devs.append(np.max(np.abs(det - 1.0)))
    assert devs[-1] < 5e-3
    assert devs[0] / devs[-1] > 8.0          # at least second order over two halvings
