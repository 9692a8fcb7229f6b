"""Adjoint identities of the oracle's transport operators.

The interpolation I_X (Sec. 2.2: a semi-Lagrangian step evaluates the field at
the departure points X) is linear in the transported field, so it has a
transpose I_X^T, a scatter: every departure point p hands w_o(p) b(p) to each
node of its stencil.  The scatter is written out here, independently of the
oracle's gather, from the cubic Lagrange basis on the nodes -1, 0, 1, 2; the
identity <I_X a, b>_h = <a, I_X^T b>_h on random a, b and a random smooth X
then fails for a wrong node offset, weight, wrap or axis order in the gather.
The same holds for the n_t-step state map S_v (m(1) = S_v m0, with the factor
c_f of the continuity model) and its transpose, the scatter applied n_t times.
"""
import math

import numpy as np
import pytest

import synth
from oracle.interp import index_grid
from oracle.transport import TransportProblem

PI = math.pi


def cubic_basis(t):
    # Lagrange polynomials of the nodes -1, 0, 1, 2 (textbook products)
    nodes = (-1.0, 0.0, 1.0, 2.0)
    out = []
    for i, xi in enumerate(nodes):
        w = np.ones_like(t)
        for j, xj in enumerate(nodes):
            if j != i:
                w = w * (t - xj) / (xi - xj)
        out.append(w)
    return out


def scatter_transpose(b, X):
    """I_X^T b: for every point p, add w(p) b(p) to each stencil node."""
    shape = b.shape
    d = b.ndim
    f = np.floor(X).astype(np.int64)
    w = [cubic_basis(X[j] - f[j]) for j in range(d)]
    out = np.zeros(shape)
    bf = b.reshape(-1)
    fl = [f[j].reshape(-1) for j in range(d)]
    wl = [[w[j][o].reshape(-1) for o in range(4)] for j in range(d)]
    for offs in np.ndindex(*([4] * d)):
        idx = tuple(np.mod(fl[j] + offs[j] - 1, shape[j]) for j in range(d))
        wt = np.ones_like(bf)
        for j in range(d):
            wt = wt * wl[j][offs[j]]
        np.add.at(out, idx, wt * bf)
    return out


def smooth_departures(shape, seed, amp):
    """X = i + a smooth periodic displacement of up to `amp` cells."""
    rng = np.random.default_rng(seed)
    disp = synth.random_velocity(shape, 3, 1.0, rng)
    disp *= amp / np.abs(disp).max()
    return index_grid(shape) + disp


def inner_h(a, b):
    cell = np.prod([2 * PI / n for n in a.shape])
    return cell * float(np.sum(a * b))


@pytest.mark.parametrize("shape,amp", [((12, 20), 2.5), ((9, 10, 14), 1.7), ((16, 6), 7.3)])
def test_interpolation_matches_its_scatter_transpose(shape, amp):
    rng = np.random.default_rng(11)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    X = smooth_departures(shape, 5, amp)
    P = TransportProblem(a, a, 1, 1.0, 1)
    Ia = P.forward(np.zeros((len(shape),) + shape), X=X)[-1]   # one step: I_X a
    lhs = inner_h(Ia, b)
    rhs = inner_h(a, scatter_transpose(b, X))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + inner_h(np.abs(Ia), np.abs(b)))


def test_scatter_transpose_catches_a_shifted_stencil():
    # the identity is not vacuous: a gather whose stencil starts one node late
    # (nodes f..f+3) breaks it by far more than rounding
    shape = (12, 20)
    rng = np.random.default_rng(3)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    X = smooth_departures(shape, 5, 2.5)
    P = TransportProblem(a, a, 1, 1.0, 1)
    Ia_wrong = P.forward(np.zeros((2,) + shape), X=X + 1.0)[-1]
    rhs = inner_h(a, scatter_transpose(b, X))
    assert abs(inner_h(Ia_wrong, b) - rhs) > 1e-3 * abs(rhs)


@pytest.mark.parametrize("model", ["advection", "continuity"])
@pytest.mark.parametrize("name,shape,nt", [("c0", (16, 24), 4), ("c2", (8, 10, 12), 2)])
def test_state_map_adjoint_identity(name, shape, nt, model):
    """<S_v a, b>_h = <a, S_v^T b>_h with S_v^T = (I_X^T diag(c_f))^{n_t}."""
    if model == "continuity" and name == "c2":
        pytest.skip("the incompressible workload is an advection problem")
    wl = synth.workload(name, shape=shape)
    rng = np.random.default_rng(21)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    P = TransportProblem(a, a, nt, 1.0, 1, model=model)
    v = 2.0 * wl.vstar
    X, Y = P.characteristics(v)
    cf, _ = P.source_factors(v, X, Y)
    if model == "continuity":
        assert cf is not None
    Sa = P.forward(v)[-1]
    t = b.copy()
    for _ in range(nt):
        t = scatter_transpose(t if cf is None else cf * t, X)
    lhs = inner_h(Sa, b)
    rhs = inner_h(a, t)
    assert abs(lhs - rhs) <= 1e-12 * inner_h(np.abs(a), np.abs(t))
