"""Periodic tensor-product cubic Lagrange interpolation.

The semi-Lagrangian scheme of Sec. 2.2 evaluates the transported field at
departure points that are off the grid.  The paper does not name the kernel;
this implementation uses a cubic (4-point) Lagrange polynomial per axis, i.e. the
tricubic (3-D) / bicubic (2-D) tensor-product stencil, without prefiltering.

Points are given in index space: xi_j is measured in cells along axis j, so the
grid node l sits at xi = l.  Per axis f = floor(xi_j), t = xi_j - f, and the
stencil nodes are f-1, f, f+1, f+2 (taken modulo n_j) with the Lagrange basis
weights of the nodes -1, 0, 1, 2 evaluated at t.
"""
from __future__ import annotations

import itertools

import numpy as np


def lagrange_weights(t: np.ndarray):
    """Weights of the nodes -1, 0, 1, 2 for the cubic through them, at t."""
    return (
        -t * (t - 1.0) * (t - 2.0) / 6.0,
        (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
        -(t + 1.0) * t * (t - 2.0) / 2.0,
        (t + 1.0) * t * (t - 1.0) / 6.0,
    )


def interpolate(u: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """I[u](xi): u of shape (n_1..n_d), xi of shape (d, ...) in index units."""
    shape = u.shape
    d = u.ndim
    base = np.floor(xi)
    t = xi - base
    base = base.astype(np.int64)
    w = [lagrange_weights(t[j]) for j in range(d)]
    out = np.zeros(xi.shape[1:])
    for offs in itertools.product(range(4), repeat=d):
        idx = tuple(np.mod(base[j] + (offs[j] - 1), shape[j]) for j in range(d))
        weight = w[0][offs[0]]
        for j in range(1, d):
            weight = weight * w[j][offs[j]]
        out += weight * u[idx]
    return out


def index_grid(shape) -> np.ndarray:
    """The grid nodes in index units, shape (d, n_1..n_d)."""
    return np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape],
                                indexing="ij"))
