"""Fourier pseudo-spectral calculus on the periodic box [0, 2pi)^d.

Paper, Sec. 2.2 ("Numerical Discretization"): functions are expanded in the
Fourier basis exp(i <k, x>), the grid is x_l = 2 pi l / n, h_i = 2 pi / n_i,
derivatives are diagonal in Fourier space, and an operator with a nontrivial
kernel is made invertible by setting its zero spectral entries to one before
inverting.

Readings used here:
  * wavenumbers k_j in {-n_j/2+1, ..., n_j/2} (the printed range lost its
    minus sign);
  * odd derivatives use k~_j = k_j with the Nyquist index (n_j even) set to 0,
    so that the discrete derivative is real and exactly skew-adjoint; even
    powers |k|^2 keep the Nyquist mode;
  * regulariser of order p: l_p(k) = |k|^(2p) (p=1: -Laplacian, H1 seminorm;
    p=2: biharmonic, the paper's H2 model in eq. e:varopt; p=3: the H3 model
    of the incompressible experiment, Sec. 3.5);
  * inverse: zero entries of l_p (only k=0) are replaced by one, so the
    zero-mode gain of (alpha L)^-1 is 1/alpha;
  * Leray projection P^(k) = I - k~ k~^T / |k~|^2 (identity where k~ = 0).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft


class Grid:
    """Uniform periodic grid on [0, 2pi)^d with n = (n_1, ..., n_d) cells."""

    def __init__(self, shape):
        self.shape = tuple(int(s) for s in shape)
        self.d = len(self.shape)
        self.h = tuple(2.0 * math.pi / n for n in self.shape)
        self.cell = float(np.prod(self.h))          # |h| = prod h_i
        self.N = int(np.prod(self.shape))

    # -- wavenumbers -----------------------------------------------------
    def k(self, j: int) -> np.ndarray:
        """Integer wavenumbers along axis j, broadcastable to the grid."""
        n = self.shape[j]
        kj = np.fft.fftfreq(n, 1.0 / n)
        if n % 2 == 0:
            kj[n // 2] = n // 2          # the Nyquist mode is +n/2
        s = [1] * self.d
        s[j] = n
        return kj.reshape(s)

    def ktilde(self, j: int) -> np.ndarray:
        """Wavenumbers for odd derivatives: Nyquist index set to zero."""
        n = self.shape[j]
        kj = self.k(j).reshape(-1).copy()
        if n % 2 == 0:
            kj[n // 2] = 0.0
        s = [1] * self.d
        s[j] = n
        return kj.reshape(s)

    def ksq(self) -> np.ndarray:
        return sum(self.k(j) ** 2 for j in range(self.d))

    # -- inner products --------------------------------------------------
    def inner(self, a: np.ndarray, b: np.ndarray) -> float:
        """<a, b>_h = |h| sum over grid points (and components)."""
        return self.cell * float(np.sum(a * b))


# Threads of the multi-dimensional transforms (scipy.fft's `workers`): the
# transform is the same unnormalised DFT whatever the count; only the CPU
# baseline raises it to the cores it may use.
WORKERS = 1


def fft(u):
    """Unnormalised forward DFT over every axis."""
    return scipy.fft.fftn(u, workers=WORKERS)


def ifft(uh):
    """Inverse DFT (scaled by 1/N), real part."""
    return np.real(scipy.fft.ifftn(uh, workers=WORKERS))


def deriv(grid: Grid, u: np.ndarray, j: int) -> np.ndarray:
    """Spectral partial derivative d/dx_j (multiplier i k~_j)."""
    return ifft(1j * grid.ktilde(j) * fft(u))


def gradient(grid: Grid, u: np.ndarray) -> np.ndarray:
    return np.stack([deriv(grid, u, j) for j in range(grid.d)])


def divergence(grid: Grid, v: np.ndarray) -> np.ndarray:
    return sum(deriv(grid, v[j], j) for j in range(grid.d))


def symbol(grid: Grid, p: int) -> np.ndarray:
    """l_p(k) = |k|^(2p)."""
    return grid.ksq() ** p


def apply_reg(grid: Grid, v: np.ndarray, p: int, alpha: float = 1.0) -> np.ndarray:
    """alpha L_p v, componentwise."""
    lp = alpha * symbol(grid, p)
    return np.stack([ifft(lp * fft(v[c])) for c in range(v.shape[0])])


def apply_reg_inverse(grid: Grid, v: np.ndarray, p: int, alpha: float) -> np.ndarray:
    """(alpha L_p)^-1 v with the zero entries of l_p set to one."""
    lp = symbol(grid, p).astype(np.float64)
    lp = np.where(lp == 0.0, 1.0, lp)
    return np.stack([ifft(fft(v[c]) / (alpha * lp)) for c in range(v.shape[0])])


def leray(grid: Grid, v: np.ndarray) -> np.ndarray:
    """Projection onto divergence-free fields: v^ - k~ (k~ . v^) / |k~|^2."""
    vh = [fft(v[c]) for c in range(grid.d)]
    kt = [grid.ktilde(j) for j in range(grid.d)]
    kt2 = sum(k * k for k in kt)
    safe = np.where(kt2 == 0.0, 1.0, kt2)
    kdotv = sum(kt[j] * vh[j] for j in range(grid.d))
    return np.stack([ifft(vh[c] - np.where(kt2 == 0.0, 0.0, kt[c] * kdotv / safe))
                     for c in range(grid.d)])


def reg_value(grid: Grid, v: np.ndarray, p: int) -> float:
    """R(v) = <v, L_p v>_h, evaluated with Parseval:
    (|h|/N) sum_c sum_k l_p(k) |v^_c(k)|^2.  For p=2 this is ||Lap v||^2."""
    lp = symbol(grid, p)
    tot = 0.0
    for c in range(v.shape[0]):
        vh = fft(v[c])
        tot += float(np.sum(lp * (vh.real ** 2 + vh.imag ** 2)))
    return grid.cell / grid.N * tot
