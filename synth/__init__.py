"""Seeded synthetic inputs shared by the GPU path and the FP64 oracle.

This module only draws images and velocity fields; it performs none of the
registration method's arithmetic (no transport, no objective, no gradient, no
regularisation or projection operator).  The paper's own datasets (hands,
NIREP, rect, the smooth sinusoid and Gaussian-density sets of the
incompressible and mass-preserving experiments) are not available, so these
generators stand in for them: smooth periodic images on [0, 2*pi)^d and smooth
stationary velocities built from a few random Fourier modes.

Conventions (shared with the oracle and the library):
  * a scalar field has shape (n_1, ..., n_d) in C order (last axis contiguous);
  * a vector field has shape (d, n_1, ..., n_d); component c acts along axis c;
  * grid points are x_l = 2*pi*l/n_j, cell sizes h_j = 2*pi/n_j.

The reference image m1 of a registration is m0 transported by v*; it is not
produced here because that needs the transport solver.  Tests obtain it from
the oracle; the benchmark obtains it from the library's own forward solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def _axis_coords(n: int) -> np.ndarray:
    return TWO_PI * np.arange(n, dtype=np.float64) / n


def wrapped_gaussian_1d(n: int, centre: float, sigma: float) -> np.ndarray:
    """A 1-D Gaussian made 2*pi-periodic by summing its images at -2pi, 0, +2pi."""
    x = _axis_coords(n)
    out = np.zeros(n)
    for s in (-1, 0, 1):
        out += np.exp(-((x - centre + TWO_PI * s) ** 2) / (2.0 * sigma * sigma))
    return out


def blob_image(shape, n_blobs: int, rng: np.random.Generator,
               anisotropic: bool = False, sigma_range=(0.3, 0.8)) -> np.ndarray:
    """Sum of separable wrapped Gaussians.

    Per blob the draw order is amplitude a~U(0.5,1), centre c~U([0,2pi)^d),
    then width: one sigma~U(sigma_range) (isotropic) or one per axis.
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    factors = [np.zeros((n_blobs, n)) for n in shape]
    for b in range(n_blobs):
        a = rng.uniform(0.5, 1.0)
        c = rng.uniform(0.0, TWO_PI, size=d)
        if anisotropic:
            sig = rng.uniform(*sigma_range, size=d)
        else:
            sig = np.full(d, rng.uniform(*sigma_range))
        for j in range(d):
            factors[j][b] = wrapped_gaussian_1d(shape[j], c[j], sig[j])
        factors[0][b] *= a
    # sum_b prod_j f_j[b, i_j] as a chain of matrix products (fast for 256^3)
    acc = factors[0].T  # (n_1, B)
    for j in range(1, d):
        acc = (acc[:, None, :] * factors[j].T[None, :, :]).reshape(-1, n_blobs) \
            if j < d - 1 else acc @ factors[j]
    return np.ascontiguousarray(acc.reshape(shape))


def _kgrid(shape):
    ks = [np.fft.fftfreq(n, 1.0 / n) for n in shape]
    return np.meshgrid(*ks, indexing="ij")


def _random_modes(shape, kmax: float, rng) -> np.ndarray:
    """Complex N(0,1)+iN(0,1) coefficients on the shell 0 < |k|_2 <= kmax."""
    kk = _kgrid(shape)
    k2 = sum(k * k for k in kk)
    mask = (k2 > 0) & (k2 <= kmax * kmax)
    coef = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return np.where(mask, coef, 0.0), kk


def _synth(spec: np.ndarray) -> np.ndarray:
    # real part of sum_k c_k exp(i k.x): a real trigonometric polynomial
    return np.real(np.fft.ifftn(spec)) * spec.size


def bandlimited_noise(shape, kmax: float, rng, peak: float) -> np.ndarray:
    """sum_{0<|k|<=kmax} a_k cos(k.x) + b_k sin(k.x), scaled to max|.| = peak."""
    spec, _ = _random_modes(shape, kmax, rng)
    eta = _synth(spec)
    return eta * (peak / np.max(np.abs(eta)))


def smoothed_noise(shape, rng, std_cells: float, peak: float) -> np.ndarray:
    """U(0,1) per voxel, Gaussian-filtered (std = std_cells*h), mean removed,
    scaled to max|.| = peak."""
    u = rng.uniform(0.0, 1.0, size=shape)
    kk = _kgrid(shape)
    h = [TWO_PI / n for n in shape]
    damp = np.ones(shape)
    for j, k in enumerate(kk):
        s = std_cells * h[j]
        damp = damp * np.exp(-0.5 * (s * k) ** 2)
    f = np.real(np.fft.ifftn(np.fft.fftn(u) * damp))
    f -= f.mean()
    return f * (peak / np.max(np.abs(f)))


def random_velocity(shape, kmax: float, max_disp_cells: float, rng,
                    divergence_free: bool = False) -> np.ndarray:
    """Smooth stationary velocity from random Fourier modes 0<|k|_2<=kmax.

    General case: each component is an independent random trigonometric
    polynomial.  Divergence-free case: every mode's amplitude vector is made
    orthogonal to its wave vector by construction (2-D: the rotated wave
    vector times a random scalar, i.e. a stream function; 3-D: the cross
    product of the wave vector with a random vector, i.e. a vector
    potential), so each mode, and hence the sum, has zero divergence.

    Scaled so that max_x |v(x)|_2 = max_disp_cells * min_j h_j (unit time).
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    if not divergence_free:
        comps = [_synth(_random_modes(shape, kmax, rng)[0]) for _ in range(d)]
    elif d == 2:
        psi, (k1, k2) = _random_modes(shape, kmax, rng)
        comps = [_synth(1j * k2 * psi), _synth(-1j * k1 * psi)]
    elif d == 3:
        a1, kk = _random_modes(shape, kmax, rng)
        a2, _ = _random_modes(shape, kmax, rng)
        a3, _ = _random_modes(shape, kmax, rng)
        k1, k2, k3 = kk
        # i k x A
        comps = [_synth(1j * (k2 * a3 - k3 * a2)),
                 _synth(1j * (k3 * a1 - k1 * a3)),
                 _synth(1j * (k1 * a2 - k2 * a1))]
    else:
        raise ValueError("divergence-free velocity needs d in {2,3}")
    v = np.stack(comps)
    speed = np.sqrt(np.sum(v * v, axis=0)).max()
    hmin = min(TWO_PI / n for n in shape)
    return np.ascontiguousarray(v * (max_disp_cells * hmin / speed))


@dataclass
class Workload:
    """One registration problem: data, velocity and solver parameters."""
    name: str
    shape: tuple
    model: str                 # "advection" or "continuity"
    incompressible: bool
    reg_order: int             # p in l_p(k) = |k|^(2p)
    alpha: float
    nt: int
    m0: np.ndarray
    vstar: np.ndarray
    dtype: str = "f64"
    checkpoint_every: int = 1
    solver: dict = field(default_factory=dict)


def workload(name: str, shape=None, seed=None) -> Workload:
    """The five configurations of the study.  `shape`/`seed` override the
    grid and seed (used for small parity cases of the same recipe).

      c0  2-D advection 64^2, H1, alpha=1e-2, nt=4, FP64
      c1  2-D continuity 256^2, H2, alpha=1e-3, nt=8, FP32
      c2  3-D incompressible advection 128^3, H1, alpha=1e-4, nt=4, FP32
      c3  3-D advection 256^3, H2, alpha=1e-4, nt=8, checkpoint every 2
      c4i one instance of the batched 2-D set (shape and seed given)
    """
    if name == "c0":
        shape = shape or (64, 64)
        rng = np.random.default_rng(0 if seed is None else seed)
        m0 = blob_image(shape, 8, rng)
        v = random_velocity(shape, 4, 2.0, rng)
        return Workload("c0", tuple(shape), "advection", False, 1, 1e-2, 4, m0, v,
                        dtype="f64",
                        solver=dict(w=5, sigma=2, tau=1, n_iter=20, eps_rel=1e-12))
    if name == "c1":
        shape = shape or (256, 256)
        rng = np.random.default_rng(1 if seed is None else seed)
        m0 = blob_image(shape, 32, rng)
        m0 = m0 + bandlimited_noise(shape, 8, rng, 0.05 * m0.max())
        # a density: strictly positive, unit mass
        m0 = m0 - m0.min() + 0.01 * (m0.max() - m0.min())
        cell = np.prod([TWO_PI / n for n in shape])
        m0 = m0 / (m0.sum() * cell)
        v = random_velocity(shape, 8, 6.0 * shape[0] / 256.0, rng)
        return Workload("c1", tuple(shape), "continuity", False, 2, 1e-3, 8, m0, v,
                        dtype="f32")
    if name == "c2":
        shape = shape or (128, 128, 128)
        rng = np.random.default_rng(2 if seed is None else seed)
        m0 = blob_image(shape, 64, rng, anisotropic=True)
        v = random_velocity(shape, 6, 4.0 * shape[0] / 128.0, rng, divergence_free=True)
        return Workload("c2", tuple(shape), "advection", True, 1, 1e-4, 4, m0, v,
                        dtype="f32",
                        solver=dict(w=5, sigma=2, tau=1, n_iter=500, eps_rel=1e-2))
    if name == "c3":
        shape = shape or (256, 256, 256)
        rng = np.random.default_rng(3 if seed is None else seed)
        m0 = blob_image(shape, 256, rng, anisotropic=True)
        m0 = m0 + smoothed_noise(shape, rng, 2.0, 0.05 * m0.max())
        v = random_velocity(shape, 10, 8.0 * shape[0] / 256.0, rng)
        return Workload("c3", tuple(shape), "advection", False, 2, 1e-4, 8, m0, v,
                        dtype="f32", checkpoint_every=2)
    if name == "c4i":
        if shape is None or seed is None:
            raise ValueError("c4i needs shape and seed")
        rng = np.random.default_rng(seed)
        alpha = [1e-2, 1e-3, 1e-4][int(rng.integers(0, 3))]
        m0 = blob_image(shape, 8, rng)
        v = random_velocity(shape, 4, 2.0 * shape[0] / 64.0, rng)
        return Workload("c4i", tuple(shape), "advection", False, 1, alpha, 4, m0, v,
                        dtype="f32", solver=dict(w=5, sigma=2, tau=1, n_iter=15, eps_rel=1e-12))
    raise KeyError(name)


def batch_workloads():
    """The batched set: 16 instances each at 96^2, 192^2 and 384^2."""
    out = []
    for i, n in enumerate([96] * 16 + [192] * 16 + [384] * 16):
        out.append(workload("c4i", shape=(n, n), seed=4000 + i))
    return out
