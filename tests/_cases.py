"""Problem builders shared by the GPU tests: seeded inputs from `synth`, the
reference image m1 and every expected value from the FP64 oracle."""
from __future__ import annotations

import numpy as np

import synth
from oracle.transport import TransportProblem


def oracle_problem(wl, nt=None, m1=None):
    nt = wl.nt if nt is None else nt
    if m1 is None:
        gen = TransportProblem(wl.m0, wl.m0, nt, wl.alpha, wl.reg_order, model=wl.model,
                               incompressible=wl.incompressible)
        m1 = gen.forward(wl.vstar)[-1]
    return TransportProblem(wl.m0, m1, nt, wl.alpha, wl.reg_order, model=wl.model,
                            incompressible=wl.incompressible)


def smooth_direction(shape, seed, divergence_free=False):
    rng = np.random.default_rng(seed)
    return synth.random_velocity(shape, 3, 1.0, rng, divergence_free=divergence_free)


def probes(wl, seed=7):
    """Fixed probe velocities: 0, v*/2 and v* + 0.1 |v*| * smooth noise."""
    noise = smooth_direction(wl.shape, seed, wl.incompressible)
    scale = np.abs(wl.vstar).max() / np.abs(noise).max()
    return {"zero": np.zeros_like(wl.vstar), "half": 0.5 * wl.vstar,
            "perturbed": wl.vstar + 0.1 * scale * noise}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relinf(a, b):
    """max |a - b| / max |b|: a wrong value at a few points (a tile, a wrap
    at one corner) stays small in the l2 ratio but not here."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0) if a.size else 0.0


def as_precision(P, prec):
    """The oracle problem on the inputs the GPU path actually receives: for the
    FP32 path, m0 and m1 rounded to float32 (then evaluated in FP64)."""
    if prec == "f64":
        return P
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return TransportProblem(r(P.m0), r(P.m1), P.nt, P.alpha, P.p, model=P.model,
                            incompressible=P.incompressible)


def round_to(v, prec):
    return v if prec == "f64" else np.asarray(v, dtype=np.float32).astype(np.float64)
