"""GPU parity of the transport map diagnostics: det grad y element by element
against the oracle (2-D and 3-D, FP64 and FP32, batches), and its invariants
at the full 128^3 size (incompressible: det grad y = 1 up to the
discretisation error)."""
import sys

import numpy as np
import pytest

import synth
from oracle import deformation as dfm
from oracle.transport import TransportProblem
from tests._cases import round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().double().cpu().numpy()


CASES = [
    ("c0", (48, 36), None, 3.0),
    ("c2", (24, 32, 18), None, 2.0),
    ("c3", (16, 24, 32), 3, 1.0),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_det_grad_y_matches_oracle(case, prec):
    import paper_2510_08782_amd as gan
    name, shape, nt, scale = case
    wl = synth.workload(name, shape=shape)
    nt = wl.nt if nt is None else nt
    dtype = torch.float64 if prec == "f64" else torch.float32
    v = round_to(scale * wl.vstar, prec)
    P = TransportProblem(wl.m0, wl.m0, nt, wl.alpha, wl.reg_order, model=wl.model,
                         incompressible=wl.incompressible)
    D, det_o = dfm.det_grad_y(P, v)
    lo, mean, hi, std = dfm.det_stats(det_o)
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    G = gan.Problem(dev(wl.m0), dev(wl.m0), nt, wl.alpha, wl.reg_order, model=wl.model,
                    incompressible=wl.incompressible)
    det, stats = G.deformation(dev(v))
    err = np.max(np.abs(host(det) - det_o))
    say(f"  {name} {shape} {prec}: det in [{lo:.6f}, {hi:.6f}], max |det - det_oracle| {err:.2e}, "
        f"stats {stats[0]}")
    tol = 1e-10 if prec == "f64" else 2e-5
    assert err <= tol * max(1.0, np.max(np.abs(det_o)))
    got = np.array(stats[0])
    np.testing.assert_allclose(got[[0, 1, 2]], [lo, mean, hi], rtol=0, atol=tol)
    assert abs(got[3] - std) <= tol + 1e-3 * std
    G.close()


def test_batch_deformation_per_problem():
    import paper_2510_08782_amd as gan
    wls = [synth.workload("c4i", shape=(32, 32), seed=s) for s in (4001, 4002, 4003)]
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    B = gan.BatchProblem(dev(np.stack([w.m0 for w in wls])), dev(np.stack([w.m0 for w in wls])),
                         wls[0].nt, [w.alpha for w in wls], wls[0].reg_order)
    det, stats = B.deformation(dev(np.stack([3.0 * w.vstar for w in wls], axis=1)))
    det = host(det)
    for i, w in enumerate(wls):
        P = TransportProblem(w.m0, w.m0, w.nt, w.alpha, w.reg_order)
        _, det_o = dfm.det_grad_y(P, 3.0 * w.vstar)
        assert np.max(np.abs(det[i] - det_o)) <= 1e-10
        np.testing.assert_allclose(np.array(stats[i])[[0, 1, 2]],
                                   np.array(dfm.det_stats(det_o))[[0, 1, 2]], atol=1e-10)
        assert abs(stats[i][1] - 1.0) < 1e-12          # 2-D: the mean is exactly 1


def test_c2_full_size_volume_preservation():
    """128^3 incompressible workload, FP32: the map of v* keeps volume up to the
    discretisation error, and its determinant is positive everywhere."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c2")
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")
    G = gan.Problem(dev(wl.m0), dev(wl.m0), wl.nt, wl.alpha, wl.reg_order,
                    incompressible=True)
    _, stats = G.deformation(dev(wl.vstar), want_det=False)
    lo, mean, hi, std = stats[0]
    say(f"  c2 128^3 det grad y: min {lo:.6f} mean {mean:.8f} max {hi:.6f} std {std:.2e}")
    assert lo > 0.99 and hi < 1.01
    assert abs(mean - 1.0) < 1e-4
    # a compressible velocity of the same size is not volume preserving
    u = dev(synth.random_velocity(wl.shape, 6, 4.0, np.random.default_rng(9)))
    _, s2 = G.deformation(u, want_det=False)
    assert s2[0][3] > 10 * std
    G.close()
