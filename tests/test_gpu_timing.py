"""Kernel-class timing: the selected classes alone are bracketed with events,
and timing leaves results unchanged."""
import numpy as np
import pytest

import synth
from tests._cases import oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_timing_selects_classes_and_changes_nothing():
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0", shape=(48, 64))
    P = oracle_problem(wl, nt=3)
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    G = gan.Problem(dev(P.m0), dev(P.m1), P.nt, P.alpha, P.p)
    v = dev(0.5 * wl.vstar)
    J0, g0 = G.eval_gradient(v)
    G.timing(True, ["sl_step"])
    G.timing_reset()
    J1, g1 = G.eval_gradient(v)
    rep = G.timing_report()
    G.timing(False)
    assert rep["sl_step"][1] == 2 * P.nt and rep["sl_step"][0] > 0.0
    assert all(c == 0 for k, (ms, c) in rep.items() if k != "sl_step")
    G.timing(True)
    G.timing_reset()
    J2, g2 = G.eval_gradient(v)
    rep = G.timing_report()
    G.timing(False)
    assert sum(1 for ms, c in rep.values() if c > 0) >= 5
    assert J0 == J1 == J2 and torch.equal(g0, g1) and torch.equal(g0, g2)
    G.close()
