"""GPU parity at the grid sizes of the batched 2-D set (96^2, 192^2, 384^2):
three problems of one size with different regularisation weights in one batch
handle, every problem checked against the FP64 oracle at fixed probe
velocities (objective, mismatch, terminal state, adjoint at t = 0, gradient and
preconditioned direction; relative l2 and max norms).  These sizes run on the
transforms compiled for lengths 96, 192 and 384."""
import sys

import numpy as np
import pytest

import synth
from oracle import ngmres as ong
from tests._cases import as_precision, oracle_problem, probes, rel, relinf, round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}
# seeds of the batched set with alpha = 1e-4, 1e-2, 1e-3 (96^2), 1e-3, 1e-4,
# 1e-2 (192^2) and 1e-2, 1e-3, 1e-4 (384^2)
SEEDS = {96: (4000, 4002, 4008), 192: (4016, 4017, 4022), 384: (4032, 4034, 4036)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().double().cpu().numpy()


def check_batch_probe(Ps, B, vs, dtype, tol, name):
    """Per-problem parity of a batch handle B at the probe velocities vs."""
    vb = torch.tensor(np.ascontiguousarray(np.stack(vs, axis=1)), dtype=dtype, device="cuda")
    Jtot = B.eval_objective(vb)
    Jv, misv = B.values()
    assert abs(Jtot - sum(Jv)) <= 1e-12 * abs(Jtot)
    _, g = B.eval_gradient(vb)
    g = host(g)
    mT = host(B.get_field("state", Ps[0].nt))
    lam0 = host(B.get_field("adjoint", 0))
    s, _ = B.apply_precond(torch.tensor(np.ascontiguousarray(g), dtype=dtype, device="cuda"))
    s = host(s)
    for i, (P, v) in enumerate(zip(Ps, vs)):
        Jo, miso, _ = P.objective(v, return_parts=True)
        _, go, st = P.gradient(v, return_states=True)
        err, errinf = rel(g[:, i], go), relinf(g[:, i], go)
        say(f"  {name} problem {i} alpha {P.alpha:g}: J {Jv[i]:.12e} / {Jo:.12e}, "
            f"g rel {err:.2e} (inf {errinf:.2e})")
        assert abs(Jv[i] - Jo) <= tol * abs(Jo)
        assert abs(misv[i] - miso) <= tol * max(abs(miso), 1e-300) + tol * abs(Jo)
        assert rel(mT[i], st["m"][-1]) <= tol and relinf(mT[i], st["m"][-1]) <= tol
        if np.abs(st["lam"][0]).max() > 0:
            kappa = np.linalg.norm(st["m"][-1]) / max(np.linalg.norm(st["lam"][-1]), 1e-300)
            tol_lam = tol + (2e-6 if tol > 1e-8 else 1e-14) * kappa
            assert rel(lam0[i], st["lam"][0]) <= tol_lam, (name, i, kappa)
        else:
            assert np.abs(lam0[i]).max() <= tol * max(np.abs(st["lam"][-1]).max(), 1e-300)
        assert err <= tol and errinf <= tol
        so, _ = ong.precond(P, g[:, i])
        assert rel(s[:, i], so) <= tol and relinf(s[:, i], so) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [96, 192, 384])
def test_batch_sizes_parity(n, prec):
    import paper_2510_08782_amd as gan
    say(f"batch {n}x{n} {prec}")
    dtype = torch.float64 if prec == "f64" else torch.float32
    wls = [synth.workload("c4i", shape=(n, n), seed=s) for s in SEEDS[n]]
    assert len({w.alpha for w in wls}) == 3
    Ps = [as_precision(oracle_problem(w), prec) for w in wls]
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    B = gan.BatchProblem(dev(np.stack([P.m0 for P in Ps])), dev(np.stack([P.m1 for P in Ps])),
                         wls[0].nt, [w.alpha for w in wls], wls[0].reg_order)
    pr = [probes(w) for w in wls]
    for pname in pr[0]:
        vs = [round_to(p[pname], prec) for p in pr]
        check_batch_probe(Ps, B, vs, dtype, TOL[prec], pname)
    B.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_group_sizes_parity(prec):
    """The three sizes in ONE group handle (two problems per size, merged
    launches): each problem's objective, mismatch, gradient and preconditioned
    direction against the FP64 oracle at v*/2 and at the perturbed probe."""
    import paper_2510_08782_amd as gan
    say(f"group 96/192/384 {prec}")
    dtype = torch.float64 if prec == "f64" else torch.float32
    tol = TOL[prec]
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    wls = [[synth.workload("c4i", shape=(n, n), seed=s) for s in SEEDS[n][:2]]
           for n in (96, 192, 384)]
    Ps = [[as_precision(oracle_problem(w), prec) for w in wc] for wc in wls]
    G = gan.GroupProblem([dev(np.stack([P.m0 for P in Pc])) for Pc in Ps],
                         [dev(np.stack([P.m1 for P in Pc])) for Pc in Ps],
                         wls[0][0].nt, [w.alpha for wc in wls for w in wc], wls[0][0].reg_order)
    pr = [[probes(w) for w in wc] for wc in wls]
    for pname in ("half", "perturbed"):
        vs = [[round_to(p[pname], prec) for p in pc] for pc in pr]
        v = G.pack_velocity([dev(np.stack(vc, axis=1)) for vc in vs])
        _, g = G.eval_gradient(v)
        Jv, misv = G.values()
        s, _ = G.apply_precond(g)
        gv, sv = G.velocity_views(g), G.velocity_views(s)
        k = 0
        for c, Pc in enumerate(Ps):
            gc, sc = host(gv[c]), host(sv[c])
            for i, P in enumerate(Pc):
                Jo, miso, _ = P.objective(vs[c][i], return_parts=True)
                _, go = P.gradient(vs[c][i])
                err, errinf = rel(gc[:, i], go), relinf(gc[:, i], go)
                say(f"  {pname} class {c} problem {i}: J {Jv[k]:.12e} / {Jo:.12e}, "
                    f"g rel {err:.2e} (inf {errinf:.2e})")
                assert abs(Jv[k] - Jo) <= tol * abs(Jo)
                assert abs(misv[k] - miso) <= tol * max(abs(miso), 1e-300) + tol * abs(Jo)
                assert err <= tol and errinf <= tol
                so, _ = ong.precond(P, gc[:, i])
                assert rel(sc[:, i], so) <= tol and relinf(sc[:, i], so) <= tol
                k += 1
    submitted, issued = G.launches()
    say(f"  launches: {submitted} by the classes, {issued} merged")
    assert issued * 2.5 <= submitted
    G.close()
