"""GPU tests of group handles: batches of 2-D problems of different grid sizes
in one handle, every phase one kernel launch for all of them.

  * each problem's objective, gradient and preconditioned direction equal
    those of the same problems on batch handles of their own size;
  * GA-NGMRES trajectories equal the per-size batch handles' and the
    oracle's, problem by problem;
  * one problem per size class matches the FP64 oracle at the parity bounds;
  * the classes' launches merge: about one launch per phase for all classes.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ngmres as ong
from tests._cases import as_precision, oracle_problem, probes, rel, relinf, round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# three size classes of the batched-set recipe, two or three problems each,
# on transform lengths compiled into the merged kernels (32, 64, 96); the
# runtime-plan lengths (24, 36 here) run as launches of their own
CLASSES = [((32, 32), (4101, 4102)), ((64, 32), (4103, 4104, 4105)), ((96, 96), (4106, 4107))]
ODD_CLASSES = [((24, 24), (4101, 4102)), ((48, 36), (4103, 4104, 4105)), ((96, 96), (4106, 4107))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().double().cpu().numpy()


def setup(prec="f64", classes=CLASSES):
    import paper_2510_08782_amd as gan
    dtype = torch.float64 if prec == "f64" else torch.float32
    dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    wls, Ps, m0s, m1s, batches = [], [], [], [], []
    for shape, seeds in classes:
        w = [synth.workload("c4i", shape=shape, seed=s) for s in seeds]
        P = [as_precision(oracle_problem(x), prec) for x in w]
        wls.append(w)
        Ps.append(P)
        m0s.append(dev(np.stack([p.m0 for p in P])))
        m1s.append(dev(np.stack([p.m1 for p in P])))
        batches.append(gan.BatchProblem(m0s[-1], m1s[-1], w[0].nt, [x.alpha for x in w],
                                        w[0].reg_order))
    alphas = [x.alpha for w in wls for x in w]
    G = gan.GroupProblem(m0s, m1s, wls[0][0].nt, alphas, wls[0][0].reg_order)
    return wls, Ps, G, batches, dtype


@pytest.mark.parametrize("prec,classes", [("f64", CLASSES), ("f32", CLASSES), ("f64", ODD_CLASSES)],
                         ids=["f64", "f32", "f64-runtime-lengths"])
def test_group_evaluations_match_batch_handles(prec, classes):
    wls, Ps, G, batches, dtype = setup(prec, classes)
    tol = 1e-12 if prec == "f64" else 1e-6
    vb = [torch.tensor(np.ascontiguousarray(np.stack([round_to(0.5 * x.vstar, prec) for x in w],
                                                     axis=1)), dtype=dtype, device="cuda")
          for w in wls]
    v = G.pack_velocity(vb)
    Jg, g = G.eval_gradient(v)
    Jv, misv = G.values()
    s, gs = G.apply_precond(g)
    gv, sv = G.velocity_views(g), G.velocity_views(s)
    mT = G.image_views(G.get_field("state", G.nt))
    k = 0
    Jsum, gssum = 0.0, 0.0
    for c, B in enumerate(batches):
        Jb, gb = B.eval_gradient(vb[c])
        Jbv, misb = B.values()
        sb, gsb = B.apply_precond(gb)
        Jsum += Jb
        gssum += gsb
        say(f"  class {c} {tuple(vb[c].shape[2:])}: g rel {rel(host(gv[c]), host(gb)):.2e}, "
            f"s rel {rel(host(sv[c]), host(sb)):.2e}")
        assert rel(host(gv[c]), host(gb)) <= tol and relinf(host(gv[c]), host(gb)) <= tol
        assert rel(host(sv[c]), host(sb)) <= tol
        assert rel(host(mT[c]), host(B.get_field("state", B.nt))) <= tol
        for i in range(len(Jbv)):
            assert abs(Jv[k + i] - Jbv[i]) <= tol * abs(Jbv[i])
            assert abs(misv[k + i] - misb[i]) <= tol * abs(Jbv[i])
        k += len(Jbv)
    assert abs(Jg - Jsum) <= tol * abs(Jsum)
    assert abs(gs - gssum) <= tol * abs(gssum)
    submitted, issued = G.launches()
    say(f"  launches: {submitted} by the classes, {issued} merged")
    # three classes: nearly every launch serves all of them (fewer where the
    # classes' transforms have runtime-plan lengths)
    assert issued * (2.5 if classes is CLASSES else 1.5) <= submitted
    for c in range(len(classes)):
        p, us = G.tile_autotune(c)
        say(f"  class {c}: tile variant {p} points per thread, us per gather {us}")
        assert p in (2, 4, 8) and min(us) > 0


def test_group_oracle_parity_one_problem_per_class():
    """The first problem of every class against the FP64 oracle at the
    probes (FP64 path, 1e-10)."""
    wls, Ps, G, batches, dtype = setup("f64")
    pr = [[probes(x) for x in w] for w in wls]
    for pname in ("zero", "half", "perturbed"):
        vb = [torch.tensor(np.ascontiguousarray(np.stack([p[pname] for p in pc], axis=1)),
                           dtype=dtype, device="cuda") for pc in pr]
        v = G.pack_velocity(vb)
        _, g = G.eval_gradient(v)
        Jv, _ = G.values()
        gv = G.velocity_views(g)
        k = 0
        for c, P in enumerate(Ps):
            Jo, go = P[0].gradient(pr[c][0][pname])
            err = rel(host(gv[c])[:, 0], go)
            say(f"  {pname} class {c}: J {Jv[k]:.12e} / {Jo:.12e}, g rel {err:.2e}")
            assert abs(Jv[k] - Jo) <= 1e-10 * abs(Jo)
            assert err <= 1e-10 and relinf(host(gv[c])[:, 0], go) <= 1e-10
            k += len(P)


@pytest.mark.parametrize("accel", ["ngmres", "aa"])
def test_group_trajectories(accel):
    """8 GA-NGMRES (or GA-AA) iterations on the group against the per-size
    batch handles (same step kinds and trials, iterates to 1e-10) and the
    oracle (iterates to 1e-8)."""
    import paper_2510_08782_amd as gan
    wls, Ps, G, batches, dtype = setup("f64")
    n_iter = 8
    params = gan.SolveParams(w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=n_iter,
                             accel=gan.ACCEL_AA if accel == "aa" else gan.ACCEL_NGMRES)
    refs = [[ong.solve(P, w=5, sigma=2, tau=1, eps_rel=1e-12, n_iter=n_iter, keep_iterates=True,
                       accel=accel) for P in Pc] for Pc in Ps]
    v = G.new_velocity()
    vbs = [B.new_velocity() for B in batches]
    for k in range(1, n_iter + 1):
        infos = G.step(params, v)
        vv = [host(x) for x in G.velocity_views(v)]
        q = 0
        for c, B in enumerate(batches):
            ib = B.step(params, vbs[c])
            vb = host(vbs[c])
            for i in range(len(ib)):
                rec = refs[c][i].records[k - 1]
                info = infos[q + i]
                assert (info.step_kind, info.n_trials) == (ib[i].step_kind, ib[i].n_trials)
                assert info.n_trials == rec.trials
                assert abs(info.J - ib[i].J) <= 1e-12 * abs(ib[i].J)
                assert rel(vv[c][:, i], vb[:, i]) <= 1e-10
                err = rel(vv[c][:, i], refs[c][i].iterates[k])
                assert err <= 1e-8, (k, c, i, err)
            q += len(ib)
        say(f"  k {k}: {infos[0].step_kind} trials {[i.n_trials for i in infos]}")
    submitted, issued = G.launches()
    say(f"  launches: {submitted} by the classes, {issued} merged")
    # the line searches of the classes take different numbers of trials (a
    # class whose problems have all accepted launches nothing meanwhile), so
    # fewer launches merge than in an evaluation
    assert issued * 1.3 <= submitted


def test_group_rejects_newton_and_bad_classes():
    import ctypes

    import paper_2510_08782_amd as gan
    wls, Ps, G, batches, dtype = setup("f64", classes=CLASSES[:2])
    with pytest.raises(gan.GanmresError):
        G.step(gan.SolveParams(accel=gan.ACCEL_NK), G.new_velocity())
    cfg = gan.Config(3, (ctypes.c_int * 3)(8, 8, 8), 4, gan.ADVECTION, 0, 1, 1e-2, gan.F64, 1)
    h = ctypes.c_void_p()
    one = (ctypes.c_int * 1)(1)
    sh = (ctypes.c_int * 2)(8, 8)
    p = (ctypes.c_void_p * 1)(ctypes.c_void_p(16))
    assert gan.lib().ganmres_create_group(ctypes.byref(cfg), 1, sh, one, None, p, p, None,
                                          ctypes.byref(h)) == -1
