"""GPU parity: the HIP library against the FP64 oracle, element by element.

Tolerances (relative l2 unless stated): 1e-10 for the FP64 path, 1e-4 for
the FP32 path, on the objective, the gradient, the terminal state, the adjoint
at t = 0 and the preconditioned direction, at fixed probe velocities.
Grids are chosen to span several LDS tiles with ragged tails (sizes that are
not multiples of the tile widths, odd 3^b sizes).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ngmres as ong
from tests._cases import as_precision, oracle_problem, probes, rel, relinf, round_to

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def make_gpu(P, wl, dtype):
    import paper_2510_08782_amd as gan
    return gan.Problem(dev(P.m0, dtype), dev(P.m1, dtype), P.nt, P.alpha, P.p, model=P.model,
                       incompressible=P.incompressible)


def inf_tol(P, tol):
    """Bound on the relative max-norm error.  The FP32 rounding of a spectral
    derivative grows with the largest wavenumber, n/2 on an n-long axis, against
    the derivative of the smooth content, so the FP32 bound scales with the
    longest axis beyond 256; the FP64 bound is the l2 one."""
    if tol < 1e-8:
        return tol
    return tol * max(1.0, max(np.shape(P.m0)) / 256.0)


def check_probe(P, G, v, dtype, tol, name):
    say(f"  probe {name}")
    tinf = inf_tol(P, tol)
    vd = dev(v, dtype)
    Jg, mis = G.eval_objective(vd, with_mismatch=True)
    Jo, miso, _ = P.objective(v, return_parts=True)
    assert abs(Jg - Jo) <= tol * abs(Jo), (name, Jg, Jo)
    assert abs(mis - miso) <= tol * max(abs(miso), 1e-300) + tol * abs(Jo), (name, mis, miso)
    Jg2, g = G.eval_gradient(vd)
    Jo2, go, st = P.gradient(v, return_states=True)
    assert abs(Jg2 - Jo2) <= tol * abs(Jo2)
    mT = host(G.get_field("state", P.nt))
    assert rel(mT, st["m"][-1]) <= tol, name
    assert relinf(mT, st["m"][-1]) <= tinf, name
    lam_scale = max(np.abs(st["lam"][-1]).max(), 1e-300)
    lam0 = host(G.get_field("adjoint", 0))
    if np.abs(st["lam"][0]).max() > 0:
        # lam^nt = m1 - m(1) cancels: the relative rounding error of m(1)
        # (<= 2e-6 in FP32 after the transport, 1e-14 in FP64) is amplified
        # by kappa = |m(1)| / |lam^nt|, which grows near the optimum
        kappa = np.linalg.norm(st["m"][-1]) / max(np.linalg.norm(st["lam"][-1]), 1e-300)
        tol_lam = tol + (2e-6 if tol > 1e-8 else 1e-14) * kappa
        assert rel(lam0, st["lam"][0]) <= tol_lam, (name, kappa)
    else:
        assert np.abs(lam0).max() <= tol * lam_scale
    err = rel(host(g), go)
    errinf = relinf(host(g), go)
    say(f"    J {Jg:.12e} / {Jo:.12e}  grad rel err {err:.3e} (inf {errinf:.3e})")
    assert err <= tol, (name, err)
    assert errinf <= tinf, (name, errinf)
    s, gs = G.apply_precond(g)
    so, gso = ong.precond(P, go)
    assert rel(host(s), so) <= tol, name
    assert relinf(host(s), so) <= tinf, name
    assert abs(gs - gso) <= 10 * tol * abs(gso), (gs, gso)


CASES = [
    # (workload, shape, nt)
    ("c0", (48, 64), 4),
    ("c1", (96, 72), 4),
    ("c2", (24, 32, 48), 2),
    ("c3", (32, 24, 36), 3),
    # a 256-long leading axis: the transforms compiled for that length along
    # the slowest axis, and many z tiles of the gather
    ("c2", (256, 24, 32), 2),
    # lengths from 192 up run the 512-thread complex passes: 192 compiled along
    # the slowest axis, 216 (= 2^3 3^3) on the runtime plan along the strided
    # 2-D axis
    ("c2", (192, 16, 24), 2),
    ("c0", (216, 48), 3),
    # the transforms compiled for length 512 (rows, complex passes, the fused
    # spectral pass and the body-force derivative), on a grid with enough
    # pencils that their tiles hold the full pencil count
    ("c0", (512, 512), 2),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_{'x'.join(map(str, c[1]))}" for c in CASES])
def test_probe_parity(case, prec):
    name, shape, nt = case
    say(f"case {name} shape {shape} nt {nt} {prec}")
    wl = synth.workload(name, shape=shape)
    P = as_precision(oracle_problem(wl, nt=nt), prec)
    dtype = torch.float64 if prec == "f64" else torch.float32
    G = make_gpu(P, wl, dtype)
    for pname, v in probes(wl).items():
        check_probe(P, G, round_to(v, prec), dtype, TOL[prec], pname)
    G.close()


EDGE = [
    ("odd27x36", "c0", (27, 36), 2, 1.0),
    ("tiny4x6", "c0", (4, 6), 1, 1.0),
    ("odd3d_9x12x27", "c3", (9, 12, 27), 1, 1.0),
    ("big_displacement", "c0", (32, 48), 2, 12.0),
    ("continuity_nt1", "c1", (16, 24), 1, 1.0),
]


@pytest.mark.parametrize("edge", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases_f64(edge):
    ename, name, shape, nt, vscale = edge
    say(f"edge {ename} shape {shape} nt {nt} vscale {vscale}")
    wl = synth.workload(name, shape=shape)
    wl.vstar = wl.vstar * vscale
    P = oracle_problem(wl, nt=nt)
    G = make_gpu(P, wl, torch.float64)
    for pname, v in probes(wl).items():
        check_probe(P, G, v, torch.float64, TOL["f64"], pname)
    G.close()


# Long, smooth displacements: tiles whose displacement floors spread less than
# the staged window's capacity take the LDS path with a shifted window, the
# others gather from global memory; both within one launch.
LARGE = [
    ("shift3d_x3", "c2", (24, 32, 64), 2, 3.0),
    ("far3d_x8", "c3", (16, 24, 32), 1, 8.0),
    ("far2d_x20", "c0", (48, 64), 2, 20.0),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("edge", LARGE, ids=[e[0] for e in LARGE])
def test_large_displacement_parity(edge, prec):
    ename, name, shape, nt, vscale = edge
    say(f"large {ename} shape {shape} nt {nt} vscale {vscale} {prec}")
    wl = synth.workload(name, shape=shape)
    wl.vstar = wl.vstar * vscale
    P = as_precision(oracle_problem(wl, nt=nt), prec)
    dtype = torch.float64 if prec == "f64" else torch.float32
    G = make_gpu(P, wl, dtype)
    for pname, v in probes(wl).items():
        check_probe(P, G, round_to(v, prec), dtype, TOL[prec], pname)
    G.close()


def test_gradient_is_deterministic():
    wl = synth.workload("c2", shape=(24, 32, 48))
    P = oracle_problem(wl, nt=2)
    G = make_gpu(P, wl, torch.float32)
    v = dev(0.5 * wl.vstar, torch.float32)
    _, g1 = G.eval_gradient(v)
    _, g2 = G.eval_gradient(v)
    J1 = G.eval_objective(v)
    J2 = G.eval_objective(v)
    assert torch.equal(g1, g2) and J1 == J2


def test_reuse_forward_matches_fresh_gradient():
    wl = synth.workload("c1", shape=(48, 64))
    P = oracle_problem(wl, nt=3)
    G = make_gpu(P, wl, torch.float64)
    v = dev(0.5 * wl.vstar, torch.float64)
    J0 = G.eval_objective(v, keep_history=True)
    J1, g1 = G.eval_gradient(v, reuse_forward=True)
    J2, g2 = G.eval_gradient(v)
    assert J0 == J1 == J2
    assert torch.equal(g1, g2)
    import paper_2510_08782_amd as gan
    G.eval_objective(v, keep_history=False)
    with pytest.raises(gan.GanmresError) as ei:
        G.eval_gradient(v, reuse_forward=True)
    assert ei.value.code == -7


@pytest.mark.parametrize("w", [5, 20])
def test_c0_trajectory_parity_f64(w):
    """Config c0 (64^2, FP64, GA-NGMRES(w; 2, 1), 20 iterations) against the
    oracle's loop: every iterate to 1e-8, J and the step kinds exactly.  The
    window w = 20 (the paper's best runs use windows of 15 to 25) takes the
    Gram matrix of up to 22 vectors through the one-pass blocked kernel."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0")
    P = oracle_problem(wl)
    sv = wl.solver
    res = ong.solve(P, w=w, sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                    n_iter=sv["n_iter"], keep_iterates=True)
    G = make_gpu(P, wl, torch.float64)
    params = gan.SolveParams(w=w, sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                             n_iter=sv["n_iter"])
    v = G.new_velocity()
    for k in range(1, sv["n_iter"] + 1):
        info = G.step(params, v)
        rec = res.records[k - 1]
        err = rel(host(v), res.iterates[k])
        say(f"  k {k} {('ngmres', 'fp')[info.step_kind]} J {info.J:.12e} / {rec.J:.12e} "
            f"iterate err {err:.2e} trials {info.n_trials}/{rec.trials}")
        assert ("ngmres", "fp")[info.step_kind] == rec.kind
        assert info.n_trials == rec.trials
        assert err <= 1e-8
        assert abs(info.J - rec.J) <= 1e-10 * abs(rec.J)
        if rec.beta is not None:
            assert info.n_beta == len(rec.beta)
            np.testing.assert_allclose(np.array(info.beta[:info.n_beta]), rec.beta, rtol=1e-6,
                                       atol=1e-9)
        if info.stop:
            break
    assert info.k == res.iterations
    if w == 20:
        assert max(len(r.beta) for r in res.records if r.beta is not None) > 8


KIND = {0: "ngmres", 1: "fp", 2: "aa"}


@pytest.mark.parametrize("variant", ["GA", "ALT"])
def test_c0_ga_aa_trajectory_parity_f64(variant):
    """GA-AA(5; 2, 1) (Alg. 2 with the alternation of Alg. 3) on the c0 recipe
    against the oracle's loop: every iterate to 1e-8, J, the step kinds and the
    line-search trial counts exactly, the mixing coefficients to 1e-6."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0")
    P = oracle_problem(wl)
    sv = wl.solver
    n_iter = 12
    res = ong.solve(P, w=sv["w"], sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                    n_iter=n_iter, keep_iterates=True, accel="aa", variant=variant)
    G = make_gpu(P, wl, torch.float64)
    params = gan.SolveParams(w=sv["w"], sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                             n_iter=n_iter, accel=gan.ACCEL_AA,
                             variant=gan.VARIANT_GA if variant == "GA" else gan.VARIANT_ALT)
    v = G.new_velocity()
    for k in range(1, n_iter + 1):
        info = G.step(params, v)
        rec = res.records[k - 1]
        err = rel(host(v), res.iterates[k])
        say(f"  k {k} {KIND[info.step_kind]} J {info.J:.12e} / {rec.J:.12e} "
            f"iterate err {err:.2e} trials {info.n_trials}/{rec.trials}")
        assert KIND[info.step_kind] == rec.kind
        assert info.n_trials == rec.trials
        assert err <= 1e-8
        assert abs(info.J - rec.J) <= 1e-10 * abs(rec.J)
        if rec.beta is not None:
            assert info.n_beta == len(rec.beta)
            np.testing.assert_allclose(np.array(info.beta[:info.n_beta]), rec.beta, rtol=1e-6,
                                       atol=1e-9)
        if info.stop:
            break
    assert info.k == res.iterations


def test_accelerator_change_needs_reset():
    """Switching between GA-NGMRES and GA-AA inside a solve is an error; after
    a reset the other accelerator starts cleanly."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0", shape=(32, 32))
    P = oracle_problem(wl)
    G = make_gpu(P, wl, torch.float64)
    v = G.new_velocity()
    G.step(gan.SolveParams(w=3, sigma=2, tau=1, n_iter=5), v)
    with pytest.raises(gan.GanmresError):
        G.step(gan.SolveParams(w=3, sigma=2, tau=1, n_iter=5, accel=gan.ACCEL_AA), v)
    G.reset()
    v.zero_()
    info = G.step(gan.SolveParams(w=3, sigma=2, tau=1, n_iter=5, accel=gan.ACCEL_AA), v)
    assert info.k == 1 and KIND[info.step_kind] == "fp"
