"""GPU parity of the Gauss--Newton--Krylov baseline against the FP64 oracle.

The Hessian matvec element by element (2-D and 3-D, compressible and
incompressible, FP64 and FP32; relative l2 1e-10 / 1e-4 as for the gradient),
the NK iteration on the c0 recipe step by step (iterates to 1e-8, J to 1e-10,
the CG iteration counts, steps and line-search trials exactly), the settings
the baseline does not cover (errors), and at the full 128^3 FP32 size the
properties that hold at any size: symmetry and positivity of H_gn up to the
discretisation gap, and an NK step that reduces the gradient.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import newton as onk
from tests._cases import as_precision, oracle_problem, rel, round_to, smooth_direction

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


def make_gpu(P, dtype, **kw):
    import paper_2510_08782_amd as gan
    return gan.Problem(dev(P.m0, dtype), dev(P.m1, dtype), P.nt, P.alpha, P.p, model=P.model,
                       incompressible=P.incompressible, **kw)


CASES = [
    ("c0", (48, 64), 4),
    ("c2", (24, 32, 18), 2),
    ("c3", (16, 24, 18), 3),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gn_matvec_parity(case, prec):
    name, shape, nt = case
    say(f"case {name} shape {shape} nt {nt} {prec}")
    wl = synth.workload(name, shape=shape)
    P = as_precision(oracle_problem(wl, nt=nt), prec)
    dtype = torch.float64 if prec == "f64" else torch.float32
    G = make_gpu(P, dtype)
    for vname, v in (("zero", np.zeros_like(wl.vstar)), ("half", 0.5 * wl.vstar)):
        v = round_to(v, prec)
        for seed in (11, 12):
            vt = round_to(smooth_direction(wl.shape, seed, wl.incompressible), prec)
            Ho = onk.gn_matvec(P, v, vt)
            Hg = host(G.hessian_matvec(dev(v, dtype), dev(vt, dtype)))
            err = rel(Hg, Ho)
            say(f"  v {vname} seed {seed}: rel err {err:.2e}")
            assert err <= TOL[prec], (vname, seed, err)
    G.close()


def test_gn_matvec_is_linear_and_leaves_the_gradient_path_intact():
    """H(a x + y) = a H x + H y to rounding, and a gradient evaluation after a
    matvec (the matvec overwrites the adjoint fields) is unchanged."""
    wl = synth.workload("c0", shape=(48, 36))
    P = oracle_problem(wl, nt=3)
    G = make_gpu(P, torch.float64)
    v = dev(0.5 * wl.vstar, torch.float64)
    x = dev(smooth_direction(wl.shape, 5), torch.float64)
    y = dev(smooth_direction(wl.shape, 6), torch.float64)
    J0, g0 = G.eval_gradient(v)
    Hx, Hy = host(G.hessian_matvec(v, x)), host(G.hessian_matvec(v, y))
    Hxy = host(G.hessian_matvec(v, 2.5 * x + y))
    assert rel(Hxy, 2.5 * Hx + Hy) <= 1e-12
    J1, g1 = G.eval_gradient(v)
    assert J1 == J0 and torch.equal(g0, g1)
    G.close()


def test_nk_trajectory_parity_f64():
    """The inexact GN-Krylov iteration on the c0 recipe (64^2, FP64) against the
    oracle's loop, to ||g||_inf <= 1e-5 ||g_0||_inf."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0")
    P = oracle_problem(wl)
    res = onk.nk_solve(P, eps_rel=1e-5, n_iter=8, keep_iterates=True)
    G = make_gpu(P, torch.float64)
    params = gan.SolveParams(eps_rel=1e-5, n_iter=8, accel=gan.ACCEL_NK)
    v = G.new_velocity()
    for k in range(1, 9):
        info = G.step(params, v)
        rec = res.records[k - 1]
        err = rel(host(v), res.iterates[k])
        say(f"  k {k} J {info.J:.12e} / {rec.J:.12e} cg {info.n_beta}/{rec.cg_iters} "
            f"rho {info.rho}/{rec.rho} trials {info.n_trials}/{rec.trials} iterate err {err:.2e}")
        assert info.step_kind == gan.STEP_NEWTON
        assert info.n_beta == rec.cg_iters
        assert info.rho == rec.rho and info.n_trials == rec.trials
        assert err <= 1e-8
        assert abs(info.J - rec.J) <= 1e-10 * abs(rec.J)
        assert abs(info.ginf - rec.ginf) <= 1e-8 * res.g0inf
        if info.stop:
            break
    assert info.k == len(res.records)
    G.close()


def test_nk_settings_outside_the_baseline_are_errors():
    import paper_2510_08782_amd as gan
    params = gan.SolveParams(n_iter=3, accel=gan.ACCEL_NK)
    wl = synth.workload("c1", shape=(16, 24))
    P = oracle_problem(wl, nt=2)
    G = make_gpu(P, torch.float64)
    v = G.new_velocity()
    with pytest.raises(gan.GanmresError) as ei:
        G.step(params, v)
    assert ei.value.code == -1
    with pytest.raises(gan.GanmresError):
        G.hessian_matvec(v, v.clone())
    G.close()
    wl = synth.workload("c0", shape=(16, 24))
    P = oracle_problem(wl, nt=4)
    G = make_gpu(P, torch.float64, checkpoint_every=2)
    with pytest.raises(gan.GanmresError) as ei:
        G.step(params, G.new_velocity())
    assert ei.value.code == -1
    G.close()
    wls = [synth.workload("c4i", shape=(16, 16), seed=s) for s in (1, 2)]
    B = gan.BatchProblem(dev(np.stack([w.m0 for w in wls]), torch.float64),
                         dev(np.stack([w.m0 for w in wls]), torch.float64), wls[0].nt,
                         [w.alpha for w in wls], wls[0].reg_order)
    with pytest.raises(gan.GanmresError) as ei:
        B.step(params, B.new_velocity())
    assert ei.value.code == -1
    B.close()


def test_c2_full_size_hessian_properties_and_nk_step():
    """128^3 incompressible FP32 (the c2 workload): <e, H d> = <d, H e> and
    <d, H d> > 0 up to the discretisation gap, and one NK step from v = 0
    lowers J and the gradient."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c2")
    P = oracle_problem(wl)
    G = make_gpu(P, torch.float32)
    cell = float(np.prod([2 * np.pi / n for n in wl.shape]))
    v = dev(0.5 * wl.vstar, torch.float32)
    d = dev(smooth_direction(wl.shape, 21, True), torch.float32)
    e = dev(smooth_direction(wl.shape, 22, True), torch.float32)
    Hd, He = G.hessian_matvec(v, d), G.hessian_matvec(v, e)
    ip = lambda a, b: cell * float((a.double() * b.double()).sum())
    a, b = ip(e, Hd), ip(d, He)
    say(f"  <e,Hd> {a:.6e} <d,He> {b:.6e} <d,Hd> {ip(d, Hd):.6e} <e,He> {ip(e, He):.6e}")
    dd, ee = ip(d, Hd), ip(e, He)
    assert dd > 0 and ee > 0
    # the gap relative to the Cauchy-Schwarz scale (3e-6 at 64^3 in the oracle)
    assert abs(a - b) <= 1e-3 * np.sqrt(dd * ee)
    v0 = G.new_velocity()
    info = G.step(gan.SolveParams(eps_rel=1e-3, n_iter=5, accel=gan.ACCEL_NK), v0)
    say(f"  NK step: J {info.J:.6e} ginf {info.ginf:.3e} / {info.g0inf:.3e} cg {info.n_beta} "
        f"rho {info.rho}")
    J0 = G.eval_objective(G.new_velocity())
    assert info.J < J0 and info.ginf < info.g0inf
    assert info.n_beta >= 1 and info.step_kind == gan.STEP_NEWTON
    G.close()


# ---- preconditioners of the Newton step ----------------------------------------
PCS = {"ireg": 0, "h0rpc": 1, "2lrpcsym": 2}


def data_term_lambda_max(P, iters=60):
    """Largest eigenvalue of Hreg^-1/2 [P] grad m0 (grad m0 . ) Hreg^-1/2 (power iteration)."""
    g = P.grid
    gm = onk.sp.gradient(g, P.m0)
    R = lambda x: onk.reg_inverse_sqrt(g, x, P.p, P.alpha, P.incompressible)

    def op(x):
        y = R(x)
        dt = np.sum(gm * y, axis=0) * gm
        return R(onk.sp.leray(g, dt) if P.incompressible else dt)

    x = np.random.default_rng(0).standard_normal((g.d,) + g.shape)
    lam = 0.0
    for _ in range(iters):
        y = op(x)
        lam = np.sqrt(g.inner(y, y) / g.inner(x, x))
        x = y / np.sqrt(g.inner(y, y))
    return lam


def oracle_pc(name, P, v, r):
    if name == "ireg":
        return onk.precond_apply(P, r)
    if name == "h0rpc":
        return onk.h0_precond_apply(P, r)
    return onk.TwoLevel(P, v).apply(r)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("pc", list(PCS))
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_newton_preconditioner_parity(case, pc, prec):
    """z = M^-1 r element by element against the oracle (the inner GMRES / coarse
    CG with the same stopping rule)."""
    name, shape, nt = case
    say(f"case {name} shape {shape} nt {nt} {pc} {prec}")
    wl = synth.workload(name, shape=shape)
    P = as_precision(oracle_problem(wl, nt=nt), prec)
    dtype = torch.float64 if prec == "f64" else torch.float32
    G = make_gpu(P, dtype)
    v = round_to(0.5 * wl.vstar, prec)
    tol = TOL[prec]
    if pc != "ireg":
        # The inner solves work on I + Hreg^-1/2 H_data Hreg^-1/2 (or the
        # left form, same spectrum): the relative error of their solution is up
        # to kappa times that of the operator, one unit of rounding of the
        # path's precision.  kappa = 1 + lambda_max, estimated by power
        # iteration on the zero-velocity data term.
        kappa = 1.0 + data_term_lambda_max(P)
        eps = np.finfo(np.float64 if prec == "f64" else np.float32).eps
        tol = max(tol, eps * kappa)
        say(f"  kappa {kappa:.4g}, tolerance {tol:.2e}")
    for seed in (31, 32):
        r = round_to(smooth_direction(wl.shape, seed, wl.incompressible), prec)
        zo = oracle_pc(pc, P, v, r)
        zg = host(G.newton_precond(PCS[pc], dev(v, dtype), dev(r, dtype)))
        err = rel(zg, zo)
        say(f"  seed {seed}: rel err {err:.2e}")
        assert err <= tol, (seed, err)
    G.close()


@pytest.mark.parametrize("pc", ["h0rpc", "2lrpcsym"])
def test_nk_trajectory_parity_with_preconditioner_f64(pc):
    """NK with the zero-velocity or the two-level preconditioner on the c0
    recipe (64^2, FP64) against the oracle's loop, to ||g||_inf <= 1e-4 ||g_0||_inf."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0")
    P = oracle_problem(wl)
    res = onk.nk_solve(P, eps_rel=1e-4, n_iter=8, keep_iterates=True, precond=pc)
    G = make_gpu(P, torch.float64)
    params = gan.SolveParams(eps_rel=1e-4, n_iter=8, accel=gan.ACCEL_NK, nk_precond=PCS[pc])
    v = G.new_velocity()
    for k in range(1, 9):
        info = G.step(params, v)
        rec = res.records[k - 1]
        err = rel(host(v), res.iterates[k])
        say(f"  k {k} J {info.J:.12e} / {rec.J:.12e} cg {info.n_beta}/{rec.cg_iters} "
            f"rho {info.rho}/{rec.rho} iterate err {err:.2e}")
        assert info.n_beta == rec.cg_iters
        assert info.rho == rec.rho and info.n_trials == rec.trials
        assert err <= 1e-8
        assert abs(info.J - rec.J) <= 1e-10 * abs(rec.J)
        if info.stop:
            break
    assert info.k == len(res.records)
    G.close()


def test_newton_preconditioner_errors():
    import paper_2510_08782_amd as gan
    wl = synth.workload("c0", shape=(27, 36))
    P = oracle_problem(wl, nt=2)
    G = make_gpu(P, torch.float64)
    v = G.new_velocity()
    r = dev(smooth_direction(wl.shape, 3), torch.float64)
    with pytest.raises(gan.GanmresError) as ei:   # odd size: no half grid
        G.newton_precond(gan.PC_2LRPCSYM, v, r)
    assert ei.value.code == -1
    with pytest.raises(gan.GanmresError):
        G.newton_precond(7, v, r)
    with pytest.raises(gan.GanmresError):
        G.step(gan.SolveParams(n_iter=2, accel=gan.ACCEL_NK, nk_precond=9), v)
    # the zero-velocity preconditioner has no size restriction
    z = host(G.newton_precond(gan.PC_H0RPC, v, r))
    assert rel(z, onk.h0_precond_apply(P, host(r))) <= 1e-10
    G.close()


@pytest.mark.parametrize("pc", ["h0rpc", "2lrpcsym"])
def test_c2_full_size_nk_step_with_preconditioner(pc):
    """128^3 incompressible FP32: one NK step from v = 0 with each inner-solve
    preconditioner lowers J and the gradient, with no more CG iterations than
    the regulariser preconditioner needs."""
    import paper_2510_08782_amd as gan
    wl = synth.workload("c2")
    P = oracle_problem(wl)
    its = {}
    for name in ("ireg", pc):
        G = make_gpu(P, torch.float32)
        v0 = G.new_velocity()
        info = G.step(gan.SolveParams(eps_rel=1e-3, n_iter=5, accel=gan.ACCEL_NK,
                                      nk_precond=PCS[name]), v0)
        say(f"  {name}: J {info.J:.6e} ginf {info.ginf:.3e} / {info.g0inf:.3e} cg {info.n_beta} "
            f"rho {info.rho}")
        its[name] = info.n_beta
        J0 = G.eval_objective(G.new_velocity())
        assert info.J < J0 and info.ginf < info.g0inf
        G.close()
    assert its[pc] <= its["ireg"]
