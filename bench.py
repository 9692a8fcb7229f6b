"""Benchmark: gradient evaluations per second of GA-NGMRES on the 3-D 128^3
incompressible advection workload (FP32 transport/FFT, FP64 Gram/LSQ), with
the FP64 path, time-to-1e-2 gradient reduction, the roofline of the dominant
kernel and the CPU oracle as a reported baseline.

A step is one GA-NGMRES(5; 2, 1) iteration of the library (ganmres_step):
preconditioner, Armijo line search (objective evaluations), gradient at q,
Gram/least squares/update on NGMRES steps, stop test.  `value` counts the
gradient evaluations those steps perform per second of wall time.
Inputs (m0, m1, v) are resident in HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(torch, gan, synth, dtype, wl):
    """Device problem of workload wl; m1 = m0 transported by v* with the
    library's own forward solve (the benchmark's reference image)."""
    dev = lambda x: torch.tensor(x, dtype=dtype, device="cuda")
    m0 = dev(wl.m0)
    vstar = dev(wl.vstar)
    gen = gan.Problem(m0, m0, wl.nt, wl.alpha, wl.reg_order, model=wl.model,
                      incompressible=wl.incompressible)
    gen.eval_objective(vstar)
    m1 = gen.get_field("state", wl.nt)
    gen.close()
    P = gan.Problem(m0, m1, wl.nt, wl.alpha, wl.reg_order, model=wl.model,
                    incompressible=wl.incompressible)
    return P, vstar


def run_steps(torch, P, params, v, nsteps):
    """nsteps GA-NGMRES iterations (restarting from v = 0 after a stop).
    Returns (gradient evaluations, objective evaluations)."""
    ngrad = nobj = 0
    for _ in range(nsteps):
        info = P.step(params, v)
        ngrad += info.n_grad
        nobj += info.n_trials
        if info.stop:
            P.reset()
            v.zero_()
    return ngrad, nobj


def time_steps(torch, P, params, steps, warmup, timing=False, classes=None):
    """steps solver iterations after warmup; timing: bracket the launches of
    `classes` (all when None) with HIP events and return the per-class report."""
    v = P.new_velocity()
    P.reset()
    run_steps(torch, P, params, v, warmup)
    if timing:
        P.timing(True, classes)
        P.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ngrad, nobj = run_steps(torch, P, params, v, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = None
    if timing:
        rep = P.timing_report()
        P.timing(False)
    return t1 - t0, ngrad, nobj, rep


def time_gradients(torch, P, v, reps):
    g = P.new_velocity()
    P.eval_gradient(v, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.eval_gradient(v, g)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def time_to_solution(torch, P, params):
    v = P.new_velocity()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v, infos = P.solve(params, v0=v)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    last = infos[-1]
    out = dict(seconds=round(t, 4), iterations=last.k,
               rel_grad=last.ginf / last.g0inf, reached=bool(last.ginf <= params.eps_rel * last.g0inf),
               grad_evals=sum(i.n_grad for i in infos),   # includes g(v^0)
               obj_evals=sum(i.n_trials for i in infos), J=last.J)
    import paper_2510_08782_amd as gan
    if params.accel == gan.ACCEL_NK:   # one Hessian matvec per CG iteration
        out["hessian_matvecs"] = sum(i.n_beta for i in infos)
    return out


def algorithmic_bytes(kernel, wl, N, s):
    """Compulsory HBM bytes of one launch of `kernel` on this workload.

    sl_step:    read source field, d displacement fields (plus the factor
                when a source term is present), write one field.
    deriv_axis: body force along one axis: read (n_t+1) states and (n_t+1)
                adjoints, write one component.
    """
    d = len(wl.shape)
    if kernel == "sl_step":
        return (1 + d + 1) * N * s
    if kernel == "deriv_axis":
        return (2 * (wl.nt + 1) + 1) * N * s
    return None


def cpu_baseline(synth_mod, min_seconds=10.0):
    """The FP64 oracle's gradient on the same recipe at 64^3 (1/8 of the
    points), repeated for at least min_seconds, scaled to the 128^3 workload
    by the point count."""
    from oracle.transport import TransportProblem
    wl = synth_mod.workload("c2", shape=(64, 64, 64))
    gen = TransportProblem(wl.m0, wl.m0, wl.nt, wl.alpha, wl.reg_order, incompressible=True)
    m1 = gen.forward(wl.vstar)[-1]
    P = TransportProblem(wl.m0, m1, wl.nt, wl.alpha, wl.reg_order, incompressible=True)
    v = 0.5 * wl.vstar
    reps = 0
    t0 = time.perf_counter()
    while True:
        P.gradient(v)
        reps += 1
        t = time.perf_counter() - t0
        if t >= min_seconds:
            break
    scale = (128 ** 3) / (64 ** 3)
    per = t / reps
    return {"value": round(1.0 / (per * scale), 6), "unit": "grad evals/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} oracle gradients of the 128^3 recipe at 64^3 ({t:.1f} s, numpy, "
                      f"single thread), time per gradient scaled x{scale:.0f} by grid points"}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of `kernel`, or None when its source changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_c2_128cubed_traffic.txt")
    src = os.path.join(ROOT, "paper_2510_08782_amd", "csrc",
                       {"sl_step": "sl.hip", "deriv_axis": "spectral.hip"}.get(kernel, ""))
    if not (os.path.exists(path) and os.path.isfile(src)):
        return None
    kv = {}
    for line in open(path):
        if "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if kv.get("source_sha256_16") != digest:
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def c3_throughput(torch, gan, synth):
    """256^3 advection, H2, nt=8: FP32 with checkpointed history (every 2nd
    state) against the plain FP64 path: grad evals/s and device workspace."""
    wl = synth.workload("c3")
    out = {}
    for name, dtype, ck in (("fp32_checkpoint2", torch.float32, 2), ("fp64_plain", torch.float64, 1)):
        dev = lambda x: torch.tensor(x, dtype=dtype, device="cuda")
        m0 = dev(wl.m0)
        vstar = dev(wl.vstar)
        gen = gan.Problem(m0, m0, wl.nt, wl.alpha, wl.reg_order, checkpoint_every=ck)
        gen.eval_objective(vstar)
        m1 = gen.get_field("state", wl.nt)
        gen.close()
        P = gan.Problem(m0, m1, wl.nt, wl.alpha, wl.reg_order, checkpoint_every=ck)
        v = (0.5 * vstar).contiguous()
        torch.cuda.reset_peak_memory_stats()
        t = time_gradients(torch, P, v, 5)
        out[name] = {"grad_evals_per_s": round(1.0 / t, 2), "ms_per_grad": round(1e3 * t, 3),
                     "workspace_bytes": P.workspace_bytes(),
                     "torch_peak_bytes": int(torch.cuda.max_memory_allocated())}
        P.close()
        del m0, m1, vstar, v
        torch.cuda.empty_cache()
    return out


def c4_throughput(torch, gan, synth):
    """The batched 2-D set: 16 problems each at 96^2, 192^2 and 384^2 (FP32,
    H1, nt=4, alpha per problem), one batch handle per size; 15 GA-NGMRES
    iterations of every problem from v = 0.  Aggregate gradient evaluations
    per second over the whole set."""
    import numpy as np
    wls = synth.batch_workloads()
    sv = wls[0].solver
    params = gan.SolveParams(w=sv["w"], sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                             n_iter=sv["n_iter"])
    groups = {}
    for w in wls:
        groups.setdefault(w.shape, []).append(w)
    batches = []
    for shape, ws in groups.items():
        dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")
        m0 = dev(np.stack([w.m0 for w in ws]))
        vstar = dev(np.stack([w.vstar for w in ws], axis=1))
        alphas = [w.alpha for w in ws]
        gen = gan.BatchProblem(m0, m0, ws[0].nt, alphas, ws[0].reg_order)
        gen.eval_objective(vstar)
        m1 = gen.get_field("state", ws[0].nt)
        gen.close()
        batches.append((shape, gan.BatchProblem(m0, m1, ws[0].nt, alphas, ws[0].reg_order)))
    # warm-up: one iteration per batch
    for _, B in batches:
        B.step(params, B.new_velocity())
        B.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ngrad = 0
    per = {}
    for shape, B in batches:
        t1 = time.perf_counter()
        v = B.new_velocity()
        for _ in range(params.n_iter):
            infos = B.step(params, v)
            ngrad += sum(i.n_grad for i in infos)
        torch.cuda.synchronize()
        per[f"{shape[0]}x{shape[1]}"] = {"problems": B.count,
                                         "seconds": round(time.perf_counter() - t1, 4),
                                         "rel_grad_max": max(i.ginf / i.g0inf for i in infos)}
        B.reset()
    dt = time.perf_counter() - t0
    # n_grad of each first step already counts g(v^0)
    for _, B in batches:
        B.close()
    return {"problems": len(wls), "iterations_each": params.n_iter, "seconds": round(dt, 4),
            "grad_evals": ngrad, "grad_evals_per_s": round(ngrad / dt, 1), "per_size": per}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 256^3 throughput figures")
    ap.add_argument("--no-c4", action="store_true", help="skip the batched 2-D set")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is designed, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_08782_amd as gan
    import synth

    wl = synth.workload("c2")
    N = int(np.prod(wl.shape))
    sv = wl.solver
    params = gan.SolveParams(w=sv["w"], sigma=sv["sigma"], tau=sv["tau"], eps_rel=sv["eps_rel"],
                             n_iter=sv["n_iter"])
    log(f"workload c2 {wl.shape} nt={wl.nt}; building FP32 problem")
    P32, vstar32 = make_problem(torch, gan, synth, torch.float32, wl)

    if args.copy_probe:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # Per-class breakdown from a pass with every launch bracketed by events;
    # the timed region then brackets only the dominant class (each event pair
    # costs the stream a few microseconds, so bracketing everything would slow
    # the measured step by about 13%).
    nb = min(args.steps, 10)
    log(f"kernel breakdown: {nb} FP32 steps with every launch timed")
    _, _, _, rep = time_steps(torch, P32, params, nb, args.warmup, timing=True)
    dname = max(rep.items(), key=lambda kv: kv[1][0])[0]
    log(f"timing {args.steps} FP32 steps after {args.warmup} warmup ({dname} launches timed)")
    dt, ngrad, nobj, drep = time_steps(torch, P32, params, args.steps, args.warmup, timing=True,
                                       classes=[dname])
    value = ngrad / dt
    log(f"FP32: {ngrad} grads in {dt:.3f}s -> {value:.1f} grad/s")

    # dominant kernel of the timed region and its roofline
    dms, dcount = drep[dname]
    bpl = algorithmic_bytes(dname, wl, N, 4)
    roofline = None
    if bpl is not None and dcount > 0:
        avg_ms = dms / dcount
        achieved = bpl / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dname), "avg_launch_us": round(avg_ms * 1e3, 2),
                    "bytes_per_launch": bpl, "launches": dcount}
    kernels = {k: {"ms": round(ms, 3), "launches": c,
                   "avg_us": round(1e3 * ms / c, 2) if c else None,
                   "share": round(ms / max(sum(x[0] for x in rep.values()), 1e-12), 4)}
               for k, (ms, c) in rep.items()}
    kernels["_note"] = f"separate pass of {nb} steps with every launch timed"
    for kname in ("sl_step", "deriv_axis"):
        b = algorithmic_bytes(kname, wl, N, 4)
        if kname in rep and rep[kname][1]:
            kernels[kname]["GBps"] = round(b / (rep[kname][0] / rep[kname][1] * 1e-3) / 1e9, 1)

    extra = {}
    v_half = (0.5 * vstar32).contiguous()
    extra["grad_eval_only_fp32_per_s"] = round(1.0 / time_gradients(torch, P32, v_half, 10), 2)
    if not args.no_tts:
        log("time-to-1e-2, FP32 GA-NGMRES")
        extra["tts_fp32_ga_ngmres"] = time_to_solution(torch, P32, params)
        for pname, pc in (("ireg", gan.PC_IREG), ("h0rpc", gan.PC_H0RPC),
                          ("2lrpcsym", gan.PC_2LRPCSYM)):
            log(f"time-to-1e-2, FP32 Gauss-Newton-Krylov baseline, {pname}")
            nk = gan.SolveParams(eps_rel=sv["eps_rel"], n_iter=sv["n_iter"], accel=gan.ACCEL_NK,
                                 nk_precond=pc)
            key = "tts_fp32_nk" if pc == gan.PC_IREG else f"tts_fp32_nk_{pname}"
            extra[key] = time_to_solution(torch, P32, nk)
    extra["peak_workspace_bytes_fp32"] = P32.workspace_bytes()
    P32.close()

    if not args.no_fp64:
        log("FP64 path")
        P64, vstar64 = make_problem(torch, gan, synth, torch.float64, wl)
        k64 = max(4, args.steps // 3)
        dt64, ng64, _, _ = time_steps(torch, P64, params, k64, 2)
        extra["fp64_grad_evals_per_s"] = round(ng64 / dt64, 2)
        extra["grad_eval_only_fp64_per_s"] = round(
            1.0 / time_gradients(torch, P64, (0.5 * vstar64).contiguous(), 5), 2)
        if not args.no_tts:
            log("time-to-1e-2, FP64 GA-NGMRES")
            extra["tts_fp64_ga_ngmres"] = time_to_solution(torch, P64, params)
        P64.close()

    if not args.no_c3:
        log("256^3 throughput (c3)")
        extra["c3_256cubed"] = c3_throughput(torch, gan, synth)

    if not args.no_c4:
        log("batched 2-D set (c4)")
        extra["c4_batched_2d"] = c4_throughput(torch, gan, synth)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle sample")
        cpu = cpu_baseline(synth)

    out = {
        "metric": "grad evals/sec at 3D 128^3 (FP32 vs FP64), time-to-1e-2 grad reduction",
        "value": round(value, 2),
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2: 3-D incompressible advection 128^3, nt=4, H1, alpha=1e-4, "
                               "GA-NGMRES(5;2,1), FP32 transport/FFT, FP64 Gram/LSQ",
                   "grid": list(wl.shape), "nt": wl.nt, "grad_evals_timed": ngrad,
                   "obj_evals_timed": nobj},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_fp32": kernels,
        **extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
