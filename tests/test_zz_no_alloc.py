"""The allocation-free objective (ganmres_eval_objective_noalloc) against the
handle-based ganmres_eval_objective, through the C ABI: two calls in a row on
each case, the second on a smaller problem, so that the shared device array
keeps the first call's contents when the second runs.  Same kernels on both
sides (twiddles computed on the device here): FP64 to 1e-10 relative, FP32
to 1e-4 (the bounds of the parity tests); an oversized problem is rejected."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from tests._cases import oracle_problem

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cfg_of(gan, shape, nt, alpha, p, model, incompressible, dtype):
    n = list(shape) + [1] * (3 - len(shape))
    return gan.Config(len(shape), (ctypes.c_int * 3)(*n), nt,
                      gan.ADVECTION if model == "advection" else gan.CONTINUITY,
                      int(incompressible), p, alpha,
                      gan.F32 if dtype == torch.float32 else gan.F64, 1)


def noalloc_objective(gan, cfg, m0, m1, v):
    J, mis = ctypes.c_double(), ctypes.c_double()
    stream = torch.cuda.current_stream().cuda_stream
    rc = gan.lib().ganmres_eval_objective_noalloc(ctypes.byref(cfg), m0.data_ptr(), m1.data_ptr(),
                                                  v.data_ptr(), ctypes.c_void_p(stream),
                                                  ctypes.byref(J), ctypes.byref(mis))
    if rc != 0:
        raise gan.GanmresError(rc, gan.lib().ganmres_last_error(None).decode())
    return J.value, mis.value


CASES = [
    # (name, first shape, second (smaller) shape, nt)
    ("c0", (64, 64), (24, 36), 4),
    ("c1", (96, 72), (32, 48), 3),
    ("c2", (32, 24, 48), (16, 12, 18), 2),
    ("c3", (24, 32, 36), (12, 16, 8), 3),
]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_objective_matches_handle(case, prec):
    import paper_2510_08782_amd as gan
    name, big, small, nt = case
    dtype = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-10 if prec == "f64" else 1e-4
    for shape in (big, small):
        say(f"noalloc {name} {shape} nt {nt} {prec}")
        wl = synth.workload(name, shape=shape)
        P = oracle_problem(wl, nt=nt)
        dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
        m0, m1 = dev(P.m0), dev(P.m1)
        G = gan.Problem(m0, m1, nt, P.alpha, P.p, model=P.model, incompressible=P.incompressible)
        cfg = cfg_of(gan, shape, nt, P.alpha, P.p, P.model, P.incompressible, dtype)
        for vname, v in (("half", 0.5 * wl.vstar), ("star", wl.vstar)):
            vd = dev(v)
            Jh, mh = G.eval_objective(vd, with_mismatch=True)
            Jn, mn = noalloc_objective(gan, cfg, m0, m1, vd)
            say(f"  {vname}: J {Jn:.15e} / {Jh:.15e}, mismatch {mn:.6e} / {mh:.6e}")
            assert abs(Jn - Jh) <= tol * abs(Jh)
            assert abs(mn - mh) <= tol * abs(mh) + tol * abs(Jh)
        G.close()


def test_noalloc_rejects_oversized_problems_before_device_work():
    import paper_2510_08782_amd as gan
    cfg = cfg_of(gan, (128, 128, 128), 4, 1e-4, 1, "advection", True, torch.float32)
    J, mis = ctypes.c_double(), ctypes.c_double()
    dummy = ctypes.c_void_p(16)   # never dereferenced: the size check fails first
    rc = gan.lib().ganmres_eval_objective_noalloc(ctypes.byref(cfg), dummy, dummy, dummy, None,
                                                  ctypes.byref(J), ctypes.byref(mis))
    assert rc == -1
    assert b"bytes" in gan.lib().ganmres_last_error(None)
    bad = cfg_of(gan, (64, 64), 0, 1e-2, 1, "advection", False, torch.float64)
    assert gan.lib().ganmres_eval_objective_noalloc(ctypes.byref(bad), dummy, dummy, dummy, None,
                                                    ctypes.byref(J), None) == -1
