"""Thin Python binding of libganmres.so, the MI355X GA-NGMRES transport library.

Argument marshalling only: every step of the objective, gradient,
preconditioner and GA-NGMRES iteration runs in the library's HIP kernels.
torch supplies device memory and the stream.  There is no fallback: if the
library is missing or a call fails, an exception is raised.

Shapes: an image is a tensor of shape (n_1, ..., n_d), a velocity one of shape
(d, n_1, ..., n_d), contiguous, float32 or float64 on the GPU, matching the
problem's dtype.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
# GANMRES_CHECKED=1 selects the build whose gathers check every interpolation
# stencil against the window staged in LDS (python -m paper_2510_08782_amd.build --checked)
LIB_PATH = os.path.join(HERE, "_lib", "libganmres_checked.so"
                        if os.environ.get("GANMRES_CHECKED") == "1" else "libganmres.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ganmres.h")

ADVECTION, CONTINUITY = 0, 1
F32, F64 = 0, 1
VARIANT_GA, VARIANT_ALT = 0, 1
STEP_NGMRES, STEP_FP, STEP_AA, STEP_NEWTON = 0, 1, 2, 3
ACCEL_NGMRES, ACCEL_AA, ACCEL_NK = 0, 1, 2
PC_IREG, PC_H0RPC, PC_2LRPCSYM = 0, 1, 2
MAX_WINDOW = 64

ERRORS = {
    -1: "GANMRES_EINVAL", -2: "GANMRES_ENOMEM", -3: "GANMRES_EDEVICE",
    -4: "GANMRES_ENONFINITE", -5: "GANMRES_ELINESEARCH", -6: "GANMRES_ELSQ",
    -7: "GANMRES_ESTATE",
}


class GanmresError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("nt", ctypes.c_int),
                ("model", ctypes.c_int), ("incompressible", ctypes.c_int),
                ("reg_order", ctypes.c_int), ("alpha", ctypes.c_double),
                ("dtype", ctypes.c_int), ("checkpoint_every", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int), ("sigma", ctypes.c_int), ("tau", ctypes.c_int),
                ("eps_rel", ctypes.c_double), ("n_iter", ctypes.c_int),
                ("c_armijo", ctypes.c_double), ("max_backtracks", ctypes.c_int),
                ("rho_cap", ctypes.c_double), ("variant", ctypes.c_int), ("accel", ctypes.c_int),
                ("nk_precond", ctypes.c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("step_kind", ctypes.c_int), ("stop", ctypes.c_int),
                ("n_trials", ctypes.c_int), ("n_grad", ctypes.c_int), ("n_beta", ctypes.c_int),
                ("lsq_fallback", ctypes.c_int),
                ("J", ctypes.c_double), ("J_q", ctypes.c_double), ("ginf", ctypes.c_double),
                ("g0inf", ctypes.c_double), ("rho", ctypes.c_double),
                ("beta", ctypes.c_double * (MAX_WINDOW + 1))]


_lib = None


def lib():
    """Load libganmres.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        flag = " --checked" if LIB_PATH.endswith("_checked.so") else ""
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2510_08782_amd.build{flag}`")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.ganmres_create.argtypes = [ctypes.POINTER(Config), vp, vp, vp, ctypes.POINTER(vp)]
    L.ganmres_create_batch.argtypes = [ctypes.POINTER(Config), ip, dp, vp, vp, vp,
                                       ctypes.POINTER(vp)]
    L.ganmres_create_group.argtypes = [ctypes.POINTER(Config), ip, ctypes.POINTER(ip),
                                       ctypes.POINTER(ip), dp, ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), vp, ctypes.POINTER(vp)]
    L.ganmres_group_launches.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong)]
    L.ganmres_tile_autotune.argtypes = [vp, ip, ctypes.POINTER(ip), dp]
    L.ganmres_batch_count.argtypes = [vp]
    L.ganmres_batch_values.argtypes = [vp, dp, dp]
    L.ganmres_deformation.argtypes = [vp, vp, vp, dp]
    L.ganmres_hessian_matvec.argtypes = [vp, vp, vp, vp]
    L.ganmres_newton_precond.argtypes = [vp, ip, vp, vp, vp]
    L.ganmres_destroy.argtypes = [vp]
    L.ganmres_last_error.argtypes = [vp]
    L.ganmres_last_error.restype = ctypes.c_char_p
    L.ganmres_eval_objective.argtypes = [vp, vp, ip, dp, dp]
    L.ganmres_eval_gradient.argtypes = [vp, vp, vp, ip, dp]
    L.ganmres_apply_precond.argtypes = [vp, vp, vp, dp]
    L.ganmres_step.argtypes = [vp, ctypes.POINTER(SolverParams), vp, ctypes.POINTER(StepInfo)]
    L.ganmres_solver_reset.argtypes = [vp]
    L.ganmres_lsq.argtypes = [ip, dp, dp, ctypes.POINTER(ctypes.c_int)]
    L.ganmres_eval_objective_noalloc.argtypes = [ctypes.POINTER(Config), vp, vp, vp, vp, dp, dp]
    L.ganmres_get_field.argtypes = [vp, ip, ip, vp]
    L.ganmres_timing_enable.argtypes = [vp, ip]
    L.ganmres_timing_reset.argtypes = [vp]
    L.ganmres_timing_select.argtypes = [vp, ctypes.c_uint]
    L.ganmres_timing_get.argtypes = [vp, ip, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.ganmres_kernel_count.argtypes = []
    L.ganmres_kernel_name.argtypes = [ip]
    L.ganmres_kernel_name.restype = ctypes.c_char_p
    L.ganmres_workspace_bytes.argtypes = [vp]
    L.ganmres_workspace_bytes.restype = ctypes.c_longlong
    _lib = L
    return L


def lsq(G):
    """beta and the fallback flag of the library's host least-squares solve for
    the Gram matrix G (K x K) of [r, g_0, .., g_{K-2}] (see ganmres_lsq)."""
    import numpy as np
    G = np.ascontiguousarray(G, dtype=np.float64)
    K = G.shape[0]
    beta = (ctypes.c_double * (K - 1))()
    fb = ctypes.c_int()
    rc = lib().ganmres_lsq(K, G.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), beta,
                           ctypes.byref(fb))
    if rc != 0:
        raise GanmresError(rc, "ganmres_lsq")
    return np.array(beta[:]), bool(fb.value)


def header_symbols():
    """Function names declared in include/ganmres.h."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(ganmres_[a-z_]+)\s*\(", txt)))


@dataclass
class SolveParams:
    w: int = 5
    sigma: int = 2
    tau: int = 1
    eps_rel: float = 1e-2
    n_iter: int = 200
    c_armijo: float = 1e-4
    max_backtracks: int = 30
    rho_cap: float = 0.0
    variant: int = VARIANT_GA
    accel: int = ACCEL_NGMRES
    nk_precond: int = PC_IREG

    def to_c(self):
        return SolverParams(self.w, self.sigma, self.tau, self.eps_rel, self.n_iter,
                            self.c_armijo, self.max_backtracks, self.rho_cap, self.variant,
                            self.accel, self.nk_precond)


class Problem:
    """A registration problem living on one GPU (one library handle).

    m0, m1: device images; the library copies them.  The handle's stream is
    torch's current stream at construction."""

    def __init__(self, m0, m1, nt, alpha, reg_order, model="advection",
                 incompressible=False, checkpoint_every=1, stream=None):
        import torch
        if not m0.is_cuda:
            raise ValueError("m0/m1 must be device tensors")
        self.torch = torch
        self.dtype = m0.dtype
        if m0.dtype not in (torch.float32, torch.float64) or m1.dtype != m0.dtype:
            raise ValueError("m0/m1 must share dtype float32 or float64")
        self.m0 = m0.contiguous()
        self.m1 = m1.contiguous()
        self.shape = tuple(m0.shape)
        self.dim = len(self.shape)
        n = list(self.shape) + [1] * (3 - self.dim)
        cfg = Config(self.dim, (ctypes.c_int * 3)(*n), int(nt),
                     ADVECTION if model == "advection" else CONTINUITY,
                     int(bool(incompressible)), int(reg_order), float(alpha),
                     F32 if m0.dtype == torch.float32 else F64, int(checkpoint_every))
        self.cfg = cfg
        self.nt = int(nt)
        self.stream = stream if stream is not None else torch.cuda.current_stream(m0.device)
        h = ctypes.c_void_p()
        rc = lib().ganmres_create(ctypes.byref(cfg), self.m0.data_ptr(), self.m1.data_ptr(),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise GanmresError(rc, lib().ganmres_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise GanmresError(rc, lib().ganmres_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().ganmres_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, v):
        if v.dtype != self.dtype or tuple(v.shape) != (self.dim,) + self.shape or not v.is_cuda:
            raise ValueError(f"expected a {self.dtype} device tensor of shape "
                             f"{(self.dim,) + self.shape}")
        if not v.is_contiguous():
            raise ValueError("velocity must be contiguous")
        return v

    def new_velocity(self):
        return self.torch.zeros((self.dim,) + self.shape, dtype=self.dtype, device=self.m0.device)

    # -- calls ----------------------------------------------------------------
    def eval_objective(self, v, keep_history=False, with_mismatch=False):
        J, mis = ctypes.c_double(), ctypes.c_double()
        self._check(lib().ganmres_eval_objective(self.h, self._vec(v).data_ptr(),
                                                 int(keep_history), ctypes.byref(J),
                                                 ctypes.byref(mis)))
        return (J.value, mis.value) if with_mismatch else J.value

    def eval_gradient(self, v, g=None, reuse_forward=False):
        g = self.new_velocity() if g is None else self._vec(g)
        J = ctypes.c_double()
        self._check(lib().ganmres_eval_gradient(self.h, self._vec(v).data_ptr(), g.data_ptr(),
                                                int(reuse_forward), ctypes.byref(J)))
        return J.value, g

    def apply_precond(self, g, s=None):
        s = self.new_velocity() if s is None else self._vec(s)
        gs = ctypes.c_double()
        self._check(lib().ganmres_apply_precond(self.h, self._vec(g).data_ptr(), s.data_ptr(),
                                                ctypes.byref(gs)))
        return s, gs.value

    def step(self, params: SolveParams, v):
        info = StepInfo()
        cp = params.to_c()
        self._check(lib().ganmres_step(self.h, ctypes.byref(cp), self._vec(v).data_ptr(),
                                       ctypes.byref(info)))
        return info

    def hessian_matvec(self, v, vt, out=None):
        """Gauss-Newton Hessian H_gn[v] applied to vt (the Newton-Krylov baseline)."""
        out = self.new_velocity() if out is None else self._vec(out)
        self._check(lib().ganmres_hessian_matvec(self.h, self._vec(v).data_ptr(),
                                                 self._vec(vt).data_ptr(), out.data_ptr()))
        return out

    def newton_precond(self, which, v, r, z=None):
        """z = M^-1 r for the Newton-step preconditioner `which` (PC_*) at velocity v."""
        z = self.new_velocity() if z is None else self._vec(z)
        self._check(lib().ganmres_newton_precond(self.h, int(which), self._vec(v).data_ptr(),
                                                 self._vec(r).data_ptr(), z.data_ptr()))
        return z

    def reset(self):
        self._check(lib().ganmres_solver_reset(self.h))

    def get_field(self, which, j):
        out = self.torch.empty(self.shape, dtype=self.dtype, device=self.m0.device)
        self._check(lib().ganmres_get_field(self.h, {"state": 0, "adjoint": 1}[which], int(j),
                                            out.data_ptr()))
        return out

    def tile_autotune(self, cls=0):
        """(points per thread chosen for the 2-D gather tiles, microseconds per
        gather launch of the variants 8, 4, 2) of class cls (0 unless a group)."""
        p = ctypes.c_int()
        us = (ctypes.c_double * 3)()
        self._check(lib().ganmres_tile_autotune(self.h, int(cls), ctypes.byref(p), us))
        return p.value, list(us)

    def workspace_bytes(self):
        return int(lib().ganmres_workspace_bytes(self.h))

    # -- timing ---------------------------------------------------------------
    def timing(self, on=True, classes=None):
        """Bracket launches with HIP events; classes: names of the kernel classes
        to time (all when None)."""
        mask = 0xFFFFFFFF
        if classes is not None:
            names = [lib().ganmres_kernel_name(k).decode() for k in range(lib().ganmres_kernel_count())]
            mask = 0
            for c in classes:
                mask |= 1 << names.index(c)
        self._check(lib().ganmres_timing_select(self.h, mask))
        self._check(lib().ganmres_timing_enable(self.h, int(on)))

    def timing_reset(self):
        self._check(lib().ganmres_timing_reset(self.h))

    def timing_report(self):
        out = {}
        for kidx in range(lib().ganmres_kernel_count()):
            ms, cnt = ctypes.c_double(), ctypes.c_longlong()
            self._check(lib().ganmres_timing_get(self.h, kidx, ctypes.byref(ms), ctypes.byref(cnt)))
            out[lib().ganmres_kernel_name(kidx).decode()] = (ms.value, cnt.value)
        return out

    def deformation(self, v, want_det=True):
        """det grad y of the transport map of v: (det image or None, list of
        (min, mean, max, std) per problem)."""
        n = lib().ganmres_batch_count(self.h)
        det = self.torch.empty(self.shape, dtype=self.dtype, device=self.m0.device) if want_det else None
        st = (ctypes.c_double * (4 * n))()
        self._check(lib().ganmres_deformation(self.h, self._vec(v).data_ptr(),
                                              det.data_ptr() if want_det else None, st))
        return det, [tuple(st[4 * i:4 * i + 4]) for i in range(n)]

    def values(self):
        """Per-problem J and mismatch of the last evaluation (lists)."""
        n = lib().ganmres_batch_count(self.h)
        J, mis = (ctypes.c_double * n)(), (ctypes.c_double * n)()
        self._check(lib().ganmres_batch_values(self.h, J, mis))
        return list(J), list(mis)

    def solve(self, params: SolveParams, v0=None, callback=None):
        """Run GA-NGMRES, GA-AA when params.accel is ACCEL_AA, or the
        Gauss-Newton-Krylov baseline when it is ACCEL_NK, from v0 (default 0)
        until the stopping rule holds."""
        v = self.new_velocity() if v0 is None else self._vec(v0).clone()
        self.reset()
        infos = []
        while True:
            info = self.step(params, v)
            infos.append(info)
            if callback:
                callback(info)
            if info.stop:
                break
        return v, infos


def transport_objective():
    """torch.autograd.Function whose forward is the library's objective and
    whose backward is the hand-written adjoint: dJ/dv = |h| g (g is the L2
    representer returned by ganmres_eval_gradient)."""
    import math

    import torch

    class TransportObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v, problem):
            v = v.detach().contiguous()
            J = problem.eval_objective(v, keep_history=True)
            ctx.problem = problem
            ctx.save_for_backward(v)
            return torch.tensor(J, dtype=torch.float64, device=v.device)

        @staticmethod
        def backward(ctx, grad_out):
            (v,) = ctx.saved_tensors
            problem = ctx.problem
            _, g = problem.eval_gradient(v, reuse_forward=True)
            cell = 1.0
            for n in problem.shape:
                cell *= 2.0 * math.pi / n
            return (grad_out.to(g.dtype) * cell) * g, None

    return TransportObjective


class BatchProblem(Problem):
    """count same-size 2-D problems stacked along a leading axis in one handle
    (one launch per kernel serves all of them).  m0, m1: device images of
    shape (count, n0, n1); alphas: one regularisation weight per problem.
    Velocities are component-major, shape (2, count, n0, n1); step() returns
    one StepInfo per problem, and the evaluation calls return sums over the
    problems (values() gives them one by one)."""

    def __init__(self, m0, m1, nt, alphas, reg_order, model="advection", stream=None):
        import torch
        if not m0.is_cuda or m0.dim() != 3:
            raise ValueError("m0/m1 must be device tensors of shape (count, n0, n1)")
        if m0.dtype not in (torch.float32, torch.float64) or m1.dtype != m0.dtype:
            raise ValueError("m0/m1 must share dtype float32 or float64")
        self.torch = torch
        self.dtype = m0.dtype
        self.m0 = m0.contiguous()
        self.m1 = m1.contiguous()
        self.count = int(m0.shape[0])
        alphas = [float(a) for a in alphas]
        if len(alphas) != self.count:
            raise ValueError("one alpha per problem")
        self.shape = tuple(m0.shape)
        self.dim = 2
        cfg = Config(2, (ctypes.c_int * 3)(int(m0.shape[1]), int(m0.shape[2]), 1), int(nt),
                     ADVECTION if model == "advection" else CONTINUITY, 0, int(reg_order),
                     alphas[0], F32 if m0.dtype == torch.float32 else F64, 1)
        self.cfg = cfg
        self.nt = int(nt)
        self.stream = stream if stream is not None else torch.cuda.current_stream(m0.device)
        h = ctypes.c_void_p()
        al = (ctypes.c_double * self.count)(*alphas)
        rc = lib().ganmres_create_batch(ctypes.byref(cfg), self.count, al, self.m0.data_ptr(),
                                        self.m1.data_ptr(),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise GanmresError(rc, lib().ganmres_last_error(None).decode())
        self.h = h

    def step(self, params: SolveParams, v):
        infos = (StepInfo * self.count)()
        cp = params.to_c()
        self._check(lib().ganmres_step(self.h, ctypes.byref(cp), self._vec(v).data_ptr(), infos))
        return list(infos)



class GroupProblem(Problem):
    """Batches of 2-D problems of different grid sizes in one handle: every
    phase of an evaluation or iteration is one kernel launch for all of them.

    m0s, m1s: per size class a device tensor of shape (count_c, n0_c, n1_c);
    alphas: one weight per problem, classes in order.  A velocity is a flat
    tensor holding the classes' batch velocities (2, count_c, n0_c, n1_c) back
    to back (velocity_views gives them); images likewise (image_views).
    step() returns one StepInfo per problem, classes in order."""

    def __init__(self, m0s, m1s, nt, alphas, reg_order, model="advection", stream=None):
        import torch
        if len(m0s) != len(m1s) or not m0s:
            raise ValueError("one m0 and one m1 per class")
        self.torch = torch
        self.dtype = m0s[0].dtype
        if self.dtype not in (torch.float32, torch.float64):
            raise ValueError("float32 or float64 images")
        for a, b in zip(m0s, m1s):
            if a.dim() != 3 or a.shape != b.shape or a.dtype != self.dtype or b.dtype != self.dtype \
                    or not a.is_cuda:
                raise ValueError("images must be device tensors (count, n0, n1) of one dtype")
        self.m0s = [a.contiguous() for a in m0s]
        self.m1s = [b.contiguous() for b in m1s]
        self.m0 = self.m0s[0]
        self.classes = [tuple(a.shape) for a in self.m0s]
        self.count = sum(c[0] for c in self.classes)
        alphas = [float(x) for x in alphas]
        if len(alphas) != self.count:
            raise ValueError("one alpha per problem")
        self.dim = 2
        self.nt = int(nt)
        self.vlen = sum(2 * c * a * b for c, a, b in self.classes)
        self.ilen = sum(c * a * b for c, a, b in self.classes)
        self.shape = (self.ilen,)
        cfg = Config(2, (ctypes.c_int * 3)(1, 1, 1), int(nt),
                     ADVECTION if model == "advection" else CONTINUITY, 0, int(reg_order),
                     alphas[0], F32 if self.dtype == torch.float32 else F64, 1)
        self.cfg = cfg
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.m0.device)
        n = len(self.classes)
        shapes = (ctypes.c_int * (2 * n))(*[x for c in self.classes for x in c[1:]])
        counts = (ctypes.c_int * n)(*[c[0] for c in self.classes])
        al = (ctypes.c_double * self.count)(*alphas)
        p0 = (ctypes.c_void_p * n)(*[a.data_ptr() for a in self.m0s])
        p1 = (ctypes.c_void_p * n)(*[b.data_ptr() for b in self.m1s])
        h = ctypes.c_void_p()
        rc = lib().ganmres_create_group(ctypes.byref(cfg), n, shapes, counts, al, p0, p1,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise GanmresError(rc, lib().ganmres_last_error(None).decode())
        self.h = h

    def _vec(self, v):
        if v.dtype != self.dtype or tuple(v.shape) != (self.vlen,) or not v.is_cuda \
                or not v.is_contiguous():
            raise ValueError(f"expected a contiguous {self.dtype} device tensor of shape "
                             f"({self.vlen},)")
        return v

    def new_velocity(self):
        return self.torch.zeros((self.vlen,), dtype=self.dtype, device=self.m0.device)

    def velocity_views(self, v):
        """Per class the view (2, count_c, n0_c, n1_c) of a group velocity."""
        out, off = [], 0
        for c, a, b in self.classes:
            out.append(v[off:off + 2 * c * a * b].view(2, c, a, b))
            off += 2 * c * a * b
        return out

    def image_views(self, img):
        """Per class the view (count_c, n0_c, n1_c) of a group image."""
        out, off = [], 0
        for c, a, b in self.classes:
            out.append(img[off:off + c * a * b].view(c, a, b))
            off += c * a * b
        return out

    def pack_velocity(self, views):
        """A group velocity from per-class batch velocities (2, count_c, n0_c, n1_c)."""
        return self.torch.cat([x.reshape(-1) for x in views]).contiguous()

    def step(self, params: SolveParams, v):
        infos = (StepInfo * self.count)()
        cp = params.to_c()
        self._check(lib().ganmres_step(self.h, ctypes.byref(cp), self._vec(v).data_ptr(), infos))
        return list(infos)

    def launches(self):
        """(launches the classes made, merged launches that ran them) so far."""
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        self._check(lib().ganmres_group_launches(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value
