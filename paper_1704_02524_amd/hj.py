"""Python binding of the C interface in include/hj.h (argument marshalling
only: every step of the solve runs in the HIP kernels of libhj.so).

Device arrays are torch tensors on a ROCm device; PyTorch provides device
memory and streams.  The library must have been built (``python -m
paper_1704_02524_amd.build``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhj.so")

HJ_OK, HJ_EINVAL, HJ_EDTYPE, HJ_ENOMEM, HJ_EDEVICE, HJ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
HJ_H_QUADRATIC, HJ_J_ELLIPSOID = 0, 0
ST_MAXITER, ST_CONVERGED, ST_STALLED, ST_DIVERGED = 0, 1, 2, 3

_dp = C.POINTER(C.c_double)


class HParams(C.Structure):
    _fields_ = [("m_kind", C.c_int32), ("e", C.c_int32), ("kappa", C.c_double),
                ("s", C.c_double), ("w", C.c_double), ("d", _dp), ("A", _dp),
                ("k", C.c_int32), ("s1", C.c_double), ("s2", C.c_double), ("c0", C.c_double),
                ("beta", C.c_double), ("gam", C.c_double), ("mu", _dp)]


class JParams(C.Structure):
    _fields_ = [("a", _dp), ("j0", C.c_double), ("rscale", C.c_double)]


class Guesses(C.Structure):
    _fields_ = [("G", C.c_int32), ("R_max", C.c_int32), ("init", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("formula", C.c_int32), ("mode", C.c_int32),
                ("quad", C.c_int32), ("max_iter", C.c_int32), ("ckpt_K", C.c_int32),
                ("cert_fp64", C.c_int32), ("lanes_per_task", C.c_int32),
                ("alpha0", C.c_double), ("fd_sigma", C.c_double), ("eps_step", C.c_double),
                ("cert_tol", C.c_double), ("v_max", C.c_double), ("acc_rel", C.c_double),
                ("armijo_c", C.c_double),
                ("stream", C.c_void_p), ("workspace", C.c_void_p), ("ws_bytes", C.c_size_t),
                ("ev_begin", C.c_void_p), ("ev_end", C.c_void_p), ("schedule", C.c_int32),
                ("max_groups", C.c_int32), ("fp64_continue", C.c_int32),
                ("ode", C.c_int32), ("M", C.c_int32), ("momentum", C.c_double),
                ("group_cfg", C.c_void_p), ("n_group_cfg", C.c_int32),
                ("cont_lanes_per_task", C.c_int32), ("tail_budget", C.c_int32),
                ("tail_lanes_per_task", C.c_int32)]


class GroupCfg(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("lanes_per_task", C.c_int32), ("ckpt_K", C.c_int32),
                ("max_groups", C.c_int32), ("cont_lanes_per_task", C.c_int32)]

SCHED_AUTO, SCHED_STATIC, SCHED_PERSISTENT = 0, 1, 2


class SlotDiag(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("rho", C.c_void_p), ("status", C.c_void_p),
                ("cert", C.c_void_p), ("iters", C.c_void_p), ("attempts", C.c_void_p),
                ("n_fwd", C.c_void_p), ("n_bwd", C.c_void_p), ("v_final", C.c_void_p)]


class Instance(C.Structure):
    _fields_ = [("n", C.c_int32), ("t", C.c_double), ("nsteps", C.c_int32), ("H", HParams),
                ("J", JParams), ("x", C.c_void_p), ("B", C.c_int64), ("guesses", Guesses),
                ("out_u", C.c_void_p), ("out_argopt", C.c_void_p), ("out_cert", C.c_void_p),
                ("diag", SlotDiag)]


class HJError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded libhj.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HJError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1704_02524_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.hj_solve.restype = C.c_int32
        L.hj_solve.argtypes = [C.c_int32, C.POINTER(HParams), C.c_int32, C.POINTER(JParams),
                               C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                               C.POINTER(Guesses), C.POINTER(Opts), C.c_void_p, C.c_void_p,
                               C.c_void_p, C.POINTER(SlotDiag)]
        L.hj_solve_noalloc.restype = C.c_int32
        L.hj_solve_noalloc.argtypes = L.hj_solve.argtypes
        L.hj_eval.restype = C.c_int32
        L.hj_eval.argtypes = [C.c_int32, C.POINTER(HParams), C.c_int32, C.POINTER(JParams),
                              C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                              C.c_void_p, C.c_int32, C.POINTER(Opts), C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p]
        L.hj_lax_friedrichs.restype = C.c_int32
        L.hj_lax_friedrichs.argtypes = [C.c_int32, C.POINTER(HParams), C.c_int32,
                                        C.POINTER(JParams), C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_int32, C.c_int32, C.c_double,
                                        C.c_int32, C.c_double, C.c_double, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        L.hj_workspace_size.restype = C.c_size_t
        L.hj_workspace_size.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                        C.POINTER(Opts)]
        L.hj_last_error.restype = C.c_char_p
        L.hj_last_error.argtypes = []
        L.hj_version.restype = C.c_int32
        L.hj_version.argtypes = []
        L.hj_batch_plan.restype = C.c_int32
        L.hj_batch_plan.argtypes = [C.c_int32, C.c_int32, C.POINTER(Instance), C.c_int32,
                                    C.POINTER(Opts), C.POINTER(C.c_void_p)]
        L.hj_batch_run.restype = C.c_int32
        L.hj_batch_run.argtypes = [C.c_void_p, C.c_void_p]
        L.hj_batch_info.restype = C.c_int32
        L.hj_batch_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]
        L.hj_batch_free.restype = C.c_int32
        L.hj_batch_free.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != HJ_OK:
        raise HJError(f"libhj error {rc}: {lib().hj_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _tdtype(dtype: int):
    return torch.float64 if dtype == W.F64 else torch.float32


class Problem:
    """Host-side H and J parameters of a workload, kept alive for the call."""

    def __init__(self, wl):
        import numpy as np
        self.n = wl.n
        self._d = np.ascontiguousarray(wl.d, dtype=np.float64)
        self._a = np.ascontiguousarray(wl.a, dtype=np.float64)
        self._A = None if wl.A is None else np.ascontiguousarray(wl.A, dtype=np.float64)
        self._mu = np.ascontiguousarray(wl.mu if wl.mu is not None else np.zeros(wl.n),
                                        dtype=np.float64)
        self.h_kind, self.j_kind = wl.h_kind, wl.j_kind
        self.H = HParams(wl.m_kind, wl.e, wl.kappa, wl.s, wl.w,
                         self._d.ctypes.data_as(_dp),
                         None if self._A is None else self._A.ctypes.data_as(_dp),
                         wl.k_split, wl.s1, wl.s2, wl.c0, wl.beta, wl.gam,
                         self._mu.ctypes.data_as(_dp))
        self.J = JParams(self._a.ctypes.data_as(_dp), wl.j0, wl.rscale)


def make_opts(wl, stream: Optional[torch.cuda.Stream] = None, events=None, **over) -> Opts:
    """hj_opts from a workload; `events` = (begin, end) torch.cuda.Event pair
    recorded by the library around its descent / evaluation kernel."""
    kw = dict(dtype=wl.dtype, formula=wl.formula, mode=wl.mode, quad=wl.quad,
              max_iter=wl.max_iter, ckpt_K=wl.ckpt_K, cert_fp64=int(wl.cert_fp64),
              alpha0=wl.alpha0, fd_sigma=wl.fd_sigma, eps_step=wl.eps_step,
              cert_tol=wl.cert_tol, v_max=wl.v_max, acc_rel=wl.acc_rel,
              armijo_c=wl.armijo_c, fp64_continue=int(wl.fp64_continue), ode=wl.ode,
              M=wl.M, momentum=wl.momentum)
    kw.update(over)
    o = Opts()
    for k, v in kw.items():
        setattr(o, k, v)
    s = stream if stream is not None else torch.cuda.current_stream()
    o.stream = C.c_void_p(s.cuda_stream)
    if events is not None:
        o.ev_begin = C.c_void_p(events[0].cuda_event)
        o.ev_end = C.c_void_p(events[1].cuda_event)
    return o


def device_inputs(wl, device="cuda"):
    """x [B, n] and guesses [B, G, R+1, n] as device tensors of the run dtype."""
    dt = _tdtype(wl.dtype)
    x = torch.as_tensor(wl.x, dtype=dt).to(device).contiguous()
    g = torch.as_tensor(wl.guesses, dtype=dt).to(device).contiguous()
    return x, g


def solve(wl, x: torch.Tensor, guesses: torch.Tensor, diag: bool = True,
          stream: Optional[torch.cuda.Stream] = None, out=None, events=None,
          noalloc: bool = False, **opt_over):
    """hj_solve (hj_solve_noalloc with noalloc=True) on device tensors
    x [B, n], guesses [B, G, R+1, n].

    Returns a dict of device tensors: u [B] (float64), argopt [B, n],
    cert [B] (int32) and, with diag, the per-slot records."""
    B, n = x.shape
    G, R1 = guesses.shape[1], guesses.shape[2]
    dev = x.device
    dt = _tdtype(wl.dtype)
    assert x.dtype == dt and guesses.dtype == dt
    assert x.is_contiguous() and guesses.is_contiguous()
    assert guesses.shape == (B, G, R1, n)
    prob = Problem(wl)
    o = make_opts(wl, stream, events, **opt_over)
    if out is None:
        out = dict(u=torch.empty(B, dtype=torch.float64, device=dev),
                   argopt=torch.empty(B, n, dtype=dt, device=dev),
                   cert=torch.empty(B, dtype=torch.int32, device=dev))
        if diag:
            out.update(
                slot_phi=torch.empty(B, G, dtype=torch.float64, device=dev),
                slot_rho=torch.empty(B, G, dtype=torch.float64, device=dev),
                slot_status=torch.empty(B, G, dtype=torch.int32, device=dev),
                slot_cert=torch.empty(B, G, dtype=torch.int32, device=dev),
                slot_iters=torch.empty(B, G, dtype=torch.int32, device=dev),
                slot_attempts=torch.empty(B, G, dtype=torch.int32, device=dev),
                slot_fwd=torch.empty(B, G, dtype=torch.int64, device=dev),
                slot_bwd=torch.empty(B, G, dtype=torch.int64, device=dev),
                slot_v=torch.empty(B, G, n, dtype=dt, device=dev))
    D = None
    if "slot_phi" in out:
        D = SlotDiag(_ptr(out["slot_phi"]), _ptr(out["slot_rho"]), _ptr(out["slot_status"]),
                     _ptr(out["slot_cert"]), _ptr(out["slot_iters"]),
                     _ptr(out["slot_attempts"]), _ptr(out["slot_fwd"]), _ptr(out["slot_bwd"]),
                     _ptr(out["slot_v"]))
    gs = Guesses(G, R1 - 1, _ptr(guesses))
    fn = lib().hj_solve_noalloc if noalloc else lib().hj_solve
    rc = fn(prob.h_kind, C.byref(prob.H), prob.j_kind, C.byref(prob.J),
            _ptr(x), B, n, float(wl.t), int(wl.nsteps), C.byref(gs), C.byref(o),
            _ptr(out["u"]), _ptr(out["argopt"]), _ptr(out["cert"]),
            C.byref(D) if D is not None else None)
    _check(rc)
    return out


def evaluate(wl, x: torch.Tensor, v: torch.Tensor, grad: bool = False, yN: bool = False,
             stream: Optional[torch.cuda.Stream] = None, **opt_over):
    """hj_eval: objective (and certificate residual, end state, exact
    gradients) at v [B, G, n] for the queries x [B, n]."""
    B, n = x.shape
    G = v.shape[1]
    dev = x.device
    dt = _tdtype(wl.dtype)
    assert x.dtype == dt and v.dtype == dt and v.shape == (B, G, n)
    assert x.is_contiguous() and v.is_contiguous()
    prob = Problem(wl)
    o = make_opts(wl, stream, **opt_over)
    out = dict(phi=torch.empty(B, G, dtype=torch.float64, device=dev),
               rho=torch.empty(B, G, dtype=torch.float64, device=dev))
    if yN:
        out["yN"] = torch.empty(B, G, 2 * n, dtype=dt, device=dev)
    if grad:
        out["grad_v"] = torch.empty(B, G, n, dtype=dt, device=dev)
        out["grad_x"] = torch.empty(B, G, n, dtype=dt, device=dev)
    rc = lib().hj_eval(prob.h_kind, C.byref(prob.H), prob.j_kind, C.byref(prob.J),
                       _ptr(x), B, n, float(wl.t), int(wl.nsteps), _ptr(v), G, C.byref(o),
                       _ptr(out["phi"]), _ptr(out.get("yN")), _ptr(out["rho"]),
                       _ptr(out.get("grad_v")), _ptr(out.get("grad_x")))
    _check(rc)
    return out


def lax_friedrichs(wl, x0, y0, dx, dy, nx, ny, dt, nt, ax, ay, device="cuda",
                   stream: Optional[torch.cuda.Stream] = None):
    """hj_lax_friedrichs: the grid solution [ny, nx] (float64, row j at y0 +
    j dy) of the workload's H and g (n = 2) at t = nt dt."""
    prob = Problem(wl)
    phi = torch.empty(ny, nx, dtype=torch.float64, device=device)
    work = torch.empty(ny, nx, dtype=torch.float64, device=device)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().hj_lax_friedrichs(prob.h_kind, C.byref(prob.H), prob.j_kind, C.byref(prob.J),
                                   x0, y0, dx, dy, nx, ny, dt, nt, ax, ay, _ptr(phi),
                                   _ptr(work), C.c_void_p(s.cuda_stream)))
    return phi


class HJFunctional(torch.autograd.Function):
    """The discretised Lax / Hopf objective as a differentiable function of
    (x, v): x [B, n], v [B, G, n] -> phi [B, G] (float64), both directions in
    libhj.so.  When a gradient can be asked for, the forward runs the RK4
    solve with checkpoints and the discrete adjoint in one kernel (hj_eval
    with gradients) and keeps d phi / d v and d phi / d x, so the backward
    only scales them by the incoming gradient: one forward solve and one
    adjoint sweep per step, never a second forward solve."""

    @staticmethod
    def forward(ctx, x, v, wl):
        # (autograd runs forward with gradients disabled: ask ctx which
        # inputs will want one)
        need = bool(ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
        out = evaluate(wl, x.detach().contiguous(), v.detach().contiguous(), grad=need)
        if need:
            ctx.save_for_backward(out["grad_x"], out["grad_v"])
        return out["phi"]

    @staticmethod
    def backward(ctx, gphi):
        gx_all, gv_all = ctx.saved_tensors
        g = gphi.to(gv_all.dtype).unsqueeze(-1)
        gv = gv_all * g if ctx.needs_input_grad[1] else None
        gx = (gx_all * g).sum(dim=1) if ctx.needs_input_grad[0] else None
        return gx, gv, None


def version() -> int:
    return lib().hj_version()


class BatchPlan:
    """hj_batch_plan over a list of workloads (same formula, quadrature,
    dtype and solve options; any n, t, N, B).  Owns the device inputs and
    outputs of every instance; run() replays the captured graph."""

    def __init__(self, wls, device="cuda", diag=True, group_cfg=None, **opt_over):
        """group_cfg: launch choices by dimension class, a list of dicts with
        n_max and any of lanes_per_task, ckpt_K, max_groups,
        cont_lanes_per_task (0 or absent: the library's choice); an instance
        takes the first entry with n <= n_max."""
        assert len(wls) > 0
        self.wls = wls
        self.inputs, self.outputs, self._probs = [], [], []
        arr = (Instance * len(wls))()
        for i, wl in enumerate(wls):
            x, g = device_inputs(wl, device)
            dt = _tdtype(wl.dtype)
            B, G, n = wl.B, wl.G, wl.n
            out = dict(u=torch.empty(B, dtype=torch.float64, device=device),
                       argopt=torch.empty(B, n, dtype=dt, device=device),
                       cert=torch.empty(B, dtype=torch.int32, device=device))
            if diag:
                out.update(
                    slot_phi=torch.empty(B, G, dtype=torch.float64, device=device),
                    slot_rho=torch.empty(B, G, dtype=torch.float64, device=device),
                    slot_status=torch.empty(B, G, dtype=torch.int32, device=device),
                    slot_cert=torch.empty(B, G, dtype=torch.int32, device=device),
                    slot_iters=torch.empty(B, G, dtype=torch.int32, device=device),
                    slot_attempts=torch.empty(B, G, dtype=torch.int32, device=device),
                    slot_fwd=torch.empty(B, G, dtype=torch.int64, device=device),
                    slot_bwd=torch.empty(B, G, dtype=torch.int64, device=device),
                    slot_v=torch.empty(B, G, n, dtype=dt, device=device))
            prob = Problem(wl)
            self._probs.append(prob)
            self.inputs.append((x, g))
            self.outputs.append(out)
            I = arr[i]
            I.n, I.t, I.nsteps = n, float(wl.t), int(wl.nsteps)
            I.H, I.J = prob.H, prob.J
            I.x, I.B = _ptr(x), B
            I.guesses = Guesses(G, wl.R_max, _ptr(g))
            I.out_u, I.out_argopt, I.out_cert = _ptr(out["u"]), _ptr(out["argopt"]), \
                _ptr(out["cert"])
            if diag:
                I.diag = SlotDiag(_ptr(out["slot_phi"]), _ptr(out["slot_rho"]),
                                  _ptr(out["slot_status"]), _ptr(out["slot_cert"]),
                                  _ptr(out["slot_iters"]), _ptr(out["slot_attempts"]),
                                  _ptr(out["slot_fwd"]), _ptr(out["slot_bwd"]),
                                  _ptr(out["slot_v"]))
        self._arr = arr
        o = make_opts(wls[0], **opt_over)
        if group_cfg:
            cfgs = sorted(group_cfg, key=lambda c: c["n_max"])
            self._gcfg = (GroupCfg * len(cfgs))(*[
                GroupCfg(int(c["n_max"]), int(c.get("lanes_per_task", 0)),
                         int(c.get("ckpt_K", 0)), int(c.get("max_groups", 0)),
                         int(c.get("cont_lanes_per_task", 0))) for c in cfgs])
            o.group_cfg = C.cast(self._gcfg, C.c_void_p)
            o.n_group_cfg = len(cfgs)
        h = C.c_void_p()
        _check(lib().hj_batch_plan(HJ_H_QUADRATIC, HJ_J_ELLIPSOID, arr, len(wls), C.byref(o),
                                   C.byref(h)))
        self.handle = h

    def info(self):
        t, g, nl = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().hj_batch_info(self.handle, C.byref(t), C.byref(g), C.byref(nl)))
        return dict(tasks=t.value, groups=g.value, launches=nl.value)

    def run(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().hj_batch_run(self.handle, C.c_void_p(s.cuda_stream)))
        return self.outputs

    def free(self):
        if getattr(self, "handle", None):
            lib().hj_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
