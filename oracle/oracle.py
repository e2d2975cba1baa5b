"""ctypes access to the FP64 CPU reference (liboracle_hj.so).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU product path never imports it.

Build with ``python oracle/oracle.py`` (``__graft_entry__.build()`` does it).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HJ_ORACLE_LIB points the tests at another build of the reference (used to
# check that the pins catch planted mistakes).
LIB_PATH = os.environ.get("HJ_ORACLE_LIB", os.path.join(HERE, "liboracle_hj.so"))
SRC = os.path.join(HERE, "hj_oracle.c")

ST_MAXITER, ST_CONVERGED, ST_STALLED, ST_DIVERGED = 0, 1, 2, 3

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("m_kind", C.c_int32), ("e", C.c_int32),
                ("formula", C.c_int32), ("quad", C.c_int32), ("nsteps", C.c_int32),
                ("kappa", C.c_double), ("s", C.c_double), ("w", C.c_double),
                ("t", C.c_double), ("j0", C.c_double),
                ("d", _dp), ("A", _dp), ("a", _dp)]


class Opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_iter", C.c_int32), ("R_max", C.c_int32),
                ("pad_", C.c_int32), ("alpha0", C.c_double), ("fd_sigma", C.c_double),
                ("eps_step", C.c_double), ("cert_tol", C.c_double),
                ("v_max", C.c_double), ("acc_rel", C.c_double), ("armijo_c", C.c_double)]


class SlotDiag(C.Structure):
    _fields_ = [("phi", _dp), ("rho", _dp), ("status", _ip), ("cert", _ip),
                ("iters", _ip), ("attempts", _ip), ("n_fwd", _lp), ("n_bwd", _lp),
                ("v_final", _dp)]


def build(force: bool = False) -> str:
    """Compile the reference with plain gcc -O2 (no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Problem)
        L.hjo_scalars.argtypes = [P, C.c_double, _dp, _dp, _dp]
        L.hjo_hamiltonian.argtypes = [P, _dp, _dp]
        L.hjo_hamiltonian.restype = C.c_double
        L.hjo_field.argtypes = [P, _dp, _dp, _dp]
        L.hjo_integrand.argtypes = [P, _dp, _dp]
        L.hjo_integrand.restype = C.c_double
        L.hjo_trajectory.argtypes = [P, _dp, _dp, _dp]
        L.hjo_eval.argtypes = [P, _dp, _dp, _dp]
        L.hjo_eval.restype = C.c_double
        L.hjo_eval_tangent.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.hjo_eval_tangent.restype = C.c_double
        L.hjo_grad_tangent.argtypes = [P, _dp, _dp, _dp, _dp]
        L.hjo_grad_tangent.restype = C.c_double
        L.hjo_grad_reverse.argtypes = [P, _dp, _dp, _dp, _dp]
        L.hjo_grad_reverse.restype = C.c_double
        L.hjo_certificate.argtypes = [P, _dp]
        L.hjo_certificate.restype = C.c_double
        L.hjo_descend.argtypes = [P, C.POINTER(Opts), _dp, _dp, _dp, _dp, _ip, _lp, _lp]
        L.hjo_descend.restype = C.c_int32
        L.hjo_solve.argtypes = [P, C.POINTER(Opts), _dp, C.c_int64, C.c_int64, C.c_int64,
                                _dp, C.c_int32, _dp, _dp, _ip, C.POINTER(SlotDiag)]
        L.hjo_solve.restype = C.c_int32
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class Oracle:
    """The reference bound to one problem (H, g, t, N, formula, quadrature).

    Arrays passed in are converted to contiguous float64; the object keeps
    references so the C side's pointers stay valid."""

    def __init__(self, n, t, nsteps, m_kind=0, e=1, kappa=0.0, s=1.0, w=0.0,
                 d=None, A=None, a=None, j0=0.0, formula=0, quad=1):
        self.n = int(n)
        self.d = _f64(np.ones(n) if d is None else d)
        self.A = None if A is None else _f64(A)
        self.a = _f64(np.ones(n) if a is None else a)
        self.formula = formula
        self.P = Problem(self.n, m_kind, e, formula, quad, int(nsteps), kappa, s, w,
                         float(t), float(j0), _ptr(self.d), _ptr(self.A), _ptr(self.a))

    @classmethod
    def from_workload(cls, wl, **over):
        kw = dict(n=wl.n, t=wl.t, nsteps=wl.nsteps, m_kind=wl.m_kind, e=wl.e,
                  kappa=wl.kappa, s=wl.s, w=wl.w, d=wl.d, A=wl.A, a=wl.a, j0=wl.j0,
                  formula=wl.formula, quad=wl.quad)
        kw.update(over)
        return cls(**kw)

    # -- pointwise functions ------------------------------------------------
    def scalars(self, r):
        m, m1, m2 = C.c_double(), C.c_double(), C.c_double()
        lib().hjo_scalars(C.byref(self.P), r, C.byref(m), C.byref(m1), C.byref(m2))
        return m.value, m1.value, m2.value

    def hamiltonian(self, gam, p):
        gam, p = _f64(gam), _f64(p)
        return lib().hjo_hamiltonian(C.byref(self.P), _ptr(gam), _ptr(p))

    def field(self, gam, p):
        gam, p = _f64(gam), _f64(p)
        out = np.empty(2 * self.n)
        lib().hjo_field(C.byref(self.P), _ptr(gam), _ptr(p), _ptr(out))
        return out

    def integrand(self, gam, p):
        gam, p = _f64(gam), _f64(p)
        return lib().hjo_integrand(C.byref(self.P), _ptr(gam), _ptr(p))

    def trajectory(self, x, v):
        x, v = _f64(x), _f64(v)
        out = np.empty((self.P.nsteps + 1, 2 * self.n))
        lib().hjo_trajectory(C.byref(self.P), _ptr(x), _ptr(v), _ptr(out))
        return out

    def eval(self, x, v):
        """Phi(v) and y_N."""
        x, v = _f64(x), _f64(v)
        yN = np.empty(2 * self.n)
        phi = lib().hjo_eval(C.byref(self.P), _ptr(x), _ptr(v), _ptr(yN))
        return phi, yN

    def eval_tangent(self, x, v, dx, dv):
        x, v, dx, dv = _f64(x), _f64(v), _f64(dx), _f64(dv)
        dphi = C.c_double()
        phi = lib().hjo_eval_tangent(C.byref(self.P), _ptr(x), _ptr(v), _ptr(dx), _ptr(dv),
                                     C.byref(dphi))
        return phi, dphi.value

    def grad_tangent(self, x, v):
        x, v = _f64(x), _f64(v)
        gv, gx = np.empty(self.n), np.empty(self.n)
        phi = lib().hjo_grad_tangent(C.byref(self.P), _ptr(x), _ptr(v), _ptr(gv), _ptr(gx))
        return phi, gv, gx

    def grad_reverse(self, x, v):
        x, v = _f64(x), _f64(v)
        gv, gx = np.empty(self.n), np.empty(self.n)
        phi = lib().hjo_grad_reverse(C.byref(self.P), _ptr(x), _ptr(v), _ptr(gv), _ptr(gx))
        return phi, gv, gx

    def certificate(self, yN):
        yN = _f64(yN)
        return lib().hjo_certificate(C.byref(self.P), _ptr(yN))

    # -- descent and full solve ---------------------------------------------
    @staticmethod
    def opts(mode=1, max_iter=200, R_max=2, alpha0=0.1, fd_sigma=1e-4, eps_step=0.5e-7,
             cert_tol=1e-8, v_max=1e6, acc_rel=64 * np.finfo(np.float64).eps, armijo_c=0.0):
        return Opts(mode, max_iter, R_max, 0, alpha0, fd_sigma, eps_step, cert_tol,
                    v_max, acc_rel, armijo_c)

    @staticmethod
    def opts_from_workload(wl, **over):
        kw = dict(mode=wl.mode, max_iter=wl.max_iter, R_max=wl.R_max, alpha0=wl.alpha0,
                  fd_sigma=wl.fd_sigma, eps_step=wl.eps_step, cert_tol=wl.cert_tol,
                  v_max=wl.v_max,
                  acc_rel=wl.acc_rel, armijo_c=wl.armijo_c)
        kw.update(over)
        return Oracle.opts(**kw)

    def descend(self, x, v0, O):
        x = _f64(x)
        v = _f64(v0).copy()
        phi, rho = C.c_double(), C.c_double()
        it = C.c_int32()
        fwd, bwd = C.c_int64(0), C.c_int64(0)
        st = lib().hjo_descend(C.byref(self.P), C.byref(O), _ptr(x), _ptr(v), C.byref(phi),
                               C.byref(rho), C.byref(it), C.byref(fwd), C.byref(bwd))
        return dict(status=st, v=v, phi=phi.value, rho=rho.value, iters=it.value,
                    n_fwd=fwd.value, n_bwd=bwd.value)

    def solve(self, x, guesses, O, b0=0, b1=None, diag=True):
        """Full multi-start solve.  x [B, n], guesses [B, G, R+1, n]."""
        x = _f64(x)
        guesses = _f64(guesses)
        B, n = x.shape
        G = guesses.shape[1]
        assert guesses.shape == (B, G, O.R_max + 1, n)
        b1 = B if b1 is None else b1
        u = np.full(B, np.nan)
        arg = np.full((B, n), np.nan)
        cert = np.full(B, -2, dtype=np.int32)
        res = dict(u=u, argopt=arg, cert=cert)
        D = None
        if diag:
            res.update(
                slot_phi=np.full((B, G), np.nan), slot_rho=np.full((B, G), np.nan),
                slot_status=np.full((B, G), -1, np.int32),
                slot_cert=np.full((B, G), -2, np.int32),
                slot_iters=np.zeros((B, G), np.int32),
                slot_attempts=np.zeros((B, G), np.int32),
                slot_fwd=np.zeros((B, G), np.int64), slot_bwd=np.zeros((B, G), np.int64),
                slot_v=np.full((B, G, n), np.nan))
            D = SlotDiag(_ptr(res["slot_phi"]), _ptr(res["slot_rho"]),
                         _ptr(res["slot_status"], _ip), _ptr(res["slot_cert"], _ip),
                         _ptr(res["slot_iters"], _ip), _ptr(res["slot_attempts"], _ip),
                         _ptr(res["slot_fwd"], _lp), _ptr(res["slot_bwd"], _lp),
                         _ptr(res["slot_v"]))
        rc = lib().hjo_solve(C.byref(self.P), C.byref(O), _ptr(x), B, b0, b1, _ptr(guesses), G,
                             _ptr(u), _ptr(arg), _ptr(cert, _ip),
                             C.byref(D) if D is not None else None)
        if rc != 0:
            raise ValueError(f"hjo_solve rejected its arguments (rc={rc})")
        return res


def solve_workload(wl, b0=0, b1=None, diag=True, **opt_over):
    o = Oracle.from_workload(wl)
    return o.solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl, **opt_over), b0, b1, diag)


if __name__ == "__main__":
    build(force=True)
    print(LIB_PATH)
