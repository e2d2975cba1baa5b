"""ctypes access to the FP64 reference of the paper's own scheme and its
further problem families (liboracle_paper.so, built from hj_paper.c).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HJ_PAPER_ORACLE_LIB", os.path.join(HERE, "liboracle_paper.so"))
SRC = os.path.join(HERE, "hj_paper.c")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("hkind", C.c_int32), ("jkind", C.c_int32),
                ("functional", C.c_int32), ("ode", C.c_int32), ("nsteps", C.c_int32),
                ("t", C.c_double), ("m_kind", C.c_int32), ("e", C.c_int32),
                ("kappa", C.c_double), ("s", C.c_double), ("w", C.c_double), ("d", _dp),
                ("k", C.c_int32), ("s1", C.c_double), ("s2", C.c_double), ("c0", C.c_double),
                ("beta", C.c_double), ("gam", C.c_double), ("mu", _dp), ("a", _dp),
                ("j0", C.c_double), ("rscale", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_iter", C.c_int32), ("R_max", C.c_int32),
                ("M", C.c_int32), ("alpha0", C.c_double), ("fd_sigma", C.c_double),
                ("eps", C.c_double), ("cert_tol", C.c_double), ("v_max", C.c_double),
                ("momentum", C.c_double), ("acc_rel", C.c_double)]


def build(force: bool = False) -> str:
    """Compile the reference with plain gcc -O2 (no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < max(os.path.getmtime(SRC),
                                            os.path.getmtime(os.path.join(HERE, "hj_paper.h"))):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Problem)
        L.hjp_hamiltonian.argtypes = [P, _dp, _dp]
        L.hjp_hamiltonian.restype = C.c_double
        L.hjp_grads.argtypes = [P, _dp, _dp, _dp, _dp]
        L.hjp_g.argtypes = [P, _dp]
        L.hjp_g.restype = C.c_double
        L.hjp_grad_g.argtypes = [P, _dp, _dp]
        L.hjp_eval.argtypes = [P, _dp, _dp, _dp, _dp]
        L.hjp_eval.restype = C.c_double
        L.hjp_descend.argtypes = [P, C.POINTER(Opts), _dp, _dp, _dp, _dp, _ip, _lp]
        L.hjp_descend.restype = C.c_int32
        L.hjp_solve.argtypes = [P, C.POINTER(Opts), _dp, C.c_int64, _dp, C.c_int32, _dp, _dp,
                                _ip, _dp, _dp, _ip, _ip, _lp]
        L.hjp_solve.restype = C.c_int32
        L.hjp_lax_friedrichs.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                         C.c_double, C.c_double, _dp]
        L.hjp_lax_friedrichs.restype = C.c_int32
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class PaperOracle:
    """The reference for one problem (H, g, t, N, functional, ODE scheme)."""

    def __init__(self, wl):
        n = wl.n
        self._d = _f64(wl.d)
        self._a = _f64(wl.a)
        self._mu = _f64(wl.mu if wl.mu is not None else np.zeros(n))
        self.n = n
        self.P = Problem(n, wl.h_kind, wl.j_kind, wl.formula, wl.ode, wl.nsteps, wl.t,
                         wl.m_kind, wl.e, wl.kappa, wl.s, wl.w, _ptr(self._d), wl.k_split,
                         wl.s1, wl.s2, wl.c0, wl.beta, wl.gam, _ptr(self._mu), _ptr(self._a),
                         wl.j0, wl.rscale)
        self.O = Opts(wl.mode - 2, wl.max_iter, wl.R_max, wl.M, wl.alpha0, wl.fd_sigma,
                      wl.eps_step, wl.cert_tol, wl.v_max, wl.momentum, wl.acc_rel)

    def hamiltonian(self, x, p):
        return lib().hjp_hamiltonian(C.byref(self.P), _ptr(_f64(x)), _ptr(_f64(p)))

    def grads(self, x, p):
        Hx, Hp = np.zeros(self.n), np.zeros(self.n)
        lib().hjp_grads(C.byref(self.P), _ptr(_f64(x)), _ptr(_f64(p)), _ptr(Hx), _ptr(Hp))
        return Hx, Hp

    def g(self, x):
        return lib().hjp_g(C.byref(self.P), _ptr(_f64(x)))

    def grad_g(self, x):
        out = np.zeros(self.n)
        lib().hjp_grad_g(C.byref(self.P), _ptr(_f64(x)), _ptr(out))
        return out

    def eval(self, x, v):
        rho = C.c_double()
        yN = np.zeros(2 * self.n)
        phi = lib().hjp_eval(C.byref(self.P), _ptr(_f64(x)), _ptr(_f64(v)), C.byref(rho),
                             _ptr(yN))
        return phi, rho.value, yN

    def descend(self, x, v0):
        v = _f64(v0).copy()
        phi, rho, it, ev = C.c_double(), C.c_double(), C.c_int32(), C.c_int64(0)
        st = lib().hjp_descend(C.byref(self.P), C.byref(self.O), _ptr(_f64(x)), _ptr(v),
                               C.byref(phi), C.byref(rho), C.byref(it), C.byref(ev))
        return dict(status=st, v=v, phi=phi.value, rho=rho.value, iters=it.value,
                    n_eval=ev.value)

    def solve(self, x, guesses):
        x = _f64(x)
        guesses = _f64(guesses)
        B, n = x.shape
        G = guesses.shape[1]
        u, arg = np.zeros(B), np.zeros((B, n))
        cert = np.zeros(B, np.int32)
        sp, sr = np.zeros((B, G)), np.zeros((B, G))
        sc, si = np.zeros((B, G), np.int32), np.zeros((B, G), np.int32)
        se = np.zeros((B, G), np.int64)
        rc = lib().hjp_solve(C.byref(self.P), C.byref(self.O), _ptr(x), B, _ptr(guesses), G,
                             _ptr(u), _ptr(arg), _ptr(cert, _ip), _ptr(sp), _ptr(sr),
                             _ptr(sc, _ip), _ptr(si, _ip), _ptr(se, _lp))
        if rc != 0:
            raise ValueError("hjp_solve rejected its arguments")
        return dict(u=u, argopt=arg, cert=cert, slot_phi=sp, slot_rho=sr, slot_cert=sc,
                    slot_iters=si, slot_eval=se)

    def lax_friedrichs(self, x0, y0, dx, dy, nx, ny, dt, nt, ax, ay):
        phi = np.zeros((ny, nx))
        rc = lib().hjp_lax_friedrichs(C.byref(self.P), x0, y0, dx, dy, nx, ny, dt, nt, ax, ay,
                                      _ptr(phi))
        if rc != 0:
            raise ValueError("hjp_lax_friedrichs rejected its arguments")
        return phi
