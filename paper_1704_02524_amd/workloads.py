"""Seeded synthetic workloads for the Lax / Hopf solver.

This module only draws inputs: query points, initial guesses (including the
restart guesses the method draws), and the per-problem parameters.  It holds
none of the method's arithmetic, and both the GPU path and the CPU reference
consume exactly the arrays it returns.

The problem family is the one of the paper's section 5 experiments (state-
dependent quadratic Hamiltonians with ellipsoid initial data, queries in a box,
random initial guesses): the Hamiltonian

    H(x, p) = <A x, p> + 1/2 m(|x|^2) sum_i d_i p_i^2 + 1/2 w |x|^2,
    m = c^e,  c in {1, 1 + kappa r/(1+r), 1 + kappa tanh(r/s)},

and the initial data g(x) = 1/2 sum_i x_i^2 / a_i^2 + j0.

Every array is generated from numpy's PCG64 seeded with a SeedSequence, with
one child stream per quantity, so that a workload with fewer points is a
prefix of the full one.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# enum values shared with the C interfaces (they are plain integers there)
M_CONST, M_RAT, M_TANH = 0, 1, 2
LAX, HOPF = 0, 1
TRAPZ, RK4AUG = 0, 1
CD_FD, GD_ADJ = 0, 1
F64, F32 = 0, 1

SEED_BASE = 170402524

# Initial step size 1/L of Algorithm 1 where a configuration states none: the
# paper's Lipschitz guess L = 3 of its smooth quadratic Example 2.
ALPHA_DEFAULT = 1.0 / 3.0

# The step is halved when a trial step fails to realise this fraction of the
# decrease its gradient predicts (Armijo).  0 means halving on ascent only,
# which the n=2 configuration states.
ARMIJO_DEFAULT = 0.1


@dataclasses.dataclass
class Workload:
    """One problem instance plus its queries and guesses."""
    name: str
    n: int
    t: float
    nsteps: int
    m_kind: int
    e: int
    kappa: float
    s: float
    w: float
    d: np.ndarray            # [n]
    A: Optional[np.ndarray]  # [n, n] or None
    a: np.ndarray            # [n]
    j0: float
    formula: int
    quad: int
    x: np.ndarray            # [B, n]
    guesses: np.ndarray      # [B, G, R_max+1, n]
    mode: int = GD_ADJ
    dtype: int = F64
    max_iter: int = 200
    alpha0: float = 0.1
    fd_sigma: float = 1e-4
    eps_step: float = 0.5e-7
    cert_tol: float = 1e-8
    ckpt_K: int = 16
    v_max: float = 1e6
    acc_rel: float = 64 * 2.220446049250313e-16
    armijo_c: float = ARMIJO_DEFAULT
    cert_fp64: bool = True
    # FP32 adjoint descent: continue in FP64 an attempt whose FP32 result the
    # FP64 certificate rejects (the FP64 reference's attempt sequence)
    fp64_continue: bool = True
    seed: int = 0

    @property
    def B(self) -> int:
        return int(self.x.shape[0])

    @property
    def G(self) -> int:
        return int(self.guesses.shape[1])

    @property
    def R_max(self) -> int:
        return int(self.guesses.shape[2]) - 1

    def subset(self, b0: int, b1: int) -> "Workload":
        """The same problem restricted to points [b0, b1)."""
        return dataclasses.replace(self, x=self.x[b0:b1].copy(),
                                   guesses=self.guesses[b0:b1].copy())

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _streams(seed: int, k: int) -> List[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(k)]


def _round_f32(arr):
    if arr is None:
        return None
    return np.asarray(arr, dtype=np.float32).astype(np.float64)


def _normal_guesses(rng, B, G, R_max, n):
    return rng.standard_normal(size=(B, G, R_max + 1, n))


def _hopf_axes(rng, n, t, kappa):
    """a ~ U[0.5, 2]^n; the first axis (the one with d_1 = -1) is redrawn
    from U[sqrt(1.25 c_max t), 2] when a_1^2 < 1.25 c_max t, so that the Hopf
    objective stays bounded below (c_max = 1 + kappa)."""
    a = rng.uniform(0.5, 2.0, size=n)
    lim = 1.25 * (1.0 + kappa) * t
    if a[0] ** 2 < lim:
        a[0] = rng.uniform(math.sqrt(lim), 2.0)
    return a


def c0_lax_n2(B: Optional[int] = None, seed: int = SEED_BASE + 0) -> Workload:
    """Lax, n=2, FP64: H = 1/2 c(x)^2 |p|^2, c = 1 + 0.25 |x|^2/(1+|x|^2),
    g = 1/2|x|^2 - 1/2, t=0.5, 64 RK4 steps with the trapezoid rule, a 32x32
    grid on [-2,2]^2, 4 guesses N(0,1), central-FD coordinate descent."""
    s_guess, = _streams(seed, 1)
    g1 = np.linspace(-2.0, 2.0, 32)
    x = np.stack(np.meshgrid(g1, g1, indexing="ij"), axis=-1).reshape(-1, 2)
    Bf = x.shape[0]
    guesses = _normal_guesses(s_guess, Bf, 4, 2, 2)
    B = Bf if B is None else B
    return Workload(
        name="lax_n2_rat_trapz", n=2, t=0.5, nsteps=64, m_kind=M_RAT, e=2,
        kappa=0.25, s=1.0, w=0.0, d=np.ones(2), A=None, a=np.ones(2), j0=-0.5,
        formula=LAX, quad=TRAPZ, x=x[:B].copy(), guesses=guesses[:B].copy(),
        mode=CD_FD, dtype=F64, max_iter=100, alpha0=0.1, fd_sigma=1e-4,
        eps_step=0.5e-7, cert_tol=1e-3, armijo_c=0.0, seed=seed)


def c1_hopf_n10(B: int = 4096, seed: int = SEED_BASE + 1, mode: int = GD_ADJ) -> Workload:
    """Hopf, n=10, FP64: H = 1/2 c(x)(sum p_i^2 - 2 p_1^2), c = 1 + 0.5
    tanh(|x|^2/10), g = 1/2 sum x_i^2/a_i^2 - 1/2, t=1, 128 RK4 steps with the
    RK4-augmented quadrature, points U[-3,3]^10, 16 guesses N(0,I)."""
    n, t, kappa = 10, 1.0, 0.5
    s_par, s_x, s_guess = _streams(seed, 3)
    a = _hopf_axes(s_par, n, t, kappa)
    d = np.ones(n)
    d[0] = -1.0
    x = s_x.uniform(-3.0, 3.0, size=(B, n))
    guesses = _normal_guesses(s_guess, B, 16, 2, n)
    return Workload(
        name="hopf_n10_tanh", n=n, t=t, nsteps=128, m_kind=M_TANH, e=1,
        kappa=kappa, s=float(n), w=0.0, d=d, A=None, a=a, j0=-0.5,
        formula=HOPF, quad=RK4AUG, x=x, guesses=guesses, mode=mode, dtype=F64,
        max_iter=200, alpha0=ALPHA_DEFAULT, fd_sigma=1e-4, eps_step=1e-12, cert_tol=1e-8,
        ckpt_K=16, seed=seed)


def c2_batched(seed: int = SEED_BASE + 2, dtype: int = F64, n_inst: int = 64,
               max_points: Optional[int] = None) -> List[Workload]:
    """64 uneven Hopf instances of the n=10 family: n in {4,8,16,32},
    t ~ U[0.2,2], steps in {32,64,128,256}, log-uniform point counts in
    [256, 8192], points U[-3,3]^n, 8 guesses, per-instance axes."""
    s_meta, = _streams(seed, 1)
    out = []
    child_seeds = np.random.SeedSequence(seed).spawn(n_inst + 1)[1:]
    for i in range(n_inst):
        n = int(s_meta.choice([4, 8, 16, 32]))
        t = float(s_meta.uniform(0.2, 2.0))
        N = int(s_meta.choice([32, 64, 128, 256]))
        B = int(round(math.exp(s_meta.uniform(math.log(256), math.log(8192)))))
        if max_points is not None:
            B = min(B, max_points)
        s_par, s_x, s_guess = [np.random.Generator(np.random.PCG64(c))
                               for c in child_seeds[i].spawn(3)]
        kappa = 0.5
        a = _hopf_axes(s_par, n, t, kappa)
        d = np.ones(n)
        d[0] = -1.0
        x = s_x.uniform(-3.0, 3.0, size=(B, n))
        guesses = _normal_guesses(s_guess, B, 8, 2, n)
        wl = Workload(
            name=f"batched_{i}_n{n}", n=n, t=t, nsteps=N, m_kind=M_TANH, e=1,
            kappa=kappa, s=float(n), w=0.0, d=d, A=None, a=a, j0=-0.5,
            formula=HOPF, quad=RK4AUG, x=x, guesses=guesses, mode=GD_ADJ,
            dtype=dtype, max_iter=200, alpha0=ALPHA_DEFAULT,
            eps_step=1e-12 if dtype == F64 else 1e-6,
            cert_tol=1e-6 if dtype == F64 else 1e-4, ckpt_K=16, seed=seed)
        out.append(_as_dtype(wl) if dtype == F32 else wl)
    return out


def c3_drift_n32(B: int = 65536, seed: int = SEED_BASE + 3, dtype: int = F64) -> Workload:
    """Lax, n=32, linear drift: H = <A x, p> + 1/2 c(x)|p|^2 with c as in the
    n=2 case, A with N(0,1/n) entries rescaled to spectral norm <= 0.9,
    g = 1/2|x|^2 - 1/2, t=1, 256 RK4 steps, points U[-2,2]^32, 8 guesses."""
    n = 32
    s_par, s_x, s_guess = _streams(seed, 3)
    A = s_par.standard_normal(size=(n, n)) / math.sqrt(n)
    nrm = float(np.linalg.norm(A, 2))
    if nrm > 0.9:
        A = A * (0.9 / nrm)
    x = s_x.uniform(-2.0, 2.0, size=(B, n))
    guesses = _normal_guesses(s_guess, B, 8, 2, n)
    wl = Workload(
        name="lax_n32_drift", n=n, t=1.0, nsteps=256, m_kind=M_RAT, e=1,
        kappa=0.25, s=1.0, w=0.0, d=np.ones(n), A=A, a=np.ones(n), j0=-0.5,
        formula=LAX, quad=RK4AUG, x=x, guesses=guesses, mode=GD_ADJ, dtype=dtype,
        max_iter=200, alpha0=ALPHA_DEFAULT, eps_step=1e-12, cert_tol=1e-6, ckpt_K=16,
        seed=seed)
    if dtype == F32:
        # the FP32 comparison run takes the step and certificate thresholds of
        # the other FP32 workload (n = 100): FP32 descent cannot drive the
        # residual to 1e-6
        wl = _as_dtype(wl.with_(eps_step=1e-6, cert_tol=1e-4))
    return wl


def c4_lax_n100(B: int = 262144, seed: int = SEED_BASE + 4) -> Workload:
    """Lax, n=100, FP32 descent with an FP64 certificate: H = 1/2 c(x)|p|^2,
    c = 1 + 0.5 tanh(|x|^2/100), g = 1/2 sum x_i^2/a_i^2 - 1/2, t=0.5, 128 RK4
    steps, points U[-2,2]^100, 4 guesses N(0,I)."""
    n = 100
    s_par, s_x, s_guess = _streams(seed, 3)
    a = s_par.uniform(0.5, 2.0, size=n)
    x = s_x.uniform(-2.0, 2.0, size=(B, n))
    guesses = _normal_guesses(s_guess, B, 4, 2, n)
    wl = Workload(
        name="lax_n100_tanh_f32", n=n, t=0.5, nsteps=128, m_kind=M_TANH, e=1,
        kappa=0.5, s=float(n), w=0.0, d=np.ones(n), A=None, a=a, j0=-0.5,
        formula=LAX, quad=RK4AUG, x=x, guesses=guesses, mode=GD_ADJ, dtype=F32,
        max_iter=300, alpha0=ALPHA_DEFAULT, eps_step=1e-6, cert_tol=1e-4, ckpt_K=8,
        cert_fp64=True, seed=seed)
    return _as_dtype(wl)


def _as_dtype(wl: Workload) -> Workload:
    """FP32 runs: round every real input to FP32 first, so that both sides
    see the same values (the FP64 reference then runs on the rounded data)."""
    return dataclasses.replace(
        wl, x=_round_f32(wl.x), guesses=_round_f32(wl.guesses), a=_round_f32(wl.a),
        A=_round_f32(wl.A), dtype=F32, acc_rel=64 * 1.1920928955078125e-07)


def make(name: str, B: Optional[int] = None, **kw) -> Workload:
    """Build a named single-instance workload."""
    table = {
        "lax_n2": c0_lax_n2,
        "hopf_n10": c1_hopf_n10,
        "lax_n32_drift": c3_drift_n32,
        "lax_n100_f32": c4_lax_n100,
    }
    fn = table[name]
    if B is None:
        return fn(**kw)
    return fn(B=B, **kw)
