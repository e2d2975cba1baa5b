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
LAX, HOPF, LAX_MIN = 0, 1, 2          # functionals F1, G, F2 (grid minimum)
TRAPZ, RK4AUG = 0, 1
CD_FD, GD_ADJ, ALG1, MOMENTUM = 0, 1, 2, 3
F64, F32 = 0, 1
RK4, EULER, STAGGERED = 0, 1, 2       # characteristic ODE scheme
H_QUADRATIC, H_NORM = 0, 1
J_ELLIPSOID, J_ROSENBROCK = 0, 1

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
    # the paper's scheme and further families (section 4.1-4.2, section 5):
    # ODE scheme, Hamiltonian and initial-data kinds, the degree-1 family's
    # parameters (H = s1 c1(x)|p_A| + s2 c2(x)|p_B|, A = first k_split
    # components, c_i = c0 (1 + beta exp(-gam |x -+ mu|^2))), the Rosenbrock
    # scale, Algorithm 1's halving period M and the heavy-ball coefficient
    ode: int = RK4
    h_kind: int = H_QUADRATIC
    j_kind: int = J_ELLIPSOID
    k_split: int = 0
    s1: float = 1.0
    s2: float = 0.0
    c0: float = 1.0
    beta: float = 0.0
    gam: float = 0.0
    mu: Optional[np.ndarray] = None
    rscale: float = 0.4e-3
    M: int = 500
    momentum: float = 0.9

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


# ---------------------------------------------------------------------------
# The paper's own experiments (section 5): a 2-D cross-section grid of query
# points in [-3,3]^2 x {0}^(d-2), guesses U[-2,2]^d, the ellipse initial data
# g(x) = 1/2(<x, A x> - 1) with A^-1 = diag(1, 25/4, 1/4, ..., 1/4) (semi-axes
# a = (1, 5/2, 1/2, ...)), step Delta s, difference step sigma, 1/L, M = 500
# and epsilon = 0.5e-7, forward Euler with the rectangle rule and Algorithm 1.
# The paper does not state its grid; `grid` points per side.
# ---------------------------------------------------------------------------
def _paper_common(n, grid, G, seed, R_max=0):
    g1 = np.linspace(-3.0, 3.0, grid)
    xy = np.stack(np.meshgrid(g1, g1, indexing="ij"), axis=-1).reshape(-1, 2)
    x = np.zeros((xy.shape[0], n))
    x[:, :2] = xy
    s_guess, = _streams(seed, 1)
    guesses = s_guess.uniform(-2.0, 2.0, size=(x.shape[0], G, R_max + 1, n))
    a = np.full(n, 0.5)
    a[0] = 1.0
    if n > 1:
        a[1] = 2.5
    return x, guesses, a


def paper_ex2(sign: int = -1, n: int = 2, t: float = 0.5, grid: int = 64, G: int = 5,
              seed: int = SEED_BASE + 5, cert_tol: float = 5e-2) -> Workload:
    """Section 5 Example 2, the harmonic oscillator H = +-1/2(|p|^2 + |x|^2),
    by the maximization (Hopf) principle: Delta s = 0.02, sigma = 0.001,
    L = 3, 5 guesses per point."""
    x, guesses, a = _paper_common(n, grid, G, seed)
    return Workload(
        name=f"paper_ex2_{'minus' if sign < 0 else 'plus'}_d{n}", n=n, t=t,
        nsteps=int(round(t / 0.02)), m_kind=M_CONST, e=1, kappa=0.0, s=1.0, w=float(sign),
        d=np.full(n, float(sign)), A=None, a=a, j0=-0.5, formula=HOPF, quad=TRAPZ, x=x,
        guesses=guesses, mode=ALG1, dtype=F64, max_iter=20000, alpha0=1.0 / 3.0,
        fd_sigma=1e-3, eps_step=0.5e-7, cert_tol=cert_tol, seed=seed, ode=EULER, M=500)


def paper_ex2_rosenbrock(t: float = 0.5, grid: int = 64, G: int = 5,
                         seed: int = SEED_BASE + 6, cert_tol: float = 5e-2) -> Workload:
    """Section 5 Example 2 with the non-convex Rosenbrock initial data (eq.
    weird) and the convex H+ = 1/2(|p|^2 + |x|^2), by the minimization (Lax)
    principle, d = 2."""
    wl = paper_ex2(sign=1, n=2, t=t, grid=grid, G=G, seed=seed, cert_tol=cert_tol)
    return wl.with_(name="paper_ex2_rosenbrock", formula=LAX, j_kind=J_ROSENBROCK,
                    rscale=0.4e-3)


def paper_ex3(sign: int = 1, n: int = 2, t: float = 0.3, grid: int = 64, G: int = 5,
              seed: int = SEED_BASE + 7, formula: int = LAX_MIN,
              cert_tol: float = 5e-2) -> Workload:
    """Section 5 Example 3, H = +-c(x)|p| with c(x) = 1 + 3 exp(-4|x -
    (1,1,0,..)|^2), by the minimization (Lax) principle: Delta s = 0.02,
    sigma = 0.001, L = 0.02; the grid-minimum functional F2 by default (the
    integrand of F1 vanishes for degree-1 H)."""
    x, guesses, a = _paper_common(n, grid, G, seed)
    mu = np.zeros(n)
    mu[:2] = 1.0
    return Workload(
        name=f"paper_ex3_{'plus' if sign > 0 else 'minus'}_d{n}", n=n, t=t,
        nsteps=int(round(t / 0.02)), m_kind=M_CONST, e=1, kappa=0.0, s=1.0, w=0.0,
        d=np.ones(n), A=None, a=a, j0=-0.5, formula=formula, quad=TRAPZ, x=x,
        guesses=guesses, mode=ALG1, dtype=F64, max_iter=20000, alpha0=1.0 / 0.02,
        fd_sigma=1e-3, eps_step=0.5e-7, cert_tol=cert_tol, seed=seed, ode=EULER, M=500,
        h_kind=H_NORM, k_split=n, s1=float(sign), s2=0.0, c0=1.0, beta=3.0, gam=4.0, mu=mu)


def paper_ex5(n: int = 2, t: float = 0.3, grid: int = 64, G: int = 20,
              seed: int = SEED_BASE + 8, cert_tol: float = 5e-2) -> Workload:
    """Section 5 Example 5, H = c1(x)|p_1| - c2(x)|p_2..d| with c1(x) = c(x),
    c2(x) = c(-x), c(x) = 2(1 + 3 exp(-4|x - (1,1,0,..)|^2)), by the
    maximization (Hopf) principle: Delta s = 0.02, sigma = 0.001, L = 50,
    20 guesses per point."""
    x, guesses, a = _paper_common(n, grid, G, seed)
    mu = np.zeros(n)
    mu[:2] = 1.0
    return Workload(
        name=f"paper_ex5_d{n}", n=n, t=t, nsteps=int(round(t / 0.02)), m_kind=M_CONST, e=1,
        kappa=0.0, s=1.0, w=0.0, d=np.ones(n), A=None, a=a, j0=-0.5, formula=HOPF,
        quad=TRAPZ, x=x, guesses=guesses, mode=ALG1, dtype=F64, max_iter=20000,
        alpha0=1.0 / 50.0, fd_sigma=1e-3, eps_step=0.5e-7, cert_tol=cert_tol, seed=seed,
        ode=EULER, M=500, h_kind=H_NORM, k_split=1, s1=1.0, s2=-1.0, c0=2.0, beta=3.0,
        gam=4.0, mu=mu)


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
