"""Pins of the FP64 CPU reference against facts fixed by the paper and by
mathematics, independent of the reference's own code:

  - closed forms of the Lax and Hopf formulas where H does not depend on x
    (the paper's Hopf Example 1, section 3.4) and for the linear-quadratic
    drift problem (Hopf Example 3's linear dynamics, section 3.4, solved by
    the matrix Riccati equation, evaluated with scipy's expm);
  - the harmonic oscillator of the paper's numerical Example 2 (section 5),
    whose value function is quadratic with coefficients tan(theta -+ t);
  - conservation of H along the characteristics and the convergence orders of
    RK4 and the two quadratures;
  - Lax == Hopf on convex problems, argopt == grad_x u (section 1 remark that
    the optimiser is the spatial gradient), brute-force global minima for n=1,2;
  - the exact discrete gradient: tangent == reverse == central differences.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.oracle import Oracle, build, ST_DIVERGED
from paper_1704_02524_amd import workloads as W

build()

LAX, HOPF = W.LAX, W.HOPF
TRAPZ, RK4AUG = W.TRAPZ, W.RK4AUG


def _tight(mode=1, **kw):
    base = dict(mode=mode, max_iter=2000, alpha0=1 / 3, eps_step=1e-13, cert_tol=1e-7,
                R_max=0)
    base.update(kw)
    return Oracle.opts(**base)


def _minimise(o, x, v0, **kw):
    r = o.descend(x, v0, _tight(**kw))
    assert r["status"] != ST_DIVERGED
    return r


# --------------------------------------------------------------------------
# problem functions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m_kind,e", [(W.M_CONST, 1), (W.M_RAT, 1), (W.M_RAT, 2),
                                      (W.M_TANH, 1), (W.M_TANH, 2)])
def test_scalars_special_values_and_derivatives(m_kind, e):
    kappa, s = 0.37, 3.0
    o = Oracle(n=1, t=1.0, nsteps=1, m_kind=m_kind, e=e, kappa=kappa, s=s)
    # r = 0: c = 1 for every kind
    assert o.scalars(0.0)[0] == pytest.approx(1.0, abs=1e-15)
    # saturation / half points of the two speed profiles
    if m_kind == W.M_RAT:
        assert o.scalars(1.0)[0] == pytest.approx((1 + kappa / 2) ** e, rel=1e-14)
        assert o.scalars(1e12)[0] == pytest.approx((1 + kappa) ** e, rel=1e-10)
    if m_kind == W.M_TANH:
        assert o.scalars(s * math.atanh(0.5))[0] == pytest.approx((1 + kappa / 2) ** e,
                                                                  rel=1e-14)
    # m' and m'' against central differences of m and m'
    for r in [0.0, 0.3, 1.7, 6.0]:
        h = 1e-5
        m, m1, m2 = o.scalars(r)
        mp, m1p, _ = o.scalars(r + h)
        mm, m1m, _ = o.scalars(r - h) if r > 0 else o.scalars(r)
        den = 2 * h if r > 0 else h
        ref1 = (mp - mm) / den
        ref2 = (m1p - m1m) / den
        tol = 1e-9 if r > 0 else 1e-4
        assert m1 == pytest.approx(ref1, abs=tol)
        assert m2 == pytest.approx(ref2, abs=tol)


def _rand_problem(rng, n, formula, m_kind=W.M_TANH, e=1, drift=False, w=0.0, quad=RK4AUG,
                  nsteps=32, t=0.7, signs=False):
    d = np.ones(n)
    if signs:
        d[: max(1, n // 3)] = -1.0
    A = rng.standard_normal((n, n)) * 0.3 if drift else None
    a = rng.uniform(1.2, 2.0, n)
    return Oracle(n=n, t=t, nsteps=nsteps, m_kind=m_kind, e=e, kappa=0.4, s=float(n), w=w,
                  d=d, A=A, a=a, j0=-0.5, formula=formula, quad=quad)


@pytest.mark.parametrize("formula", [LAX, HOPF])
@pytest.mark.parametrize("drift", [False, True])
def test_field_is_minus_Hp_plus_Hx(formula, drift):
    """f(y) = (-dH/dp, +dH/dx), checked against central differences of H."""
    rng = np.random.default_rng(1)
    n = 5
    o = _rand_problem(rng, n, formula, m_kind=W.M_RAT, e=2, drift=drift, w=0.3, signs=True)
    gam, p = rng.standard_normal(n), rng.standard_normal(n)
    f = o.field(gam, p)
    h = 1e-6
    for i in range(n):
        e_i = np.zeros(n)
        e_i[i] = h
        Hp = (o.hamiltonian(gam, p + e_i) - o.hamiltonian(gam, p - e_i)) / (2 * h)
        Hx = (o.hamiltonian(gam + e_i, p) - o.hamiltonian(gam - e_i, p)) / (2 * h)
        assert f[i] == pytest.approx(-Hp, abs=1e-8)
        assert f[n + i] == pytest.approx(Hx, abs=1e-8)


@pytest.mark.parametrize("m_kind,e,formula,drift,signs,w", [
    (W.M_RAT, 2, LAX, False, False, 0.0),
    (W.M_TANH, 1, HOPF, False, True, 0.0),
    (W.M_RAT, 1, LAX, True, False, 0.0),
    (W.M_TANH, 1, LAX, False, False, 0.0),
    (W.M_CONST, 1, HOPF, False, False, 1.0),
])
def test_hamiltonian_conserved_at_fourth_order(m_kind, e, formula, drift, signs, w):
    """H is autonomous, so it is constant along exact characteristics; RK4
    keeps it to O(h^4)."""
    rng = np.random.default_rng(2)
    n = 6
    errs = []
    for N in [16, 32, 64]:
        o = _rand_problem(np.random.default_rng(3), n, formula, m_kind=m_kind, e=e,
                          drift=drift, signs=signs, w=w, nsteps=N, t=1.0)
        x, v = rng.standard_normal(n), rng.standard_normal(n)
        rng = np.random.default_rng(2)
        traj = o.trajectory(x, v)
        H0 = o.hamiltonian(traj[0, :n], traj[0, n:])
        HN = o.hamiltonian(traj[-1, :n], traj[-1, n:])
        errs.append(abs(HN - H0))
    assert errs[-1] < 1e-6
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    # at least fourth order (a linear flow, w != 0 with m = 1, does better)
    assert r1 > 12 and r2 > 12, errs


@pytest.mark.parametrize("formula", [LAX, HOPF])
def test_integrand_simplified_forms_match_definitions(formula):
    """The reference evaluates the action with the definitions <p,H_p> - H
    (Lax) and H - <H_x,gamma> (Hopf); its tangent mode uses the simplified
    forms.  Their objective values must agree to rounding."""
    rng = np.random.default_rng(4)
    for m_kind, e in [(W.M_RAT, 2), (W.M_TANH, 1)]:
        for quad in [TRAPZ, RK4AUG]:
            o = _rand_problem(rng, 4, formula, m_kind=m_kind, e=e, w=0.2, quad=quad,
                              drift=True)
            x, v = rng.standard_normal(4), rng.standard_normal(4)
            phi, _ = o.eval(x, v)
            phi_t, _ = o.eval_tangent(x, v, np.zeros(4), np.zeros(4))
            assert phi_t == pytest.approx(phi, rel=1e-13, abs=1e-13)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("quad", [TRAPZ, RK4AUG])
@pytest.mark.parametrize("mode", [0, 1])
def test_free_particle_lax_closed_form(quad, mode):
    """H = 1/2|p|^2, g = 1/2|x|^2: u = |x|^2 / (2(1+t)), argmin x/(1+t).
    RK4 is exact on the linear flow and the integrand is constant along it,
    so the discrete objective has the same minimum."""
    t = 0.8
    o = Oracle(n=3, t=t, nsteps=8, formula=LAX, quad=quad)
    x = np.array([0.4, -1.3, 2.2])
    phi, yN = o.eval(x, x / (1 + t))
    assert phi == pytest.approx(x @ x / (2 * (1 + t)), rel=1e-14)
    assert o.certificate(yN) < 1e-14
    r = _minimise(o, x, np.zeros(3), mode=mode)
    assert r["phi"] == pytest.approx(x @ x / (2 * (1 + t)), rel=1e-12)
    np.testing.assert_allclose(r["v"], x / (1 + t), atol=1e-8)
    assert r["rho"] < 1e-8


@pytest.mark.parametrize("formula", [LAX, HOPF])
def test_x_independent_H_reduces_to_classical_hopf_lax(formula):
    """kappa = 0: H = 1/2 sum d_i p_i^2.  Lax (d = 1) and Hopf (signed d, convex
    g) both give u = 1/2 sum x_i^2/(a_i^2 + t d_i) + j0 (the Hopf formula of
    the paper's Hopf Example 1), with the optimum v = x/(a^2 + t d)."""
    rng = np.random.default_rng(5)
    n, t, j0 = 5, 0.6, -0.5
    a = rng.uniform(1.0, 2.0, n)
    d = np.ones(n)
    if formula == HOPF:
        d[:2] = -1.0
    o = Oracle(n=n, t=t, nsteps=12, d=d, a=a, j0=j0, formula=formula, quad=RK4AUG)
    x = rng.uniform(-2, 2, n)
    u_exact = 0.5 * np.sum(x ** 2 / (a ** 2 + t * d)) + j0
    vstar = x / (a ** 2 + t * d)
    phi, yN = o.eval(x, vstar)
    u = phi if formula == LAX else -phi
    assert u == pytest.approx(u_exact, rel=1e-14)
    assert o.certificate(yN) < 1e-14
    r = _minimise(o, x, rng.standard_normal(n))
    u = r["phi"] if formula == LAX else -r["phi"]
    assert u == pytest.approx(u_exact, rel=1e-12)
    np.testing.assert_allclose(r["v"], vstar, atol=1e-9)


def _oscillator(sign, n, t, N, quad, formula, a):
    # H = sign * 1/2 (|p|^2 + |x|^2): m = 1, d = sign, w = sign
    return Oracle(n=n, t=t, nsteps=N, m_kind=W.M_CONST, d=sign * np.ones(n), w=float(sign),
                  a=a, j0=-0.5, formula=formula, quad=quad)


@pytest.mark.parametrize("sign,formula", [(+1, HOPF), (-1, HOPF), (+1, LAX)])
def test_harmonic_oscillator_closed_form_and_orders(sign, formula):
    """The paper's Example 2: H = +-1/2(|p|^2 + |x|^2) with ellipsoid data has
    u = 1/2 sum tan(theta_i -+ t) x_i^2 + j0, theta_i = atan(1/a_i^2) (a
    quadratic solution of the HJ PDE: the Riccati equation a' = -+(a^2 + 1)).
    The trapezoid rule converges at order 2, the RK4-augmented rule at 4."""
    n, t = 2, 0.5
    a = np.array([1.4, 1.2])   # theta + t stays well inside (-pi/2, pi/2)
    x = np.array([0.7, -0.4])
    theta = np.arctan(1.0 / a ** 2)
    u_exact = 0.5 * np.sum(np.tan(theta - sign * t) * x ** 2) - 0.5
    for quad, order in [(TRAPZ, 2), (RK4AUG, 4)]:
        errs = []
        for N in [16, 32, 64]:
            o = _oscillator(sign, n, t, N, quad, formula, a)
            r = _minimise(o, x, np.zeros(n), alpha0=0.2)
            u = r["phi"] if formula == LAX else -r["phi"]
            errs.append(abs(u - u_exact))
        ratio = errs[1] / errs[2]
        assert 2 ** order * 0.7 < ratio < 2 ** order * 1.4, (quad, errs)
        assert errs[-1] < (1e-5 if order == 2 else 1e-9)


@pytest.mark.parametrize("formula", [LAX])
def test_linear_drift_riccati_closed_form(formula):
    """H = <A x, p> + 1/2|p|^2, g = 1/2|x|^2 + j0 (a linear-quadratic control
    problem, the paper's Hopf Example 3 family): u = 1/2 x^T P(t) x + j0 with
    P' = -(A^T P + P A + P^2), P(0) = I, i.e. P = Y X^{-1} where
    [X; Y] = expm(t [[A, I], [0, -A^T]]) [I; I].  A is not symmetric, so a
    transposed drift operand changes the answer."""
    rng = np.random.default_rng(6)
    n, t = 4, 0.9
    A = rng.standard_normal((n, n)) * 0.5
    M = np.block([[A, np.eye(n)], [np.zeros((n, n)), -A.T]])
    XY = expm(t * M) @ np.vstack([np.eye(n), np.eye(n)])
    P = XY[n:] @ np.linalg.inv(XY[:n])
    x = rng.uniform(-1.5, 1.5, n)
    u_exact = 0.5 * x @ P @ x - 0.5
    errs = []
    for N in [16, 32, 64]:
        o = Oracle(n=n, t=t, nsteps=N, A=A, j0=-0.5, formula=formula, quad=RK4AUG)
        r = _minimise(o, x, np.zeros(n))
        errs.append(abs(r["phi"] - u_exact))
    assert errs[-1] < 1e-8, errs
    assert 16 * 0.6 < errs[0] / errs[1] < 16 * 1.5, errs
    # the optimum is the spatial gradient P x
    np.testing.assert_allclose(r["v"], P @ x, atol=1e-6)
    # the transposed operand gives a different value
    XYt = expm(t * np.block([[A.T, np.eye(n)], [np.zeros((n, n)), -A]])) @ \
        np.vstack([np.eye(n), np.eye(n)])
    Pt = XYt[n:] @ np.linalg.inv(XYt[:n])
    assert abs(0.5 * x @ Pt @ x - 0.5 - r["phi"]) > 1e-3


# --------------------------------------------------------------------------
# consistency on state-dependent problems
# --------------------------------------------------------------------------

def test_lax_equals_hopf_on_convex_state_dependent_problem():
    """For convex H and convex g both formulas give the viscosity solution
    (sections 3.3 and 3.4), so the two discrete optima converge together."""
    n, t = 2, 0.5
    x = np.array([0.9, -0.6])
    diffs = []
    for N in [16, 32]:
        kw = dict(n=n, t=t, nsteps=N, m_kind=W.M_RAT, e=2, kappa=0.25, j0=-0.5, quad=RK4AUG)
        lax = _minimise(Oracle(formula=LAX, **kw), x, np.zeros(n))
        hop = _minimise(Oracle(formula=HOPF, **kw), x, np.zeros(n))
        diffs.append(abs(lax["phi"] - (-hop["phi"])))
    assert diffs[-1] < 1e-8, diffs
    assert diffs[0] / diffs[1] > 8, diffs


@pytest.mark.parametrize("formula,signs", [(LAX, False), (HOPF, True)])
def test_argopt_is_spatial_gradient(formula, signs):
    """The optimiser v equals grad_x u where u is smooth."""
    rng = np.random.default_rng(7)
    n = 3
    a = np.array([1.6, 1.1, 1.3]) if formula == HOPF else np.ones(n)
    d = np.array([-1.0, 1, 1]) if signs else np.ones(n)
    o = Oracle(n=n, t=0.5, nsteps=32, m_kind=W.M_TANH, kappa=0.5, s=3.0, d=d, a=a, j0=-0.5,
               formula=formula, quad=RK4AUG)
    x = rng.uniform(-1, 1, n)
    sgn = 1 if formula == LAX else -1
    r = _minimise(o, x, np.zeros(n))
    h = 1e-4
    for i in range(n):
        e_i = np.zeros(n)
        e_i[i] = h
        up = sgn * _minimise(o, x + e_i, r["v"])["phi"]
        um = sgn * _minimise(o, x - e_i, r["v"])["phi"]
        assert r["v"][i] == pytest.approx((up - um) / (2 * h), abs=1e-6)


def _brute_force_1d(f, lo, hi, step):
    grid = np.arange(lo, hi + step / 2, step)
    vals = np.array([f(g) for g in grid])
    k = int(np.argmin(vals))
    a, b = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    gr = (math.sqrt(5) - 1) / 2
    c, d = b - gr * (b - a), a + gr * (b - a)
    fc, fd = f(c), f(d)
    while b - a > 1e-10:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = f(d)
    return min(fc, fd)


def test_descent_finds_global_minimum_n1_hopf():
    """n = 1, non-convex H (d = -1, state-dependent speed): the descent's
    certified value equals a brute-force global minimum over [-4, 4]."""
    for xv in [-2.5, -0.7, 0.4, 1.9]:
        o = Oracle(n=1, t=0.6, nsteps=32, m_kind=W.M_TANH, kappa=0.5, s=1.0,
                   d=np.array([-1.0]), a=np.array([1.5]), j0=-0.5, formula=HOPF,
                   quad=RK4AUG)
        x = np.array([xv])
        ref = _brute_force_1d(lambda v: o.eval(x, np.array([v]))[0], -4, 4, 0.01)
        best = min(_minimise(o, x, np.array([v0]))["phi"] for v0 in [-1.0, 0.0, 1.0])
        assert best == pytest.approx(ref, rel=1e-9, abs=1e-9)


def test_descent_finds_global_minimum_n2_lax():
    """n = 2 Lax with the state-dependent speed of the n=2 workload: grid
    search with per-coordinate golden-section refinement."""
    wl = W.c0_lax_n2(B=1024)
    o = Oracle.from_workload(wl)
    for b in [0, 200, 517, 1000]:
        x = wl.x[b]
        g = np.arange(-4, 4.001, 0.05)
        vals = np.array([[o.eval(x, np.array([p, q]))[0] for q in g] for p in g])
        i, j = np.unravel_index(np.argmin(vals), vals.shape)
        v = np.array([g[i], g[j]])
        for _ in range(4):  # alternate golden-section line minimisations
            v[0] = _argmin_1d(lambda s: o.eval(x, np.array([s, v[1]]))[0], v[0] - .1, v[0] + .1)
            v[1] = _argmin_1d(lambda s: o.eval(x, np.array([v[0], s]))[0], v[1] - .1, v[1] + .1)
        ref = o.eval(x, v)[0]
        r = _minimise(o, x, np.zeros(2))
        assert r["phi"] == pytest.approx(ref, rel=1e-9, abs=1e-9)


def _argmin_1d(f, a, b):
    gr = (math.sqrt(5) - 1) / 2
    c, d = b - gr * (b - a), a + gr * (b - a)
    fc, fd = f(c), f(d)
    while b - a > 1e-11:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


def test_lax_n2_workload_symmetry():
    """The n=2 workload is invariant under x_i -> -x_i and under swapping the
    coordinates; its grid is mapped onto itself."""
    wl = W.c0_lax_n2()
    O = Oracle.opts_from_workload(wl, eps_step=1e-12, max_iter=400, cert_tol=1e-6)
    o = Oracle.from_workload(wl)
    idx = lambda i, j: 32 * i + j  # noqa: E731
    for (i, j) in [(3, 7), (10, 25), (0, 31)]:
        pts = [(i, j), (31 - i, j), (i, 31 - j), (j, i)]
        us = []
        for (p, q) in pts:
            b = idx(p, q)
            r = o.descend(wl.x[b], np.zeros(2), O)
            us.append(r["phi"])
        np.testing.assert_allclose(us, us[0], rtol=1e-9)


# --------------------------------------------------------------------------
# exact discrete gradient
# --------------------------------------------------------------------------

@pytest.mark.parametrize("formula,m_kind,e,drift,signs,quad,w", [
    (LAX, W.M_RAT, 2, False, False, TRAPZ, 0.0),
    (HOPF, W.M_TANH, 1, False, True, RK4AUG, 0.0),
    (LAX, W.M_RAT, 1, True, False, RK4AUG, 0.0),
    (HOPF, W.M_CONST, 1, True, False, TRAPZ, -0.7),
    (LAX, W.M_TANH, 2, False, False, RK4AUG, 0.4),
])
def test_gradient_tangent_reverse_fd(formula, m_kind, e, drift, signs, quad, w):
    rng = np.random.default_rng(8)
    n = 4
    o = _rand_problem(rng, n, formula, m_kind=m_kind, e=e, drift=drift, signs=signs, w=w,
                      quad=quad, nsteps=24)
    x, v = rng.standard_normal(n), rng.standard_normal(n)
    phi_t, gv_t, gx_t = o.grad_tangent(x, v)
    phi_r, gv_r, gx_r = o.grad_reverse(x, v)
    assert phi_t == pytest.approx(phi_r, rel=1e-13)
    np.testing.assert_allclose(gv_r, gv_t, rtol=1e-12, atol=1e-12 * np.abs(gv_t).max())
    np.testing.assert_allclose(gx_r, gx_t, rtol=1e-12, atol=1e-12 * np.abs(gx_t).max())
    h = 1e-6
    for i in range(n):
        e_i = np.zeros(n)
        e_i[i] = h
        fd_v = (o.eval(x, v + e_i)[0] - o.eval(x, v - e_i)[0]) / (2 * h)
        fd_x = (o.eval(x + e_i, v)[0] - o.eval(x - e_i, v)[0]) / (2 * h)
        assert gv_r[i] == pytest.approx(fd_v, rel=1e-7, abs=1e-8)
        assert gx_r[i] == pytest.approx(fd_x, rel=1e-7, abs=1e-8)


def test_gradient_vanishes_where_certificate_holds():
    """In the continuous limit grad_v F = (d gamma_0/dv)^T (grad g(gamma_0) -
    p_0): at a certified optimum the exact discrete gradient is zero up to
    the discretisation error."""
    wl = W.c1_hopf_n10(B=2)
    o = Oracle.from_workload(wl)
    r = _minimise(o, wl.x[0], wl.guesses[0, 0, 0])
    _, gv, _ = o.grad_reverse(wl.x[0], r["v"])
    assert np.abs(gv).max() < 1e-11
    assert r["rho"] < 1e-9


# --------------------------------------------------------------------------
# multi-start, certificate, restart and selection logic
# --------------------------------------------------------------------------

def test_solve_selection_and_fallbacks():
    wl = W.c1_hopf_n10(B=3)
    wl = wl.with_(guesses=wl.guesses[:, :2])
    o = Oracle.from_workload(wl)
    # a NaN guess diverges at once; the other slot certifies
    g = wl.guesses.copy()
    g[0, 0] = np.nan
    res = o.solve(wl.x, g, Oracle.opts_from_workload(wl))
    assert res["cert"][0] == 1
    assert res["slot_cert"][0, 0] == -1 and res["slot_cert"][0, 1] == 1
    assert res["slot_attempts"][0, 0] == 3
    # all guesses NaN: no finite slot
    g[1] = np.nan
    res = o.solve(wl.x, g, Oracle.opts_from_workload(wl))
    assert res["cert"][1] == -1 and np.isnan(res["u"][1])
    # tolerance 0: nothing certifies; the best finite slot is reported
    res = o.solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl, cert_tol=0.0))
    assert (res["cert"] == 0).all()
    assert (res["slot_attempts"] == 3).all()
    for b in range(3):
        k = int(np.argmin(res["slot_phi"][b]))
        assert res["u"][b] == -res["slot_phi"][b, k]
        np.testing.assert_array_equal(res["argopt"][b], res["slot_v"][b, k])


def test_slot_stops_at_its_first_certified_attempt():
    """Section 5's independent trials stop once a trial is certified: a slot
    whose first guess certifies runs one attempt, with the work of that one
    descent only."""
    wl = W.c1_hopf_n10(B=2)
    wl = wl.with_(guesses=wl.guesses[:, :1])
    O = Oracle.opts_from_workload(wl)
    o = Oracle.from_workload(wl)
    res = o.solve(wl.x, wl.guesses, O)
    for b in range(2):
        one = o.descend(wl.x[b], wl.guesses[b, 0, 0], O)
        assert res["slot_cert"][b, 0] == 1
        assert res["slot_attempts"][b, 0] == 1
        assert res["slot_fwd"][b, 0] == one["n_fwd"]
        assert res["slot_phi"][b, 0] == one["phi"]


def test_ill_posed_hopf_instance_is_not_certified():
    """With a_1^2 < c t the Hopf objective is unbounded below in v_1; every
    run must end diverged or uncertified, never certified."""
    wl = W.c1_hopf_n10(B=2)
    a = wl.a.copy()
    a[0] = 0.8
    wl = wl.with_(a=a, guesses=wl.guesses[:, :2])
    res = Oracle.from_workload(wl).solve(wl.x, wl.guesses, Oracle.opts_from_workload(wl,
                                                                                     v_max=1e3))
    assert (res["cert"] <= 0).all()
    assert (res["slot_status"][res["slot_cert"] >= 0] != 1).all() or (res["cert"] == 0).all()


def test_workload_prefix_property():
    a = W.c1_hopf_n10(B=64)
    b = W.c1_hopf_n10(B=16)
    np.testing.assert_array_equal(a.x[:16], b.x)
    np.testing.assert_array_equal(a.guesses[:16], b.guesses)
    np.testing.assert_array_equal(a.a, b.a)
    assert a.a[0] ** 2 >= 1.25 * 1.5 * a.t


@pytest.mark.parametrize("mode", [0, 1])
def test_first_step_follows_the_exact_gradient(mode):
    """On a quadratic objective (x-independent H) central differences are
    exact, so the first coordinate move of the sweep (mode 0) and the first
    gradient step (mode 1) equal -alpha times the closed-form gradient
    (a_i^2 + t d_i) v_i - x_i of the Hopf objective."""
    n, t, alpha = 3, 0.5, 0.05
    a = np.array([1.5, 1.2, 1.8])
    d = np.array([-1.0, 1.0, 1.0])
    o = Oracle(n=n, t=t, nsteps=4, d=d, a=a, j0=-0.5, formula=HOPF, quad=RK4AUG)
    x = np.array([0.3, -0.8, 1.1])
    v0 = np.array([0.4, 0.2, -0.5])
    O = Oracle.opts(mode=mode, max_iter=1, alpha0=alpha, eps_step=0.0, R_max=0)
    r = o.descend(x, v0, O)
    if mode == 1:
        g = (a ** 2 + t * d) * v0 - x
        np.testing.assert_allclose(r["v"], v0 - alpha * g, rtol=1e-10, atol=1e-12)
    else:
        v = v0.copy()
        for j in range(n):  # Gauss-Seidel: each coordinate sees the updated ones
            gj = (a[j] ** 2 + t * d[j]) * v[j] - x[j]
            v[j] -= alpha * gj
        np.testing.assert_allclose(r["v"], v, rtol=1e-9, atol=1e-11)
    assert r["n_fwd"] == (1 + 3 * n if mode == 0 else 2)
    assert r["n_bwd"] == (0 if mode == 0 else 2)


@pytest.mark.parametrize("mode", [0, 1])
def test_sufficient_decrease_rejects_overshoot(mode):
    """n = 1 quadratic Hopf objective 1/2 lam v^2 - x v (lam = a^2 + t d): a
    step with alpha lam = 1.9 lowers the objective by only 5% of alpha g^2, so
    the plain ascent test accepts it while the sufficient-decrease test with
    armijo_c = 0.1 rejects it and halves the step."""
    a, t = 1.5, 0.4
    lam = a * a + t
    o = Oracle(n=1, t=t, nsteps=4, a=np.array([a]), j0=0.0, formula=HOPF, quad=RK4AUG)
    x, v0 = np.array([0.7]), np.array([1.3])
    g = lam * v0 - x
    alpha = 1.9 / lam
    for c, moved in [(0.0, True), (0.1, False)]:
        r = o.descend(x, v0, Oracle.opts(mode=mode, max_iter=1, alpha0=alpha, eps_step=0.0,
                                         R_max=0, armijo_c=c))
        if moved:
            np.testing.assert_allclose(r["v"], v0 - alpha * g, rtol=1e-9)
        else:
            np.testing.assert_array_equal(r["v"], v0)


def test_uncertified_slot_reports_its_best_attempt():
    """With nothing certified, a slot reports the attempt with the lowest
    objective among its restarts."""
    wl = W.c1_hopf_n10(B=2)
    wl = wl.with_(guesses=wl.guesses[:, :1] * 3.0)
    O = Oracle.opts_from_workload(wl, cert_tol=0.0, max_iter=1)
    o = Oracle.from_workload(wl)
    res = o.solve(wl.x, wl.guesses, O)
    for b in range(2):
        phis = [o.descend(wl.x[b], wl.guesses[b, 0, r], O)["phi"] for r in range(3)]
        assert len(set(phis)) == 3
        assert res["slot_phi"][b, 0] == min(phis)
        assert res["u"][b] == -min(phis)


def test_equal_objectives_select_the_lowest_slot():
    """At x = 0 the n=2 workload is symmetric under v -> -v (negation is exact
    in floating point), so the guesses g and -g give bit-identical objectives
    with opposite optimisers; the lowest slot must win the tie."""
    wl = W.c0_lax_n2(B=1)
    x = np.zeros((1, 2))
    g0 = np.array([0.7, -0.3])
    guesses = np.stack([g0, -g0])[None, :, None, :].repeat(3, axis=2)
    o = Oracle.from_workload(wl)
    O = Oracle.opts_from_workload(wl, max_iter=2, cert_tol=0.0)
    res = o.solve(x, guesses, O)
    assert res["slot_phi"][0, 0] == res["slot_phi"][0, 1]
    np.testing.assert_array_equal(res["slot_v"][0, 0], -res["slot_v"][0, 1])
    np.testing.assert_array_equal(res["argopt"][0], res["slot_v"][0, 0])
    # and the same with the slots swapped
    res2 = o.solve(x, guesses[:, ::-1].copy(), O)
    np.testing.assert_array_equal(res2["argopt"][0], res["slot_v"][0, 1])
