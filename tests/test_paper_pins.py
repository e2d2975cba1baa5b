"""Pins of the reference of the paper's own scheme (forward Euler, rectangle
rule, forward differences, Algorithm 1), the degree-1 homogeneous
Hamiltonians and the grid-minimum functional F2, the Rosenbrock initial data,
heavy-ball descent and the Lax-Friedrichs grid solver (oracle/hj_paper.c).
Each pin is fixed by the mathematics, not by the reference itself: closed
forms where the Euler scheme is exact, convergence orders, homogeneity,
finite differences of H and g, and brute force."""
import math

import numpy as np
import pytest

from oracle.paper_oracle import PaperOracle, build
from paper_1704_02524_amd import workloads as W

build()


def _wl(n=2, **kw):
    base = dict(name="pin", n=n, t=0.5, nsteps=25, m_kind=W.M_CONST, e=1, kappa=0.0, s=1.0,
                w=0.0, d=np.ones(n), A=None, a=np.ones(n), j0=-0.5, formula=W.LAX,
                quad=W.TRAPZ, x=np.zeros((1, n)), guesses=np.zeros((1, 1, 1, n)),
                mode=W.ALG1, max_iter=20000, alpha0=0.5, fd_sigma=1e-7, eps_step=1e-10,
                cert_tol=1e-3, ode=W.EULER, M=500)
    base.update(kw)
    return W.Workload(**base)


def test_euler_free_particle_lax_is_exact_and_algorithm1_finds_it():
    """H = 1/2|p|^2 moves on straight lines with constant p, so the Euler
    characteristics and the rectangle rule are exact: F(v) = 1/2|x - t v|^2
    + t/2 |v|^2 + j0, minimised at v = x/(1+t) with u = |x|^2/(2(1+t)) + j0."""
    wl = _wl(t=0.6, nsteps=7)
    o = PaperOracle(wl)
    x = np.array([0.7, -1.3])
    for v in (np.array([0.1, 0.2]), np.array([-1.0, 0.5])):
        phi, _, _ = o.eval(x, v)
        exact = 0.5 * np.sum((x - wl.t * v) ** 2) + 0.5 * wl.t * v @ v - 0.5
        assert phi == pytest.approx(exact, abs=1e-14)
    r = o.descend(x, np.array([1.5, 1.5]))
    assert r["status"] == 1  # converged: d consecutive moves below epsilon
    np.testing.assert_allclose(r["v"], x / (1 + wl.t), atol=1e-6)
    assert r["phi"] == pytest.approx(x @ x / (2 * (1 + wl.t)) - 0.5, abs=1e-11)
    assert r["rho"] < 1e-6


def test_algorithm1_first_update_by_hand():
    """The first update of Algorithm 1 moves coordinate 1 only, by alpha
    times the forward difference (F(v + sigma e_1) - F(v)) / sigma."""
    wl = _wl(t=0.6, nsteps=7, fd_sigma=1e-3, max_iter=1, alpha0=0.25)
    o = PaperOracle(wl)
    x, v0 = np.array([0.7, -1.3]), np.array([0.3, -0.2])
    F = lambda v: 0.5 * np.sum((x - 0.6 * v) ** 2) + 0.3 * v @ v - 0.5
    e1 = np.array([1.0, 0.0])
    g1 = (F(v0 + 1e-3 * e1) - F(v0)) / 1e-3
    # one sweep = two coordinate updates
    r = o.descend(x, v0)
    g2 = (F(v0 - 0.25 * g1 * e1 + 1e-3 * np.array([0.0, 1.0])) - F(v0 - 0.25 * g1 * e1)) / 1e-3
    expect = v0 - 0.25 * np.array([g1, g2])
    np.testing.assert_allclose(r["v"], expect, atol=1e-12)
    assert r["iters"] == 2 and r["n_eval"] == 5


def test_alpha_halves_every_M_updates():
    """Algorithm 1's step-size rule: alpha halves after every M coordinate updates
    and never otherwise (no acceptance test).  The run is followed update by
    update in Python on the reference's own objective, with M = 2 over five
    updates (alpha, alpha, alpha/2, alpha/2, alpha/4)."""
    wl = _wl(t=0.6, nsteps=7, fd_sigma=1e-3, M=2, max_iter=3, alpha0=0.7,
             eps_step=1e-30)
    o = PaperOracle(wl)
    x, v = np.array([0.7, -1.3]), np.array([0.3, -0.2])
    F = lambda u: o.eval(x, u)[0]
    alpha, phi = 0.7, F(v)
    for k in range(6):
        j = k % 2
        e = np.zeros(2)
        e[j] = 1e-3
        g = (F(v + e) - phi) / 1e-3
        v = v.copy()
        v[j] -= alpha * g
        phi = F(v)
        if (k + 1) % 2 == 0:
            alpha /= 2
    r = o.descend(x, np.array([0.3, -0.2]))
    assert r["iters"] == 6
    np.testing.assert_allclose(r["v"], v, rtol=0, atol=1e-14)


def _osc_exact(x, a, t, sign):
    """u of H = sign 1/2(|p|^2 + |x|^2) with g = 1/2 sum x^2/a^2 - 1/2:
    1/2 sum tan(theta_i - sign t) x_i^2 - 1/2, theta_i = arctan(1/a_i^2)
    (Riccati equation alpha' = -sign (alpha^2 + 1))."""
    th = np.arctan(1.0 / a ** 2)
    return 0.5 * np.sum(np.tan(th - sign * t) * x ** 2) - 0.5


@pytest.mark.parametrize("sign", [1, -1])
def test_euler_hopf_oscillator_converges_at_first_order(sign):
    """The paper's Example 2 oscillator with the Hopf functional: the Euler
    discretisation's value (minimised with a tight tolerance) converges to
    the closed form at first order in the step."""
    a = np.array([1.0, 2.5])
    x = np.array([0.8, -1.1])
    errs = []
    for N in (20, 40, 80):
        wl = _wl(t=0.5, nsteps=N, d=np.full(2, float(sign)), w=float(sign), a=a,
                 formula=W.HOPF, alpha0=1 / 3, fd_sigma=1e-8, eps_step=1e-12)
        r = PaperOracle(wl).descend(x, np.array([0.2, -0.2]))
        errs.append(abs(-r["phi"] - _osc_exact(x, a, 0.5, sign)))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs


def test_staggered_free_particle_lax_is_exact():
    """The staggered Lax form of the section 3 lemma is exact for H = 1/2|p|^2
    (p constant, x_n - x_{n-1} = delta p): F(v) = 1/2|x - t v|^2 + t/2|v|^2
    - 1/2, and Algorithm 1 finds v = x/(1+t), u = |x|^2/(2(1+t)) - 1/2."""
    wl = _wl(t=0.6, nsteps=7, ode=W.STAGGERED)
    o = PaperOracle(wl)
    x = np.array([0.7, -1.3])
    for v in (np.array([0.1, 0.2]), np.array([-1.0, 0.5])):
        phi, _, _ = o.eval(x, v)
        assert phi == pytest.approx(0.5 * np.sum((x - 0.6 * v) ** 2) + 0.3 * v @ v - 0.5,
                                    abs=1e-14)
    r = o.descend(x, np.array([1.5, 1.5]))
    assert r["status"] == 1
    np.testing.assert_allclose(r["v"], x / 1.6, atol=1e-6)
    assert r["rho"] < 1e-6


def test_staggered_hopf_x_independent_solve_is_exact():
    """The staggered Hopf form with H = 1/2 sum d p^2 keeps p_n = v and
    moves x_0 = x - t D v, so G = <x,v> - g*(v) - t/2 sum d v^2 exactly and
    u = 1/2 sum x^2/(a^2 + t d) + j0 (section 3.4's first example)."""
    a, d = np.array([1.5, 2.0]), np.array([-1.0, 1.0])
    wl = _wl(t=0.5, nsteps=9, d=d, a=a, j0=-0.3, formula=W.HOPF, alpha0=1 / 3,
             fd_sigma=1e-8, eps_step=1e-12, cert_tol=1e-5, ode=W.STAGGERED)
    x = np.array([[0.8, -1.1], [-0.4, 0.3]])
    r = PaperOracle(wl).solve(x, np.zeros((2, 1, 1, 2)))
    assert (r["cert"] == 1).all()
    np.testing.assert_allclose(r["u"], 0.5 * (x ** 2 / (a ** 2 + 0.5 * d)).sum(1) - 0.3,
                               atol=1e-6)


@pytest.mark.parametrize("sign,formula", [(1, W.HOPF), (-1, W.HOPF), (1, W.LAX)])
def test_staggered_oscillator_converges_at_first_order(sign, formula):
    """Example 2's oscillator with the staggered forms (x-dependent H_x, so
    p and x alternate): the discrete value converges to the closed form at
    first order in the step, for Hopf (both signs) and Lax (convex H)."""
    a = np.array([1.0, 2.5])
    x = np.array([0.8, -1.1])
    errs = []
    for N in (20, 40, 80):
        wl = _wl(t=0.5, nsteps=N, d=np.full(2, float(sign)), w=float(sign), a=a,
                 formula=formula, alpha0=1 / 3, fd_sigma=1e-8, eps_step=1e-12,
                 ode=W.STAGGERED)
        r = PaperOracle(wl).descend(x, np.array([0.2, -0.2]))
        u = -r["phi"] if formula == W.HOPF else r["phi"]
        errs.append(abs(u - _osc_exact(x, a, 0.5, sign)))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3, errs


@pytest.mark.parametrize("formula", [W.LAX, W.HOPF])
def test_staggered_state_dependent_converges_to_the_rk4_value(formula):
    """With a state-dependent speed (H_p depends on x, so each staggered step
    solves an implicit equation) the staggered functional at fixed v
    converges at first order to the continuous one, computed independently
    by the RK4 reference at a fine step."""
    from oracle.oracle import Oracle
    n, t = 3, 0.6
    d = np.array([-1.0, 1.0, 1.0]) if formula == W.HOPF else np.ones(n)
    a = np.array([1.8, 1.2, 0.9])
    kw = dict(m_kind=W.M_TANH, e=1, kappa=0.5, s=float(n), w=0.0, d=d, a=a, j0=-0.5,
              formula=formula)
    x = np.array([0.6, -0.4, 0.9])
    v = np.array([0.3, 0.5, -0.2])
    ref = Oracle(n=n, t=t, nsteps=800, m_kind=W.M_TANH, e=1, kappa=0.5, s=float(n), w=0.0,
                 d=d, a=a, j0=-0.5, formula=formula, quad=W.RK4AUG)
    exact = ref.eval(x, v)[0]
    errs = []
    for N in (40, 80, 160):
        o = PaperOracle(_wl(n=n, t=t, nsteps=N, ode=W.STAGGERED, **kw))
        errs.append(abs(o.eval(x, v)[0] - exact))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3, errs


@pytest.mark.parametrize("formula", [W.LAX, W.HOPF])
def test_staggered_dynamics_are_the_stationarity_conditions(formula):
    """Section 3's lemmas obtain the staggered recursions as the
    stationarity conditions of the discrete functional in the interior
    points, so at a critical point of the value as a function of v the
    remaining end condition holds exactly: grad g(x_0) equals the co-state
    carried past n = 0 (Lax), grad g*(p_1) equals x_0 (Hopf).  A descent to
    that critical point, with a state-dependent H (implicit steps), must
    therefore certify to the descent's accuracy, not to O(delta)."""
    n = 3
    d = np.array([-1.0, 1.0, 1.0]) if formula == W.HOPF else np.ones(n)
    wl = _wl(n=n, t=0.6, nsteps=10, m_kind=W.M_TANH, e=1, kappa=0.5, s=float(n), d=d,
             a=np.array([1.8, 1.2, 0.9]), formula=formula, ode=W.STAGGERED, alpha0=1 / 3,
             fd_sigma=1e-8, eps_step=1e-12, M=2000)
    o = PaperOracle(wl)
    x = np.array([0.6, -0.4, 0.9])
    r = o.descend(x, np.zeros(n))
    assert r["status"] == 1
    h = 1e-6
    grad = [(o.eval(x, r["v"] + h * e)[0] - o.eval(x, r["v"] - h * e)[0]) / (2 * h)
            for e in np.eye(n)]
    assert np.max(np.abs(grad)) < 1e-6
    assert r["rho"] < 1e-6


def test_rk4_option_converges_at_fourth_order():
    a = np.array([1.0, 2.5])
    x = np.array([0.8, -1.1])
    errs = []
    for N in (5, 10, 20):
        wl = _wl(t=0.5, nsteps=N, d=np.full(2, -1.0), w=-1.0, a=a, formula=W.HOPF,
                 ode=W.RK4, alpha0=1 / 3, fd_sigma=1e-8, eps_step=1e-12)
        o = PaperOracle(wl)
        # the exact optimum of the continuous problem: v = grad u(x)
        th = np.arctan(1.0 / a ** 2)
        v = np.tan(th + 0.5) * x
        phi, _, _ = o.eval(x, v)
        errs.append(abs(-phi - _osc_exact(x, a, 0.5, -1)))
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs


@pytest.mark.parametrize("m_kind,e", [(W.M_CONST, 1), (W.M_RAT, 1), (W.M_RAT, 2),
                                       (W.M_TANH, 1), (W.M_TANH, 2)])
def test_quadratic_hamiltonian_derivatives(m_kind, e):
    """H_x and H_p of the state-dependent quadratic family against central
    differences of H itself (every speed profile, c and c^2)."""
    rng = np.random.default_rng(5)
    n = 3
    wl = _wl(n=n, m_kind=m_kind, e=e, kappa=0.7, s=1.3, w=-0.4, d=np.array([-1.0, 0.5, 2.0]))
    o = PaperOracle(wl)
    h = 1e-6
    for _ in range(4):
        x, p = rng.normal(size=n), rng.normal(size=n)
        Hx, Hp = o.grads(x, p)
        for i in range(n):
            ei = np.zeros(n)
            ei[i] = h
            fx = (o.hamiltonian(x + ei, p) - o.hamiltonian(x - ei, p)) / (2 * h)
            fp = (o.hamiltonian(x, p + ei) - o.hamiltonian(x, p - ei)) / (2 * h)
            assert Hx[i] == pytest.approx(fx, rel=1e-7, abs=1e-8)
            assert Hp[i] == pytest.approx(fp, rel=1e-7, abs=1e-8)


def test_hopf_solve_reports_minus_the_minimum():
    """u = -min G for the Hopf functional: with an x-independent H the Euler
    characteristics are exact straight lines, so the discrete problem has
    the closed form of section 3.4's first example, u = 1/2 sum x_i^2 /
    (a_i^2 + t d_i) + j0, and hjp_solve must return it with its sign."""
    a = np.array([1.5, 2.0])
    d = np.array([-1.0, 1.0])
    wl = _wl(t=0.5, nsteps=9, d=d, a=a, j0=-0.3, formula=W.HOPF, alpha0=1 / 3,
             fd_sigma=1e-8, eps_step=1e-12, cert_tol=1e-5)
    x = np.array([[0.8, -1.1], [-0.4, 0.3]])
    r = PaperOracle(wl).solve(x, np.zeros((2, 1, 1, 2)))
    exact = 0.5 * (x ** 2 / (a ** 2 + 0.5 * d)).sum(axis=1) - 0.3
    assert (r["cert"] == 1).all()
    np.testing.assert_allclose(r["u"], exact, atol=1e-6)


def _norm_wl(n=2, **kw):
    mu = np.zeros(n)
    mu[:2] = 1.0
    base = dict(h_kind=W.H_NORM, k_split=n, s1=1.0, s2=0.0, c0=1.0, beta=3.0, gam=4.0, mu=mu)
    base.update(kw)
    return _wl(n=n, **base)


def test_norm_hamiltonian_derivatives_and_homogeneity():
    rng = np.random.default_rng(3)
    for wl in (_norm_wl(n=3), _norm_wl(n=4, k_split=1, s2=-1.0, c0=2.0)):
        o = PaperOracle(wl)
        for _ in range(5):
            x, p = rng.normal(size=wl.n), rng.normal(size=wl.n)
            Hx, Hp = o.grads(x, p)
            h = 1e-6
            for i in range(wl.n):
                e = np.zeros(wl.n)
                e[i] = h
                assert Hx[i] == pytest.approx((o.hamiltonian(x + e, p) - o.hamiltonian(x - e, p))
                                              / (2 * h), rel=1e-6, abs=1e-8)
                assert Hp[i] == pytest.approx((o.hamiltonian(x, p + e) - o.hamiltonian(x, p - e))
                                              / (2 * h), rel=1e-6, abs=1e-8)
            # degree 1 in p: H(x, 3p) = 3 H(x, p), <p, H_p> = H
            assert o.hamiltonian(x, 3 * p) == pytest.approx(3 * o.hamiltonian(x, p), rel=1e-13)
            assert p @ Hp == pytest.approx(o.hamiltonian(x, p), rel=1e-12)
            # the zero subgradient at p_A = 0
            q = p.copy()
            q[:wl.k_split] = 0.0
            _, Hq = o.grads(x, q)
            assert np.all(Hq[:wl.k_split] == 0.0)


@pytest.mark.parametrize("ode", [W.EULER, W.STAGGERED])
def test_huygens_functional_closed_form_ball_minimum(ode):
    """H = c|p| with constant c: the value is the minimum of g over the ball
    of radius c t (Huygens).  For g = 1/2|x|^2 - 1/2 and |x| > c t it is
    1/2(|x| - c t)^2 - 1/2, reached by v along x at the last grid point, so
    F2's grid minimum is exact; F1 (the sphere only) agrees there, and inside
    the ball (|x| < c t) F2 finds the interior minimum -1/2 where F1 cannot."""
    c, t = 1.5, 0.4
    wl = _norm_wl(beta=0.0, c0=c, t=t, nsteps=20, formula=W.LAX_MIN, ode=ode)
    o = PaperOracle(wl)
    x = np.array([1.2, -0.9])
    v = x / np.linalg.norm(x)
    phi, rho, _ = o.eval(x, v)
    assert phi == pytest.approx(0.5 * (np.linalg.norm(x) - c * t) ** 2 - 0.5, abs=1e-13)
    assert rho < 1e-12
    # other directions give more
    for ang in (0.3, 1.0, 2.5):
        rot = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
        assert o.eval(x, rot @ v)[0] > phi
    # inside the ball: F2 reaches the minimum of g, F1 stays on the sphere
    xi = np.array([0.3, 0.0])  # |x| = 0.3 < c t = 0.6, on a grid point at s = 0.2
    phi2, _, _ = o.eval(xi, np.array([1.0, 0.0]))
    assert phi2 == pytest.approx(-0.5, abs=1e-13)
    o1 = PaperOracle(wl.with_(formula=W.LAX))
    phi1, _, _ = o1.eval(xi, np.array([1.0, 0.0]))
    assert phi1 == pytest.approx(0.5 * (c * t - 0.3) ** 2 - 0.5, abs=1e-13)


@pytest.mark.parametrize("ode", [W.EULER, W.STAGGERED])
def test_hopf_nonconvex_norm_closed_form(ode):
    """H = c1|p_1| - c2|p_2| with constant c1, c2 and ellipsoid g: the Euler
    and the staggered schemes are exact (p constant, integrand equal to H)
    and the Hopf value is separable: 1/2 max(|x1| - t c1, 0)^2/a1^2 + 1/2
    (|x2| + t c2)^2/a2^2 - 1/2."""
    t = 0.3  # c1 = c2 = c0 = 1 (beta = 0)
    a = np.array([1.0, 2.5])
    wl = _norm_wl(k_split=1, s1=1.0, s2=-1.0, c0=1.0, beta=0.0, t=t, nsteps=15, a=a,
                  formula=W.HOPF, fd_sigma=1e-9, eps_step=1e-12, alpha0=0.2, ode=ode)
    o = PaperOracle(wl)
    x = np.array([1.4, -0.7])
    exact = 0.5 * max(abs(x[0]) - t, 0) ** 2 / a[0] ** 2 + \
        0.5 * (abs(x[1]) + t) ** 2 / a[1] ** 2 - 0.5
    v_opt = np.array([np.sign(x[0]) * (abs(x[0]) - t) / a[0] ** 2,
                      np.sign(x[1]) * (abs(x[1]) + t) / a[1] ** 2])
    phi, rho, _ = o.eval(x, v_opt)
    assert -phi == pytest.approx(exact, abs=1e-13)
    assert rho < 1e-12
    r = o.descend(x, np.array([0.5, -0.5]))
    assert -r["phi"] == pytest.approx(exact, abs=1e-7)
    np.testing.assert_allclose(r["v"], v_opt, atol=1e-4)


def test_rosenbrock_gradient_and_minimum():
    wl = _wl(j_kind=W.J_ROSENBROCK, rscale=0.4e-3)
    o = PaperOracle(wl)
    assert o.g(np.array([1.0, 0.0])) == pytest.approx(-0.04, abs=1e-16)
    np.testing.assert_allclose(o.grad_g(np.array([1.0, 0.0])), 0.0, atol=1e-16)
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.normal(size=2)
        h = 1e-6
        fd = [(o.g(x + h * e) - o.g(x - h * e)) / (2 * h) for e in np.eye(2)]
        np.testing.assert_allclose(o.grad_g(x), fd, rtol=1e-7, atol=1e-10)


def test_rosenbrock_lax_matches_brute_force():
    """Section 5 Example 2 with Rosenbrock data and H+ (n = 2): the best
    result of Algorithm 1 over several guesses equals the minimum of the same
    discrete functional found by a grid search refined by golden sections."""
    wl = W.paper_ex2_rosenbrock(grid=4, G=5).with_(fd_sigma=1e-7, eps_step=1e-11)
    o = PaperOracle(wl)
    x = np.array([0.4, -0.6])
    best = min(o.descend(x, g)["phi"] for g in wl.guesses[3, :, 0])
    F = lambda v: o.eval(x, v)[0]
    gs = np.linspace(-4, 4, 161)
    vals = np.array([[F(np.array([a, b])) for b in gs] for a in gs])
    i, j = np.unravel_index(np.argmin(vals), vals.shape)
    v = np.array([gs[i], gs[j]])
    for _ in range(6):  # coordinate golden-section refinement
        for k in range(2):
            lo, hi = v[k] - 0.06, v[k] + 0.06
            for _ in range(60):
                m1, m2 = lo + 0.382 * (hi - lo), lo + 0.618 * (hi - lo)
                v1, v2 = v.copy(), v.copy()
                v1[k], v2[k] = m1, m2
                if F(v1) < F(v2):
                    hi = m2
                else:
                    lo = m1
            v[k] = 0.5 * (lo + hi)
    assert best == pytest.approx(F(v), abs=1e-8)


def test_momentum_descent_reaches_the_closed_form():
    wl = _wl(t=0.6, nsteps=7, mode=W.MOMENTUM, alpha0=0.5, momentum=0.9,
             acc_rel=1e-15, eps_step=1e-11, max_iter=5000)
    o = PaperOracle(wl)
    x = np.array([0.7, -1.3])
    r = o.descend(x, np.array([1.5, 1.5]))
    assert r["status"] == 1
    np.testing.assert_allclose(r["v"], x / 1.6, atol=1e-6)
    # one iteration costs n + 1 evaluations
    assert (r["n_eval"] - 1) % 3 == 0


def test_momentum_iterates_follow_the_heavy_ball_recurrence():
    """For the free particle the Euler objective is exactly quadratic in v,
    F(v) = 1/2|x - t v|^2 + 1/2 t |v|^2 - 1/2 with Hessian lambda = t^2 + t,
    so heavy-ball iterates obey v_{k+1} - v* = (1 + beta - alpha lambda)
    (v_k - v*) - beta (v_{k-1} - v*), v* = x / (1 + t) (the forward
    difference adds lambda sigma / 2 to every gradient component)."""
    t, alpha, beta, sig = 0.6, 0.3, 0.5, 1e-7
    lam = t * t + t
    x = np.array([0.7, -1.3])
    v0 = np.array([1.5, 1.5])
    vs = x / (1 + t)
    ref = [v0, v0]
    for _ in range(3):
        vk, vkm = ref[-1], ref[-2]
        g = lam * (vk - vs) + 0.5 * lam * sig
        ref.append(vk - alpha * g + beta * (vk - vkm))
    for k in (1, 2, 3):
        wl = _wl(t=t, nsteps=7, mode=W.MOMENTUM, alpha0=alpha, momentum=beta,
                 acc_rel=1e-15, eps_step=1e-14, max_iter=k, fd_sigma=sig)
        r = PaperOracle(wl).descend(x, v0)
        np.testing.assert_allclose(r["v"], ref[k + 1], atol=1e-7)


def test_lax_friedrichs_converges_to_the_free_particle():
    """phi_t + 1/2|grad phi|^2 = 0, phi(., 0) = 1/2|x|^2 - 1/2 has the
    solution |x|^2/(2(1+t)) - 1/2; the first-order Lax-Friedrichs scheme
    converges to it at first order in the mesh (interior points)."""
    wl = _wl()
    o = PaperOracle(wl)
    errs, edge = [], []
    for dx in (0.04, 0.02):
        nx = int(round(4.0 / dx)) + 1
        dt = dx / 5.0
        nt = int(round(0.5 / dt))
        phi = o.lax_friedrichs(-2.0, -2.0, dx, dx, nx, nx, dt, nt, 2.5, 2.5)
        g1 = np.linspace(-2, 2, nx)
        X, Y = np.meshgrid(g1, g1, indexing="xy")
        exact = (X ** 2 + Y ** 2) / (2 * 1.5) - 0.5
        inner = (np.abs(X) <= 1.0) & (np.abs(Y) <= 1.0)
        err = np.abs(phi - exact)
        errs.append(err[inner].max())
        # the characteristics leave the square, so the boundary rule (linear
        # extrapolation of the neighbour across the edge) keeps first order
        # up to and on the edge
        edge.append(np.r_[err[0], err[-1], err[:, 0], err[:, -1]].max())
        # H and g are even in each coordinate and symmetric under x <-> y, and
        # the stencil and the boundary rule respect that on this grid
        scale = np.abs(phi).max()
        np.testing.assert_allclose(phi, phi[:, ::-1], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(phi, phi[::-1, :], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(phi, phi.T, rtol=0, atol=1e-12 * scale)
    assert errs[1] < errs[0] and 1.6 < errs[0] / errs[1] < 2.4, errs
    assert 1.6 < edge[0] / edge[1] < 2.4 and edge[1] < 1.5 * errs[1], (edge, errs)


def test_formula_solutions_match_the_viscosity_solution():
    """The independent check of section 5: on the n = 2 Lax problem of the
    benchmark (H = 1/2 c(x)^2 |p|^2, c = 1 + 0.25|x|^2/(1+|x|^2), g =
    1/2|x|^2 - 1/2, t = 0.5), the RK4 reference's certified values at
    scattered points and the Lax-Friedrichs grid solution differ by O(dx):
    the difference halves with the mesh."""
    from oracle.oracle import Oracle
    wl = W.c0_lax_n2()
    pts = np.array([[0.5, 0.5], [1.0, -0.5], [-1.5, 0.25], [0.0, 0.0], [1.25, 1.25]])
    sub = wl.with_(x=pts, guesses=wl.guesses[:len(pts)])
    ref = Oracle.from_workload(sub).solve(sub.x, sub.guesses, Oracle.opts_from_workload(sub))
    assert (ref["cert"] == 1).all()
    po = PaperOracle(wl.with_(mode=W.ALG1))
    diffs = []
    for dx in (0.04, 0.02):
        nx = int(round(6 / dx)) + 1
        phi = po.lax_friedrichs(-3.0, -3.0, dx, dx, nx, nx, dx / 12, int(round(6.0 / dx)),
                                5.0, 5.0)
        idx = np.round((pts + 3) / dx).astype(int)
        diffs.append(np.abs(phi[idx[:, 1], idx[:, 0]] - ref["u"]).max())
    assert diffs[0] < 0.1 and 1.7 < diffs[0] / diffs[1] < 2.4, diffs
