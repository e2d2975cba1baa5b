/*
 * hj_paper.c -- plain, slow, single-threaded FP64 reference of the paper's
 * own scheme and of its further problem families (notation in hj_paper.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product path.  Each
 * function follows its definition in the paper with no blocking, fusion or
 * reordering.
 *
 * Readings of the paper that this file commits to:
 *  - the paper's ODE solver is forward Euler (section 4.2) applied to the
 *    bi-characteristics in reversed time tau = t - s from (x, v), with N
 *    uniform steps of h = t / N; its rectangle rule (eq. num_int, whose
 *    index range the paper leaves open) takes the integrand at the state
 *    each Euler step starts from: h sum_{k=0}^{N-1} iota(y_k);
 *  - Algorithm 1 is read literally: one coordinate update per k, no
 *    acceptance test, alpha halved every M updates, stop once d consecutive
 *    updates moved less than epsilon, with a cap of max_iter
 *    sweeps as a safety net the paper does not need;
 *  - for degree-1 homogeneous H the scale of p is free (H_p does not depend
 *    on it), so the certificate p(0) in dg(gamma(0)) of section 4.3 is
 *    checked on directions: |p/|p| - grad g/|grad g||_inf; for F2 it is
 *    checked at the minimising grid state;
 *  - at p_A = 0 (p_B = 0) the norm family's H_p takes the zero subgradient.
 */
#include "hj_paper.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* The Hamiltonians.                                                    */
/* ------------------------------------------------------------------ */

static double sq_norm(int n, const double *v)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        s += v[i] * v[i];
    return s;
}

/* quadratic family: m(r) = c(r)^e and dm/dr */
static void quad_m(const hjp_problem *P, double r, double *m, double *m1)
{
    double c, c1;
    if (P->m_kind == 1) {
        c = 1.0 + P->kappa * r / (1.0 + r);
        c1 = P->kappa / ((1.0 + r) * (1.0 + r));
    } else if (P->m_kind == 2) {
        double th = tanh(r / P->s);
        c = 1.0 + P->kappa * th;
        c1 = P->kappa / P->s * (1.0 - th * th);
    } else {
        c = 1.0;
        c1 = 0.0;
    }
    if (P->e == 2) {
        *m = c * c;
        *m1 = 2.0 * c * c1;
    } else {
        *m = c;
        *m1 = c1;
    }
}

/* norm family: c_i(x) = c0 (1 + beta exp(-gam |x - mu_i|^2)), mu_1 = mu,
 * mu_2 = -mu, and its gradient */
static double bump(const hjp_problem *P, const double *x, double sgn, double *grad)
{
    double r = 0.0;
    for (int i = 0; i < P->n; ++i) {
        double dx = x[i] - sgn * P->mu[i];
        r += dx * dx;
    }
    double E = exp(-P->gam * r);
    if (grad)
        for (int i = 0; i < P->n; ++i)
            grad[i] = P->c0 * P->beta * E * (-2.0 * P->gam) * (x[i] - sgn * P->mu[i]);
    return P->c0 * (1.0 + P->beta * E);
}

static double block_norm(const double *p, int lo, int hi)
{
    double s = 0.0;
    for (int i = lo; i < hi; ++i)
        s += p[i] * p[i];
    return sqrt(s);
}

double hjp_hamiltonian(const hjp_problem *P, const double *x, const double *p)
{
    const int n = P->n;
    if (P->hkind == HJP_H_NORM) {
        double c1 = bump(P, x, 1.0, NULL), c2 = bump(P, x, -1.0, NULL);
        return P->s1 * c1 * block_norm(p, 0, P->k) + P->s2 * c2 * block_norm(p, P->k, n);
    }
    double m, m1, q = 0.0;
    quad_m(P, sq_norm(n, x), &m, &m1);
    for (int i = 0; i < n; ++i)
        q += P->d[i] * p[i] * p[i];
    return 0.5 * m * q + 0.5 * P->w * sq_norm(n, x);
}

void hjp_grads(const hjp_problem *P, const double *x, const double *p, double *Hx, double *Hp)
{
    const int n = P->n;
    if (P->hkind == HJP_H_NORM) {
        double *g1 = (double *)malloc(sizeof(double) * 2 * n), *g2 = g1 + n;
        double c1 = bump(P, x, 1.0, g1), c2 = bump(P, x, -1.0, g2);
        double nA = block_norm(p, 0, P->k), nB = block_norm(p, P->k, n);
        for (int i = 0; i < n; ++i) {
            Hx[i] = P->s1 * nA * g1[i] + P->s2 * nB * g2[i];
            if (i < P->k)
                Hp[i] = nA > 0.0 ? P->s1 * c1 * p[i] / nA : 0.0;
            else
                Hp[i] = nB > 0.0 ? P->s2 * c2 * p[i] / nB : 0.0;
        }
        free(g1);
        return;
    }
    double m, m1, q = 0.0;
    quad_m(P, sq_norm(n, x), &m, &m1);
    for (int i = 0; i < n; ++i)
        q += P->d[i] * p[i] * p[i];
    for (int i = 0; i < n; ++i) {
        Hp[i] = m * P->d[i] * p[i];
        Hx[i] = (q * m1 + P->w) * x[i];
    }
}

/* ------------------------------------------------------------------ */
/* Initial data.                                                        */
/* ------------------------------------------------------------------ */

double hjp_g(const hjp_problem *P, const double *x)
{
    if (P->jkind == HJP_J_ROSENBROCK) {
        double a = 1.0 - x[0], b = 1.0 + x[1] - x[0] * x[0];
        return P->rscale * (-100.0 + a * a + 100.0 * b * b);
    }
    double s = 0.0;
    for (int i = 0; i < P->n; ++i)
        s += x[i] * x[i] / (P->a[i] * P->a[i]);
    return 0.5 * s + P->j0;
}

void hjp_grad_g(const hjp_problem *P, const double *x, double *out)
{
    if (P->jkind == HJP_J_ROSENBROCK) {
        double b = 1.0 + x[1] - x[0] * x[0];
        out[0] = P->rscale * (-2.0 * (1.0 - x[0]) - 400.0 * x[0] * b);
        out[1] = P->rscale * 200.0 * b;
        for (int i = 2; i < P->n; ++i)
            out[i] = 0.0;
        return;
    }
    for (int i = 0; i < P->n; ++i)
        out[i] = x[i] / (P->a[i] * P->a[i]);
}

/* conjugate of the ellipsoid data: g*(p) = 1/2 sum a^2 p^2 - j0 */
static double gstar(const hjp_problem *P, const double *p)
{
    double s = 0.0;
    for (int i = 0; i < P->n; ++i)
        s += P->a[i] * P->a[i] * p[i] * p[i];
    return 0.5 * s - P->j0;
}

/* ------------------------------------------------------------------ */
/* Characteristics and the discrete functionals.                        */
/* ------------------------------------------------------------------ */

/* reversed-time field f(gamma, p) = (-H_p, +H_x) */
static void field(const hjp_problem *P, const double *y, double *f)
{
    const int n = P->n;
    hjp_grads(P, y, y + n, f + n, f);
    for (int i = 0; i < n; ++i)
        f[i] = -f[i];
}

/* integrand: Lax <p, H_p> - H, Hopf H - <H_x, gamma> */
static double integrand(const hjp_problem *P, const double *y)
{
    const int n = P->n;
    double *Hx = (double *)malloc(sizeof(double) * 2 * n), *Hp = Hx + n;
    hjp_grads(P, y, y + n, Hx, Hp);
    double H = hjp_hamiltonian(P, y, y + n), v;
    if (P->functional == HJP_HOPF) {
        double s = 0.0;
        for (int i = 0; i < n; ++i)
            s += Hx[i] * y[i];
        v = H - s;
    } else {
        double s = 0.0;
        for (int i = 0; i < n; ++i)
            s += y[n + i] * Hp[i];
        v = s - H;
    }
    free(Hx);
    return v;
}

/* The trajectory y_0 .. y_N ([(N+1) * 2n]) and the action quadrature:
 * Euler with the left rectangle rule, or RK4 with the RK4-augmented rule. */
static double trajectory(const hjp_problem *P, const double *x, const double *v, double *traj)
{
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    const double h = P->t / N;
    double *w = (double *)malloc(sizeof(double) * 6 * n2);
    double *K1 = w, *K2 = w + n2, *K3 = w + 2 * n2, *K4 = w + 3 * n2, *Y = w + 4 * n2;
    double q = 0.0;
    memcpy(traj, x, sizeof(double) * n);
    memcpy(traj + n, v, sizeof(double) * n);
    for (int k = 0; k < N; ++k) {
        const double *y = traj + (size_t)k * n2;
        double *yn = traj + (size_t)(k + 1) * n2;
        if (P->ode == HJP_EULER) {
            field(P, y, K1);
            q += h * integrand(P, y);
            for (int i = 0; i < n2; ++i)
                yn[i] = y[i] + h * K1[i];
        } else {
            double i1 = integrand(P, y);
            field(P, y, K1);
            for (int i = 0; i < n2; ++i)
                Y[i] = y[i] + 0.5 * h * K1[i];
            double i2 = integrand(P, Y);
            field(P, Y, K2);
            for (int i = 0; i < n2; ++i)
                Y[i] = y[i] + 0.5 * h * K2[i];
            double i3 = integrand(P, Y);
            field(P, Y, K3);
            for (int i = 0; i < n2; ++i)
                Y[i] = y[i] + h * K3[i];
            double i4 = integrand(P, Y);
            field(P, Y, K4);
            for (int i = 0; i < n2; ++i)
                yn[i] = y[i] + h / 6.0 * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
            q += h / 6.0 * (i1 + 2.0 * i2 + 2.0 * i3 + i4);
        }
    }
    free(w);
    return q;
}

static void unit(int n, const double *v, double *out)
{
    double s = sqrt(sq_norm(n, v));
    for (int i = 0; i < n; ++i)
        out[i] = s > 0.0 ? v[i] / s : 0.0;
}

/* certificate of the Lax functionals at (gamma, p): p = grad g(gamma),
 * compared on directions for the degree-1 family */
static double lax_residual(const hjp_problem *P, const double *gam, const double *p)
{
    const int n = P->n;
    double *gg = (double *)malloc(sizeof(double) * 3 * n), *u1 = gg + n, *u2 = gg + 2 * n;
    hjp_grad_g(P, gam, gg);
    double r = 0.0;
    if (P->hkind == HJP_H_NORM) {
        unit(n, p, u1);
        unit(n, gg, u2);
    } else {
        memcpy(u1, p, sizeof(double) * n);
        memcpy(u2, gg, sizeof(double) * n);
    }
    for (int i = 0; i < n; ++i) {
        double d = fabs(u1[i] - u2[i]);
        if (d > r || d != d)
            r = d;
    }
    free(gg);
    return r;
}

/* The staggered discrete schemes of the section 3 lemmas, in the paper's
 * index n = 0..N with x_N = x, p_N = v and delta = t / N:
 *   Lax  (eq. hahalolXDform):  p_{n-1} = p_n + delta H_x(x_n, p_n),
 *                              x_n - x_{n-1} = delta H_p(x_{n-1}, p_{n-1})
 *        (explicit in p, implicit in x_{n-1});
 *   Hopf (eq. hahalolXDform2): x_{n-1} = x_n - delta H_p(x_n, p_n),
 *                              p_{n-1} - p_n = delta H_x(x_{n-1}, p_{n-1})
 *        (explicit in x, implicit in p_{n-1}; needed for n - 1 >= 1).
 * The implicit equations are solved by fixed-point iteration from the
 * explicit guess, to a step below 1e-14 (1 + |z|_inf) or 60 sweeps.
 * X and Pm hold [(N+1) n] (row n). */
static void stagger_solve(const hjp_problem *P, const double *rhs0, const double *other,
                          int implicit_x, double delta, double *z)
{
    /* implicit_x: z = rhs0 - delta H_p(z, other)  (Lax, z = x_{n-1})
     * else:       z = rhs0 + delta H_x(other, z)  (Hopf, z = p_{n-1}) */
    const int n = P->n;
    double *w = (double *)malloc(sizeof(double) * 3 * n), *Hx = w, *Hp = w + n, *zn = w + 2 * n;
    for (int it = 0; it < 60; ++it) {
        if (implicit_x) {
            hjp_grads(P, z, other, Hx, Hp);
            for (int i = 0; i < n; ++i)
                zn[i] = rhs0[i] - delta * Hp[i];
        } else {
            hjp_grads(P, other, z, Hx, Hp);
            for (int i = 0; i < n; ++i)
                zn[i] = rhs0[i] + delta * Hx[i];
        }
        double dz = 0.0, nz = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = fabs(zn[i] - z[i]);
            if (d > dz || d != d)
                dz = d;
            if (fabs(zn[i]) > nz)
                nz = fabs(zn[i]);
            z[i] = zn[i];
        }
        if (!(dz > 1e-14 * (1.0 + nz)))
            break;
    }
    free(w);
}

static void staggered(const hjp_problem *P, const double *x, const double *v, double *X,
                      double *Pm)
{
    const int n = P->n, N = P->nsteps;
    const double delta = P->t / N;
    double *w = (double *)malloc(sizeof(double) * 2 * n), *Hx = w, *Hp = w + n;
    memcpy(X + (size_t)N * n, x, sizeof(double) * n);
    memcpy(Pm + (size_t)N * n, v, sizeof(double) * n);
    for (int m = N; m >= 1; --m) {
        double *xm = X + (size_t)m * n, *pm = Pm + (size_t)m * n;
        double *xl = X + (size_t)(m - 1) * n, *pl = Pm + (size_t)(m - 1) * n;
        hjp_grads(P, xm, pm, Hx, Hp);
        if (P->functional != HJP_HOPF) {
            for (int i = 0; i < n; ++i) {
                pl[i] = pm[i] + delta * Hx[i];
                xl[i] = xm[i] - delta * Hp[i];  /* explicit guess */
            }
            stagger_solve(P, xm, pl, 1, delta, xl);
        } else {
            for (int i = 0; i < n; ++i) {
                xl[i] = xm[i] - delta * Hp[i];
                pl[i] = pm[i];                  /* guess (p_0 is not used) */
            }
            if (m - 1 >= 1)
                stagger_solve(P, pm, xl, 0, delta, pl);
        }
    }
    free(w);
}

/* The staggered functionals and their certificates.
 *   Lax:  F = g(x_0) + sum_{n=0}^{N-1} <p_n, x_{n+1} - x_n> - delta sum_{n=0}^{N-1} H(x_n, p_n),
 *         certificate p_{-1} = p_0 + delta H_x(x_0, p_0) = grad g(x_0)
 *         (stationarity in x_0);
 *   F2:   min_n g(x_n), certificate at the first minimiser from n = N down;
 *   Hopf: G = <p_N, x> - g*(p_1) - delta sum_{n=1}^{N} H(x_n, p_n)
 *             + sum_{n=1}^{N-1} <p_n - p_{n+1}, x_n>, minimised as -G,
 *         certificate x_0 = grad g*(p_1) (stationarity in p_1). */
static double stagger_eval(const hjp_problem *P, const double *x, const double *v, double *rho,
                           double *yN)
{
    const int n = P->n, N = P->nsteps;
    const double delta = P->t / N;
    double *X = (double *)malloc(sizeof(double) * (size_t)(N + 1) * n);
    double *Pm = (double *)malloc(sizeof(double) * (size_t)(N + 1) * n);
    staggered(P, x, v, X, Pm);
    double phi, r = 0.0;
    const double *xc, *pc;
    if (P->functional == HJP_HOPF) {
        double G = 0.0;
        for (int i = 0; i < n; ++i)
            G += Pm[(size_t)N * n + i] * x[i];
        G -= gstar(P, Pm + n);
        for (int m = 1; m <= N; ++m)
            G -= delta * hjp_hamiltonian(P, X + (size_t)m * n, Pm + (size_t)m * n);
        for (int m = 1; m <= N - 1; ++m)
            for (int i = 0; i < n; ++i)
                G += (Pm[(size_t)m * n + i] - Pm[(size_t)(m + 1) * n + i]) * X[(size_t)m * n + i];
        phi = -G;
        xc = X;
        pc = Pm + n;
        for (int i = 0; i < n; ++i) {
            double d = fabs(xc[i] - P->a[i] * P->a[i] * pc[i]);
            if (d > r || d != d)
                r = d;
        }
    } else if (P->functional == HJP_LAX_MIN) {
        int mb = N;
        phi = hjp_g(P, X + (size_t)N * n);
        for (int m = N - 1; m >= 0; --m) {
            double gm = hjp_g(P, X + (size_t)m * n);
            if (gm < phi || (gm != gm && phi == phi)) {
                phi = gm;
                mb = m;
            }
        }
        xc = X + (size_t)mb * n;
        pc = Pm + (size_t)mb * n;
        r = lax_residual(P, xc, pc);
    } else {
        phi = hjp_g(P, X);
        for (int m = 0; m <= N - 1; ++m) {
            for (int i = 0; i < n; ++i)
                phi += Pm[(size_t)m * n + i] *
                       (X[(size_t)(m + 1) * n + i] - X[(size_t)m * n + i]);
            phi -= delta * hjp_hamiltonian(P, X + (size_t)m * n, Pm + (size_t)m * n);
        }
        /* the co-state recursion carried one step past n = 0: its value
         * p_0 + delta H_x(x_0, p_0) meets grad g(x_0) exactly where F is
         * stationary in v (the x_0-derivative of the functional) */
        double *w = (double *)malloc(sizeof(double) * 2 * n), *Hx = w, *Hp = w + n;
        hjp_grads(P, X, Pm, Hx, Hp);
        for (int i = 0; i < n; ++i)
            Pm[i] += delta * Hx[i];
        free(w);
        xc = X;
        pc = Pm;
        r = lax_residual(P, xc, pc);
    }
    if (rho)
        *rho = r;
    if (yN) {
        memcpy(yN, xc, sizeof(double) * n);
        memcpy(yN + n, pc, sizeof(double) * n);
    }
    free(X);
    free(Pm);
    return phi;
}

double hjp_eval(const hjp_problem *P, const double *x, const double *v, double *rho,
                double *yN)
{
    if (P->ode == HJP_STAGGERED)
        return stagger_eval(P, x, v, rho, yN);
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    double *traj = (double *)malloc(sizeof(double) * (size_t)(N + 1) * n2);
    double q = trajectory(P, x, v, traj);
    const double *end = traj + (size_t)N * n2;
    double phi, r;
    if (P->functional == HJP_HOPF) {
        /* G(v) = g*(p_N) + sum - <x, v>;  certificate gamma_N = a^2 p_N */
        double xv = 0.0;
        for (int i = 0; i < n; ++i)
            xv += x[i] * v[i];
        phi = gstar(P, end + n) + q - xv;
        r = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = fabs(end[i] - P->a[i] * P->a[i] * end[n + i]);
            if (d > r || d != d)
                r = d;
        }
    } else if (P->functional == HJP_LAX_MIN) {
        /* F2(v) = min_k g(gamma_k), k = 0..N (eq. num_min); the first
         * minimising state carries the certificate */
        int kb = 0;
        phi = hjp_g(P, traj);
        for (int k = 1; k <= N; ++k) {
            double gk = hjp_g(P, traj + (size_t)k * n2);
            if (gk < phi || (gk != gk && phi == phi)) {
                phi = gk;
                kb = k;
            }
        }
        end = traj + (size_t)kb * n2;
        r = lax_residual(P, end, end + n);
    } else {
        phi = hjp_g(P, end) + q;
        r = lax_residual(P, end, end + n);
    }
    if (rho)
        *rho = r;
    if (yN)
        memcpy(yN, end, sizeof(double) * n2);
    free(traj);
    return phi;
}

/* ------------------------------------------------------------------ */
/* Descent.                                                             */
/* ------------------------------------------------------------------ */

static double inf_norm(int n, const double *v)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a > s || a != a)
            s = a;
    }
    return s;
}

/* Algorithm 1 (section 4.1) with forward differences (eq. num_diff): two
 * objective evaluations per coordinate update. */
static int32_t descend_alg1(const hjp_problem *P, const hjp_opts *O, const double *x, double *v,
                            double *phi_out, double *rho_out, int32_t *iters, int64_t *n_eval)
{
    const int n = P->n;
    double rho, alpha = O->alpha0;
    double phi = hjp_eval(P, x, v, &rho, NULL);
    int64_t ev = 1;
    int32_t count = 0, kM = 0, upd = 0, status = HJP_ST_MAXITER;
    int j = 0;
    if (!isfinite(phi))
        status = HJP_ST_DIVERGED;
    while (status == HJP_ST_MAXITER && upd < O->max_iter * n) {
        double vj = v[j];
        v[j] = vj + O->fd_sigma;
        double fp = hjp_eval(P, x, v, NULL, NULL);
        double gj = (fp - phi) / O->fd_sigma;
        double step = alpha * gj;
        v[j] = vj - step;
        phi = hjp_eval(P, x, v, &rho, NULL);
        ev += 2;
        ++upd;
        if (++kM == O->M) {
            kM = 0;
            alpha *= 0.5;
        }
        if (fabs(step) > O->eps)
            count = 0;
        else if (fabs(step) < O->eps)
            ++count;
        j = (j + 1) % n;
        if (!isfinite(phi) || !(inf_norm(n, v) <= O->v_max))
            status = HJP_ST_DIVERGED;
        else if (count == n)
            status = HJP_ST_CONVERGED;
    }
    *phi_out = phi;
    *rho_out = status == HJP_ST_DIVERGED ? NAN : rho;
    *iters = upd;
    *n_eval += ev;
    return status;
}

/* Heavy-ball descent with a forward-difference gradient: v' = v - alpha g +
 * beta (v - v_prev); a trial that increases the objective (beyond the
 * rounding allowance) is rejected, the momentum dropped and alpha halved. */
static int32_t descend_momentum(const hjp_problem *P, const hjp_opts *O, const double *x,
                                double *v, double *phi_out, double *rho_out, int32_t *iters,
                                int64_t *n_eval)
{
    const int n = P->n;
    double *w = (double *)malloc(sizeof(double) * 3 * n), *g = w, *vp = w + n, *vt = w + 2 * n;
    double rho, alpha = O->alpha0;
    const double floor_a = O->alpha0 * ldexp(1.0, -40);
    double phi = hjp_eval(P, x, v, &rho, NULL);
    int64_t ev = 1;
    int32_t it = 0, status = HJP_ST_MAXITER;
    memcpy(vp, v, sizeof(double) * n);
    if (!isfinite(phi))
        status = HJP_ST_DIVERGED;
    while (status == HJP_ST_MAXITER && it < O->max_iter) {
        ++it;
        for (int j = 0; j < n; ++j) {
            double vj = v[j];
            v[j] = vj + O->fd_sigma;
            g[j] = (hjp_eval(P, x, v, NULL, NULL) - phi) / O->fd_sigma;
            v[j] = vj;
        }
        double smax = 0.0;
        for (int j = 0; j < n; ++j) {
            vt[j] = v[j] - alpha * g[j] + O->momentum * (v[j] - vp[j]);
            double d = fabs(vt[j] - v[j]);
            if (d > smax || d != d)
                smax = d;
        }
        double rt, ft = hjp_eval(P, x, vt, &rt, NULL);
        ev += n + 1;
        memcpy(vp, v, sizeof(double) * n);
        if (ft <= phi + O->acc_rel * fabs(phi)) {
            memcpy(v, vt, sizeof(double) * n);
            phi = ft;
            rho = rt;
        } else {
            alpha *= 0.5;
        }
        if (!isfinite(phi) || !(inf_norm(n, v) <= O->v_max))
            status = HJP_ST_DIVERGED;
        else if (smax < O->eps)
            status = HJP_ST_CONVERGED;
        else if (alpha < floor_a)
            status = HJP_ST_STALLED;
    }
    free(w);
    *phi_out = phi;
    *rho_out = status == HJP_ST_DIVERGED ? NAN : rho;
    *iters = it;
    *n_eval += ev;
    return status;
}

int32_t hjp_descend(const hjp_problem *P, const hjp_opts *O, const double *x, double *v,
                    double *phi, double *rho, int32_t *iters, int64_t *n_eval)
{
    if (O->mode == HJP_MOMENTUM)
        return descend_momentum(P, O, x, v, phi, rho, iters, n_eval);
    return descend_alg1(P, O, x, v, phi, rho, iters, n_eval);
}

int32_t hjp_solve(const hjp_problem *P, const hjp_opts *O, const double *x, int64_t B,
                  const double *guesses, int32_t G, double *out_u, double *out_argopt,
                  int32_t *out_cert, double *slot_phi, double *slot_rho, int32_t *slot_cert,
                  int32_t *slot_iters, int64_t *slot_eval)
{
    const int n = P->n, R = O->R_max;
    if (n < 1 || G < 1 || R < 0 || P->nsteps < 1)
        return -1;
    double *v = (double *)malloc(sizeof(double) * n);
    double *sv = (double *)malloc(sizeof(double) * (size_t)G * n);
    double *sp = (double *)malloc(sizeof(double) * G);
    int32_t *sc = (int32_t *)malloc(sizeof(int32_t) * G);
    for (int64_t b = 0; b < B; ++b) {
        const double *xb = x + b * n;
        for (int g = 0; g < G; ++g) {
            double bphi = NAN, brho = NAN;
            int32_t bcert = -1, iters = 0;
            int64_t ev = 0;
            for (int r = 0; r <= R; ++r) {
                memcpy(v, guesses + (((size_t)b * G + g) * (R + 1) + r) * n,
                       sizeof(double) * n);
                double phi, rho;
                int32_t it;
                int32_t st = hjp_descend(P, O, xb, v, &phi, &rho, &it, &ev);
                iters += it;
                int fin = st != HJP_ST_DIVERGED && isfinite(phi);
                int cert = fin && rho <= O->cert_tol;
                if (cert || (fin && (bcert < 0 || phi < bphi))) {
                    bphi = phi;
                    brho = rho;
                    bcert = cert ? 1 : 0;
                    memcpy(sv + (size_t)g * n, v, sizeof(double) * n);
                }
                if (cert)
                    break;
            }
            if (bcert < 0)
                for (int i = 0; i < n; ++i)
                    sv[(size_t)g * n + i] = NAN;
            sp[g] = bphi;
            sc[g] = bcert;
            size_t k = (size_t)b * G + g;
            if (slot_phi) slot_phi[k] = bphi;
            if (slot_rho) slot_rho[k] = brho;
            if (slot_cert) slot_cert[k] = bcert;
            if (slot_iters) slot_iters[k] = iters;
            if (slot_eval) slot_eval[k] = ev;
        }
        /* selection: certified first, lowest objective, ties to the lowest slot */
        int pick = -1, pc = -1;
        double best = 0.0;
        for (int g = 0; g < G; ++g) {
            if (sc[g] < 0)
                continue;
            if (sc[g] > pc || (sc[g] == pc && sp[g] < best)) {
                pick = g;
                pc = sc[g];
                best = sp[g];
            }
        }
        out_cert[b] = pc;
        if (pick < 0) {
            out_u[b] = NAN;
            for (int i = 0; i < n; ++i)
                out_argopt[b * n + i] = NAN;
        } else {
            out_u[b] = P->functional == HJP_HOPF ? -best : best;
            memcpy(out_argopt + b * n, sv + (size_t)pick * n, sizeof(double) * n);
        }
    }
    free(v);
    free(sv);
    free(sp);
    free(sc);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Lax-Friedrichs grid solver (two space dimensions).                   */
/* ------------------------------------------------------------------ */

int32_t hjp_lax_friedrichs(const hjp_problem *P, double x0, double y0, double dx, double dy,
                           int32_t nx, int32_t ny, double dt, int32_t nt, double ax, double ay,
                           double *phi)
{
    if (P->n != 2 || P->hkind != HJP_H_QUADRATIC || nx < 3 || ny < 3)
        return -1;
    double *nw = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    double pt[2];
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            pt[0] = x0 + i * dx;
            pt[1] = y0 + j * dy;
            phi[(size_t)j * nx + i] = hjp_g(P, pt);
        }
    for (int s = 0; s < nt; ++s) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double c = phi[(size_t)j * nx + i];
                /* neighbours, with linear extrapolation across the boundary */
                double l = i > 0 ? phi[(size_t)j * nx + i - 1] : 2.0 * c - phi[(size_t)j * nx + 1];
                double r = i < nx - 1 ? phi[(size_t)j * nx + i + 1]
                                      : 2.0 * c - phi[(size_t)j * nx + nx - 2];
                double d = j > 0 ? phi[(size_t)(j - 1) * nx + i] : 2.0 * c - phi[(size_t)nx + i];
                double u = j < ny - 1 ? phi[(size_t)(j + 1) * nx + i]
                                      : 2.0 * c - phi[(size_t)(ny - 2) * nx + i];
                double pp = (r - c) / dx, pm = (c - l) / dx;
                double qp = (u - c) / dy, qm = (c - d) / dy;
                double p[2] = {0.5 * (pp + pm), 0.5 * (qp + qm)};
                pt[0] = x0 + i * dx;
                pt[1] = y0 + j * dy;
                double Hn = hjp_hamiltonian(P, pt, p) - 0.5 * ax * (pp - pm) -
                            0.5 * ay * (qp - qm);
                nw[(size_t)j * nx + i] = c - dt * Hn;
            }
        memcpy(phi, nw, sizeof(double) * (size_t)nx * ny);
    }
    free(nw);
    return 0;
}
