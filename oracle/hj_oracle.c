/*
 * hj_oracle.c -- plain, slow, single-threaded FP64 reference of the
 * generalized Lax / Hopf solver (arXiv:1704.02524, sections 3.3, 3.4 and 4).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product path.  It is
 * written for readability, not speed: no blocking, fusion or reordering
 * beyond what each definition states.  Notation is in hj_oracle.h.
 *
 * Readings of the paper that this file commits to (the paper leaves them
 * open or uses simpler choices on purpose):
 *  - the characteristic ODE is integrated with classical RK4 (the paper
 *    allows "any ODE solver", section 4.1, and uses forward Euler in its
 *    experiments, section 4.2);
 *  - the action integral uses the trapezoid rule on the RK4 nodes or the
 *    RK4-augmented rule (RK4 applied to a' = integrand); the paper's
 *    rectangular rule (eq. num_int) is the same family of quadratures;
 *  - derivatives are central differences (the paper's eq. num_diff is a
 *    forward difference) or the exact gradient of the discrete objective;
 *  - Algorithm 1 (cyclic coordinate descent) halves the step whenever a
 *    trial step does not decrease the objective (up to a rounding
 *    allowance), and one iteration is one sweep over all coordinates.
 */
#include "hj_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Problem functions (paper section 2.1, eq. HJeqn; the family of H).  */
/* ------------------------------------------------------------------ */

/* m(r) = c(r)^e and its first two derivatives with respect to r = |x|^2. */
void hjo_scalars(const hjo_problem *P, double r, double *m, double *m1, double *m2)
{
    double c, c1, c2;
    if (P->m_kind == HJO_M_RAT) {
        /* c = 1 + kappa r / (1 + r) */
        double q = 1.0 + r;
        c = 1.0 + P->kappa * r / q;
        c1 = P->kappa / (q * q);
        c2 = -2.0 * P->kappa / (q * q * q);
    } else if (P->m_kind == HJO_M_TANH) {
        /* c = 1 + kappa tanh(r / s) */
        double th = tanh(r / P->s);
        double sech2 = 1.0 - th * th;
        c = 1.0 + P->kappa * th;
        c1 = P->kappa / P->s * sech2;
        c2 = -2.0 * P->kappa / (P->s * P->s) * th * sech2;
    } else {
        c = 1.0;
        c1 = 0.0;
        c2 = 0.0;
    }
    if (P->e == 2) {
        *m = c * c;
        *m1 = 2.0 * c * c1;
        *m2 = 2.0 * c1 * c1 + 2.0 * c * c2;
    } else {
        *m = c;
        *m1 = c1;
        *m2 = c2;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

/* q(p) = sum_i d_i p_i^2 */
static double kinetic(const hjo_problem *P, const double *p)
{
    double q = 0.0;
    for (int i = 0; i < P->n; ++i)
        q += P->d[i] * p[i] * p[i];
    return q;
}

/* <A gam, p> */
static double drift_pair(const hjo_problem *P, const double *gam, const double *p)
{
    if (!P->A)
        return 0.0;
    double s = 0.0;
    for (int i = 0; i < P->n; ++i)
        for (int j = 0; j < P->n; ++j)
            s += p[i] * P->A[i * P->n + j] * gam[j];
    return s;
}

double hjo_hamiltonian(const hjo_problem *P, const double *gam, const double *p)
{
    double r = dot(P->n, gam, gam), m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    return drift_pair(P, gam, p) + 0.5 * m * kinetic(P, p) + 0.5 * P->w * r;
}

/* H_p = A gam + m D p ;  H_x = A^T p + (q m' + w) gam.
 * The final-value problem gam' = H_p, p' = -H_x (paper section 4.1) becomes,
 * in reversed time tau = t - s, y' = f(y) with f = (-H_p, +H_x). */
void hjo_field(const hjo_problem *P, const double *gam, const double *p, double *out)
{
    const int n = P->n;
    double r = dot(n, gam, gam), m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    double q = kinetic(P, p);
    for (int i = 0; i < n; ++i) {
        double Hp = m * P->d[i] * p[i];
        double Hx = (q * m1 + P->w) * gam[i];
        if (P->A) {
            for (int j = 0; j < n; ++j) {
                Hp += P->A[i * n + j] * gam[j];
                Hx += P->A[j * n + i] * p[j];
            }
        }
        out[i] = -Hp;
        out[n + i] = Hx;
    }
}

/* Lax (eq. lax_formula):  <p, H_p> - H       = 1/2 m q - 1/2 w r
 * Hopf (eq. hopf_formula): H - <H_x, gamma>  = 1/2 m q - q m' r - 1/2 w r
 * Written here from the definitions, not from the simplified forms. */
double hjo_integrand(const hjo_problem *P, const double *gam, const double *p)
{
    const int n = P->n;
    double f[2 * 512];
    double *buf = (2 * n <= 1024) ? f : (double *)malloc(sizeof(double) * 2 * n);
    hjo_field(P, gam, p, buf);
    double H = hjo_hamiltonian(P, gam, p);
    double val;
    if (P->formula == HJO_LAX) {
        /* H_p = -f_gamma */
        double pHp = 0.0;
        for (int i = 0; i < n; ++i)
            pHp += p[i] * (-buf[i]);
        val = pHp - H;
    } else {
        /* H_x = +f_p */
        double xHx = 0.0;
        for (int i = 0; i < n; ++i)
            xHx += buf[n + i] * gam[i];
        val = H - xHx;
    }
    if (buf != f)
        free(buf);
    return val;
}

/* Initial data g (ellipsoid) and its conjugate g* (paper section 5 uses
 * g = 1/2(<x, A x> - 1) with a diagonal A). */
static double g_val(const hjo_problem *P, const double *x)
{
    double s = 0.0;
    for (int i = 0; i < P->n; ++i)
        s += x[i] * x[i] / (P->a[i] * P->a[i]);
    return 0.5 * s + P->j0;
}

static double gstar_val(const hjo_problem *P, const double *p)
{
    double s = 0.0;
    for (int i = 0; i < P->n; ++i)
        s += P->a[i] * P->a[i] * p[i] * p[i];
    return 0.5 * s - P->j0;
}

/* ------------------------------------------------------------------ */
/* Evaluation of the objective (section 4.2): ODE solve + quadrature.  */
/* ------------------------------------------------------------------ */

/* One classical RK4 step of y' = f(y) with step h, accumulating the
 * RK4-augmented quadrature of the integrand into *acc when requested. */
static void rk4_step(const hjo_problem *P, double h, const double *y, double *ynext,
                     double *acc, int augment, double *work)
{
    const int n2 = 2 * P->n, n = P->n;
    double *K1 = work, *K2 = work + n2, *K3 = work + 2 * n2, *K4 = work + 3 * n2;
    double *Y = work + 4 * n2;
    int i;

    /* stage 1 */
    hjo_field(P, y, y + n, K1);
    double i1 = augment ? hjo_integrand(P, y, y + n) : 0.0;
    /* stage 2 */
    for (i = 0; i < n2; ++i)
        Y[i] = y[i] + 0.5 * h * K1[i];
    hjo_field(P, Y, Y + n, K2);
    double i2 = augment ? hjo_integrand(P, Y, Y + n) : 0.0;
    /* stage 3 */
    for (i = 0; i < n2; ++i)
        Y[i] = y[i] + 0.5 * h * K2[i];
    hjo_field(P, Y, Y + n, K3);
    double i3 = augment ? hjo_integrand(P, Y, Y + n) : 0.0;
    /* stage 4 */
    for (i = 0; i < n2; ++i)
        Y[i] = y[i] + h * K3[i];
    hjo_field(P, Y, Y + n, K4);
    double i4 = augment ? hjo_integrand(P, Y, Y + n) : 0.0;

    for (i = 0; i < n2; ++i)
        ynext[i] = y[i] + h / 6.0 * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
    if (augment)
        *acc += h / 6.0 * (i1 + 2.0 * i2 + 2.0 * i3 + i4);
}

void hjo_trajectory(const hjo_problem *P, const double *x, const double *v, double *traj)
{
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    const double h = P->t / N;
    double *work = (double *)malloc(sizeof(double) * 5 * n2);
    double dummy = 0.0;
    memcpy(traj, x, sizeof(double) * n);
    memcpy(traj + n, v, sizeof(double) * n);
    for (int k = 0; k < N; ++k)
        rk4_step(P, h, traj + (size_t)k * n2, traj + (size_t)(k + 1) * n2, &dummy, 0, work);
    free(work);
}

/* Objective Phi(v): paper functionals F^1 (Lax) and G (Hopf), section 4.1. */
double hjo_eval(const hjo_problem *P, const double *x, const double *v, double *yN)
{
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    const double h = P->t / N;
    double *work = (double *)malloc(sizeof(double) * 7 * n2);
    double *y = work + 5 * n2, *ynext = work + 6 * n2;
    double acc = 0.0;
    int aug = (P->quad == HJO_RK4AUG);

    memcpy(y, x, sizeof(double) * n);
    memcpy(y + n, v, sizeof(double) * n);
    if (!aug)
        acc += 0.5 * h * hjo_integrand(P, y, y + n);
    for (int k = 0; k < N; ++k) {
        rk4_step(P, h, y, ynext, &acc, aug, work);
        memcpy(y, ynext, sizeof(double) * n2);
        if (!aug)
            acc += (k + 1 < N ? h : 0.5 * h) * hjo_integrand(P, y, y + n);
    }
    double phi;
    if (P->formula == HJO_LAX)
        phi = g_val(P, y) + acc;
    else
        phi = gstar_val(P, y + n) + acc - dot(n, x, v);
    if (yN)
        memcpy(yN, y, sizeof(double) * n2);
    free(work);
    return phi;
}

/* ------------------------------------------------------------------ */
/* Exact derivative of the discrete objective, forward (tangent) mode. */
/* Every quantity u is carried with its directional derivative du.     */
/* ------------------------------------------------------------------ */

/* f and its directional derivative along (dgam, dp). */
static void field_tangent(const hjo_problem *P, const double *gam, const double *p,
                          const double *dgam, const double *dp, double *f, double *df)
{
    const int n = P->n;
    double r = dot(n, gam, gam), dr = 2.0 * dot(n, gam, dgam);
    double m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    double dm = m1 * dr, dm1 = m2 * dr;
    double q = 0.0, dq = 0.0;
    for (int i = 0; i < n; ++i) {
        q += P->d[i] * p[i] * p[i];
        dq += 2.0 * P->d[i] * p[i] * dp[i];
    }
    for (int i = 0; i < n; ++i) {
        double Hp = m * P->d[i] * p[i];
        double dHp = dm * P->d[i] * p[i] + m * P->d[i] * dp[i];
        double Hx = (q * m1 + P->w) * gam[i];
        double dHx = (dq * m1 + q * dm1) * gam[i] + (q * m1 + P->w) * dgam[i];
        if (P->A) {
            for (int j = 0; j < n; ++j) {
                Hp += P->A[i * n + j] * gam[j];
                dHp += P->A[i * n + j] * dgam[j];
                Hx += P->A[j * n + i] * p[j];
                dHx += P->A[j * n + i] * dp[j];
            }
        }
        f[i] = -Hp;
        df[i] = -dHp;
        f[n + i] = Hx;
        df[n + i] = dHx;
    }
}

/* Integrand and its directional derivative, from the simplified forms
 * 1/2 m q - 1/2 w r (Lax) and 1/2 m q - q m' r - 1/2 w r (Hopf), which the
 * tests check against hjo_integrand (the definitions). */
static double integrand_tangent(const hjo_problem *P, const double *gam, const double *p,
                                const double *dgam, const double *dp, double *dval)
{
    const int n = P->n;
    double r = dot(n, gam, gam), dr = 2.0 * dot(n, gam, dgam);
    double m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    double dm = m1 * dr, dm1 = m2 * dr;
    double q = 0.0, dq = 0.0;
    for (int i = 0; i < n; ++i) {
        q += P->d[i] * p[i] * p[i];
        dq += 2.0 * P->d[i] * p[i] * dp[i];
    }
    double val = 0.5 * m * q - 0.5 * P->w * r;
    double dv = 0.5 * dm * q + 0.5 * m * dq - 0.5 * P->w * dr;
    if (P->formula == HJO_HOPF) {
        val -= q * m1 * r;
        dv -= dq * m1 * r + q * dm1 * r + q * m1 * dr;
    }
    *dval = dv;
    return val;
}

double hjo_eval_tangent(const hjo_problem *P, const double *x, const double *v,
                        const double *dx, const double *dv, double *dphi)
{
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    const double h = P->t / N;
    const int aug = (P->quad == HJO_RK4AUG);
    /* y, dy, stage buffers Y, dY, K1..K4 and dK1..dK4 */
    double *mem = (double *)malloc(sizeof(double) * 14 * n2);
    double *y = mem, *dy = mem + n2, *Y = mem + 2 * n2, *dY = mem + 3 * n2;
    double *K[4], *dK[4];
    for (int s = 0; s < 4; ++s) {
        K[s] = mem + (4 + s) * n2;
        dK[s] = mem + (8 + s) * n2;
    }
    double *yn = mem + 12 * n2, *dyn = mem + 13 * n2;
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    const double bw[4] = {1.0, 2.0, 2.0, 1.0};
    double acc = 0.0, dacc = 0.0, di;

    memcpy(y, x, sizeof(double) * n);
    memcpy(y + n, v, sizeof(double) * n);
    memcpy(dy, dx, sizeof(double) * n);
    memcpy(dy + n, dv, sizeof(double) * n);
    if (!aug) {
        acc += 0.5 * h * integrand_tangent(P, y, y + n, dy, dy + n, &di);
        dacc += 0.5 * h * di;
    }
    for (int k = 0; k < N; ++k) {
        for (int s = 0; s < 4; ++s) {
            for (int i = 0; i < n2; ++i) {
                Y[i] = s ? y[i] + cst[s] * h * K[s - 1][i] : y[i];
                dY[i] = s ? dy[i] + cst[s] * h * dK[s - 1][i] : dy[i];
            }
            field_tangent(P, Y, Y + n, dY, dY + n, K[s], dK[s]);
            if (aug) {
                double val = integrand_tangent(P, Y, Y + n, dY, dY + n, &di);
                acc += h / 6.0 * bw[s] * val;
                dacc += h / 6.0 * bw[s] * di;
            }
        }
        for (int i = 0; i < n2; ++i) {
            yn[i] = y[i] + h / 6.0 * (K[0][i] + 2.0 * K[1][i] + 2.0 * K[2][i] + K[3][i]);
            dyn[i] = dy[i] + h / 6.0 * (dK[0][i] + 2.0 * dK[1][i] + 2.0 * dK[2][i] + dK[3][i]);
        }
        memcpy(y, yn, sizeof(double) * n2);
        memcpy(dy, dyn, sizeof(double) * n2);
        if (!aug) {
            double wk = (k + 1 < N) ? h : 0.5 * h;
            acc += wk * integrand_tangent(P, y, y + n, dy, dy + n, &di);
            dacc += wk * di;
        }
    }
    double phi, dphi_v;
    if (P->formula == HJO_LAX) {
        phi = g_val(P, y) + acc;
        dphi_v = dacc;
        for (int i = 0; i < n; ++i)
            dphi_v += y[i] / (P->a[i] * P->a[i]) * dy[i];
    } else {
        phi = gstar_val(P, y + n) + acc - dot(n, x, v);
        dphi_v = dacc - dot(n, dx, v) - dot(n, x, dv);
        for (int i = 0; i < n; ++i)
            dphi_v += P->a[i] * P->a[i] * y[n + i] * dy[n + i];
    }
    *dphi = dphi_v;
    free(mem);
    return phi;
}

double hjo_grad_tangent(const hjo_problem *P, const double *x, const double *v,
                        double *grad_v, double *grad_x)
{
    const int n = P->n;
    double *e = (double *)calloc(2 * n, sizeof(double));
    double *zero = e + n, phi = 0.0;
    for (int i = 0; i < n; ++i) {
        e[i] = 1.0;
        if (grad_v)
            phi = hjo_eval_tangent(P, x, v, zero, e, &grad_v[i]);
        if (grad_x)
            phi = hjo_eval_tangent(P, x, v, e, zero, &grad_x[i]);
        e[i] = 0.0;
    }
    if (!grad_v && !grad_x)
        phi = hjo_eval(P, x, v, NULL);
    free(e);
    return phi;
}

/* ------------------------------------------------------------------ */
/* Exact gradient of the discrete objective, reverse (adjoint) mode.   */
/* ------------------------------------------------------------------ */

/* (mu_gam, mu_p) = J_f(gam, p)^T (lam_gam, lam_p), from the derivative of
 * f = (-(A gam + m D p), A^T p + (q m' + w) gam):
 *   mu_gam = -A^T lam_g - 2 m' <D p, lam_g> gam
 *            + (q m' + w) lam_p + 2 q m'' <gam, lam_p> gam
 *   mu_p   = -m D lam_g + A lam_p + 2 m' <gam, lam_p> D p            */
static void field_vjp(const hjo_problem *P, const double *gam, const double *p,
                      const double *lam, double *mu)
{
    const int n = P->n;
    const double *lg = lam, *lp = lam + n;
    double r = dot(n, gam, gam), m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    double q = kinetic(P, p);
    double Dp_lg = 0.0, gam_lp = dot(n, gam, lp);
    for (int i = 0; i < n; ++i)
        Dp_lg += P->d[i] * p[i] * lg[i];
    for (int i = 0; i < n; ++i) {
        double mg = -2.0 * m1 * Dp_lg * gam[i] + (q * m1 + P->w) * lp[i]
                    + 2.0 * q * m2 * gam_lp * gam[i];
        double mp = -m * P->d[i] * lg[i] + 2.0 * m1 * gam_lp * P->d[i] * p[i];
        if (P->A) {
            for (int j = 0; j < n; ++j) {
                mg -= P->A[j * n + i] * lg[j];
                mp += P->A[i * n + j] * lp[j];
            }
        }
        mu[i] = mg;
        mu[n + i] = mp;
    }
}

/* Gradient of the integrand: grad_gam, grad_p into out[2n]. */
static void integrand_grad(const hjo_problem *P, const double *gam, const double *p,
                           double *out)
{
    const int n = P->n;
    double r = dot(n, gam, gam), m, m1, m2;
    hjo_scalars(P, r, &m, &m1, &m2);
    double q = kinetic(P, p);
    double cg, cp;
    if (P->formula == HJO_LAX) {
        /* 1/2 m q - 1/2 w r */
        cg = q * m1 - P->w;
        cp = m;
    } else {
        /* 1/2 m q - q m' r - 1/2 w r */
        cg = q * m1 - 2.0 * q * (m2 * r + m1) - P->w;
        cp = m - 2.0 * r * m1;
    }
    for (int i = 0; i < n; ++i) {
        out[i] = cg * gam[i];
        out[n + i] = cp * P->d[i] * p[i];
    }
}

double hjo_grad_reverse(const hjo_problem *P, const double *x, const double *v,
                        double *grad_v, double *grad_x)
{
    const int n = P->n, n2 = 2 * n, N = P->nsteps;
    const double h = P->t / N;
    const int aug = (P->quad == HJO_RK4AUG);
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    const double bw[4] = {1.0, 2.0, 2.0, 1.0};
    double *traj = (double *)malloc(sizeof(double) * (size_t)(N + 1) * n2);
    double *mem = (double *)malloc(sizeof(double) * 14 * n2);
    double *Ys[4], *Ks[4];
    for (int s = 0; s < 4; ++s) {
        Ys[s] = mem + s * n2;
        Ks[s] = mem + (4 + s) * n2;
    }
    double *lam = mem + 8 * n2, *ybar = mem + 9 * n2, *Kbar = mem + 10 * n2;
    double *Ybar = mem + 11 * n2, *tmp = mem + 12 * n2, *ig = mem + 13 * n2;

    /* forward: the objective and the stored trajectory */
    double phi = hjo_eval(P, x, v, NULL);
    hjo_trajectory(P, x, v, traj);

    /* seed with the derivative of the terminal term at y_N */
    const double *yN = traj + (size_t)N * n2;
    for (int i = 0; i < n; ++i) {
        if (P->formula == HJO_LAX) {
            lam[i] = yN[i] / (P->a[i] * P->a[i]);
            lam[n + i] = 0.0;
        } else {
            lam[i] = 0.0;
            lam[n + i] = P->a[i] * P->a[i] * yN[n + i];
        }
    }
    if (!aug) {
        integrand_grad(P, yN, yN + n, ig);
        for (int i = 0; i < n2; ++i)
            lam[i] += 0.5 * h * ig[i];
    }

    for (int k = N - 1; k >= 0; --k) {
        const double *yk = traj + (size_t)k * n2;
        /* recompute the stages of step k */
        for (int s = 0; s < 4; ++s) {
            for (int i = 0; i < n2; ++i)
                Ys[s][i] = s ? yk[i] + cst[s] * h * Ks[s - 1][i] : yk[i];
            hjo_field(P, Ys[s], Ys[s] + n, Ks[s]);
        }
        /* y_{k+1} = y_k + h/6 sum_s b_s K_s,  K_s = f(Y_s),
         * Y_s = y_k + c_s h K_{s-1}; (RK4AUG) acc += h/6 sum_s b_s iota(Y_s). */
        memcpy(ybar, lam, sizeof(double) * n2);
        /* Ybar of the stage above, used to form Kbar of the stage below */
        memset(Ybar, 0, sizeof(double) * n2);
        for (int s = 3; s >= 0; --s) {
            for (int i = 0; i < n2; ++i)
                Kbar[i] = h / 6.0 * bw[s] * lam[i] + (s < 3 ? cst[s + 1] * h * Ybar[i] : 0.0);
            field_vjp(P, Ys[s], Ys[s] + n, Kbar, tmp);
            if (aug) {
                integrand_grad(P, Ys[s], Ys[s] + n, ig);
                for (int i = 0; i < n2; ++i)
                    tmp[i] += h / 6.0 * bw[s] * ig[i];
            }
            memcpy(Ybar, tmp, sizeof(double) * n2);
            for (int i = 0; i < n2; ++i)
                ybar[i] += Ybar[i];
        }
        if (!aug) {
            double wk = (k == 0) ? 0.5 * h : h;
            integrand_grad(P, yk, yk + n, ig);
            for (int i = 0; i < n2; ++i)
                ybar[i] += wk * ig[i];
        }
        memcpy(lam, ybar, sizeof(double) * n2);
    }
    /* lam = d Phi / d y_0 except for the explicit -<x, v> of the Hopf form */
    for (int i = 0; i < n; ++i) {
        double hop_v = (P->formula == HJO_HOPF) ? x[i] : 0.0;
        double hop_x = (P->formula == HJO_HOPF) ? v[i] : 0.0;
        if (grad_v)
            grad_v[i] = lam[n + i] - hop_v;
        if (grad_x)
            grad_x[i] = lam[i] - hop_x;
    }
    free(mem);
    free(traj);
    return phi;
}

/* ------------------------------------------------------------------ */
/* Certificate of correctness (section 4.3): p(0) in dg(gamma(0)).     */
/* ------------------------------------------------------------------ */

double hjo_certificate(const hjo_problem *P, const double *yN)
{
    const int n = P->n;
    double rho = 0.0;
    for (int i = 0; i < n; ++i) {
        double res;
        if (P->formula == HJO_LAX)          /* primal: p_N - grad g(gamma_N)   */
            res = yN[n + i] - yN[i] / (P->a[i] * P->a[i]);
        else                                 /* dual: gamma_N - grad g*(p_N)    */
            res = yN[i] - P->a[i] * P->a[i] * yN[n + i];
        res = fabs(res);
        if (!(res <= rho))                   /* propagates NaN */
            rho = res;
    }
    return rho;
}

/* ------------------------------------------------------------------ */
/* Descent (Algorithm 1, section 4.1) and multi-start (section 5).     */
/* ------------------------------------------------------------------ */

/* A trial step counts as an ascent when it raises the objective by more than
 * a rounding allowance acc_rel * |Phi|; the allowance keeps rounding noise of
 * the objective from halving the step size near the optimum. */
static int accept_step(const hjo_opts *O, double trial, double cur, double decrease)
{
    /* decrease = alpha * (directional derivative along the step), >= 0; the
     * trial must realise the fraction armijo_c of it (Armijo's sufficient
     * decrease; armijo_c = 0 is the plain "no ascent" test) */
    return trial <= cur - O->armijo_c * decrease + O->acc_rel * fabs(cur);
}

/* max(s, a) that keeps a NaN once one has been seen */
static double nan_max(double s, double a)
{
    return (a > s || a != a) ? a : s;
}

static double inf_norm(int n, const double *v)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        s = nan_max(s, fabs(v[i]));
    return s;
}

int32_t hjo_descend(const hjo_problem *P, const hjo_opts *O, const double *x,
                    double *v, double *phi_out, double *rho_out, int32_t *iters_out,
                    int64_t *n_fwd, int64_t *n_bwd)
{
    const int n = P->n;
    double *mem = (double *)malloc(sizeof(double) * 6 * n);
    double *vt = mem, *g = mem + n, *yN = mem + 2 * n, *yNt = mem + 4 * n;
    double alpha = O->alpha0;
    const double alpha_floor = O->alpha0 * ldexp(1.0, -40);
    int32_t status = HJO_ST_MAXITER, it = 0;
    int64_t fwd = 0, bwd = 0;
    double phi;

    phi = hjo_eval(P, x, v, yN);
    fwd += 1;
    if (O->mode == HJO_GD && isfinite(phi)) {
        hjo_grad_reverse(P, x, v, g, NULL);
        bwd += 1;
    }
    if (!isfinite(phi))
        status = HJO_ST_DIVERGED;

    /* status stays HJO_ST_MAXITER while the run goes on */
    while (status == HJO_ST_MAXITER && it < O->max_iter) {
        double smax = 0.0;
        ++it;
        if (O->mode == HJO_CD_FD) {
            /* one sweep of cyclic coordinate descent */
            for (int j = 0; j < n; ++j) {
                memcpy(vt, v, sizeof(double) * n);
                vt[j] = v[j] + O->fd_sigma;
                double fp = hjo_eval(P, x, vt, NULL);
                vt[j] = v[j] - O->fd_sigma;
                double fm = hjo_eval(P, x, vt, NULL);
                double gj = (fp - fm) / (2.0 * O->fd_sigma);
                double step = alpha * gj;
                smax = nan_max(smax, fabs(step));
                vt[j] = v[j] - step;
                double ft = hjo_eval(P, x, vt, yNt);
                fwd += 3;
                if (accept_step(O, ft, phi, alpha * gj * gj)) {
                    v[j] = vt[j];
                    phi = ft;
                    memcpy(yN, yNt, sizeof(double) * 2 * n);
                } else {
                    alpha *= 0.5;
                }
            }
        } else {
            /* one full-gradient step with the exact discrete gradient */
            smax = alpha * inf_norm(n, g);
            for (int i = 0; i < n; ++i)
                vt[i] = v[i] - alpha * g[i];
            double ft = hjo_eval(P, x, vt, yNt);
            fwd += 1;
            if (accept_step(O, ft, phi, alpha * dot(n, g, g))) {
                memcpy(v, vt, sizeof(double) * n);
                phi = ft;
                memcpy(yN, yNt, sizeof(double) * 2 * n);
                hjo_grad_reverse(P, x, v, g, NULL);
                bwd += 1;
            } else {
                alpha *= 0.5;
            }
        }
        if (!isfinite(phi) || !(inf_norm(n, v) <= O->v_max))
            status = HJO_ST_DIVERGED;
        else if (smax < O->eps_step)
            status = HJO_ST_CONVERGED;
        else if (alpha < alpha_floor)
            status = HJO_ST_STALLED;
    }
    *phi_out = phi;
    *rho_out = (status == HJO_ST_DIVERGED) ? NAN : hjo_certificate(P, yN);
    *iters_out = it;
    *n_fwd += fwd;
    *n_bwd += bwd;
    free(mem);
    return status;
}

int32_t hjo_solve(const hjo_problem *P, const hjo_opts *O, const double *x,
                  int64_t B, int64_t b0, int64_t b1, const double *guesses, int32_t G,
                  double *out_u, double *out_argopt, int32_t *out_cert,
                  const hjo_slot_diag *diag)
{
    const int n = P->n, R = O->R_max;
    if (n < 1 || G < 1 || R < 0 || b0 < 0 || b1 > B || b0 > b1 || P->nsteps < 1)
        return -1;
    double *v = (double *)malloc(sizeof(double) * n);
    double *slot_v = (double *)malloc(sizeof(double) * (size_t)G * n);
    double *slot_phi = (double *)malloc(sizeof(double) * G);
    int32_t *slot_cert = (int32_t *)malloc(sizeof(int32_t) * G);

    for (int64_t b = b0; b < b1; ++b) {
        const double *xb = x + (size_t)b * n;
        for (int g = 0; g < G; ++g) {
            /* attempts of one slot: stop at the first certified one; else
             * report the attempt with the lowest finite objective */
            double best_phi = NAN, best_rho = NAN;
            int32_t best_cert = -1, best_status = HJO_ST_DIVERGED, iters = 0, att = 0;
            int64_t fwd = 0, bwd = 0;
            for (int r = 0; r <= R; ++r) {
                const double *v0 = guesses + (((size_t)b * G + g) * (R + 1) + r) * n;
                memcpy(v, v0, sizeof(double) * n);
                double phi, rho;
                int32_t it;
                int32_t st = hjo_descend(P, O, xb, v, &phi, &rho, &it, &fwd, &bwd);
                iters += it;
                att = r + 1;
                int finite = (st != HJO_ST_DIVERGED) && isfinite(phi);
                int certified = finite && (rho <= O->cert_tol);
                if (certified || (finite && (best_cert < 0 || phi < best_phi))) {
                    best_phi = phi;
                    best_rho = rho;
                    best_cert = certified ? 1 : 0;
                    best_status = st;
                    memcpy(slot_v + (size_t)g * n, v, sizeof(double) * n);
                }
                if (certified)
                    break;
            }
            if (best_cert < 0) {
                for (int i = 0; i < n; ++i)
                    slot_v[(size_t)g * n + i] = NAN;
            }
            slot_phi[g] = best_phi;
            slot_cert[g] = best_cert;
            if (diag) {
                size_t k = (size_t)b * G + g;
                if (diag->phi) diag->phi[k] = best_phi;
                if (diag->rho) diag->rho[k] = best_rho;
                if (diag->status) diag->status[k] = best_status;
                if (diag->cert) diag->cert[k] = best_cert;
                if (diag->iters) diag->iters[k] = iters;
                if (diag->attempts) diag->attempts[k] = att;
                if (diag->n_fwd) diag->n_fwd[k] = fwd;
                if (diag->n_bwd) diag->n_bwd[k] = bwd;
                if (diag->v_final)
                    memcpy(diag->v_final + k * n, slot_v + (size_t)g * n, sizeof(double) * n);
            }
        }
        /* selection over slots: certified first, then finite; lowest
         * objective; ties go to the lowest slot index */
        int pick = -1, pick_cert = -1;
        for (int g = 0; g < G; ++g) {
            if (slot_cert[g] < 0)
                continue;
            if (slot_cert[g] > pick_cert
                || (slot_cert[g] == pick_cert && slot_phi[g] < slot_phi[pick])) {
                pick = g;
                pick_cert = slot_cert[g];
            }
        }
        if (pick < 0) {
            out_u[b] = NAN;
            for (int i = 0; i < n; ++i)
                out_argopt[(size_t)b * n + i] = NAN;
            out_cert[b] = -1;
        } else {
            double phi = slot_phi[pick];
            out_u[b] = (P->formula == HJO_LAX) ? phi : -phi;
            memcpy(out_argopt + (size_t)b * n, slot_v + (size_t)pick * n, sizeof(double) * n);
            out_cert[b] = pick_cert;
        }
    }
    free(v);
    free(slot_v);
    free(slot_phi);
    free(slot_cert);
    return 0;
}
