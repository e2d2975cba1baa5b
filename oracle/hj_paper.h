/*
 * hj_paper.h -- plain, slow, single-threaded FP64 reference of the paper's
 * own scheme and of its further problem families (arXiv:1704.02524):
 *
 *  - the paper's scheme: forward Euler characteristics in reversed time with
 *    the rectangle rule for the action (section 4.2, eq. num_int), forward
 *    differences for derivatives (eq. num_diff), and Algorithm 1 (section
 *    4.1: cyclic coordinate descent with alpha = 1/L halved every M
 *    coordinate updates, stopped after d consecutive moves below epsilon);
 *    or the staggered discrete Lax and Hopf forms of the section 3 lemmas
 *    (eqs. hahalolXDform, hahalolXDform2) in place of Euler and the
 *    rectangle rule;
 *  - degree-1 homogeneous Hamiltonians (section 5 Examples 3 and 5)
 *        H(x, p) = s1 c1(x) |p_A| + s2 c2(x) |p_B|,
 *        A = {1..k}, B = {k+1..n}, c_i(x) = c0 (1 + beta exp(-gam |x - mu_i|^2)),
 *        mu_1 = mu, mu_2 = -mu,
 *    and the grid-minimum functional F2(v) = min_i g(gamma_i) (section 4.1,
 *    its grid form eq. num_min);
 *  - the Rosenbrock initial data of section 5 Example 2 (eq. weird)
 *        g(x) = r (-100 + (1 - x_1)^2 + 100 (1 + x_2 - x_1^2)^2),  n = 2;
 *  - heavy-ball momentum descent (section 5 Example 5 suggests momentum for
 *    trench-shaped functionals);
 *  - a first-order Lax-Friedrichs grid solver for two space dimensions, the
 *    independent check the paper compares against (section 5).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library.  The quadratic family (m, d, w) is the one of hj_oracle.h.
 */
#ifndef HJ_PAPER_H
#define HJ_PAPER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HJP_H_QUADRATIC = 0, HJP_H_NORM = 1 };
enum { HJP_J_ELLIPSOID = 0, HJP_J_ROSENBROCK = 1 };
enum { HJP_LAX = 0, HJP_HOPF = 1, HJP_LAX_MIN = 2 };   /* F1, G, F2 */
enum { HJP_RK4 = 0, HJP_EULER = 1, HJP_STAGGERED = 2 };  /* ODE + quadrature */
enum { HJP_ALG1 = 0, HJP_MOMENTUM = 1 };                /* descent */
enum { HJP_ST_MAXITER = 0, HJP_ST_CONVERGED = 1, HJP_ST_STALLED = 2, HJP_ST_DIVERGED = 3 };

typedef struct {
    int32_t n, hkind, jkind, functional, ode, nsteps;
    double t;
    /* quadratic family: H = 1/2 m(|x|^2) sum d_i p_i^2 + 1/2 w |x|^2, m = c^e */
    int32_t m_kind, e;            /* 0 const, 1 1 + kappa r/(1+r), 2 1 + kappa tanh(r/s) */
    double kappa, s, w;
    const double *d;              /* [n] */
    /* norm family */
    int32_t k;                    /* split A = {0..k-1}, B = {k..n-1} */
    double s1, s2, c0, beta, gam;
    const double *mu;             /* [n] */
    /* initial data */
    const double *a;              /* [n] ellipsoid semi-axes */
    double j0;                    /* ellipsoid constant */
    double rscale;                /* Rosenbrock scale r */
} hjp_problem;

typedef struct {
    int32_t mode, max_iter, R_max, M;  /* M: alpha halves every M coordinate updates */
    double alpha0, fd_sigma, eps, cert_tol, v_max;
    double momentum, acc_rel;          /* heavy ball: beta, rounding allowance */
} hjp_opts;

double hjp_hamiltonian(const hjp_problem *P, const double *x, const double *p);
/* H_x and H_p; at p_A = 0 (or p_B = 0) the norm family takes the zero
 * subgradient for that block. */
void hjp_grads(const hjp_problem *P, const double *x, const double *p, double *Hx, double *Hp);
double hjp_g(const hjp_problem *P, const double *x);
void hjp_grad_g(const hjp_problem *P, const double *x, double *out);
/* The discrete objective (F1, G or F2) at v; the certificate residual in
 * *rho; the end state (or, for F2, the minimising grid state) in yN [2n]. */
double hjp_eval(const hjp_problem *P, const double *x, const double *v, double *rho,
                double *yN);
/* One descent run from v (in/out). */
int32_t hjp_descend(const hjp_problem *P, const hjp_opts *O, const double *x, double *v,
                    double *phi, double *rho, int32_t *iters, int64_t *n_eval);
/* Multi-start solve of points [0, B): guesses [B, G, R+1, n]; per-slot
 * outputs [B, G] may be NULL. */
int32_t hjp_solve(const hjp_problem *P, const hjp_opts *O, const double *x, int64_t B,
                  const double *guesses, int32_t G, double *out_u, double *out_argopt,
                  int32_t *out_cert, double *slot_phi, double *slot_rho, int32_t *slot_cert,
                  int32_t *slot_iters, int64_t *slot_eval);

/* Lax-Friedrichs solution of phi_t + H(x, grad phi) = 0, phi(., 0) = g, on
 * the grid x_i = x0 + i dx (i < nx), y_j = y0 + j dy (j < ny), n = 2, H of
 * the quadratic family, nt steps of dt; ax, ay are the artificial
 * viscosity coefficients (bounds of |H_p1|, |H_p2|).  phi [ny * nx], row j
 * at y_j. */
int32_t hjp_lax_friedrichs(const hjp_problem *P, double x0, double y0, double dx, double dy,
                           int32_t nx, int32_t ny, double dt, int32_t nt, double ax, double ay,
                           double *phi);

#ifdef __cplusplus
}
#endif
#endif
