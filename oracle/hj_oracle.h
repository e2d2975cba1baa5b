/*
 * hj_oracle.h -- plain, slow, single-threaded FP64 reference of the
 * generalized Lax / Hopf solver of Chow, Darbon, Osher and Yin,
 * "Algorithm for overcoming the curse of dimensionality for state-dependent
 * Hamilton-Jacobi equations" (arXiv:1704.02524).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU product
 * path.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no header, helper or table with the GPU
 * library; its only shared input is the seeded workload generator, which holds
 * none of the method's arithmetic.
 *
 * Notation (paper section 4, "Numerical methods"):
 *   H(x,p)  = <A x, p> + 1/2 m(r) sum_i d_i p_i^2 + 1/2 w r,   r = |x|^2,
 *   m = c^e, c in {1, 1 + kappa r/(1+r), 1 + kappa tanh(r/s)},
 *   g(x)    = 1/2 sum_i x_i^2 / a_i^2 + j0        (ellipsoid initial data),
 *   g*(p)   = 1/2 sum_i a_i^2 p_i^2 - j0           (its convex conjugate).
 * The bi-characteristic final-value problem gamma(t) = x, p(t) = v is solved
 * in reversed time tau = t - s with classical RK4 on N uniform steps.
 * Lax objective  F(v) = g(gamma(0)) + int_0^t <p, H_p> - H ds     (minimised)
 * Hopf objective G(v) = g*(p(0)) + int_0^t H - <H_x, gamma> ds - <x, v>
 *                 (minimised; the Hopf value is -min G).
 */
#ifndef HJ_ORACLE_H
#define HJ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HJO_M_CONST = 0, HJO_M_RAT = 1, HJO_M_TANH = 2 };
enum { HJO_LAX = 0, HJO_HOPF = 1 };
enum { HJO_TRAPZ = 0, HJO_RK4AUG = 1 };
enum { HJO_CD_FD = 0, HJO_GD = 1 };

/* Per-slot stop status of one descent run. */
enum {
    HJO_ST_MAXITER   = 0,  /* iteration cap reached                        */
    HJO_ST_CONVERGED = 1,  /* a whole iteration moved less than eps_step    */
    HJO_ST_STALLED   = 2,  /* step size fell below alpha0 * 2^-40          */
    HJO_ST_DIVERGED  = 3   /* objective not finite or |v|_inf > v_max      */
};

typedef struct {
    int32_t n;          /* space dimension d                               */
    int32_t m_kind;     /* HJO_M_*                                         */
    int32_t e;          /* exponent of c in m = c^e (1 or 2)               */
    int32_t formula;    /* HJO_LAX or HJO_HOPF                             */
    int32_t quad;       /* HJO_TRAPZ or HJO_RK4AUG                         */
    int32_t nsteps;     /* N, number of RK4 steps                          */
    double  kappa;      /* amplitude of the state dependence of c          */
    double  s;          /* tanh scale                                      */
    double  w;          /* coefficient of the 1/2 w |x|^2 potential        */
    double  t;          /* horizon                                         */
    double  j0;         /* constant of the ellipsoid initial data          */
    const double *d;    /* [n]   signs / weights of the kinetic term       */
    const double *A;    /* [n*n] row-major drift matrix, or NULL           */
    const double *a;    /* [n]   ellipsoid semi-axes                       */
} hjo_problem;

typedef struct {
    int32_t mode;       /* HJO_CD_FD or HJO_GD                             */
    int32_t max_iter;   /* sweeps (CD_FD) or steps (GD)                    */
    int32_t R_max;      /* restarts per slot after the first attempt       */
    int32_t pad_;
    double  alpha0;     /* initial step size                               */
    double  fd_sigma;   /* central finite-difference step                  */
    double  eps_step;   /* stop when an iteration's largest move is below  */
    double  cert_tol;   /* certificate tolerance on rho                    */
    double  v_max;      /* divergence bound on |v|_inf                     */
    double  acc_rel;    /* relative rounding allowance of the ascent test  */
    double  armijo_c;   /* required decrease fraction (0: plain ascent test) */
} hjo_opts;

/* Scalars m, m', m'' of the state-dependent speed as functions of r. */
void hjo_scalars(const hjo_problem *P, double r, double *m, double *m1, double *m2);

/* H(gamma, p). */
double hjo_hamiltonian(const hjo_problem *P, const double *gam, const double *p);

/* Reversed-time vector field f(gamma,p) = (-H_p, +H_x); out is [2n]. */
void hjo_field(const hjo_problem *P, const double *gam, const double *p, double *out);

/* Integrand of the action: Lax <p,H_p> - H, Hopf H - <H_x, gamma>. */
double hjo_integrand(const hjo_problem *P, const double *gam, const double *p);

/* RK4 trajectory y_0..y_N, traj is [(N+1) * 2n] with y_k = (gamma, p). */
void hjo_trajectory(const hjo_problem *P, const double *x, const double *v, double *traj);

/* Objective Phi(v) (F for Lax, G for Hopf) and the end state y_N ([2n]). */
double hjo_eval(const hjo_problem *P, const double *x, const double *v, double *yN);

/* Exact derivative of the discrete objective along (dx, dv): forward mode. */
double hjo_eval_tangent(const hjo_problem *P, const double *x, const double *v,
                        const double *dx, const double *dv, double *dphi);

/* Gradient of the discrete objective by n forward-mode sweeps per input. */
double hjo_grad_tangent(const hjo_problem *P, const double *x, const double *v,
                        double *grad_v, double *grad_x);

/* Gradient of the discrete objective by one reverse (adjoint) sweep. */
double hjo_grad_reverse(const hjo_problem *P, const double *x, const double *v,
                        double *grad_v, double *grad_x);

/* Certificate residual rho at the end state: Lax |p_N - grad g(gamma_N)|_inf,
 * Hopf |gamma_N - grad g*(p_N)|_inf. */
double hjo_certificate(const hjo_problem *P, const double *yN);

/* One descent run from v (in/out).  Returns the status; fills phi, rho,
 * iteration count, and the numbers of forward solves and adjoint sweeps. */
int32_t hjo_descend(const hjo_problem *P, const hjo_opts *O, const double *x,
                    double *v, double *phi, double *rho, int32_t *iters,
                    int64_t *n_fwd, int64_t *n_bwd);

/* Per-slot diagnostics of a solve; every pointer may be NULL.  Arrays are
 * [B, G] (v_final is [B, G, n]) and indexed by absolute point b. */
typedef struct {
    double  *phi;       /* objective of the slot's reported attempt        */
    double  *rho;       /* its certificate residual                        */
    int32_t *status;    /* its HJO_ST_* stop status                        */
    int32_t *cert;      /* 1 certified, 0 finite but uncertified, -1 none  */
    int32_t *iters;     /* iterations summed over all attempts             */
    int32_t *attempts;  /* attempts used (1 .. R_max+1)                    */
    int64_t *n_fwd;     /* forward solves summed over all attempts         */
    int64_t *n_bwd;     /* adjoint sweeps summed over all attempts         */
    double  *v_final;   /* the slot's reported v                           */
} hjo_slot_diag;

/* Full solve over points [b0, b1) of B points.
 *   x        [B, n]
 *   guesses  [B, G, R_max+1, n]  attempt r of slot g starts at guesses[b,g,r]
 *   out_u [B], out_argopt [B, n], out_cert [B]  (indexed by absolute b)
 * Returns 0, or -1 on invalid arguments. */
int32_t hjo_solve(const hjo_problem *P, const hjo_opts *O, const double *x,
                  int64_t B, int64_t b0, int64_t b1, const double *guesses, int32_t G,
                  double *out_u, double *out_argopt, int32_t *out_cert,
                  const hjo_slot_diag *diag);

#ifdef __cplusplus
}
#endif
#endif
