/*
 * hj.h -- C interface of the MI355X (gfx950) solver for state-dependent
 * Hamilton-Jacobi equations by the generalized Lax and Hopf formulas of
 * Chow, Darbon, Osher and Yin (arXiv:1704.02524).
 *
 * Problem (paper section 2.1, eqs. HJeqn / HJinitial): find phi(x, t) with
 *     phi_t + H(x, grad phi) = 0,   phi(x, 0) = g(x),
 * for the Hamiltonian family
 *     H(x, p) = <A x, p> + 1/2 m(|x|^2) sum_i d_i p_i^2 + 1/2 w |x|^2,
 *     m = c^e,  c = 1 | 1 + kappa r/(1+r) | 1 + kappa tanh(r/s),  r = |x|^2,
 * and ellipsoid initial data g(x) = 1/2 sum_i x_i^2 / a_i^2 + j0, whose
 * conjugate is g*(p) = 1/2 sum_i a_i^2 p_i^2 - j0.
 *
 * Method (sections 3.3, 3.4, 4): for each query x and each initial guess v,
 * integrate the bi-characteristics gamma' = H_p, p' = -H_x backward from
 * gamma(t) = x, p(t) = v with classical RK4 on nsteps uniform steps, add the
 * action integral by a quadrature rule, and minimise over v
 *   Lax  (convex H):      F(v) = g(gamma(0)) + int_0^t <p, H_p> - H ds,
 *                          phi = min F;
 *   Hopf (convex g):      G(v) = g*(p(0)) + int_0^t H - <H_x, gamma> ds - <x, v>,
 *                          phi = -min G;
 * by cyclic coordinate descent with central differences (Algorithm 1 with
 * step halving on ascent) or by gradient descent with the exact gradient of
 * the discretised objective (a discrete adjoint with RK4 checkpoints).  The
 * certificate of section 4.3 (Lax: p(0) = grad g(gamma(0)); Hopf, dual form:
 * gamma(0) = grad g*(p(0))) accepts a result; a run that fails it restarts
 * from the next guess (section 5: multiple random guesses).  The optimiser v
 * is reported as argopt, the spatial gradient of phi where phi is smooth
 * (section 1).
 *
 * Conventions for every entry point:
 *  - Device arrays are caller-owned device pointers (hipMalloc'd or torch
 *    tensors' data_ptr()), row-major and contiguous; "dtype" arrays hold
 *    double for HJ_F64 and float for HJ_F32.
 *  - Parameter arrays inside hj_h_params / hj_j_params are HOST pointers to
 *    double and are copied during the call.
 *  - Work is enqueued on opts->stream (a hipStream_t; NULL = the null stream)
 *    and the call returns without waiting for the device: the parameter
 *    arrays are passed to the device inside kernel arguments, so the host
 *    memory they occupy may be reused as soon as the call returns.  Results
 *    are valid once that stream has completed.  Scratch memory comes from
 *    opts->workspace when it is given (ws_bytes >= hj_workspace_size), else
 *    from an allocation the library caches per device and grows as needed
 *    (growing it waits for the device once); calls that share that cache
 *    must be ordered on one stream.
 *  - Return value: HJ_OK (0) or a negative HJ_E* code; the message of the
 *    last error on the calling thread is returned by hj_last_error().  No
 *    entry point aborts the process.
 */
#ifndef HJ_H
#define HJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HJ_VERSION 1

/* return codes */
#define HJ_OK            0
#define HJ_EINVAL       -1  /* bad size, count or pointer                   */
#define HJ_EDTYPE       -2  /* unknown dtype                                */
#define HJ_ENOMEM       -3  /* workspace too small or allocation failed     */
#define HJ_EDEVICE      -4  /* a HIP call failed                            */
#define HJ_EUNSUPPORTED -5  /* valid but not built (e.g. n above the limit) */

#define HJ_MAX_G    64      /* guesses per point                            */
#define HJ_MAX_N   128      /* space dimension                              */
#define HJ_MAX_N_DRIFT 64   /* space dimension with a drift matrix A        */

/* H_kind: the quadratic family above, or the degree-1 homogeneous family
 * of section 5 Examples 3 and 5,
 *     H(x, p) = s1 c1(x) |p_A| + s2 c2(x) |p_B|,  A = {1..k}, B = {k+1..n},
 *     c1(x) = c0 (1 + beta exp(-gam |x - mu|^2)), c2(x) = c1(-x) with the
 *     same constants (the zero subgradient where p_A or p_B vanishes). */
enum { HJ_H_QUADRATIC = 0, HJ_H_NORM = 1 };
/* J_kind: the ellipsoid g above, or the Rosenbrock initial data of section 5
 * Example 2 (eq. weird), n = 2 and Lax functionals only:
 *     g(x) = rscale (-100 + (1 - x_1)^2 + 100 (1 + x_2 - x_1^2)^2). */
enum { HJ_J_ELLIPSOID = 0, HJ_J_ROSENBROCK = 1 };
enum { HJ_M_CONST = 0, HJ_M_RAT = 1, HJ_M_TANH = 2 };
/* formula: the Lax functional F1, the Hopf functional G, or the grid-minimum
 * functional F2(v) = min_k g(gamma_k) over the characteristic's nodes
 * (section 4.1, eq. num_min; minimised, phi = min F2) */
enum { HJ_LAX = 0, HJ_HOPF = 1, HJ_LAX_MIN = 2 };
enum { HJ_TRAPZ = 0, HJ_RK4AUG = 1 };     /* trapezoid on the RK4 nodes, or
                                             RK4 applied to a' = integrand */
/* descent: central-difference coordinate descent with step halving on
 * insufficient decrease, adjoint gradient descent, Algorithm 1 of section
 * 4.1 read literally (forward differences, eq. num_diff; no acceptance test;
 * alpha halved every M coordinate updates; stop after n consecutive moves
 * below eps_step), or heavy-ball descent on forward differences
 * (v' = v - alpha g + momentum (v - v_prev), a rising trial rejected with
 * the momentum dropped and alpha halved) */
enum { HJ_CD_FD = 0, HJ_GD_ADJ = 1, HJ_ALG1 = 2, HJ_MOMENTUM = 3 };
/* characteristic ODE: classical RK4, forward Euler with the rectangle
 * rule h sum_{k<N} integrand(y_k) (section 4.2, eq. num_int), or the
 * staggered discrete forms of the section 3 lemmas (eqs. hahalolXDform and
 * hahalolXDform2: one half of each step explicit, the other implicit and
 * solved by fixed-point iteration to 1e-14 (1 + |z|) or 60 sweeps; the
 * value is the discrete functional itself, and the Lax certificate compares
 * grad g(x_0) with p_0 + delta H_x(x_0, p_0), the Hopf one x_0 with
 * a^2 p_1) */
enum { HJ_RK4 = 0, HJ_EULER = 1, HJ_STAGGERED = 2 };
enum { HJ_F64 = 0, HJ_F32 = 1 };
/* stop status of one descent run */
enum { HJ_ST_MAXITER = 0, HJ_ST_CONVERGED = 1, HJ_ST_STALLED = 2, HJ_ST_DIVERGED = 3 };

typedef struct {
    int32_t m_kind;       /* HJ_M_*                                        */
    int32_t e;            /* 1 or 2: m = c^e                               */
    double  kappa;        /* amplitude of the state dependence of c        */
    double  s;            /* tanh scale (HJ_M_TANH), > 0                   */
    double  w;            /* potential 1/2 w |x|^2                         */
    const double *d;      /* host [n] kinetic weights (usually +-1)        */
    const double *A;      /* host [n*n] row-major drift (finite), or NULL.
                             With A the kernels run on the matrix cores:
                             n <= HJ_MAX_N_DRIFT, 4 lanes per task, not in
                             batched plans (HJ_EUNSUPPORTED otherwise)     */
    /* HJ_H_NORM only (d, m_kind, e, kappa, s, w and A are then unused)    */
    int32_t k;            /* size of block A, 0..n                         */
    double  s1, s2;       /* signs (or weights) of the two blocks          */
    double  c0, beta, gam;
    const double *mu;     /* host [n] centre of the bump                   */
} hj_h_params;

typedef struct {
    const double *a;      /* host [n] ellipsoid semi-axes, nonzero (may be
                             NULL for HJ_J_ROSENBROCK)                      */
    double j0;
    double rscale;        /* HJ_J_ROSENBROCK: the factor r                 */
} hj_j_params;

typedef struct {
    int32_t G;            /* guesses (slots) per point, 1..HJ_MAX_G        */
    int32_t R_max;        /* restarts per slot after the first attempt     */
    const void *init;     /* device dtype [B, G, R_max+1, n]: attempt r of
                             slot g at point b starts at init[b, g, r, :]  */
} hj_guesses;

typedef struct {
    int32_t dtype;        /* HJ_F64 or HJ_F32: descent arithmetic          */
    int32_t formula;      /* HJ_LAX or HJ_HOPF                             */
    int32_t mode;         /* HJ_CD_FD or HJ_GD_ADJ                         */
    int32_t quad;         /* HJ_TRAPZ or HJ_RK4AUG                         */
    int32_t max_iter;     /* sweeps (CD_FD) or gradient steps (GD_ADJ)     */
    int32_t ckpt_K;       /* adjoint checkpoint interval in steps (>= 1)   */
    int32_t cert_fp64;    /* HJ_F32: re-evaluate objective and certificate
                             in FP64 at each run's final v                 */
    int32_t lanes_per_task; /* 0: the library's choice; else 1, 2, 4, 8 or
                             16 lanes of a wavefront share one (point,
                             guess) task, each holding ceil(n / lanes)
                             components (HJ_EUNSUPPORTED if no such
                             kernel is built)                              */
    double  alpha0;       /* initial step size (1/L of Algorithm 1)        */
    double  fd_sigma;     /* central-difference step                       */
    double  eps_step;     /* stop when an iteration's largest move < this  */
    double  cert_tol;     /* certified iff residual <= cert_tol            */
    double  v_max;        /* diverged when |v|_inf exceeds this            */
    double  acc_rel;      /* rounding allowance of the step test (below)   */
    double  armijo_c;     /* a trial step v' = v - alpha d is accepted iff
                             F(v') <= F(v) - armijo_c alpha <g, d> + acc_rel |F(v)|
                             with g the (FD or exact) gradient; else alpha
                             is halved.  armijo_c = 0: halve on ascent.   */
    void   *stream;       /* hipStream_t                                   */
    void   *workspace;    /* optional device scratch                       */
    size_t  ws_bytes;
    void   *ev_begin;     /* optional hipEvent_t recorded on the stream just
                             before the descent (or evaluation) kernel     */
    void   *ev_end;       /* optional hipEvent_t recorded just after it    */
    int32_t schedule;     /* HJ_SCHED_*: how (point, guess) tasks reach the
                             lanes                                          */
    int32_t max_groups;   /* persistent schedule: at most this many lane
                             groups (0: as many as the device holds)       */
    int32_t fp64_continue; /* HJ_F32 with cert_fp64 and HJ_GD_ADJ: a slot
                             whose FP32 attempt ends finite but fails the
                             FP64 certificate continues in FP64 -- gradient
                             descent from that attempt's v (step reset to
                             alpha0, up to max_iter iterations), then FP64
                             restarts from its remaining guesses -- in a
                             second launch over the handed-off slots only.
                             0: the FP32 attempts alone decide.            */
    int32_t ode;          /* HJ_RK4, HJ_EULER or HJ_STAGGERED              */
    int32_t M;            /* HJ_ALG1: alpha halves every M updates (>= 1)  */
    double  momentum;     /* HJ_MOMENTUM: the heavy-ball coefficient       */
    /* hj_batch_plan only: launch choices by dimension class (NULL: the
     * options above for every instance); an instance takes the first entry
     * with n <= n_max */
    const struct hj_group_cfg_s *group_cfg;
    int32_t n_group_cfg;
    /* FP32 with fp64_continue: lanes per task of the FP64 continuation
     * launch (0: those of the descent).  The shape must have the descent
     * shape's padded dimension; the continuation runs few, long tasks, so
     * more lanes per task shorten them.  HJ_EUNSUPPORTED if not compiled. */
    int32_t cont_lanes_per_task;
    /* hj_solve, FP64 adjoint descent (HJ_GD_ADJ) of one problem without a
     * drift matrix: a slot still descending after tail_budget objective
     * evaluations (0: never) is handed, with its whole descent state (v,
     * gradient, step size, iteration and attempt counts, best attempt), to
     * a second launch of tail_lanes_per_task lanes per task (0: 2), which
     * resumes it exactly where it stopped.  The slow tail of the slots then
     * runs on wider lane groups instead of holding a one-lane wave for the
     * whole launch.  Results equal those without the hand-off up to the
     * rounding of the wider shape's sums (bit for bit with the descent's own
     * lanes per task).  The continuation takes the library's shape for n
     * with that many lanes (its own parameter rows where its padded
     * dimension differs); shapes of more than 4 lanes per task, FP32, other
     * descent modes, drift and batch plans are HJ_EUNSUPPORTED.  Adds
     * (14 + 2n) x 8 bytes per slot and the continuation's checkpoints to the
     * workspace. */
    int32_t tail_budget;
    int32_t tail_lanes_per_task;
} hj_opts;

/* Launch choices of the instances up to a dimension (an autotuner's table):
 * lanes per task (0: the library's shape for n; with FP32 the shape also
 * fixes one or two waves per SIMD), checkpoint interval (0: opts->ckpt_K),
 * lane groups of the persistent launch (0: opts->max_groups), lanes per
 * task of the FP64 continuation (0: opts->cont_lanes_per_task). */
typedef struct hj_group_cfg_s {
    int32_t n_max;
    int32_t lanes_per_task;
    int32_t ckpt_K;
    int32_t max_groups;
    int32_t cont_lanes_per_task;
} hj_group_cfg;

enum {
    HJ_SCHED_AUTO = 0,       /* persistent when tasks outnumber resident lanes */
    HJ_SCHED_STATIC = 1,     /* one task per lane group                       */
    HJ_SCHED_PERSISTENT = 2  /* resident lane groups pop tasks from a queue;
                                scratch is sized by resident lanes only      */
};

/* Optional per-slot outputs, device pointers, each NULL or [B, G] (v_final
 * [B, G, n] in dtype).  A slot's reported attempt is its first certified
 * one, else its finite attempt with the lowest objective. */
typedef struct {
    double  *phi;         /* objective of the reported attempt (FP64)      */
    double  *rho;         /* its certificate residual (FP64)               */
    int32_t *status;      /* its HJ_ST_* stop status                       */
    int32_t *cert;        /* 1 certified, 0 finite uncertified, -1 none    */
    int32_t *iters;       /* iterations over all attempts                  */
    int32_t *attempts;    /* attempts used                                 */
    int64_t *n_fwd;       /* forward solves over all attempts              */
    int64_t *n_bwd;       /* adjoint sweeps over all attempts              */
    void    *v_final;     /* the reported attempt's v                      */
} hj_slot_diag;

/* The paper's scheme and families run in a kernel of their own: a solve
 * with mode HJ_ALG1 or HJ_MOMENTUM (the only modes for HJ_H_NORM,
 * HJ_J_ROSENBROCK, HJ_LAX_MIN, HJ_EULER or HJ_STAGGERED) takes FP64, no
 * drift matrix,
 * n <= 16, one lane per (point, guess) (lanes_per_task and the schedule are
 * ignored) and the RK4-augmented rule with HJ_RK4; other combinations are
 * HJ_EUNSUPPORTED.  hj_eval evaluates these functionals without gradients. */

/* hj_solve -- phi(x_b, t) for B query points (sections 3.3-3.4, Algorithm 1,
 * certificate of section 4.3, multiple guesses of section 5).
 *   x          device dtype [B, n]
 *   out_u      device double [B]: phi (Lax: min F; Hopf: -min G)
 *   out_argopt device dtype [B, n]: the selected v (grad_x phi)
 *   out_cert   device int32 [B]: 1 certified; 0 no slot certified, u and
 *              argopt from the finite slot with the lowest objective;
 *              -1 no finite slot (u = NaN)
 *   diag       optional per-slot outputs (NULL for none)
 * Selection: among certified slots the lowest objective, ties to the lowest
 * slot index.  B = 0 is a no-op.  Errors: HJ_EINVAL for n < 1, nsteps < 1,
 * t <= 0, G outside [1, HJ_MAX_G], R_max < 0, max_iter < 0, NULL arrays,
 * non-finite drift entries; HJ_EUNSUPPORTED for n > HJ_MAX_N, an unknown
 * H_kind / J_kind, or a drift matrix with n > HJ_MAX_N_DRIFT or
 * lanes_per_task other than 0 or 4. */
int32_t hj_solve(int32_t H_kind, const hj_h_params *H, int32_t J_kind, const hj_j_params *J,
                 const void *x, int64_t B, int32_t n, double t, int32_t nsteps,
                 const hj_guesses *guesses, const hj_opts *opts,
                 double *out_u, void *out_argopt, int32_t *out_cert,
                 const hj_slot_diag *diag);

/* hj_solve_noalloc -- hj_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, checks and results as hj_solve; the
 * scratch memory is a fixed array of HJ_NOALLOC_BYTES that the library holds
 * on every device it runs on (until the process ends), so the call allocates
 * nothing.  opts->workspace must be NULL.  When the requested schedule needs
 * more scratch than the array holds, the solve runs persistent with fewer
 * lane groups (results are identical); when even 64 groups do not fit (the
 * per-slot records grow with B * G), the call returns HJ_ENOMEM with the
 * needed size in hj_last_error().  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (different streams, different threads) race, so order them on one
 * stream. */
#define HJ_NOALLOC_BYTES ((size_t)64 << 20)
int32_t hj_solve_noalloc(int32_t H_kind, const hj_h_params *H, int32_t J_kind,
                         const hj_j_params *J, const void *x, int64_t B, int32_t n, double t,
                         int32_t nsteps, const hj_guesses *guesses, const hj_opts *opts,
                         double *out_u, void *out_argopt, int32_t *out_cert,
                         const hj_slot_diag *diag);

/* hj_eval -- the discretised objective at given v (section 4.2) and,
 * optionally, its exact gradient by the discrete adjoint of the RK4 solve
 * and the quadrature.
 *   x          device dtype [B, n];  v  device dtype [B, G, n]
 *   out_phi    device double [B, G]: F (Lax) or G (Hopf)
 *   out_yN     device dtype [B, G, 2n] or NULL: (gamma(0), p(0))
 *   out_rho    device double [B, G] or NULL: certificate residual
 *   out_grad_v device dtype [B, G, n] or NULL: d objective / d v
 *   out_grad_x device dtype [B, G, n] or NULL: d objective / d x
 * opts supplies dtype, formula, quad, ckpt_K, stream and workspace. */
int32_t hj_eval(int32_t H_kind, const hj_h_params *H, int32_t J_kind, const hj_j_params *J,
                const void *x, int64_t B, int32_t n, double t, int32_t nsteps,
                const void *v, int32_t G, const hj_opts *opts,
                double *out_phi, void *out_yN, double *out_rho,
                void *out_grad_v, void *out_grad_x);

/* hj_lax_friedrichs -- the independent grid check of section 5: the
 * first-order Lax-Friedrichs scheme for phi_t + H(x, grad phi) = 0,
 * phi(x, 0) = g(x), in two space dimensions, on the grid x_i = x0 + i dx
 * (i < nx), y_j = y0 + j dy (j < ny), nt forward-Euler steps of dt with the
 * numerical Hamiltonian H(x, (D+x + D-x)/2, (D+y + D-y)/2) - ax (D+x -
 * D-x)/2 - ay (D+y - D-y)/2 (one-sided differences, linear extrapolation
 * across the boundary).  ax, ay bound |dH/dp_1|, |dH/dp_2| (stability:
 * dt (ax/dx + ay/dy) <= 1).  H: HJ_H_QUADRATIC without drift, n = 2; g:
 * either J kind.
 *   phi   device double [ny, nx]: the solution at t = nt dt (row j is y_j)
 *   work  device double [ny, nx] scratch, or NULL (the library's scratch)
 * Enqueued on `stream`; errors as in hj_solve. */
int32_t hj_lax_friedrichs(int32_t H_kind, const hj_h_params *H, int32_t J_kind,
                          const hj_j_params *J, double x0, double y0, double dx, double dy,
                          int32_t nx, int32_t ny, double dt, int32_t nt, double ax, double ay,
                          double *phi, double *work, void *stream);

/* One problem instance of a batched solve (all device arrays as in
 * hj_solve; H and J parameter arrays are host pointers copied at planning). */
typedef struct {
    int32_t      n;
    double       t;
    int32_t      nsteps;
    hj_h_params  H;
    hj_j_params  J;
    const void  *x;           /* device dtype [B, n]                        */
    int64_t      B;
    hj_guesses   guesses;     /* G, R_max, device init [B, G, R_max+1, n]  */
    double      *out_u;       /* device [B]                                 */
    void        *out_argopt;  /* device dtype [B, n]                        */
    int32_t     *out_cert;    /* device [B]                                 */
    hj_slot_diag diag;        /* optional per-slot outputs (NULL members)   */
} hj_instance;

typedef struct hj_batch_plan_s *hj_batch;

/* hj_batch_plan -- prepare a batched solve of n_inst independent problems
 * of uneven dimension, horizon, step count and point count (the method of
 * hj_solve applied to each).  Instances are grouped by lane shape (from n,
 * or from the opts->group_cfg entry covering n), speed profile and launch
 * choices; each group runs as ONE persistent launch whose resident
 * lane groups take (instance, point, guess) tasks from a queue, longest
 * instances first, and a finished group takes the next task.  The whole
 * sequence (queue resets, the descent launches, the selection) is captured
 * into a hipGraph that hj_batch_run replays, the shape groups as parallel
 * branches (they share no memory; one stream per group is created for the
 * capture, at the default priority); device pointers are fixed at
 * planning, their contents may change between runs.  opts supplies the
 * shared options (formula, quadrature, dtype, iterations, tolerances; mode
 * must be HJ_GD_ADJ).  The plan owns its device scratch.  Errors as in
 * hj_solve; *out is set on success. */
int32_t hj_batch_plan(int32_t H_kind, int32_t J_kind, const hj_instance *inst, int32_t n_inst,
                      const hj_opts *opts, hj_batch *out);

/* Enqueue the planned solve on `stream` (a hipStream_t, NULL = null stream). */
int32_t hj_batch_run(hj_batch plan, void *stream);

/* Tasks, lane groups launched, and launches (lane-shape groups) of a plan. */
int32_t hj_batch_info(hj_batch plan, int64_t *tasks, int64_t *groups, int32_t *launches);

/* Release a plan (waits for its work to finish). */
int32_t hj_batch_free(hj_batch plan);

/* Scratch bytes hj_solve / hj_eval need for B points of G slots, with the
 * schedule hj_solve picks on the current device (persistent launches hold
 * checkpoints for resident lane groups only). */
size_t hj_workspace_size(int32_t n, int64_t B, int32_t G, int32_t nsteps,
                         const hj_opts *opts);

/* Message of the last error on the calling thread ("" when none). */
const char *hj_last_error(void);

/* HJ_VERSION of the library. */
int32_t hj_version(void);

#ifdef __cplusplus
}
#endif
#endif
