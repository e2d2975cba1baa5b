// hj_launch.hpp -- kernel argument blocks, launcher declarations and the
// table of compiled lane shapes, shared by the host dispatch (hj_api.hip) and
// the instantiation units (hj_inst_*.hip).
#pragma once

#include "hj_device.hpp"

namespace hj {

// Per-slot result records (device arrays [B*G], v in [B*G, n]).
template <typename T> struct SlotOut {
  double* phi;
  double* rho;
  int32_t* status;
  int32_t* cert;
  int32_t* iters;
  int32_t* attempts;
  int64_t* n_fwd;
  int64_t* n_bwd;
  T* v;
};

// One problem instance of a batched solve (all instances of one launch share
// the lane shape, hence the component count per lane).
template <typename T> struct InstDesc {
  Problem<T> P;
  Problem<double> P64;
  const T* x;        // [B, n]
  const T* guesses;  // [B, G, R+1, n]
  int64_t B;
  int G, R;
  int64_t task0;     // global index of the instance's first task
  int64_t point0;    // global index of the instance's first point
  double* out_u;     // [B]
  T* out_arg;        // [B, n]
  int32_t* out_cert; // [B]
  SlotOut<T> diag;   // optional per-slot copies [B, G] (null members)
};

template <typename T> struct SolveArgs {
  Problem<T> P;
  Problem<double> P64;  // the same problem in FP64 (certificate of FP32 runs)
  const T* x;           // [B, n]
  const T* guesses;     // [B, G, R+1, n]
  int64_t B;
  int G, R;
  int max_iter, K;
  int cert_fp64;
  T alpha0, sigma, eps_step, acc_rel, armijo_c, v_max;
  double cert_tol;
  T* ck;                // adjoint checkpoints, SoA over `stride` lanes
  T* seg;               // adjoint segment scratch
  size_t stride;
  SlotOut<T> out;       // per-slot records, indexed by global task
  // work distribution: ntask tasks; with `queue` set, the launch is
  // persistent and a task group that finishes pops the next task index from
  // *queue (which must start at the number of task groups launched)
  int64_t ntask;
  unsigned long long* queue;
  // batched instances (nullptr: the single problem above)
  const InstDesc<T>* inst;
  int n_inst;
  // FP32 runs with an FP64 continuation (null otherwise): a slot whose FP32
  // attempt ends finite but rejected by the FP64 certificate is handed off,
  // its record written and its task index appended to `handoff`
  int64_t* handoff;                 // [ntask]
  unsigned long long* handoff_n;    // entries in handoff (starts at 0)
  // FP64 single-problem adjoint descent with a tail hand-off (0 / null
  // otherwise): a slot still descending after tail_budget objective
  // evaluations leaves its whole descent state in a record of `tail`
  // (kTailHead values, then v and g, tail_stride doubles per record; the
  // record index from *tail_n, which starts at 0), and a second launch of a
  // wider lane shape resumes it from there (RESUME: the records to resume
  // are tail[0 .. *tail_n), handed out through `queue`, which starts at 0)
  int tail_budget;
  int tail_stride;
  double* tail;
  unsigned long long* tail_n;
};

// Head of a tail record: task, iteration, attempt, alpha, phi, rho, then
// the slot's best attempt so far (phi, rho, cert, status, iterations,
// attempts, forward and adjoint counts); v and g follow.
constexpr int kTailHead = 14;

// FP64 continuation of the slots an FP32 launch handed off: each resumes the
// descent in FP64 from its FP32 result (then restarts in FP64 from its
// remaining guesses), and its record is updated in place.
template <typename TS> struct ContArgs {
  SolveArgs<TS> S;          // the FP32 launch: problems (P64 used), inputs,
                            // records, instance table, hand-off list
  int max_iter, K;
  double alpha0, eps_step, acc_rel, armijo_c, v_max;
  double* ck;               // FP64 adjoint checkpoints over `stride` lanes
  double* seg;
  size_t stride;
  unsigned long long* queue;  // next index into S.handoff (starts at 0)
};

template <typename T> struct EvalArgs {
  Problem<T> P;
  const T* x;   // [B, n]
  const T* v;   // [B, G, n]
  int64_t B;
  int G, K;
  double* phi;  // [B, G]
  double* rho;  // [B, G] or null
  T* yN;        // [B, G, 2n] or null
  T* gv;        // [B, G, n] or null
  T* gx;        // [B, G, n] or null
  T* ck;
  T* seg;
  size_t stride;
};

// The paper's scheme and families (hj_paper.hpp): the problem by value, n <=
// kPaperMaxN, padded components zero.
constexpr int kPaperMaxN = 16;

struct PaperProblem {
  int n, hkind, jkind, functional, ode, N, m_kind, e, k;
  double h, kappa, inv_s, w, s1, s2, c0, beta, gam, j0, rscale;
  double d[kPaperMaxN], a2[kPaperMaxN], ia2[kPaperMaxN], mu[kPaperMaxN];
};

struct PaperArgs {
  PaperProblem P;
  int mode, max_iter, R, G, M;
  double alpha0, sigma, eps, cert_tol, v_max, momentum, acc_rel;
  const double* x;        // [B, n]
  const double* guesses;  // [B, G, R+1, n]
  int64_t ntask;
  SlotOut<double> out;    // per-slot records [B * G]
};

// One lane per task over A.ntask tasks (hj_inst_paper.hip).
hipError_t launch_solve_paper(const PaperArgs& A, hipStream_t st);
// The functional at v [B, G, n]: phi and rho [B, G].
hipError_t launch_eval_paper(const PaperProblem& P, const double* x, const double* v, int64_t B,
                             int G, double* phi, double* rho, hipStream_t st);

// Lax-Friedrichs: nt steps from phi(., 0) = g on an nx x ny grid, ping-pong
// between phi and work; the result ends in phi.
hipError_t launch_lax_friedrichs(const PaperProblem& P, double x0, double y0, double dx,
                                 double dy, int nx, int ny, double dt, int nt, double ax,
                                 double ay, double* phi, double* work, hipStream_t st);

// Launch a descent kernel over A.ntask tasks.  grid_groups = 0: one task
// group per task (no queue); otherwise a persistent launch of grid_groups
// task groups fed by A.queue (reset by this call with a small kernel, so the
// sequence can be captured in a graph).
template <class C>
hipError_t launch_solve(const SolveArgs<typename C::T>& A, int mode, int64_t grid_groups,
                        hipStream_t st);
// Task groups the device holds at once for this kernel (occupancy x CUs).
template <class C>
int64_t resident_groups(int mode);
template <class C>
hipError_t launch_eval(const EvalArgs<typename C::T>& A, hipStream_t st);
// The FP64 continuation of an FP32 launch's hand-off list: grid_groups lane
// groups of the FP64 configuration C pop list indices from A.queue (reset to
// 0 by this call).  multi: the FP32 launch was batched.
template <class C>
hipError_t launch_continue(const ContArgs<float>& A, bool multi, int64_t grid_groups,
                           hipStream_t st);
template <class C>
int64_t resident_continue_groups();
// The continuation of a tail hand-off (FP64, one problem, no drift):
// grid_groups lane groups of configuration C pop indices of A.tail's
// *A.tail_n records from A.queue (reset to 0 by this call) and resume them.
template <class C>
hipError_t launch_resume(const SolveArgs<double>& A, int64_t grid_groups, hipStream_t st);
template <class C>
int64_t resident_resume_groups();
template <typename T>
hipError_t launch_select(int64_t B, int G, int n, int formula, const double* s_phi,
                         const int32_t* s_cert, const T* s_v, double* out_u, T* out_arg,
                         int32_t* out_cert, hipStream_t st);
// Selection for batched instances: total_points points over n_inst
// instances (each instance's points are [point0, point0 + B)).
template <typename T>
hipError_t launch_select_batched(const InstDesc<T>* inst, int n_inst, int64_t total_points,
                                 int n, int formula, const double* s_phi,
                                 const int32_t* s_cert, const T* s_v, hipStream_t st);
// Copy the per-slot records of a batched launch to the instances' diag arrays.
template <typename T>
hipError_t launch_scatter_diag(const InstDesc<T>* inst, int n_inst, int64_t total_tasks, int n,
                               SlotOut<T> rec, hipStream_t st);

// Lane shapes compiled for both arithmetic types and both speed profiles
// (components per lane NPL x lanes per task LPT), in order of preference
// for a given n when no shape is requested: the first entry whose NPL * LPT
// covers n.
struct Shape {
  int npl, lpt;
  bool dr = false;  // matrix-core layout with linear drift (lpt = 4)
  constexpr int npad() const { return npl * lpt; }
};
constexpr Shape kShapes[] = {
    {2, 1}, {4, 1}, {4, 2}, {5, 2}, {3, 4}, {4, 4}, {8, 4}, {8, 8}, {13, 8}, {16, 8},
    // alternatives reachable through an explicit lanes-per-task request
    {2, 2}, {8, 1}, {2, 4}, {10, 1}, {8, 2}, {4, 8}, {7, 16},
};
constexpr int kNumDefaultShapes = 10;
// FP32 default for 64 < n <= 112: 16 lanes of 7 components, whose descent
// kernel runs two waves per SIMD (the wider FP32 shapes run one)
constexpr Shape kF32Wide = {7, 16};
// Components per lane of the linear-drift (matrix-core) instances; the
// padded dimension 4 * NPL is a multiple of 16, the MFMA block size.
constexpr int kDriftNpl[] = {4, 8, 16};
static_assert(4 * kDriftNpl[2] == HJ_MAX_N_DRIFT, "drift shapes cover HJ_MAX_N_DRIFT");

}  // namespace hj

// X-macro over the shape table, for instantiation and dispatch.
#define HJ_FOR_EACH_SHAPE(X) \
  X(2, 1) X(4, 1) X(4, 2) X(5, 2) X(3, 4) X(4, 4) X(8, 4) X(8, 8) X(13, 8) X(16, 8) \
  X(2, 2) X(8, 1) X(2, 4) X(10, 1) X(8, 2) X(4, 8) X(7, 16)
#define HJ_FOR_EACH_DRIFT_NPL(X) X(4) X(8) X(16)
// FP64 shapes with a tail-continuation kernel (at most 4 lanes per task)
#define HJ_FOR_EACH_RESUME_SHAPE(X) \
  X(2, 1) X(4, 1) X(2, 2) X(8, 1) X(2, 4) X(4, 2) X(5, 2) X(10, 1) X(3, 4) X(4, 4) X(8, 2) X(8, 4)
