// hj_kernels.hpp -- the solver kernels: objective evaluation (with optional
// exact gradient), central-difference coordinate descent, adjoint gradient
// descent (single problem or a batch of instances), and per-point selection
// over the guess slots.  Each kernel is a template over a Cfg (arithmetic
// type, components per lane, lanes per task, speed profile); hj_inst_*.hip
// instantiate them and hj_api.hip dispatches.
#pragma once

#include <algorithm>

#include "hj_device.hpp"
#include "hj_launch.hpp"

namespace hj {

// load n-vector row into the lane's NPL components (0 beyond n)
template <class C>
__device__ __forceinline__ void load_row(const typename C::T* base, int n, int sub,
                                         typename C::T (&out)[C::NPL]) {
#pragma unroll
  for (int k = 0; k < C::NPL; ++k) {
    const int i = C::comp(sub, k);
    out[k] = (i < n) ? base[i] : typename C::T(0);
  }
}
template <class C>
__device__ __forceinline__ void store_row(typename C::T* base, int n, int sub,
                                          const typename C::T (&in)[C::NPL]) {
#pragma unroll
  for (int k = 0; k < C::NPL; ++k) {
    const int i = C::comp(sub, k);
    if (i < n) base[i] = in[k];
  }
}

// Copy the drift operand table and the padded weights d into the
// workgroup's LDS (every thread of the block takes part; the matrix-core
// kernels never leave before this point).
template <class C>
__device__ __forceinline__ void stage_drift(const typename C::T* table, const typename C::T* d,
                                            typename C::T* dst) {
  for (int i = threadIdx.x; i < C::kDriftTable; i += blockDim.x) dst[i] = table[i];
  for (int i = threadIdx.x; i < 4 * C::NPL; i += blockDim.x) dst[C::kDriftTable + i] = d[i];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// objective evaluation (and exact gradient)
// ---------------------------------------------------------------------------
// The evaluation and coordinate-descent kernels keep d in registers: the LDS
// weights (Cfg::DL) pay off in the descent kernel's adjoint sweeps only, and
// cost the forward-only coordinate descent a third of its speed (measured).
template <class C0>
using NoDl = Cfg<typename C0::T, C0::NPL, C0::LPT, C0::MK, C0::DR, false>;

template <class C0>
__global__ __launch_bounds__(256) void k_eval(EvalArgs<typename C0::T> A) {
  using C = NoDl<C0>;
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  __shared__ T s_aop[C::DR ? C::kDriftTable + 4 * NPL : 1];
  const size_t lane = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int sub = C::sub_of(threadIdx.x);
  int64_t task = C::task_of(lane);
  // matrix-core kernels keep lanes past the last task as idle wave members
  const bool live = task < A.B * A.G;
  if constexpr (!C::DR) {
    if (!live) return;
  }
  if (!live) task = 0;
  const int64_t b = task / A.G;
  const int n = A.P.n;
  LaneParams<C> L;
  L.load(A.P, sub);
  if constexpr (C::DR) {
    stage_drift<C>(A.P.aop, A.P.d, s_aop);
    L.aop = s_aop;
    L.set_dl(s_aop + C::kDriftTable);
  }
  T x[NPL], v[1][NPL], phi[1], rho[1], yg[1][NPL], yp[1][NPL];
  load_row<C>(A.x + b * n, n, sub, x);
  load_row<C>(A.v + task * n, n, sub, v[0]);
  const bool grad = (A.gv != nullptr) || (A.gx != nullptr);
  if (grad)
    forward<C, 1, true>(A.P, L, x, v, phi, rho, A.ck, A.stride, lane, A.K, yg, yp);
  else
    forward<C, 1, false>(A.P, L, x, v, phi, rho, nullptr, 0, 0, 1, yg, yp);
  if (live && sub == 0) {
    A.phi[task] = (double)phi[0];
    if (A.rho) A.rho[task] = (double)rho[0];
  }
  if (live && A.yN) {
    store_row<C>(A.yN + task * 2 * n, n, sub, yg[0]);
    store_row<C>(A.yN + task * 2 * n + n, n, sub, yp[0]);
  }
  if (grad) {
    T gv[NPL], gx[NPL];
    backward<C>(A.P, L, x, v[0], A.ck, A.seg, A.stride, lane, A.K, gv, gx);
    if (live && A.gv) store_row<C>(A.gv + task * n, n, sub, gv);
    if (live && A.gx) store_row<C>(A.gx + task * n, n, sub, gx);
  }
}

// The gradient sweep of a descent iteration: gt = d(objective)/dv at v.
// With C::kStash the point x and the iterate v wait in LDS while the sweep
// runs (the sweep reads them on its last line only), and on the matrix-core
// layout the last gradient as well (the sweep does not read it); that frees
// their registers for the sweep.  Every lane reads back what it wrote, so
// no barrier is needed, and the result is the same bit for bit.  (Without
// drift, parking the gradient too costs one segment state of LDS and
// measured even.)
template <class C>
__device__ __forceinline__ void grad_sweep(const Problem<typename C::T>& P,
                                           const LaneParams<C>& L, typename C::T (&x)[C::NPL],
                                           typename C::T (&v)[C::NPL],
                                           typename C::T (&g)[C::NPL], const typename C::T* ck,
                                           typename C::T* seg, size_t stride, size_t lane, int K,
                                           typename C::T (&gt)[C::NPL]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  T gx[NPL];
  if constexpr (C::kStash) {
    constexpr bool SG = C::DR;  // the gradient too
    __shared__ T s_st[(SG ? 3 : 2) * NPL * 256];
    T* const sx = s_st + threadIdx.x;
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      sx[k * 256] = x[k];
      sx[(NPL + k) * 256] = v[k];
      if constexpr (SG) sx[(2 * NPL + k) * 256] = g[k];
    }
    // the values now live in LDS only: the compiler may neither keep them
    // in registers across the sweep nor skip the reloads
    asm volatile("" ::: "memory");
    T z[NPL];
#pragma unroll
    for (int k = 0; k < NPL; ++k) z[k] = T(0);
    backward<C>(P, L, z, z, ck, seg, stride, lane, K, gt, gx);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      x[k] = sx[k * 256];
      v[k] = sx[(NPL + k) * 256];
      if constexpr (SG) g[k] = sx[(2 * NPL + k) * 256];
      if (P.formula == HJ_HOPF) gt[k] -= x[k];  // as backward's last line
    }
  } else {
    backward<C>(P, L, x, v, ck, seg, stride, lane, K, gt, gx);
  }
}

// ---------------------------------------------------------------------------
// task context: the problem, query point and guesses of the task a lane
// group is working on.  Single problem: the problem lives in the kernel
// arguments (wave-uniform, scalar registers).  Batched: it is loaded from the
// instance table whenever the group takes a task (per lane).
// ---------------------------------------------------------------------------
template <class C, bool MULTI> struct TaskCtx {
  using T = typename C::T;
  Problem<T> Pl;
  Problem<double> P64l;
  LaneParams<C> L;
  T x[C::NPL];
  const T* g0;  // guesses of the task: [R+1, n]
  int R;

  __device__ __forceinline__ const Problem<T>& P(const SolveArgs<T>& A) const {
    if constexpr (MULTI) return Pl;
    else return A.P;
  }
  __device__ __forceinline__ const Problem<double>& P64(const SolveArgs<T>& A) const {
    if constexpr (MULTI) return P64l;
    else return A.P64;
  }
  __device__ __forceinline__ void bind(const SolveArgs<T>& A, int64_t task, int sub) {
    const T* xb;
    if constexpr (MULTI) {
      int lo = 0, hi = A.n_inst - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.inst[mid].task0 <= task)
          lo = mid;
        else
          hi = mid - 1;
      }
      const InstDesc<T>& I = A.inst[lo];
      Pl = I.P;
      P64l = I.P64;
      L.load(Pl, sub);
      const int n = Pl.n;
      const int64_t lt = task - I.task0;
      R = I.R;
      xb = I.x + (lt / I.G) * n;
      g0 = I.guesses + lt * (int64_t)(I.R + 1) * n;
    } else {
      const int n = A.P.n;
      R = A.R;
      xb = A.x + (task / A.G) * n;
      g0 = A.guesses + task * (int64_t)(A.R + 1) * n;
    }
    load_row<C>(xb, P(A).n, sub, x);
  }
};

// Next task for a lane group: the group's leader takes an index from the
// queue and the group shares it.
template <class C>
__device__ __forceinline__ int64_t pop_task(unsigned long long* queue, int sub) {
  unsigned long long t = 0;
  if (sub == 0) t = atomicAdd(queue, 1ULL);
  if (C::LPT > 1) {
    const int leader = C::leader(threadIdx.x, sub);
    const int lo = __shfl((int)(t & 0xffffffffULL), leader, 64);
    const int hi = __shfl((int)(t >> 32), leader, 64);
    t = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  }
  return (int64_t)t;
}

// ---------------------------------------------------------------------------
// shared per-slot bookkeeping
// ---------------------------------------------------------------------------
struct SlotBest {
  double phi, rho;
  int32_t cert, status, iters, attempts;
  int64_t n_fwd, n_bwd;
  __device__ __forceinline__ void reset() {
    phi = __builtin_nan("");
    rho = __builtin_nan("");
    cert = -1;
    status = HJ_ST_DIVERGED;
    iters = 0;
    attempts = 0;
    n_fwd = 0;
    n_bwd = 0;
  }
};

// Objective and residual of a finished attempt in FP64.  FP32 runs with the
// FP64 certificate re-solve the characteristic in FP64 at the final v.
// `ending` marks the lanes whose attempt ends now; on the matrix-core layout
// the re-solve runs on the whole wave when any lane needs it.
template <class C, bool MULTI>
__device__ __forceinline__ void attempt_values(const SolveArgs<typename C::T>& A,
                                               const TaskCtx<C, MULTI>& tc, int sub,
                                               const typename C::T (&v)[C::NPL],
                                               typename C::T phi, typename C::T rho, int status,
                                               bool ending, double& phi64, double& rho64) {
  phi64 = (double)phi;
  rho64 = (status == HJ_ST_DIVERGED) ? __builtin_nan("") : (double)rho;
  if constexpr (sizeof(typename C::T) == 4) {
    const bool need = ending && status != HJ_ST_DIVERGED;
    if (A.cert_fp64 && wave_if<C>(need)) {
      using C64 = Cfg<double, C::NPL, C::LPT, C::MK, C::DR, false>;
      const Problem<double>& P64 = tc.P64(A);
      LaneParams<C64> L64;
      L64.load(P64, sub);
      double x64[C::NPL], v64[1][C::NPL], ph[1], rh[1];
#pragma unroll
      for (int k = 0; k < C::NPL; ++k) {
        x64[k] = (double)tc.x[k];
        v64[0][k] = (double)v[k];
      }
      forward<C64, 1, false>(P64, L64, x64, v64, ph, rh);
      if (need) {
        phi64 = ph[0];
        rho64 = rh[0];
      }
    }
  }
}

// Record the end of one attempt with its FP64 objective and residual;
// returns true when the slot is finished.
template <class C, bool MULTI>
__device__ __forceinline__ bool end_attempt(const SolveArgs<typename C::T>& A,
                                            const TaskCtx<C, MULTI>& tc, int sub, int64_t task,
                                            const typename C::T (&v)[C::NPL], double phi64,
                                            double rho64, int status, int it, int att,
                                            SlotBest& best) {
  best.iters += it;
  best.attempts = att + 1;
  const bool fin = (status != HJ_ST_DIVERGED) && isfinite(phi64);
  const bool certified = fin && (rho64 <= A.cert_tol);
  if (certified || (fin && (best.cert < 0 || phi64 < best.phi))) {
    best.phi = phi64;
    best.rho = rho64;
    best.cert = certified ? 1 : 0;
    best.status = status;
    const int n = tc.P(A).n;
    // slot records use the row stride A.P.n (the largest n of a batch)
    store_row<C>(A.out.v + task * A.P.n, n, sub, v);
  }
  return certified || (att + 1 > tc.R);
}

template <class C, bool MULTI>
__device__ __forceinline__ void write_slot(const SolveArgs<typename C::T>& A,
                                           const TaskCtx<C, MULTI>& tc, int sub, int64_t task,
                                           const SlotBest& best) {
  using T = typename C::T;
  const int n = tc.P(A).n;
  if (best.cert < 0) {
    T nanv[C::NPL];
#pragma unroll
    for (int k = 0; k < C::NPL; ++k) nanv[k] = T(__builtin_nan(""));
    store_row<C>(A.out.v + task * A.P.n, n, sub, nanv);
  }
  if (sub != 0) return;
  if (A.out.phi) A.out.phi[task] = best.phi;
  if (A.out.rho) A.out.rho[task] = best.rho;
  if (A.out.status) A.out.status[task] = best.status;
  if (A.out.cert) A.out.cert[task] = best.cert;
  if (A.out.iters) A.out.iters[task] = best.iters;
  if (A.out.attempts) A.out.attempts[task] = best.attempts;
  if (A.out.n_fwd) A.out.n_fwd[task] = best.n_fwd;
  if (A.out.n_bwd) A.out.n_bwd[task] = best.n_bwd;
}

// Step test: the trial must realise the fraction armijo_c of the decrease
// alpha <g, d> its gradient predicts, up to a rounding allowance acc_rel |F|
// (armijo_c = 0: no ascent).
template <class AT, typename T>
__device__ __forceinline__ bool accept_step(const AT& A, T trial, T cur, T decrease) {
  return trial <= cur - T(A.armijo_c) * decrease + T(A.acc_rel) * dabs(cur);
}

// Stop tests at the end of an iteration, in the order of the reference.
template <class C, class AT>
__device__ __forceinline__ int stop_status(const AT& A, const typename C::T (&v)[C::NPL],
                                           typename C::T phi, typename C::T smax,
                                           typename C::T alpha, int it) {
  using T = typename C::T;
  const T alpha_floor = T(A.alpha0) * T(9.094947017729282e-13);  // alpha0 * 2^-40
  T vmax = T(0);
#pragma unroll
  for (int k = 0; k < C::NPL; ++k) vmax = nanmax(vmax, dabs(v[k]));
  vmax = cmax<C>(vmax);
  if (!isfinite(phi) || !(vmax <= T(A.v_max))) return HJ_ST_DIVERGED;
  if (smax < T(A.eps_step)) return HJ_ST_CONVERGED;
  if (alpha < alpha_floor) return HJ_ST_STALLED;
  if (it >= A.max_iter) return HJ_ST_MAXITER;
  return -1;
}

// After a slot: the next task of the group, or -1 when there is none.
template <class C>
__device__ __forceinline__ int64_t next_task(const SolveArgs<typename C::T>& A, int sub) {
  if (!A.queue) return -1;
  const int64_t t = pop_task<C>(A.queue, sub);
  return t < A.ntask ? t : -1;
}

// ---------------------------------------------------------------------------
// cyclic coordinate descent with central differences (Algorithm 1; one
// iteration = one sweep over the n coordinates; the step halves when a trial
// fails the step test)
// ---------------------------------------------------------------------------
template <class C0>
__global__ __launch_bounds__(256) void k_solve_cd(SolveArgs<typename C0::T> A) {
  using C = NoDl<C0>;
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  __shared__ T s_aop[C::DR ? C::kDriftTable + 4 * NPL : 1];
  const size_t lane = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int sub = C::sub_of(threadIdx.x);
  int64_t task = C::task_of(lane);
  // matrix-core kernels keep lanes without a task as idle wave members
  int live = task < A.ntask ? 1 : 0;
  if constexpr (!C::DR) {
    if (!live) return;
  }
  TaskCtx<C, false> tc;
  tc.L.load(A.P, sub);
  if constexpr (C::DR) {
    stage_drift<C>(A.P.aop, A.P.d, s_aop);
    tc.L.aop = s_aop;
    tc.L.set_dl(s_aop + C::kDriftTable);
  }
  tc.bind(A, live != 0 ? task : 0, sub);
  const int n = A.P.n;
  T v[NPL];
  load_row<C>(tc.g0, n, sub, v);
  SlotBest best;
  best.reset();
  // it < 0 marks the first pass of an attempt (its start point is evaluated).
  // The attempt start is kept in this many-valued counter rather than in a
  // loop-carried flag: the compiler's lowering of such a flag in this loop
  // (a per-lane mask) has lost the restart of a new task.
  int att = 0, it = -1, j = 0;
  T alpha = A.alpha0, phi = T(0), rho = T(0), smax = T(0);
  while (true) {
    const bool start = it < 0;
    // pair: the two central-difference points (or the start point)
    T va[2][NPL], fp[2], rp[2];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const bool on = !start && (C::comp(sub, k) == j);
      va[0][k] = on ? v[k] + A.sigma : v[k];
      va[1][k] = on ? v[k] - A.sigma : v[k];
    }
    forward<C, 2, false>(A.P, tc.L, tc.x, va, fp, rp);
    // trial step along coordinate j
    const T gj = (fp[0] - fp[1]) / (T(2) * A.sigma);
    const T step = alpha * gj;
    T vt[1][NPL], ft[1], rt[1];
#pragma unroll
    for (int k = 0; k < NPL; ++k) vt[0][k] = (C::comp(sub, k) == j) ? v[k] - step : v[k];
    if (wave_if<C>(!start)) forward<C, 1, false>(A.P, tc.L, tc.x, vt, ft, rt);
    int status = -1;
    if (start) {
      best.n_fwd += 1;
      phi = fp[0];
      rho = rp[0];
      it = 0;
      j = 0;
      smax = T(0);
      alpha = A.alpha0;
      if (!isfinite(phi))
        status = HJ_ST_DIVERGED;
      else if (A.max_iter == 0)
        status = HJ_ST_MAXITER;
    } else {
      smax = nanmax(smax, dabs(step));
      best.n_fwd += 3;
      if (accept_step(A, ft[0], phi, alpha * gj * gj)) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) v[k] = vt[0][k];
        phi = ft[0];
        rho = rt[0];
      } else {
        alpha *= T(0.5);
      }
      if (++j == n) {
        j = 0;
        ++it;
        status = stop_status<C>(A, v, phi, smax, alpha, it);
        smax = T(0);
      }
    }
    const bool ending = live != 0 && status >= 0;
    double phi64, rho64;
    attempt_values<C, false>(A, tc, sub, v, phi, rho, status, ending, phi64, rho64);
    if (ending) {
      if (end_attempt<C, false>(A, tc, sub, task, v, phi64, rho64, status, it, att, best)) {
        write_slot<C, false>(A, tc, sub, task, best);
        task = next_task<C>(A, sub);
        att = 0;
        if (task < 0) {
          if constexpr (!C::DR) break;
          live = 0;
        } else {
          tc.bind(A, task, sub);
          best.reset();
        }
      } else {
        ++att;
      }
      load_row<C>(tc.g0 + (int64_t)att * n, n, sub, v);
      it = -1;
    }
    if constexpr (C::DR) {
      if (!wave_if<C>(live != 0)) break;
    }
  }
}

// ---------------------------------------------------------------------------
// gradient descent with the exact discrete gradient (adjoint + checkpoints)
// ---------------------------------------------------------------------------
// Save or restore the descent state of a slot in tail record r.
template <class C>
__device__ __forceinline__ void tail_save(const SolveArgs<double>& A, int sub, int64_t r,
                                          int64_t task, int it, int att, double alpha,
                                          double phi, double rho, const SlotBest& best,
                                          const double (&v)[C::NPL], const double (&g)[C::NPL]) {
  const int n = A.P.n;
  double* rec = A.tail + r * A.tail_stride;
  if (sub == 0) {
    rec[0] = (double)task;
    rec[1] = (double)it;
    rec[2] = (double)att;
    rec[3] = alpha;
    rec[4] = phi;
    rec[5] = rho;
    rec[6] = best.phi;
    rec[7] = best.rho;
    rec[8] = (double)best.cert;
    rec[9] = (double)best.status;
    rec[10] = (double)best.iters;
    rec[11] = (double)best.attempts;
    rec[12] = (double)best.n_fwd;
    rec[13] = (double)best.n_bwd;
  }
  store_row<C>(rec + kTailHead, n, sub, v);
  store_row<C>(rec + kTailHead + n, n, sub, g);
}
template <class C>
__device__ __forceinline__ int64_t tail_restore(const SolveArgs<double>& A, int sub, int64_t r,
                                                int& it, int& att, double& alpha, double& phi,
                                                double& rho, SlotBest& best,
                                                double (&v)[C::NPL], double (&g)[C::NPL]) {
  const int n = A.P.n;
  const double* rec = A.tail + r * A.tail_stride;
  it = (int)rec[1];
  att = (int)rec[2];
  alpha = rec[3];
  phi = rec[4];
  rho = rec[5];
  best.phi = rec[6];
  best.rho = rec[7];
  best.cert = (int32_t)rec[8];
  best.status = (int32_t)rec[9];
  best.iters = (int32_t)rec[10];
  best.attempts = (int32_t)rec[11];
  best.n_fwd = (int64_t)rec[12];
  best.n_bwd = (int64_t)rec[13];
  load_row<C>(rec + kTailHead, n, sub, v);
  load_row<C>(rec + kTailHead + n, n, sub, g);
  return (int64_t)rec[0];
}

// TAIL (FP64, one problem, no drift): kTailOff, the plain descent;
// kTailHandOff, a descent that hands slots over its evaluation budget to
// records; kTailResume, the continuation launch: lane groups pop record
// indices and carry each slot on from its saved state, exactly where the
// first launch left it.  (The hand-off is a variant of its own so that the
// plain descent keeps its register allocation.)
enum { kTailOff = 0, kTailHandOff = 1, kTailResume = 2 };
template <class C, bool MULTI, int TAIL>
__global__ __launch_bounds__(256, C::kWaves) void k_solve_gd(SolveArgs<typename C::T> A) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  static_assert(!(MULTI && C::DR), "batched instances carry no drift");
  static_assert(TAIL == kTailOff || (sizeof(T) == 8 && !MULTI && !C::DR),
                "tail hand-offs are FP64 single-problem descents without drift");
  constexpr bool RESUME = TAIL == kTailResume;
  __shared__ T s_aop[C::DR ? C::kDriftTable + 4 * NPL : 1];
  const size_t lane = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int sub = C::sub_of(threadIdx.x);
  int64_t task = 0, ridx = 0, rcount = 0;
  int live;
  if constexpr (RESUME) {
    rcount = (int64_t)*A.tail_n;
    ridx = pop_task<C>(A.queue, sub);
    live = ridx < rcount ? 1 : 0;
  } else {
    task = C::task_of(lane);
    // matrix-core kernels keep lanes without a task as idle wave members
    live = task < A.ntask ? 1 : 0;
  }
  if constexpr (!C::DR) {
    if (!live) return;
  }
  TaskCtx<C, MULTI> tc;
  if constexpr (!MULTI) tc.L.load(A.P, sub);
  if constexpr (C::DR) {
    stage_drift<C>(A.P.aop, A.P.d, s_aop);
    tc.L.aop = s_aop;
    tc.L.set_dl(s_aop + C::kDriftTable);
  }
  T v[NPL], g[NPL];
  SlotBest best;
  // it < 0 marks the first pass of an attempt (see k_solve_cd)
  int att = 0, it = -1;
  T alpha = A.alpha0, phi = T(0), rho = T(0);
  if constexpr (RESUME) {
    task = tail_restore<C>(A, sub, ridx, it, att, alpha, phi, rho, best, v, g);
    tc.bind(A, task, sub);
  } else {
    tc.bind(A, live != 0 ? task : 0, sub);
    load_row<C>(tc.g0, tc.P(A).n, sub, v);
#pragma unroll
    for (int k = 0; k < NPL; ++k) g[k] = T(0);
    best.reset();
  }
  while (true) {
    const bool start = it < 0;
    const Problem<T>& P = tc.P(A);
    // trial point
    T vt[1][NPL], ft[1], rt[1], smax = T(0), gg = T(0);
    if (start) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) vt[0][k] = v[k];
    } else {
      T gm = T(0);
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        gm = nanmax(gm, dabs(g[k]));
        vt[0][k] = fmaT(-alpha, g[k], v[k]);
      }
      smax = alpha * cmax<C>(gm);
      gg = csum<C>(dot2<NPL>(g, g));
    }
    forward<C, 1, true>(P, tc.L, tc.x, vt, ft, rt, A.ck, A.stride, lane, A.K);
    best.n_fwd += 1;
    const bool acc = start || accept_step(A, ft[0], phi, alpha * gg);
    if (acc) {
      if (!start) {
        // the trial point again, from the same operands (bit-identical), so
        // that it need not stay live across the solve; the empty asm keeps
        // the compiler from reusing the first computation
        T a = alpha;
        asm volatile("" : "+v"(a));
#pragma unroll
        for (int k = 0; k < NPL; ++k) v[k] = fmaT(-a, g[k], v[k]);
      }
      phi = ft[0];
      rho = rt[0];
    } else {
      alpha *= T(0.5);
    }
    const bool need_grad = acc && isfinite(phi);
    if (wave_if<C>(need_grad)) {
      T gt[NPL];
      grad_sweep<C>(P, tc.L, tc.x, v, g, A.ck, A.seg, A.stride, lane, A.K, gt);
      if (need_grad) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) g[k] = gt[k];
        best.n_bwd += 1;
      }
    }
    int status = -1;
    if (start) {
      it = 0;
      alpha = A.alpha0;
      if (!isfinite(phi))
        status = HJ_ST_DIVERGED;
      else if (A.max_iter == 0)
        status = HJ_ST_MAXITER;
    } else {
      ++it;
      status = stop_status<C>(A, v, phi, smax, alpha, it);
    }
    if constexpr (TAIL == kTailHandOff) {
      // tail hand-off: the slot is still descending after its budget of
      // objective evaluations; its state goes to a record and the group
      // takes the next task
      if (A.tail_budget > 0 && status < 0 && best.n_fwd >= A.tail_budget) {
        const int64_t r = pop_task<C>(A.tail_n, sub);
        tail_save<C>(A, sub, r, task, it, att, alpha, phi, rho, best, v, g);
        task = next_task<C>(A, sub);
        if (task < 0) break;
        tc.bind(A, task, sub);
        best.reset();
        att = 0;
        load_row<C>(tc.g0, tc.P(A).n, sub, v);
        it = -1;
        continue;
      }
    }
    const bool ending = live != 0 && status >= 0;
    double phi64, rho64;
    attempt_values<C, MULTI>(A, tc, sub, v, phi, rho, status, ending, phi64, rho64);
    if (ending) {
      bool done = end_attempt<C, MULTI>(A, tc, sub, task, v, phi64, rho64, status, it, att, best);
      // FP64 continuation: the first finite attempt the FP64 certificate
      // rejects ends the slot here (best.cert == 0 only then: earlier
      // attempts were not finite) and goes to the hand-off list
      const bool handoff = sizeof(T) == 4 && A.handoff != nullptr && best.cert == 0;
      if (done || handoff) {
        write_slot<C, MULTI>(A, tc, sub, task, best);
        if (handoff && sub == 0) A.handoff[atomicAdd(A.handoff_n, 1ULL)] = task;
        if constexpr (RESUME) {
          ridx = pop_task<C>(A.queue, sub);
          if (ridx >= rcount) break;
          task = tail_restore<C>(A, sub, ridx, it, att, alpha, phi, rho, best, v, g);
          tc.bind(A, task, sub);
          continue;
        }
        task = next_task<C>(A, sub);
        att = 0;
        if (task < 0) {
          if constexpr (!C::DR) break;
          live = 0;
        } else {
          tc.bind(A, task, sub);
          best.reset();
        }
      } else {
        ++att;
      }
      load_row<C>(tc.g0 + (int64_t)att * tc.P(A).n, tc.P(A).n, sub, v);
      it = -1;
    }
    if constexpr (C::DR) {
      if (!wave_if<C>(live != 0)) break;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 continuation of handed-off FP32 slots (same lane shape, FP64
// arithmetic): the slot's record gives its state after the FP32 attempt
// (attempts used, counts, the attempt's v); the descent resumes from that v
// with the step size reset, and an attempt the certificate still rejects is
// followed by FP64 restarts from the slot's remaining guesses, exactly as in
// k_solve_gd.  Every lane group pops list indices until the list (whose
// length the FP32 launch left in device memory) is exhausted.
// ---------------------------------------------------------------------------
template <class C> struct ContCtx {
  Problem<double> P;
  LaneParams<C> L;
  double x[C::NPL];
  const float* g0;  // guesses of the task: [R+1, n]
  int R;
  template <bool MULTI>
  __device__ __forceinline__ void bind(const SolveArgs<float>& S, int64_t task, int sub) {
    const float* xb;
    if constexpr (MULTI) {
      int lo = 0, hi = S.n_inst - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.inst[mid].task0 <= task)
          lo = mid;
        else
          hi = mid - 1;
      }
      const InstDesc<float>& I = S.inst[lo];
      P = I.P64;
      const int64_t lt = task - I.task0;
      R = I.R;
      xb = I.x + (lt / I.G) * P.n;
      g0 = I.guesses + lt * (int64_t)(I.R + 1) * P.n;
    } else {
      P = S.P64;
      R = S.R;
      xb = S.x + (task / S.G) * P.n;
      g0 = S.guesses + task * (int64_t)(S.R + 1) * P.n;
    }
    if constexpr (!C::DR) L.load(P, sub);
#pragma unroll
    for (int k = 0; k < C::NPL; ++k) {
      const int i = C::comp(sub, k);
      x[k] = (i < P.n) ? (double)xb[i] : 0.0;
    }
  }
  // an FP32 row as FP64 components (0 beyond n)
  __device__ __forceinline__ void load_f32(const float* base, int sub, double (&out)[C::NPL]) const {
#pragma unroll
    for (int k = 0; k < C::NPL; ++k) {
      const int i = C::comp(sub, k);
      out[k] = (i < P.n) ? (double)base[i] : 0.0;
    }
  }
};

template <class C, bool MULTI>
__global__ __launch_bounds__(256, 1) void k_continue_gd(ContArgs<float> A) {
  static_assert(sizeof(typename C::T) == 8, "the continuation runs in FP64");
  static_assert(!(MULTI && C::DR), "batched instances carry no drift");
  constexpr int NPL = C::NPL;
  const SolveArgs<float>& S = A.S;
  __shared__ double s_aop[C::DR ? C::kDriftTable + 4 * NPL : 1];
  const size_t lane = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int sub = C::sub_of(threadIdx.x);
  const int64_t count = (int64_t)*S.handoff_n;
  int64_t idx = pop_task<C>(A.queue, sub);
  int live = idx < count ? 1 : 0;
  if constexpr (!C::DR) {
    if (!live) return;
  }
  ContCtx<C> tc;
  if constexpr (C::DR) {
    stage_drift<C>(S.P64.aop, S.P64.d, s_aop);
    tc.L.load(S.P64, sub);
    tc.L.aop = s_aop;
    tc.L.set_dl(s_aop + C::kDriftTable);
    if (!wave_if<C>(live != 0)) return;  // after the block's only barrier
  }
  const int vs = S.P.n;  // row stride of the slot records
  int64_t task = live ? S.handoff[idx] : 0;
  SlotBest best;
  double v[NPL], g[NPL];
  int att = 0, it = -1;
  // resume a handed-off slot: bind its problem and point, read its record
  auto resume = [&]() {
    tc.template bind<MULTI>(S, task, sub);
    best.phi = S.out.phi[task];
    best.rho = S.out.rho[task];
    best.cert = S.out.cert[task];
    best.status = S.out.status[task];
    best.iters = S.out.iters[task];
    best.attempts = S.out.attempts[task];
    best.n_fwd = S.out.n_fwd[task];
    best.n_bwd = S.out.n_bwd[task];
    att = best.attempts - 1;
    tc.load_f32(S.out.v + task * vs, sub, v);
    it = -1;
  };
  resume();
#pragma unroll
  for (int k = 0; k < NPL; ++k) g[k] = 0.0;
  double alpha = A.alpha0, phi = 0.0, rho = 0.0;
  while (true) {
    const bool start = it < 0;
    const Problem<double>& P = tc.P;
    double vt[1][NPL], ft[1], rt[1], smax = 0.0, gg = 0.0;
    if (start) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) vt[0][k] = v[k];
    } else {
      double gm = 0.0;
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        gm = nanmax(gm, dabs(g[k]));
        vt[0][k] = fmaT(-alpha, g[k], v[k]);
      }
      smax = alpha * cmax<C>(gm);
      gg = csum<C>(dot2<NPL>(g, g));
    }
    forward<C, 1, true>(P, tc.L, tc.x, vt, ft, rt, A.ck, A.stride, lane, A.K);
    best.n_fwd += 1;
    const bool acc = start || accept_step(A, ft[0], phi, alpha * gg);
    if (acc) {
      if (!start) {
        double a = alpha;
        asm volatile("" : "+v"(a));
#pragma unroll
        for (int k = 0; k < NPL; ++k) v[k] = fmaT(-a, g[k], v[k]);
      }
      phi = ft[0];
      rho = rt[0];
    } else {
      alpha *= 0.5;
    }
    const bool need_grad = acc && isfinite(phi);
    if (wave_if<C>(need_grad)) {
      double gt[NPL];
      grad_sweep<C>(P, tc.L, tc.x, v, g, A.ck, A.seg, A.stride, lane, A.K, gt);
      if (need_grad) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) g[k] = gt[k];
        best.n_bwd += 1;
      }
    }
    int status = -1;
    if (start) {
      it = 0;
      alpha = A.alpha0;
      if (!isfinite(phi))
        status = HJ_ST_DIVERGED;
      else if (A.max_iter == 0)
        status = HJ_ST_MAXITER;
    } else {
      ++it;
      status = stop_status<C>(A, v, phi, smax, alpha, it);
    }
    if (live != 0 && status >= 0) {
      // end of an attempt, as end_attempt: FP64 objective and residual
      best.iters += it;
      best.attempts = att + 1;
      const bool fin = (status != HJ_ST_DIVERGED) && isfinite(phi);
      const double r64 = (status == HJ_ST_DIVERGED) ? __builtin_nan("") : rho;
      const bool certified = fin && (r64 <= S.cert_tol);
      if (certified || (fin && (best.cert < 0 || phi < best.phi))) {
        best.phi = phi;
        best.rho = r64;
        best.cert = certified ? 1 : 0;
        best.status = status;
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const int i = C::comp(sub, k);
          if (i < P.n) S.out.v[task * vs + i] = (float)v[k];
        }
      }
      if (certified || att + 1 > tc.R) {
        if (best.cert < 0) {
#pragma unroll
          for (int k = 0; k < NPL; ++k) {
            const int i = C::comp(sub, k);
            if (i < P.n) S.out.v[task * vs + i] = __builtin_nanf("");
          }
        }
        if (sub == 0) {
          S.out.phi[task] = best.phi;
          S.out.rho[task] = best.rho;
          S.out.status[task] = best.status;
          S.out.cert[task] = best.cert;
          S.out.iters[task] = best.iters;
          S.out.attempts[task] = best.attempts;
          S.out.n_fwd[task] = best.n_fwd;
          S.out.n_bwd[task] = best.n_bwd;
        }
        idx = pop_task<C>(A.queue, sub);
        if (idx >= count) {
          if constexpr (!C::DR) break;
          live = 0;
        } else {
          task = S.handoff[idx];
          resume();
          continue;
        }
      } else {
        // restart in FP64 from the slot's next guess
        ++att;
        tc.load_f32(tc.g0 + (int64_t)att * P.n, sub, v);
        it = -1;
      }
    }
    if constexpr (C::DR) {
      if (!wave_if<C>(live != 0)) break;
    }
  }
}

// ---------------------------------------------------------------------------
// selection over the G slots of each point (certified first, lowest
// objective, ties to the lowest slot)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void select_point(int64_t b, int64_t task0, int G, int n,
                                             int vstride, int formula,
                                             const double* s_phi, const int32_t* s_cert,
                                             const T* s_v, double* out_u, T* out_arg,
                                             int32_t* out_cert) {
  int pick = -1, pc = -1;
  double best = 0.0;
  for (int g = 0; g < G; ++g) {
    const int c = s_cert[task0 + g];
    if (c < 0) continue;
    const double ph = s_phi[task0 + g];
    if (c > pc || (c == pc && ph < best)) {
      pick = g;
      pc = c;
      best = ph;
    }
  }
  out_cert[b] = pc;
  if (pick < 0) {
    out_u[b] = __builtin_nan("");
    for (int i = 0; i < n; ++i) out_arg[b * n + i] = T(__builtin_nan(""));
  } else {
    out_u[b] = (formula == HJ_LAX) ? best : -best;
    for (int i = 0; i < n; ++i) out_arg[b * n + i] = s_v[(task0 + pick) * vstride + i];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_select(int64_t B, int G, int n, int formula,
                                                const double* s_phi, const int32_t* s_cert,
                                                const T* s_v, double* out_u, T* out_arg,
                                                int32_t* out_cert) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= B) return;
  select_point<T>(b, b * G, G, n, n, formula, s_phi, s_cert, s_v, out_u, out_arg, out_cert);
}

template <typename T>
__global__ __launch_bounds__(256) void k_select_batched(const InstDesc<T>* inst, int n_inst,
                                                        int64_t total, int n, int formula,
                                                        const double* s_phi,
                                                        const int32_t* s_cert, const T* s_v) {
  const int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gp >= total) return;
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].point0 <= gp)
      lo = mid;
    else
      hi = mid - 1;
  }
  const InstDesc<T>& I = inst[lo];
  const int64_t b = gp - I.point0;
  select_point<T>(b, I.task0 + b * I.G, I.G, I.P.n, n, formula, s_phi, s_cert, s_v, I.out_u,
                  I.out_arg, I.out_cert);
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_diag(const InstDesc<T>* inst, int n_inst,
                                                      int64_t total, int n, SlotOut<T> rec) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].task0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const SlotOut<T>& D = inst[lo].diag;
  const int64_t lt = t - inst[lo].task0;
  if (D.phi) D.phi[lt] = rec.phi[t];
  if (D.rho) D.rho[lt] = rec.rho[t];
  if (D.status) D.status[lt] = rec.status[t];
  if (D.cert) D.cert[lt] = rec.cert[t];
  if (D.iters) D.iters[lt] = rec.iters[t];
  if (D.attempts) D.attempts[lt] = rec.attempts[t];
  if (D.n_fwd) D.n_fwd[lt] = rec.n_fwd[t];
  if (D.n_bwd) D.n_bwd[lt] = rec.n_bwd[t];
  if (D.v)
    for (int i = 0; i < inst[lo].P.n; ++i) D.v[lt * inst[lo].P.n + i] = rec.v[t * n + i];
}

static __global__ void k_queue_reset(unsigned long long* q, unsigned long long v) { *q = v; }

// ---------------------------------------------------------------------------
// launchers (explicitly instantiated in hj_inst_*.hip)
// ---------------------------------------------------------------------------
template <class C>
int64_t resident_groups(int mode) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e;
  if (mode == HJ_CD_FD)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve_cd<C>, 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve_gd<C, false, kTailOff>, 256, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return (int64_t)cus * per_cu * (256 / C::LPT);
}

template <class C>
hipError_t launch_solve(const SolveArgs<typename C::T>& A, int mode, int64_t grid_groups,
                        hipStream_t st) {
  const int block = 256;
  const int64_t groups = grid_groups > 0 ? std::min<int64_t>(grid_groups, A.ntask) : A.ntask;
  const int64_t grid = (groups * C::LPT + block - 1) / block;
  // the queue hands out tasks after the ones every launched group starts with
  if (A.queue) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, st, A.queue,
                       (unsigned long long)(grid * block / C::LPT));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (mode == HJ_CD_FD) {
    hipLaunchKernelGGL(k_solve_cd<C>, dim3((unsigned)grid), dim3(block), 0, st, A);
  } else if (A.inst) {
    if constexpr (C::DR) {
      return hipErrorInvalidValue;  // batches carry no drift
    } else {
      hipLaunchKernelGGL((k_solve_gd<C, true, kTailOff>), dim3((unsigned)grid), dim3(block), 0, st, A);
    }
  } else if (A.tail_budget > 0) {
    if constexpr (sizeof(typename C::T) == 8 && !C::DR) {
      hipLaunchKernelGGL((k_solve_gd<C, false, kTailHandOff>), dim3((unsigned)grid), dim3(block),
                         0, st, A);
    } else {
      return hipErrorInvalidValue;  // hand-offs are FP64 descents without drift
    }
  } else {
    hipLaunchKernelGGL((k_solve_gd<C, false, kTailOff>), dim3((unsigned)grid), dim3(block), 0,
                       st, A);
  }
  return hipGetLastError();
}

template <class C>
int64_t resident_continue_groups() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_continue_gd<C, false>, 256, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int64_t)cus * per_cu * (256 / C::LPT);
}

template <class C>
hipError_t launch_continue(const ContArgs<float>& A, bool multi, int64_t grid_groups,
                           hipStream_t st) {
  const int block = 256;
  const int64_t grid = (grid_groups * C::LPT + block - 1) / block;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, st, A.queue, 0ULL);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (multi) {
    if constexpr (C::DR) {
      return hipErrorInvalidValue;  // batches carry no drift
    } else {
      hipLaunchKernelGGL((k_continue_gd<C, true>), dim3((unsigned)grid), dim3(block), 0, st, A);
    }
  } else {
    hipLaunchKernelGGL((k_continue_gd<C, false>), dim3((unsigned)grid), dim3(block), 0, st, A);
  }
  return hipGetLastError();
}

template <class C>
int64_t resident_resume_groups() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve_gd<C, false, kTailResume>, 256,
                                                   0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int64_t)cus * per_cu * (256 / C::LPT);
}

template <class C>
hipError_t launch_resume(const SolveArgs<double>& A, int64_t grid_groups, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (grid_groups * C::LPT + block - 1) / block;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, st, A.queue, 0ULL);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_gd<C, false, kTailResume>), dim3((unsigned)grid), dim3(block), 0, st, A);
  return hipGetLastError();
}

template <class C>
hipError_t launch_eval(const EvalArgs<typename C::T>& A, hipStream_t st) {
  const int64_t threads = A.B * A.G * C::LPT;
  const int block = 256;
  const int64_t grid = (threads + block - 1) / block;
  hipLaunchKernelGGL(k_eval<C>, dim3((unsigned)grid), dim3(block), 0, st, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_select(int64_t B, int G, int n, int formula, const double* s_phi,
                         const int32_t* s_cert, const T* s_v, double* out_u, T* out_arg,
                         int32_t* out_cert, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (B + block - 1) / block;
  hipLaunchKernelGGL(k_select<T>, dim3((unsigned)grid), dim3(block), 0, st, B, G, n, formula,
                     s_phi, s_cert, s_v, out_u, out_arg, out_cert);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_select_batched(const InstDesc<T>* inst, int n_inst, int64_t total_points,
                                 int n, int formula, const double* s_phi,
                                 const int32_t* s_cert, const T* s_v, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (total_points + block - 1) / block;
  hipLaunchKernelGGL(k_select_batched<T>, dim3((unsigned)grid), dim3(block), 0, st, inst,
                     n_inst, total_points, n, formula, s_phi, s_cert, s_v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter_diag(const InstDesc<T>* inst, int n_inst, int64_t total_tasks, int n,
                               SlotOut<T> rec, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (total_tasks + block - 1) / block;
  hipLaunchKernelGGL(k_scatter_diag<T>, dim3((unsigned)grid), dim3(block), 0, st, inst, n_inst,
                     total_tasks, n, rec);
  return hipGetLastError();
}

}  // namespace hj

// Explicit instantiation of the launchers of one Cfg.
#define HJ_INSTANTIATE(T, NPL, LPT, MK)                                                     \
  template hipError_t hj::launch_solve<hj::Cfg<T, NPL, LPT, MK>>(const hj::SolveArgs<T>&,  \
                                                                 int, int64_t, hipStream_t); \
  template int64_t hj::resident_groups<hj::Cfg<T, NPL, LPT, MK>>(int);                     \
  template hipError_t hj::launch_eval<hj::Cfg<T, NPL, LPT, MK>>(const hj::EvalArgs<T>&,    \
                                                                hipStream_t);
#define HJ_INSTANTIATE_BOTH(T, NPL, LPT) \
  HJ_INSTANTIATE(T, NPL, LPT, HJ_M_TANH) \
  HJ_INSTANTIATE(T, NPL, LPT, HJ_M_RAT)
// The matrix-core (linear drift) instances of one NPL (4 lanes per task).
#define HJ_INSTANTIATE_DRIFT_MK(T, NPL, MK)                                                  \
  template hipError_t hj::launch_solve<hj::Cfg<T, NPL, 4, MK, true>>(                        \
      const hj::SolveArgs<T>&, int, int64_t, hipStream_t);                                   \
  template int64_t hj::resident_groups<hj::Cfg<T, NPL, 4, MK, true>>(int);                 \
  template hipError_t hj::launch_eval<hj::Cfg<T, NPL, 4, MK, true>>(const hj::EvalArgs<T>&, \
                                                                    hipStream_t);
#define HJ_INSTANTIATE_DRIFT(T, NPL)              \
  HJ_INSTANTIATE_DRIFT_MK(T, NPL, HJ_M_TANH)      \
  HJ_INSTANTIATE_DRIFT_MK(T, NPL, HJ_M_RAT)
// The FP64 continuation kernels of the FP32 lane shape (NPL, LPT), without
// and with linear drift.
#define HJ_INSTANTIATE_CONT_MK(NPL, LPT, MK, DR)                                           \
  template hipError_t hj::launch_continue<hj::Cfg<double, NPL, LPT, MK, DR>>(              \
      const hj::ContArgs<float>&, bool, int64_t, hipStream_t);                              \
  template int64_t hj::resident_continue_groups<hj::Cfg<double, NPL, LPT, MK, DR>>();
// The tail-continuation kernels of one FP64 lane shape.
#define HJ_INSTANTIATE_RESUME_MK(NPL, LPT, MK)                                         \
  template hipError_t hj::launch_resume<hj::Cfg<double, NPL, LPT, MK>>(                \
      const hj::SolveArgs<double>&, int64_t, hipStream_t);                            \
  template int64_t hj::resident_resume_groups<hj::Cfg<double, NPL, LPT, MK>>();
#define HJ_INSTANTIATE_RESUME(NPL, LPT)            \
  HJ_INSTANTIATE_RESUME_MK(NPL, LPT, HJ_M_TANH)    \
  HJ_INSTANTIATE_RESUME_MK(NPL, LPT, HJ_M_RAT)
#define HJ_INSTANTIATE_CONT(NPL, LPT)                     \
  HJ_INSTANTIATE_CONT_MK(NPL, LPT, HJ_M_TANH, false)      \
  HJ_INSTANTIATE_CONT_MK(NPL, LPT, HJ_M_RAT, false)
#define HJ_INSTANTIATE_CONT_DRIFT(NPL)                 \
  HJ_INSTANTIATE_CONT_MK(NPL, 4, HJ_M_TANH, true)      \
  HJ_INSTANTIATE_CONT_MK(NPL, 4, HJ_M_RAT, true)
