// hj_device.hpp -- device-side building blocks of the Lax / Hopf solver for
// gfx950: the Hamiltonian family, the RK4 characteristic solve with the
// action quadrature, the discrete adjoint, and wave-level reductions.
//
// Layout: one "task" is one (query point, guess slot).  A task is held by LPT
// lanes of a wavefront, each owning NPL vector components of gamma, p, v, ...
// in registers (padding components carry d = 0, x = v = 0 and stay exactly
// zero).  Two lane layouts exist:
//  * adjacent: the task's lanes are LPT neighbouring lanes, and lane `sub`
//    owns components sub*NPL .. sub*NPL+NPL-1;
//  * matrix-core (linear drift): 16 tasks per wave, task j on lanes
//    j, j+16, j+32, j+48, lane `sub` (= lane / 16) owning components
//    4k + sub.  This is the operand layout of the 16x16x4 MFMA, so A gamma
//    and A^T p for the 16 tasks of a wave are MFMA chains with no data
//    movement (see matvec2).
// Sums over components are butterfly reductions inside the group, so every
// lane of a group holds bit-identical scalars and takes identical branches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hj.h"

namespace hj {

// ---------------------------------------------------------------------------
// math helpers
// ---------------------------------------------------------------------------
// Fused multiply-add in the operands' own precision (__builtin_fma is the
// double one: on floats it converts to double and back around an FP64 FMA).
__device__ __forceinline__ double fmaT(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Coefficients 1/j! (j = 13 .. 2) of the Taylor polynomial of expm1, in
// constant memory so that the wave-uniform loads land in scalar registers and
// every Horner step is one v_fma_f64 with a scalar operand.
static __constant__ double kExpm1Coef[12] = {
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
    1.0 / 362880.0,     1.0 / 40320.0,     1.0 / 5040.0,     1.0 / 720.0,
    1.0 / 120.0,        1.0 / 24.0,        1.0 / 6.0,        0.5};

// expm1(y) for y <= 0 in FP64: Cody-Waite reduction y = k ln2 + f with
// |f| <= ln2/2 (ln2 split into a 32-bit head and a tail), Taylor polynomial
// of expm1(f) to degree 13 (truncation below 1e-17 relative), and
// expm1(y) = 2^k expm1(f) + (2^k - 1).  Relative error a few ulp.
__device__ __forceinline__ double expm1_neg(double y) {
  const double ln2_hi = 6.93147180369123816490e-01;  // head of ln 2 (exact in 32 bits)
  const double ln2_lo = 1.90821492927058770002e-10;  // ln 2 - ln2_hi
  const double inv_ln2 = 1.44269504088896338700e+00;
  const double k = __builtin_rint(y * inv_ln2);
  double f = fmaT(-k, ln2_hi, y);
  f = fmaT(-k, ln2_lo, f);
  double p = kExpm1Coef[0];
#pragma unroll
  for (int j = 1; j < 12; ++j) p = fmaT(p, f, kExpm1Coef[j]);
  p = fmaT(p * f, f, f);                          // f + f^2 (1/2 + ...)
  const double s = __builtin_ldexp(1.0, (int)k);  // exact; 0 for very negative k
  return fmaT(s, p, s - 1.0);
}

// a / b for b in [1, 2]: hardware reciprocal, one Newton step and one
// residual correction of the quotient (error about one ulp).
__device__ __forceinline__ double div_1_2(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fmaT(fmaT(-b, r, 1.0), r, r);
  const double q = a * r;
  return fmaT(fmaT(-b, q, a), r, q);
}

// 1 / b for b >= 1 (no denormal results) the same way, in the operand's
// precision: about one ulp in five instructions, where a correctly rounded
// division takes about ten.
__device__ __forceinline__ double recip_ge1(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fmaT(fmaT(-b, r, 1.0), r, r);
  return fmaT(fmaT(-b, r, 1.0), r, r);
}
__device__ __forceinline__ float recip_ge1(float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  return fmaT(fmaT(-b, r, 1.0f), r, r);
}

// tanh in FP64 from expm1: tanh|z| = -e / (2 + e), e = expm1(-2|z|) in
// (-1, 0].  |z| is clamped to 20 (tanh(20) rounds to 1), which keeps the
// code branch-free.
__device__ __forceinline__ double dtanh(double z) {
  const double az = __builtin_fabs(z);
  const double e = expm1_neg(-2.0 * (az < 20.0 ? az : 20.0));
  double t = div_1_2(-e, 2.0 + e);
  if (z != z) t = z;
  return __builtin_copysign(t, z);
}
__device__ __forceinline__ float dtanh(float x) { return tanhf(x); }
__device__ __forceinline__ double dabs(double x) { return fabs(x); }
__device__ __forceinline__ float dabs(float x) { return fabsf(x); }
template <typename T> __device__ __forceinline__ bool finite_(T x) { return isfinite(x); }

// Max that propagates NaN: once NaN, stays NaN.
template <typename T> __device__ __forceinline__ T nanmax(T s, T a) {
  return (a > s || a != a) ? a : s;
}

// Cross-lane exchange inside a row of 16 lanes with DPP (no LDS traffic).
//   step 0: quad_perm [1,0,3,2]  (lane ^ 1)
//   step 1: quad_perm [2,3,0,1]  (lane ^ 2)
//   step 2: row_half_mirror      (lane i of 8 <-> 7 - i: swaps the two quads)
//   step 3: row_mirror           (lane i of 16 <-> 15 - i: swaps the halves)
// After step s every lane of an aligned group of 2^(s+1) lanes has combined
// the same two partial values, so a butterfly of k steps reduces groups of
// 2^k lanes and leaves bit-identical results in all of them (the combining
// operations are commutative).
template <int STEP> __device__ __forceinline__ int dpp_i(int v) {
  constexpr int ctrl = STEP == 0 ? 0xB1 : STEP == 1 ? 0x4E : STEP == 2 ? 0x141 : 0x140;
  return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
}
template <int STEP> __device__ __forceinline__ float dpp_x(float v) {
  return __builtin_bit_cast(float, dpp_i<STEP>(__builtin_bit_cast(int, v)));
}
template <int STEP> __device__ __forceinline__ double dpp_x(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<STEP>((int)(unsigned)u);
  const unsigned hi = (unsigned)dpp_i<STEP>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum / max over the LPT lanes of a task group (LPT in 1, 2, 4, 8, 16).
template <int LPT, typename T> __device__ __forceinline__ T gsum(T v) {
  static_assert(LPT == 1 || LPT == 2 || LPT == 4 || LPT == 8 || LPT == 16, "LPT");
  if (LPT >= 2) v += dpp_x<0>(v);
  if (LPT >= 4) v += dpp_x<1>(v);
  if (LPT >= 8) v += dpp_x<2>(v);
  if (LPT >= 16) v += dpp_x<3>(v);
  return v;
}
template <int LPT, typename T> __device__ __forceinline__ T gmax(T v) {
  if (LPT >= 2) v = nanmax(v, dpp_x<0>(v));
  if (LPT >= 4) v = nanmax(v, dpp_x<1>(v));
  if (LPT >= 8) v = nanmax(v, dpp_x<2>(v));
  if (LPT >= 16) v = nanmax(v, dpp_x<3>(v));
  return v;
}

// Sum / max over the four 16-lane rows of a wave (the matrix-core layout).
// gfx950's permlane32 swap of a register with itself gives every lane the
// values of rows {0,1} and of rows {2,3} at its position; permlane16 gives
// rows {0,2} and {1,3}.  Combining the pair in a fixed order leaves the same
// bits in all four lanes of a task.
template <int HALF> __device__ __forceinline__ void xrow_u(unsigned v, unsigned& a, unsigned& b) {
  if constexpr (HALF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0];
    b = r[1];
  }
}
template <int HALF> __device__ __forceinline__ void xrow(float v, float& a, float& b) {
  unsigned ua, ub;
  xrow_u<HALF>(__builtin_bit_cast(unsigned, v), ua, ub);
  a = __builtin_bit_cast(float, ua);
  b = __builtin_bit_cast(float, ub);
}
template <int HALF> __device__ __forceinline__ void xrow(double v, double& a, double& b) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  unsigned la, lb, ha, hb;
  xrow_u<HALF>((unsigned)u, la, lb);
  xrow_u<HALF>((unsigned)(u >> 32), ha, hb);
  a = __builtin_bit_cast(double, ((unsigned long long)ha << 32) | la);
  b = __builtin_bit_cast(double, ((unsigned long long)hb << 32) | lb);
}
template <typename T> __device__ __forceinline__ T rsum4(T v) {
  T a, b;
  xrow<32>(v, a, b);
  xrow<16>(a + b, a, b);
  return a + b;
}
template <typename T> __device__ __forceinline__ T rmax4(T v) {
  T a, b;
  xrow<32>(v, a, b);
  xrow<16>(nanmax(a, b), a, b);
  return nanmax(a, b);
}

// Sum of NPL terms as a balanced tree (short dependency chains).
template <int NPL, typename T> __device__ __forceinline__ T tree_sum(const T (&a)[NPL]) {
  if constexpr (NPL == 1) {
    return a[0];
  } else {
    constexpr int H = NPL / 2;
    T lo[H], hi[NPL - H];
#pragma unroll
    for (int k = 0; k < H; ++k) lo[k] = a[k];
#pragma unroll
    for (int k = H; k < NPL; ++k) hi[k - H] = a[k];
    return tree_sum<H>(lo) + tree_sum<NPL - H>(hi);
  }
}


// ---------------------------------------------------------------------------
// LDS plan of the one-wave-per-SIMD kernels
// ---------------------------------------------------------------------------
// Waves per SIMD a descent kernel is compiled for (register budget 512 /
// waves per lane): FP32 without drift at two where at most 5 components sit
// on a lane or 16 lanes share a task (they fit 256 registers), one otherwise.
constexpr int kernel_waves(int npl, int lpt, int tsize, bool dr) {
  return (!dr && tsize == 4 && (lpt == 16 || npl <= 5)) ? 2 : 1;
}
// Bytes of the matrix-core operand table and weights a drift kernel stages.
constexpr int drift_lds_bytes(int npl, int tsize, bool dr) {
  return dr ? (2 * (npl / 4) * npl * 64 + 4 * npl) * tsize : 0;
}
// A one-wave kernel runs one 256-lane block per CU, so a block may take the
// whole 160 KiB of LDS.  Beside the drift table it keeps there what a
// gradient sweep reads only on its last line (the point x and the iterate
// v, and with drift the last gradient: stashed around the sweep to free
// registers) and the states of the checkpointed trajectory that the sweep
// recomputes (2 npl values each), which would otherwise go to HBM and back
// once per step.  The number of segment states that fit, at most 15,
// bounds the checkpoint interval of these kernels at one more than that
// (FP64 n = 10 on one lane: 3 states, interval 4; FP64 n = 32 with drift:
// 2 states, interval 3).
// Two-wave kernels, and shapes where not even one state fits beside the
// stash, keep both in HBM and registers.  Host and device both use this
// function.
constexpr int kLdsBlockBytes = 160 * 1024;
// values a lane stashes around a sweep: x and v, and with drift the last
// gradient too (there it measured faster; without drift even, and the LDS
// is worth more as segment states)
constexpr int stash_values(int npl, bool dr) { return (dr ? 3 : 2) * npl; }
constexpr int seg_lds_fit(int npl, int tsize, bool dr) {
  return (kLdsBlockBytes - drift_lds_bytes(npl, tsize, dr) - stash_values(npl, dr) * tsize * 256) /
         (2 * npl * tsize * 256);
}
constexpr int seg_lds_states(int npl, int lpt, int tsize, bool dr) {
  return kernel_waves(npl, lpt, tsize, dr) != 1 || seg_lds_fit(npl, tsize, dr) < 1
             ? 0
             : (seg_lds_fit(npl, tsize, dr) < 15 ? seg_lds_fit(npl, tsize, dr) : 15);
}

// ---------------------------------------------------------------------------
// compile-time configuration of a kernel instance
// ---------------------------------------------------------------------------
// T: arithmetic type; NPL: components per lane; LPT: lanes per task;
// MK: speed profile (HJ_M_TANH, or HJ_M_RAT which also serves HJ_M_CONST
// with kappa = 0: c = 1 and c' = c'' = 0 exactly); DR: linear drift
// <A x, p> in H, on the matrix-core layout (LPT = 4, NPL a multiple of 4).
template <typename T_, int NPL_, int LPT_, int MK_, bool DR_ = false,
          bool DL_ = DR_ && sizeof(T_) == 8>
struct Cfg {
  using T = T_;
  static constexpr int NPL = NPL_;
  static constexpr int LPT = LPT_;
  static constexpr int MK = MK_;
  static constexpr bool DR = DR_;
  // weights d read from LDS at every use (see LaneParams::dk)
  static constexpr bool DL = DL_;
  static_assert(!DL || DR, "LDS weights belong to the matrix-core layout");
  static_assert(!DR || (LPT == 4 && NPL % 4 == 0), "drift layout: 4 lanes, NPL % 4 == 0");
  // vector component held in slot k of lane `sub`
  static __device__ __forceinline__ int comp(int sub, int k) {
    return DR ? k * 4 + sub : sub * NPL + k;
  }
  // lane's index within its task group, and the task of a global lane
  static __device__ __forceinline__ int sub_of(unsigned tid) {
    return DR ? (int)((tid & 63) >> 4) : (int)(tid % LPT);
  }
  static __device__ __forceinline__ int64_t task_of(size_t lane) {
    return DR ? (int64_t)((lane >> 6) * 16 + (lane & 15)) : (int64_t)(lane / LPT);
  }
  // lane (within the wave) of the group member with sub == 0
  static __device__ __forceinline__ int leader(unsigned tid, int sub) {
    return DR ? (int)(tid & 15) : (int)(tid % 64) - sub;
  }
  // elements of the MFMA operand table of A and A^T: [2][NPL/4][NPL][64]
  static constexpr int kDriftTable = DR ? 2 * (NPL / 4) * NPL * 64 : 0;
  // waves per SIMD the descent kernel is compiled for (register budget 512 /
  // kWaves per lane).  FP32 with at most 5 components per lane fits two
  // waves without spilling, and 7 x 16 with a few hundred bytes that stay
  // out of the RK4 loops; there the second wave's latency hiding pays
  // (measured).  FP64 and wider FP32 shapes lose more to spills at two
  // waves than they gain.
  static constexpr int kWaves = kernel_waves(NPL, LPT, (int)sizeof(T), DR);
  // segment states held in LDS (0: the segment goes to the global scratch)
  // and the stash of x and v (with drift also the gradient) around a sweep
  static constexpr int kSegLds = seg_lds_states(NPL, LPT, (int)sizeof(T), DR);
  static constexpr bool kStash = kSegLds > 0;
  static_assert(kSegLds == 0 || kWaves == 1, "the LDS plan assumes one block per CU");
};

// Sum / max over the lanes of a task group.
template <class C, typename T> __device__ __forceinline__ T csum(T v) {
  if constexpr (C::DR) return rsum4(v);
  else return gsum<C::LPT>(v);
}
template <class C, typename T> __device__ __forceinline__ T cmax(T v) {
  if constexpr (C::DR) return rmax4(v);
  else return gmax<C::LPT>(v);
}

// Branch condition for a block of work that needs all lanes of the wave: the
// matrix-core kernels run every MFMA with the whole wave active (an MFMA
// reads its matrix operand from all 64 lanes), so a block that some task
// needs runs on every lane and the other tasks discard its results.  Other
// layouts branch per lane.
template <class C> __device__ __forceinline__ bool wave_if(bool p) {
  if constexpr (C::DR) return __builtin_amdgcn_ballot_w64(p) != 0;
  else return p;
}

// problem description, in the arithmetic type T
template <typename T> struct Problem {
  int n;        // true dimension
  int N;        // RK4 steps
  int e;        // 1 or 2
  int formula;  // HJ_LAX / HJ_HOPF
  int quad;     // HJ_TRAPZ / HJ_RK4AUG
  T kappa, inv_s, w, j0, h;
  const T* d;    // [npad] kinetic weights, 0 in padding
  const T* a2;   // [npad] a_i^2, 1 in padding
  const T* ia2;  // [npad] 1 / a_i^2, 1 in padding
  const T* aop;  // drift: MFMA operand table of A and A^T (Cfg::kDriftTable), or null
};

// Component parameters of a lane: the kinetic weights, used in every stage,
// are held in registers (uniform across the wave when LPT == 1, so scalar
// registers); the ellipsoid axes, used once per trajectory, are read from
// memory where needed.
template <class C> struct LaneParams {
  using T = typename C::T;
  T d[C::NPL];
  const T* a2p;   // [npad] a_i^2
  const T* ia2p;  // [npad] 1 / a_i^2
  const T* aop;   // drift operand table (LDS or global), matrix-core layout only
  int sub;
  __device__ __forceinline__ void load(const Problem<T>& P, int sub_) {
    sub = sub_;
#pragma unroll
    for (int k = 0; k < C::NPL; ++k) d[k] = P.d[C::comp(sub, k)];
    a2p = P.a2;
    ia2p = P.ia2;
    aop = P.aop;
  }
  // The FP64 matrix-core descent kernel reads d from LDS (element 4k + sub
  // is the lane's slot k) at every use, through a pointer the compiler
  // cannot see through: held in registers for the whole kernel, as it would
  // hoist them, the per-lane weights are what spills first on that layout,
  // and the reloads then wait behind the checkpoint stores (5% of the n = 32
  // solve).  In FP32 kernels, and in their FP64 certificate solve, they fit
  // and the reads would only cost (measured).
  static constexpr bool kDlds = C::DL;
  typedef const __attribute__((address_space(3))) T* lds_ptr;
  lds_ptr dl;
  __device__ __forceinline__ void set_dl(const T* p) { dl = (lds_ptr)(p + sub); }
  __device__ __forceinline__ T dk(int k) const {
    if constexpr (kDlds) {
      lds_ptr q = dl;
      asm volatile("" : "+v"(q));
      return q[4 * k];
    } else {
      return d[k];
    }
  }
  __device__ __forceinline__ T a2(int k) const { return a2p[C::comp(sub, k)]; }
  __device__ __forceinline__ T ia2(int k) const { return ia2p[C::comp(sub, k)]; }
};

// ---------------------------------------------------------------------------
// linear drift on the matrix cores
// ---------------------------------------------------------------------------
typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dvec4 mfma4(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fvec4 mfma4(float a, float b, fvec4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Vec4;
template <> struct Vec4<double> { using type = dvec4; };
template <> struct Vec4<float> { using type = fvec4; };

// ya = Ma xa and yb = Mb xb for the 16 tasks of the wave, with Ma, Mb in
// {A, A^T} (mat index 0 = A, 1 = A^T).  One 16x16x4 MFMA multiplies the 16x4
// block (ib, kb) of M by the 4 x 16 block of inputs whose row `sub` is slot
// kb of the lanes of each task, which is where the layout keeps component
// 4 kb + sub.  The operand table holds, per lane, the element of each block
// that lane supplies; its host-side row order makes result register r of row
// block ib land in slot 4 ib + r of the lane owning the component.  The two
// products are interleaved as independent accumulation chains.
template <class C>
__device__ __forceinline__ void matvec2(const typename C::T* aop, int mat_a,
                                        const typename C::T (&xa)[C::NPL],
                                        typename C::T (&ya)[C::NPL], int mat_b,
                                        const typename C::T (&xb)[C::NPL],
                                        typename C::T (&yb)[C::NPL]) {
  using T = typename C::T;
  using V = typename Vec4<T>::type;
  constexpr int NPL = C::NPL, NB = NPL / 4;
  const int l = threadIdx.x & 63;
  const T* pa = aop + mat_a * (NB * NPL * 64) + l;
  const T* pb = aop + mat_b * (NB * NPL * 64) + l;
#pragma unroll
  for (int ib = 0; ib < NB; ++ib) {
    V ca = {T(0), T(0), T(0), T(0)}, cb = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int kb = 0; kb < NPL; ++kb) {
      ca = mfma4(pa[(ib * NPL + kb) * 64], xa[kb], ca);
      cb = mfma4(pb[(ib * NPL + kb) * 64], xb[kb], cb);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ya[4 * ib + r] = ca[r];
      yb[4 * ib + r] = cb[r];
    }
  }
}

// m = c^e and its derivatives in r = |gamma|^2.
template <class C, bool NEED2>
__device__ __forceinline__ void speed(const Problem<typename C::T>& P, typename C::T r,
                                      typename C::T& m, typename C::T& m1, typename C::T& m2) {
  using T = typename C::T;
  T c, c1, c2 = T(0);
  if constexpr (C::MK == HJ_M_TANH) {
    const T th = dtanh(r * P.inv_s);
    const T sech2 = T(1) - th * th;
    c = T(1) + P.kappa * th;
    c1 = P.kappa * P.inv_s * sech2;
    if (NEED2) c2 = T(-2) * P.kappa * P.inv_s * P.inv_s * th * sech2;
  } else {
    const T q = recip_ge1(T(1) + r);  // r >= 0
    c = T(1) + P.kappa * r * q;
    c1 = P.kappa * q * q;
    if (NEED2) c2 = T(-2) * P.kappa * q * q * q;
  }
  if (P.e == 2) {
    m = c * c;
    m1 = T(2) * c * c1;
    m2 = NEED2 ? T(2) * c1 * c1 + T(2) * c * c2 : T(0);
  } else {
    m = c;
    m1 = c1;
    m2 = c2;
  }
}

// Integrand of the action at a state with scalars (r, q, m, m1):
//   Lax  <p, H_p> - H       = 1/2 m q - 1/2 w r
//   Hopf H - <H_x, gamma>   = 1/2 m q - q m' r - 1/2 w r
template <typename T>
__device__ __forceinline__ T integrand(const Problem<T>& P, T r, T q, T m, T m1) {
  T v = T(0.5) * m * q - T(0.5) * P.w * r;
  if (P.formula == HJ_HOPF) v -= q * m1 * r;
  return v;
}

// ---------------------------------------------------------------------------
// RK4 in reversed time: y' = f(y), f(gamma, p) = (-(A gamma + m D p),
// A^T p + (q m' + w) gamma) (the A terms with drift only).  NT independent
// trajectories are advanced together so their instruction streams interleave.
// ---------------------------------------------------------------------------

// Sum of a[k] * b[k] over the lane's components as two interleaved FMA
// chains (half the dependency depth of one chain, no extra instructions).
template <int NPL, typename T>
__device__ __forceinline__ T dot2(const T (&a)[NPL], const T (&b)[NPL]) {
  T s0 = a[0] * b[0], s1 = T(0);
#pragma unroll
  for (int k = 1; k < NPL; ++k) {
    if (k & 1)
      s1 = fmaT(a[k], b[k], s1);
    else
      s0 = fmaT(a[k], b[k], s0);
  }
  return s0 + s1;
}

// r = |gamma|^2 and q = sum d p^2 at the stage state (G, Pp) for NT
// trajectories, and the products dp = D p that the stage update reuses.
template <class C, int NT>
__device__ __forceinline__ void reduce_rq(const typename C::T (&G)[NT][C::NPL],
                                          const typename C::T (&Pp)[NT][C::NPL],
                                          const LaneParams<C>& L, typename C::T (&r)[NT],
                                          typename C::T (&q)[NT],
                                          typename C::T (&dp)[NT][C::NPL]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int k = 0; k < C::NPL; ++k) dp[t][k] = L.dk(k) * Pp[t][k];
    r[t] = dot2<C::NPL>(G[t], G[t]);
    q[t] = dot2<C::NPL>(dp[t], Pp[t]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    r[t] = csum<C>(r[t]);
    q[t] = csum<C>(q[t]);
  }
}
template <class C, int NT>
__device__ __forceinline__ void reduce_rq(const typename C::T (&G)[NT][C::NPL],
                                          const typename C::T (&Pp)[NT][C::NPL],
                                          const LaneParams<C>& L, typename C::T (&r)[NT],
                                          typename C::T (&q)[NT]) {
  typename C::T dp[NT][C::NPL];
  reduce_rq<C, NT>(G, Pp, L, r, q, dp);
}

// One RK4 step y -> y_next for NT trajectories.  With QUAD the RK4-augmented
// quadrature of the integrand is added into acc.  The y update is the same
// instruction sequence with or without QUAD, which keeps the adjoint's
// recomputation bit-identical to the forward solve.
//
// Stage s evaluates K = f(Y) = (-m D p, (q m' + w) gamma) and folds it into
// the weighted sum S = K1 + 2 K2 + 2 K3 + K4 and the next stage state
// Y' = y + c h K with scalar coefficients, so each component costs seven
// FP64 operations per stage (D p, two reduction FMAs, four update FMAs); the
// step ends with y + h/6 S.  The stage sum is kept apart from y on purpose:
// folding each stage into y directly rounds four times at the scale of y,
// which doubles the objective's rounding noise and, near an optimum, makes
// the step test fail on noise (measured on the n=10 workload).  With drift,
// A G and A^T P come from the matrix cores; there the stage derivative K is
// formed explicitly (two FMAs per component) and enters the stage sum and
// the next stage state through one FMA each, five or seven operations per
// component and stage instead of nine.
template <class C, int NT, bool QUAD>
__device__ __forceinline__ void rk4_step(const Problem<typename C::T>& P, const LaneParams<C>& L,
                                         typename C::T (&g)[NT][C::NPL],
                                         typename C::T (&p)[NT][C::NPL],
                                         typename C::T (&acc)[NT]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  const T h = P.h, h2 = T(0.5) * P.h, h6 = P.h / T(6);
  T G[NT][NPL], Pp[NT][NPL], ag[NT][NPL], ap[NT][NPL], dp[NT][NPL];
  T r[NT], q[NT], m[NT], m1[NT], m2[NT], ia[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ia[t] = T(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      G[t][k] = g[t][k];
      Pp[t][k] = p[t][k];
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    T AG[NT][NPL], ATP[NT][NPL];  // drift: A G and A^T P
    if constexpr (C::DR) {
#pragma unroll
      for (int t = 0; t < NT; ++t) matvec2<C>(L.aop, 0, G[t], AG[t], 1, Pp[t], ATP[t]);
    }
    reduce_rq<C, NT>(G, Pp, L, r, q, dp);
#pragma unroll
    for (int t = 0; t < NT; ++t) speed<C, false>(P, r[t], m[t], m1[t], m2[t]);
    const T bw = (s == 0 || s == 3) ? T(1) : T(2);  // RK4 weights (1, 2, 2, 1)
    const T cn = (s == 2) ? h : h2;                 // next stage offset c_{s+1} h
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (QUAD) ia[t] += bw * integrand(P, r[t], q[t], m[t], m1[t]);
      const T cx = q[t] * m1[t] + P.w;
      const T ag_c = -(bw * m[t]), ap_c = bw * cx;  // stage-sum coefficients
      const T gn_c = -(cn * m[t]), pn_c = cn * cx;  // next-stage coefficients
      if constexpr (C::DR) {
        // with drift the stage derivative K = (-(A G + m D P), A^T P + cx G)
        // is formed once (two FMAs) and enters the stage sum and the next
        // stage state through one FMA each
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const T kg = fmaT(-m[t], dp[t][k], -AG[t][k]);
          const T kp = fmaT(cx, G[t][k], ATP[t][k]);
          ag[t][k] = s == 0 ? kg : fmaT(bw, kg, ag[t][k]);
          ap[t][k] = s == 0 ? kp : fmaT(bw, kp, ap[t][k]);
          if (s < 3) {
            G[t][k] = fmaT(cn, kg, g[t][k]);
            Pp[t][k] = fmaT(cn, kp, p[t][k]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const T ag0 = s == 0 ? T(0) : ag[t][k], ap0 = s == 0 ? T(0) : ap[t][k];
          ag[t][k] = fmaT(ag_c, dp[t][k], ag0);
          ap[t][k] = fmaT(ap_c, G[t][k], ap0);
          if (s < 3) {
            Pp[t][k] = fmaT(pn_c, G[t][k], p[t][k]);
            G[t][k] = fmaT(gn_c, dp[t][k], g[t][k]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (QUAD) acc[t] += h6 * ia[t];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      g[t][k] = fmaT(h6, ag[t][k], g[t][k]);
      p[t][k] = fmaT(h6, ap[t][k], p[t][k]);
    }
  }
}

// Integrand at a node (trapezoid rule).
template <class C, int NT>
__device__ __forceinline__ void node_integrand(const Problem<typename C::T>& P,
                                               const LaneParams<C>& L,
                                               const typename C::T (&g)[NT][C::NPL],
                                               const typename C::T (&p)[NT][C::NPL],
                                               typename C::T (&out)[NT]) {
  using T = typename C::T;
  T r[NT], q[NT];
  reduce_rq<C, NT>(g, p, L, r, q);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T m, m1, m2;
    speed<C, false>(P, r[t], m, m1, m2);
    out[t] = integrand(P, r[t], q[t], m, m1);
  }
}

// Checkpoint storage, blocked by wavefront: the 2 NPL values of slot c of
// the 64 lanes of wave w form one block of 2 NPL x 64 elements at block index
// c * (stride / 64) + w, component-major inside (stride = lanes of the
// arrays, a multiple of 64).  Loads and stores are coalesced across the wave
// and the per-component offsets are small compile-time constants, so no
// per-component address registers are needed.
template <typename T, int NPL>
__device__ __forceinline__ T* state_block(T* base, size_t stride, size_t lane, int c) {
  const size_t blk = (size_t)c * (stride >> 6) + (lane >> 6);
  return base + blk * (2 * NPL * 64) + (lane & 63);
}
template <typename T, int NPL>
__device__ __forceinline__ void store_state(T* base, size_t stride, size_t lane, int c,
                                            const T (&g)[NPL], const T (&p)[NPL]) {
  T* b = state_block<T, NPL>(base, stride, lane, c);
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    b[k * 64] = g[k];
    b[(NPL + k) * 64] = p[k];
  }
}
template <typename T, int NPL>
__device__ __forceinline__ void load_state(const T* base, size_t stride, size_t lane, int c,
                                           T (&g)[NPL], T (&p)[NPL]) {
  const T* b = state_block<T, NPL>(const_cast<T*>(base), stride, lane, c);
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    g[k] = b[k * 64];
    p[k] = b[(NPL + k) * 64];
  }
}

// Objective (paper section 4.1 functionals F and G, discretised) for NT
// trajectories started at (x, v[t]); also the certificate residual rho and,
// with STORE, the states y_{cK} (c = 0 .. ceil(N/K)-1) and y_N (slot
// ceil(N/K)) for the adjoint of trajectory 0.
template <class C, int NT, bool STORE>
__device__ __forceinline__ void forward(const Problem<typename C::T>& P, const LaneParams<C>& L,
                                        const typename C::T (&x)[C::NPL],
                                        const typename C::T (&v)[NT][C::NPL],
                                        typename C::T (&phi)[NT], typename C::T (&rho)[NT],
                                        typename C::T* ck = nullptr, size_t stride = 0,
                                        size_t lane = 0, int K = 1,
                                        typename C::T (*yN_g)[C::NPL] = nullptr,
                                        typename C::T (*yN_p)[C::NPL] = nullptr) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  T g[NT][NPL], p[NT][NPL], acc[NT], xv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = T(0);
    xv[t] = T(0);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      g[t][k] = x[k];
      p[t][k] = v[t][k];
      if (P.formula == HJ_HOPF) xv[t] += x[k] * v[t][k];  // <x, v> of the Hopf objective
    }
  }
  const bool aug = (P.quad == HJ_RK4AUG);
  if (!aug) {
    T io[NT];
    node_integrand<C, NT>(P, L, g, p, io);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] += T(0.5) * P.h * io[t];
  }
  for (int s = 0; s < P.N; ++s) {
    if (STORE && (s % K) == 0) store_state<T, NPL>(ck, stride, lane, s / K, g[0], p[0]);
    if (aug) {
      rk4_step<C, NT, true>(P, L, g, p, acc);
    } else {
      rk4_step<C, NT, false>(P, L, g, p, acc);
      T io[NT];
      node_integrand<C, NT>(P, L, g, p, io);
      const T wk = (s + 1 < P.N) ? P.h : T(0.5) * P.h;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] += wk * io[t];
    }
  }
  if (STORE) store_state<T, NPL>(ck, stride, lane, (P.N + K - 1) / K, g[0], p[0]);
  // terminal term, residual
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T term = T(0), res = T(0);
    if (P.formula == HJ_LAX) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        term += g[t][k] * g[t][k] * L.ia2(k);
        res = nanmax(res, dabs(p[t][k] - g[t][k] * L.ia2(k)));
      }
      term = T(0.5) * csum<C>(term) + P.j0;
    } else {
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        term += L.a2(k) * p[t][k] * p[t][k];
        res = nanmax(res, dabs(g[t][k] - L.a2(k) * p[t][k]));
      }
      term = T(0.5) * csum<C>(term) - P.j0 - csum<C>(xv[t]);
    }
    phi[t] = term + acc[t];
    rho[t] = cmax<C>(res);
    if (yN_g) {
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        yN_g[t][k] = g[t][k];
        yN_p[t][k] = p[t][k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Discrete adjoint (exact gradient of the discretised objective).
// ---------------------------------------------------------------------------

// Scalars of one stage state.
template <typename T> struct StageScal {
  T r, q, m, m1, m2;
};

template <class C>
__device__ __forceinline__ StageScal<typename C::T> stage_scalars(
    const Problem<typename C::T>& P, const LaneParams<C>& L, const typename C::T (&G)[C::NPL],
    const typename C::T (&Pp)[C::NPL]) {
  using T = typename C::T;
  StageScal<T> S;
  T dp[C::NPL];
#pragma unroll
  for (int k = 0; k < C::NPL; ++k) dp[k] = L.dk(k) * Pp[k];
  S.r = csum<C>(dot2<C::NPL>(G, G));
  S.q = csum<C>(dot2<C::NPL>(dp, Pp));
  speed<C, true>(P, S.r, S.m, S.m1, S.m2);
  return S;
}

// Coefficients of the integrand gradient: grad_gamma = cg gamma,
// grad_p = cp D p.
template <typename T>
__device__ __forceinline__ void integrand_grad_coef(const Problem<T>& P, const StageScal<T>& S,
                                                    T& cg, T& cp) {
  if (P.formula == HJ_LAX) {
    cg = S.q * S.m1 - P.w;
    cp = S.m;
  } else {
    cg = -(S.q * (S.m1 + T(2) * S.r * S.m2) + P.w);
    cp = S.m - T(2) * S.r * S.m1;
  }
}

// Vector-Jacobian product of f at a stage state, plus wb * grad(integrand):
//   out_gamma = -A^T kg - 2 m' <D p, kg> gamma + 2 q m'' <gamma, kp> gamma
//               + (q m' + w) kp + wb cg gamma
//   out_p     = A kp + D (-m kg + 2 m' <gamma, kp> p + wb cp p)
// (the A terms with drift only).  (kg, kp) is read from and out is written
// to the same arrays.
template <class C>
__device__ __forceinline__ void vjp_stage(const Problem<typename C::T>& P, const LaneParams<C>& L,
                                          const typename C::T (&G)[C::NPL],
                                          const typename C::T (&Pp)[C::NPL],
                                          const StageScal<typename C::T>& S, typename C::T wb,
                                          typename C::T (&kg)[C::NPL],
                                          typename C::T (&kp)[C::NPL]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  T dp[NPL];
#pragma unroll
  for (int k = 0; k < NPL; ++k) dp[k] = L.dk(k) * Pp[k];
  const T s1 = csum<C>(dot2<NPL>(dp, kg));
  const T s2 = csum<C>(dot2<NPL>(G, kp));
  T cg = T(0), cp = T(0);
  if (wb != T(0)) integrand_grad_coef(P, S, cg, cp);
  const T ag = T(-2) * S.m1 * s1 + T(2) * S.q * S.m2 * s2 + wb * cg;
  const T al = S.q * S.m1 + P.w;
  const T ap = T(2) * S.m1 * s2 + wb * cp;
  if constexpr (C::DR) {
    T ATk[NPL], Ak[NPL];
    matvec2<C>(L.aop, 1, kg, ATk, 0, kp, Ak);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const T og = fmaT(al, kp[k], fmaT(ag, G[k], -ATk[k]));
      const T op = fmaT(ap, dp[k], fmaT(-S.m, L.dk(k) * kg[k], Ak[k]));
      kg[k] = og;
      kp[k] = op;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const T og = fmaT(al, kp[k], ag * G[k]);
      const T op = fmaT(ap, dp[k], -S.m * (L.dk(k) * kg[k]));
      kg[k] = og;
      kp[k] = op;
    }
  }
}

// Reverse sweep through one RK4 step from y_k = (g, p): lam holds d(obj)/d
// y_{k+1} on entry and d(obj)/d y_k on exit.  This form recomputes the stage
// states once and keeps them in registers; with drift they are not local to
// a component (A mixes them), so the drift kernels use it.
template <class C>
__device__ __forceinline__ void reverse_step_stored(const Problem<typename C::T>& P,
                                             const LaneParams<C>& L,
                                             const typename C::T (&g)[C::NPL],
                                             const typename C::T (&p)[C::NPL], bool aug,
                                             typename C::T (&lg)[C::NPL],
                                             typename C::T (&lp)[C::NPL]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  const T h = P.h, h2 = T(0.5) * P.h, h6 = P.h / T(6), h3 = P.h / T(3);
  T YG[3][NPL], YP[3][NPL];  // stage states 2..4 (stage 1 is y_k itself)
  StageScal<T> S[4];
  S[0] = stage_scalars<C>(P, L, g, p);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const T cn = (s == 2) ? h : h2;
    const T cx = S[s].q * S[s].m1 + P.w;
    const T gn_c = -(cn * S[s].m), pn_c = cn * cx;  // as in rk4_step
    if constexpr (C::DR) {
      T AG[NPL], ATP[NPL];
      if (s == 0)
        matvec2<C>(L.aop, 0, g, AG, 1, p, ATP);
      else
        matvec2<C>(L.aop, 0, YG[s - 1], AG, 1, YP[s - 1], ATP);
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        const T gs = s ? YG[s - 1][k] : g[k];
        const T ps = s ? YP[s - 1][k] : p[k];
        const T kg = fmaT(-S[s].m, L.dk(k) * ps, -AG[k]);  // as in rk4_step
        const T kp = fmaT(cx, gs, ATP[k]);
        YG[s][k] = fmaT(cn, kg, g[k]);
        YP[s][k] = fmaT(cn, kp, p[k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        const T gs = s ? YG[s - 1][k] : g[k];
        const T ps = s ? YP[s - 1][k] : p[k];
        YG[s][k] = fmaT(gn_c, L.dk(k) * ps, g[k]);
        YP[s][k] = fmaT(pn_c, gs, p[k]);
      }
    }
    S[s + 1] = stage_scalars<C>(P, L, YG[s], YP[s]);
  }
  // ybar accumulates d/dy_k; bg/bp carries Ybar of the stage above.
  T yg[NPL], yp[NPL], bg[NPL], bp[NPL];
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    yg[k] = lg[k];
    yp[k] = lp[k];
  }
#pragma unroll
  for (int s = 3; s >= 0; --s) {
    const T wb = (s == 0 || s == 3) ? h6 : h3;
    const T cn = (s == 2) ? h : h2;  // c_{s+1} h: offset of stage s+1 on K_s
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      if (s == 3) {
        bg[k] = wb * lg[k];
        bp[k] = wb * lp[k];
      } else {
        bg[k] = wb * lg[k] + cn * bg[k];
        bp[k] = wb * lp[k] + cn * bp[k];
      }
    }
    if (s == 0)
      vjp_stage<C>(P, L, g, p, S[0], aug ? wb : T(0), bg, bp);
    else
      vjp_stage<C>(P, L, YG[s - 1], YP[s - 1], S[s], aug ? wb : T(0), bg, bp);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      yg[k] += bg[k];
      yp[k] += bp[k];
    }
  }
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    lg[k] = yg[k];
    lp[k] = yp[k];
  }
}

// Without drift, stage s + 1 of the RK4 step is, component by component,
//   G_{s+1} = g - c_s h m_s d P_s,   P_{s+1} = p + c_s h (q_s m'_s + w) G_s,
// so once the stage scalars are known every stage state follows from
// (g, p) with a few FMAs per component.  This form finds the scalars with one
// pass over the stages and recomputes each stage state where its
// vector-Jacobian product needs it, instead of holding all of them: the same
// arithmetic (bit for bit) with four fewer vectors live.
template <class C>
__device__ __forceinline__ void reverse_step_lean(const Problem<typename C::T>& P,
                                                  const LaneParams<C>& L,
                                                  const typename C::T (&g)[C::NPL],
                                                  const typename C::T (&p)[C::NPL], bool aug,
                                                  typename C::T (&lg)[C::NPL],
                                                  typename C::T (&lp)[C::NPL]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  const T h = P.h, h2 = T(0.5) * P.h, h6 = P.h / T(6), h3 = P.h / T(3);
  StageScal<T> S[4];
  T G[NPL], Pp[NPL];  // the stage state being visited
  // pass 1: stage scalars; leaves stage 3 in (G, Pp)
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    G[k] = g[k];
    Pp[k] = p[k];
  }
  S[0] = stage_scalars<C>(P, L, G, Pp);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const T cn = (s == 2) ? h : h2;
    const T gn_c = -(cn * S[s].m), pn_c = cn * (S[s].q * S[s].m1 + P.w);  // as in rk4_step
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      const T gs = G[k], ps = Pp[k];
      G[k] = fmaT(gn_c, L.dk(k) * ps, g[k]);
      Pp[k] = fmaT(pn_c, gs, p[k]);
    }
    S[s + 1] = stage_scalars<C>(P, L, G, Pp);
  }
  // pass 2: adjoint of the stages, last to first
  T yg[NPL], yp[NPL], bg[NPL], bp[NPL];
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    yg[k] = lg[k];
    yp[k] = lp[k];
  }
#pragma unroll
  for (int s = 3; s >= 0; --s) {
    const T wb = (s == 0 || s == 3) ? h6 : h3;
    const T cn = (s == 2) ? h : h2;  // c_{s+1} h: offset of stage s+1 on K_s
    if (s < 3) {
      // stage state s from (g, p) through the recurrence
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        G[k] = g[k];
        Pp[k] = p[k];
      }
#pragma unroll
      for (int u = 0; u < s; ++u) {
        const T cu = (u == 2) ? h : h2;
        T gn_c = -(cu * S[u].m), pn_c = cu * (S[u].q * S[u].m1 + P.w);
        // opaque copies: otherwise the compiler recognises the pass-1 values
        // and keeps those stage states live instead of recomputing them
        asm volatile("" : "+v"(gn_c), "+v"(pn_c));
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const T gs = G[k], ps = Pp[k];
          G[k] = fmaT(gn_c, L.dk(k) * ps, g[k]);
          Pp[k] = fmaT(pn_c, gs, p[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      if (s == 3) {
        bg[k] = wb * lg[k];
        bp[k] = wb * lp[k];
      } else {
        bg[k] = wb * lg[k] + cn * bg[k];
        bp[k] = wb * lp[k] + cn * bp[k];
      }
    }
    vjp_stage<C>(P, L, G, Pp, S[s], aug ? wb : T(0), bg, bp);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
      yg[k] += bg[k];
      yp[k] += bp[k];
    }
  }
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    lg[k] = yg[k];
    lp[k] = yp[k];
  }
}

template <class C>
__device__ __forceinline__ void reverse_step(const Problem<typename C::T>& P,
                                             const LaneParams<C>& L,
                                             const typename C::T (&g)[C::NPL],
                                             const typename C::T (&p)[C::NPL], bool aug,
                                             typename C::T (&lg)[C::NPL],
                                             typename C::T (&lp)[C::NPL]) {
  if constexpr (C::DR)
    reverse_step_stored<C>(P, L, g, p, aug, lg, lp);
  else
    reverse_step_lean<C>(P, L, g, p, aug, lg, lp);
}

// lam += wk * grad(integrand)(y)   (trapezoid node term)
template <class C>
__device__ __forceinline__ void add_node_grad(const Problem<typename C::T>& P,
                                              const LaneParams<C>& L,
                                              const typename C::T (&g)[C::NPL],
                                              const typename C::T (&p)[C::NPL], typename C::T wk,
                                              typename C::T (&lg)[C::NPL],
                                              typename C::T (&lp)[C::NPL]) {
  using T = typename C::T;
  const StageScal<T> S = stage_scalars<C>(P, L, g, p);
  T cg, cp;
  integrand_grad_coef(P, S, cg, cp);
#pragma unroll
  for (int k = 0; k < C::NPL; ++k) {
    lg[k] += wk * cg * g[k];
    lp[k] += wk * cp * L.dk(k) * p[k];
  }
}

// Gradient of the objective w.r.t. (x, v) from the checkpoints written by
// forward<STORE>.  seg is per-lane scratch for K states.
template <class C>
__device__ __forceinline__ void backward(const Problem<typename C::T>& P, const LaneParams<C>& L,
                                         const typename C::T (&x)[C::NPL],
                                         const typename C::T (&v)[C::NPL],
                                         const typename C::T* ck, typename C::T* seg,
                                         size_t stride, size_t lane, int K,
                                         typename C::T (&gv)[C::NPL],
                                         typename C::T (&gx)[C::NPL]) {
  using T = typename C::T;
  constexpr int NPL = C::NPL;
  const bool aug = (P.quad == HJ_RK4AUG);
  const int nseg = (P.N + K - 1) / K;
  // the recomputed states y_{k0+1} .. y_{k1-1} of a segment: in LDS
  // (C::kSegLds states; the host keeps K <= C::kSegLds + 1) or in the
  // global scratch, in the same blocked layout
  constexpr int SL = C::kSegLds;
  __shared__ T s_seg[SL > 0 ? SL * 2 * NPL * 256 : 1];
  T* const segp = SL > 0 ? s_seg : seg;
  const size_t sstride = SL > 0 ? 256 : stride;
  const size_t slane = SL > 0 ? (size_t)threadIdx.x : lane;
  T lg[NPL], lp[NPL], g[NPL], p[NPL];
  load_state<T, NPL>(ck, stride, lane, nseg, g, p);  // y_N
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    if (P.formula == HJ_LAX) {
      lg[k] = g[k] * L.ia2(k);
      lp[k] = T(0);
    } else {
      lg[k] = T(0);
      lp[k] = L.a2(k) * p[k];
    }
  }
  if (!aug) add_node_grad<C>(P, L, g, p, T(0.5) * P.h, lg, lp);
  for (int c = nseg - 1; c >= 0; --c) {
    const int k0 = c * K;
    const int k1 = (k0 + K < P.N) ? k0 + K : P.N;
    // recompute y_{k0+1} .. y_{k1-1} from checkpoint c with the forward's
    // own step function
    load_state<T, NPL>(ck, stride, lane, c, g, p);
    for (int j = k0 + 1; j < k1; ++j) {
      T gg[1][NPL], pp[1][NPL], dummy[1] = {T(0)};
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        gg[0][k] = g[k];
        pp[0][k] = p[k];
      }
      rk4_step<C, 1, false>(P, L, gg, pp, dummy);
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        g[k] = gg[0][k];
        p[k] = pp[0][k];
      }
      store_state<T, NPL>(segp, sstride, slane, j - k0 - 1, g, p);
    }
    // reverse sweep over the segment, from y_{k1-1} (in registers); each
    // earlier state is loaded where its step needs it (no state is carried
    // ahead: the registers are worth more than the hidden latency)
    for (int j = k1 - 1; j >= k0; --j) {
      if (j < k1 - 1) {
        if (j > k0)
          load_state<T, NPL>(segp, sstride, slane, j - k0 - 1, g, p);
        else
          load_state<T, NPL>(ck, stride, lane, c, g, p);
      }
      reverse_step<C>(P, L, g, p, aug, lg, lp);
      if (!aug) add_node_grad<C>(P, L, g, p, j == 0 ? T(0.5) * P.h : P.h, lg, lp);
    }
  }
#pragma unroll
  for (int k = 0; k < NPL; ++k) {
    gv[k] = lp[k] - (P.formula == HJ_HOPF ? x[k] : T(0));
    gx[k] = lg[k] - (P.formula == HJ_HOPF ? v[k] : T(0));
  }
}

}  // namespace hj
