// hj_api.hip -- host side of the C interface declared in include/hj.h:
// argument checks, parameter staging, workspace layout, and the dispatch of
// the kernel instances by (dtype, lane shape, speed profile).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hj.h"
#include "hj_launch.hpp"

// Scratch of hj_solve_noalloc: a file-scope device array, one copy per
// device, that the library holds until the process ends.  Host code never
// passes the array's name to a kernel or a copy (in host code the name is a
// host-side stand-in, not a device address): each device's address comes
// from hipGetSymbolAddress, taken once with that device current.
static __device__ __align__(256) unsigned char scratch[HJ_NOALLOC_BYTES];

namespace {

using hj::Shape;

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HJ_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(HJ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

// Library-owned scratch, one grow-only allocation per device.
struct DevScratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
DevScratch g_ws[64];

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The lane shape for n: with drift, the smallest matrix-core shape covering
// n (4 lanes per task); otherwise with lpt == 0 the first default shape
// covering n (FP32 with 64 < n <= 112: 16 lanes of 7 components), else the
// smallest compiled shape with that many lanes per task.
bool pick_shape(int n, int lpt, bool drift, bool f32, Shape& s) {
  if (drift) {
    if (lpt != 0 && lpt != 4) return false;
    for (int npl : hj::kDriftNpl)
      if (n <= 4 * npl) {
        s = Shape{npl, 4, true};
        return true;
      }
    return false;
  }
  if (lpt == 0) {
    if (f32 && n > 64 && n <= hj::kF32Wide.npad()) {
      s = hj::kF32Wide;
      return true;
    }
    for (int i = 0; i < hj::kNumDefaultShapes; ++i)
      if (n <= hj::kShapes[i].npad()) {
        s = hj::kShapes[i];
        return true;
      }
    return false;
  }
  bool found = false;
  for (const Shape& t : hj::kShapes)
    if (t.lpt == lpt && n <= t.npad() && (!found || t.npl < s.npl)) {
      s = t;
      found = true;
    }
  return found;
}

// Elements of the MFMA operand table of A and A^T for NPL components per lane.
size_t drift_table_len(int npl) { return (size_t)2 * (npl / 4) * npl * 64; }

// The table itself: element [m][ib][kb][l] = M_m[16 ib + row(l % 16)][4 kb + l / 16]
// with M_0 = A, M_1 = A^T (zero outside n x n): lane l supplies that element
// of the 16x4 block (ib, kb) as the MFMA's first operand.  The FP64 16x16x4
// MFMA returns block row 4 r + l / 16 in register r of lane l, the FP32 one
// row 4 (l / 16) + r; row() reorders the FP32 rows so that in both cases
// register r of lane `sub` receives component 16 ib + 4 r + sub, which that
// lane owns (slot 4 ib + r).  Built on the device from A (row-major, FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_drift_table(const double* A, int n, int npl, T* table) {
  const int NB = npl / 4;
  const int total = 2 * NB * npl * 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int l = idx % 64, kb = (idx / 64) % npl, ib = (idx / (64 * npl)) % NB;
  const int m = idx / (64 * npl * NB);
  const int i = l % 16;
  const int ri = sizeof(T) == 8 ? i : 4 * (i % 4) + i / 4;
  const int row = 16 * ib + ri, col = 4 * kb + l / 16;
  double val = 0.0;
  if (row < n && col < n) val = (m == 0) ? A[row * n + col] : A[col * n + row];
  table[idx] = (T)val;
}

// Stream-ordered upload of small host data (the per-component parameters,
// the drift matrix) into device memory through kernel arguments: the
// runtime copies a launch's argument block when the launch is enqueued, so
// the host needs no staging buffer, returns without waiting, and may reuse
// its memory at once; the copy is ordered after earlier work on the stream.
constexpr int kUploadWords = 736;  // 2944 bytes of payload per launch
struct Upload {
  uint64_t off;  // destination offset in 32-bit words
  uint32_t n;    // words used in w
  uint32_t pad_;
  uint32_t w[kUploadWords];
};
__global__ __launch_bounds__(256) void k_upload(uint32_t* dst, Upload u) {
  for (uint32_t i = threadIdx.x; i < u.n; i += blockDim.x) dst[u.off + i] = u.w[i];
}

class Uploader {
 public:
  Uploader(void* dst, hipStream_t st) : dst_(static_cast<uint32_t*>(dst)), st_(st) {
    u_.off = 0;
    u_.n = 0;
    u_.pad_ = 0;
  }
  template <typename T> void put(T v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized values");
    uint32_t w[sizeof(T) / 4];
    std::memcpy(w, &v, sizeof(T));
    for (uint32_t x : w) {
      if (u_.n == kUploadWords) (void)flush();
      u_.w[u_.n++] = x;
    }
  }
  // continue at a byte offset (a multiple of 4) at or after the current one
  void seek(size_t byte_off) {
    (void)flush();
    u_.off = byte_off / 4;
  }
  hipError_t flush() {
    if (u_.n > 0 && err_ == hipSuccess) {
      hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st_, dst_, u_);
      err_ = hipGetLastError();
    }
    u_.off += u_.n;
    u_.n = 0;
    return err_;
  }

 private:
  uint32_t* dst_;
  hipStream_t st_;
  Upload u_;
  hipError_t err_ = hipSuccess;
};

// Layout of the scratch memory of one call.
struct WsLayout {
  size_t params = 0, slots = 0, queue = 0, ck = 0, seg = 0, total = 0;
  size_t stride = 0;  // lanes of the SoA checkpoint arrays
  // FP64 continuation of FP32 slots: hand-off list, its counters (entries,
  // continuation queue), FP64 checkpoints over stride64 lanes
  size_t handoff = 0, cont_ctr = 0, ck64 = 0, seg64 = 0, stride64 = 0;
  // FP64 tail hand-off: the records (the continuation uses cont_ctr and the
  // ck64 / seg64 checkpoints above) and, for a continuation shape of another
  // padded dimension, its own parameter rows
  size_t tail = 0, params2 = 0;
};

// lanes: lanes that hold adjoint checkpoints (0: one lane group per task);
// cont_lanes: lanes of the FP64 continuation launch (0: none)
// tail_rec: doubles per tail hand-off record (0: no hand-off); tail_npad:
// padded dimension of the continuation's parameter rows (0: the descent's)
WsLayout layout(const Shape& s, int n, int64_t B, int G, int nsteps, int dtype, int mode, int K,
                bool grad, bool solve, size_t lanes = 0, size_t cont_lanes = 0,
                int cont_npl = 0, int cont_K = 0, int tail_rec = 0, int tail_npad = 0) {
  if (cont_npl == 0) cont_npl = s.npl;
  WsLayout L;
  const size_t tsz = dtype == HJ_F32 ? 4 : 8;
  const size_t BG = (size_t)B * (size_t)G;
  size_t off = 0;
  L.params = off;
  off += align_up((size_t)s.npad() * 3 * (8 + tsz), 256);
  if (s.dr) off += align_up(drift_table_len(s.npl) * (8 + tsz) + (size_t)n * n * 8, 256);
  if (solve) {
    L.slots = off;
    off += align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256) + align_up(BG * (size_t)n * tsz, 256);
    L.queue = off;
    off += 256;
  }
  const bool need_adj = grad || (solve && mode == HJ_GD_ADJ);
  const int Kc = std::max(1, std::min(K, nsteps));
  const size_t nck = (size_t)((nsteps + Kc - 1) / Kc) + 1;
  if (need_adj) {
    if (lanes == 0) lanes = align_up(BG * (size_t)s.lpt, 256);
    L.stride = lanes;
    L.ck = off;
    off += align_up(nck * 2 * s.npl * lanes * tsz, 256);
    L.seg = off;
    off += align_up((size_t)Kc * 2 * s.npl * lanes * tsz, 256);
  }
  if (solve && cont_lanes > 0) {
    const int K64 = cont_K > 0 ? std::max(1, std::min(cont_K, nsteps)) : Kc;
    const size_t nck64 = (size_t)((nsteps + K64 - 1) / K64) + 1;
    L.handoff = off;
    off += align_up(BG * 8, 256);
    L.cont_ctr = off;
    off += 256;
    L.stride64 = cont_lanes;
    L.ck64 = off;
    off += align_up(nck64 * 2 * cont_npl * cont_lanes * 8, 256);
    L.seg64 = off;
    off += align_up((size_t)K64 * 2 * cont_npl * cont_lanes * 8, 256);
    if (tail_rec > 0) {
      L.tail = off;
      off += align_up(BG * (size_t)tail_rec * 8, 256);
    }
    if (tail_npad > 0) {
      L.params2 = off;
      off += align_up((size_t)tail_npad * 3 * (8 + 8), 256);
    }
  }
  L.total = off;
  return L;
}

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, then kept).
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64];

int noalloc_scratch(void** out) {
  int dev = 0;
  HJ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HJ_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HJ_EDEVICE, "hipGetSymbolAddress returned no address for the scratch");
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return HJ_OK;
}

int get_workspace(const hj_opts* o, size_t need, void** out) {
  if (o && o->workspace) {
    if (o->ws_bytes < need)
      return fail(HJ_ENOMEM, "workspace of " + std::to_string(o->ws_bytes) +
                                 " bytes is smaller than the " + std::to_string(need) +
                                 " bytes needed");
    *out = o->workspace;
    return HJ_OK;
  }
  int dev = 0;
  HJ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HJ_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  DevScratch& w = g_ws[dev];
  if (w.bytes < need) {
    if (w.ptr) {
      // the previous buffer may still be in use by queued work
      HJ_HIP(hipDeviceSynchronize());
      HJ_HIP(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t bytes = std::max(need, (size_t)1 << 20);
    if (hipMalloc(&w.ptr, bytes) != hipSuccess) {
      w.ptr = nullptr;
      return fail(HJ_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    w.bytes = bytes;
  }
  *out = w.ptr;
  return HJ_OK;
}

int check_problem(int H_kind, const hj_h_params* H, int J_kind, const hj_j_params* J, int n,
                  double t, int nsteps) {
  if (H_kind != HJ_H_QUADRATIC && H_kind != HJ_H_NORM)
    return fail(HJ_EUNSUPPORTED, "unknown H_kind");
  if (J_kind != HJ_J_ELLIPSOID && J_kind != HJ_J_ROSENBROCK)
    return fail(HJ_EUNSUPPORTED, "unknown J_kind");
  if (!H || !J) return fail(HJ_EINVAL, "H and J parameters are required");
  if (n < 1) return fail(HJ_EINVAL, "n must be >= 1");
  if (n > HJ_MAX_N) return fail(HJ_EUNSUPPORTED, "n above HJ_MAX_N");
  if (!(t > 0.0) || !std::isfinite(t)) return fail(HJ_EINVAL, "t must be finite and > 0");
  if (nsteps < 1) return fail(HJ_EINVAL, "nsteps must be >= 1");
  if (H_kind == HJ_H_QUADRATIC) {
    if (H->m_kind < HJ_M_CONST || H->m_kind > HJ_M_TANH) return fail(HJ_EINVAL, "bad m_kind");
    if (H->e != 1 && H->e != 2) return fail(HJ_EINVAL, "e must be 1 or 2");
    if (H->m_kind == HJ_M_TANH && !(H->s > 0.0))
      return fail(HJ_EINVAL, "tanh scale s must be > 0");
    if (!H->d) return fail(HJ_EINVAL, "the weights d are required");
    if (H->A)
      for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(H->A[i]))
          return fail(HJ_EINVAL, "drift matrix entries must be finite");
  } else {
    if (!H->mu) return fail(HJ_EINVAL, "the centre mu is required");
    if (H->k < 0 || H->k > n) return fail(HJ_EINVAL, "block size k must be in [0, n]");
    if (!std::isfinite(H->s1) || !std::isfinite(H->s2) || !std::isfinite(H->c0) ||
        !std::isfinite(H->beta) || !(H->gam >= 0.0) || !std::isfinite(H->gam))
      return fail(HJ_EINVAL, "s1, s2, c0, beta must be finite and gam >= 0");
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(H->mu[i])) return fail(HJ_EINVAL, "mu must be finite");
  }
  if (J_kind == HJ_J_ROSENBROCK) {
    if (n != 2) return fail(HJ_EUNSUPPORTED, "the Rosenbrock initial data take n = 2");
    if (!std::isfinite(J->rscale)) return fail(HJ_EINVAL, "rscale must be finite");
  } else {
    if (!J->a) return fail(HJ_EINVAL, "the ellipsoid axes a are required");
    for (int i = 0; i < n; ++i)
      if (!(J->a[i] != 0.0) || !std::isfinite(J->a[i]))
        return fail(HJ_EINVAL, "ellipsoid axes must be finite and nonzero");
  }
  return HJ_OK;
}

// Host copies of the per-component parameters, padded to npad.
template <typename T> struct HostParams {
  std::vector<T> d, a2, ia2;
};
template <typename T>
HostParams<T> host_params(const hj_h_params* H, const hj_j_params* J, int n, int npad) {
  HostParams<T> p;
  p.d.assign(npad, T(0));
  p.a2.assign(npad, T(1));
  p.ia2.assign(npad, T(1));
  for (int i = 0; i < n; ++i) {
    const double a = J->a[i];
    p.d[i] = (T)H->d[i];
    p.a2[i] = (T)(a * a);
    p.ia2[i] = (T)(1.0 / (a * a));
  }
  return p;
}

// Kernel speed profile: TANH, or RAT (which with kappa = 0 is CONST).
int kernel_mk(const hj_h_params* H) { return H->m_kind == HJ_M_TANH ? HJ_M_TANH : HJ_M_RAT; }

template <typename T>
hj::Problem<T> make_problem(const hj_h_params* H, const hj_j_params* J, int n, double t,
                            int nsteps, int formula, int quad, const T* base, int npad) {
  hj::Problem<T> P;
  P.n = n;
  P.N = nsteps;
  P.e = H->e;
  P.formula = formula;
  P.quad = quad;
  P.kappa = (T)(H->m_kind == HJ_M_CONST ? 0.0 : H->kappa);
  P.inv_s = (T)(H->m_kind == HJ_M_TANH ? 1.0 / H->s : 1.0);
  P.w = (T)H->w;
  P.j0 = (T)J->j0;
  P.h = (T)(t / nsteps);
  P.d = base;
  P.a2 = base + npad;
  P.ia2 = base + 2 * npad;
  P.aop = nullptr;
  return P;
}

// Stage d, a^2, 1/a^2 (in T and in double) into the params region through
// kernel-argument uploads, followed with drift by A (FP64) and the MFMA
// operand tables built from it on the device (in double and in T).  Every
// step is enqueued on the stream, ordered after earlier calls' kernels that
// read the region; the host does not wait.
template <typename T>
int stage_params(const hj_h_params* H, const hj_j_params* J, int n, const Shape& s,
                 char* region, hipStream_t st, const T** dT, const double** dD,
                 const T** aT, const double** aD) {
  const int npad = s.npad();
  const size_t plen = (size_t)npad * 3 * (sizeof(T) + 8);
  const size_t tlen = s.dr ? drift_table_len(s.npl) : 0;
  Uploader up(region, st);
  // d, a^2, 1/a^2 in T, then in double; padding: d = 0, a = 1
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = 0; q < 3; ++q)
      for (int i = 0; i < npad; ++i) {
        double val = (q == 0) ? 0.0 : 1.0;
        if (i < n) {
          const double a = J->a[i];
          val = q == 0 ? H->d[i] : q == 1 ? a * a : 1.0 / (a * a);
        }
        if (pass == 0)
          up.put<T>((T)val);
        else
          up.put<double>(val);
      }
  }
  if (tlen) {
    // A after the two tables
    up.seek(plen + tlen * (8 + sizeof(T)));
    for (int i = 0; i < n * n; ++i) up.put<double>(H->A[i]);
  }
  HJ_HIP(up.flush());
  *dT = reinterpret_cast<const T*>(region);
  *dD = reinterpret_cast<const double*>(region + 3 * npad * sizeof(T));
  *aD = nullptr;
  *aT = nullptr;
  if (tlen) {
    double* t64 = reinterpret_cast<double*>(region + plen);
    T* tT = reinterpret_cast<T*>(region + plen + tlen * 8);
    const double* Ad = reinterpret_cast<const double*>(region + plen + tlen * (8 + sizeof(T)));
    const unsigned grid = (unsigned)((tlen + 255) / 256);
    hipLaunchKernelGGL(k_drift_table<double>, dim3(grid), dim3(256), 0, st, Ad, n, s.npl, t64);
    HJ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_drift_table<T>, dim3(grid), dim3(256), 0, st, Ad, n, s.npl, tT);
    HJ_HIP(hipGetLastError());
    *aD = t64;
    *aT = tT;
  }
  return HJ_OK;
}

// Launchers by shape and speed profile.
template <typename T>
hipError_t dispatch_solve(const Shape& s, int mk, const hj::SolveArgs<T>& A, int mode,
                          int64_t grid_groups, hipStream_t st) {
  if (s.dr) {
#define HJ_DCASE(NPL)                                                                         \
  if (s.npl == NPL)                                                                           \
    return mk == HJ_M_TANH ? hj::launch_solve<hj::Cfg<T, NPL, 4, HJ_M_TANH, true>>(          \
                                 A, mode, grid_groups, st)                                    \
                           : hj::launch_solve<hj::Cfg<T, NPL, 4, HJ_M_RAT, true>>(           \
                                 A, mode, grid_groups, st);
    HJ_FOR_EACH_DRIFT_NPL(HJ_DCASE)
#undef HJ_DCASE
    return hipErrorInvalidValue;
  }
#define HJ_CASE(NPL, LPT)                                                                   \
  if (s.npl == NPL && s.lpt == LPT)                                                         \
    return mk == HJ_M_TANH                                                                  \
               ? hj::launch_solve<hj::Cfg<T, NPL, LPT, HJ_M_TANH>>(A, mode, grid_groups, st) \
               : hj::launch_solve<hj::Cfg<T, NPL, LPT, HJ_M_RAT>>(A, mode, grid_groups, st);
  HJ_FOR_EACH_SHAPE(HJ_CASE)
#undef HJ_CASE
  return hipErrorInvalidValue;
}

template <typename T>
int64_t dispatch_resident(const Shape& s, int mk, int mode) {
  if (s.dr) {
#define HJ_DCASE(NPL)                                                                \
  if (s.npl == NPL)                                                                  \
    return mk == HJ_M_TANH                                                           \
               ? hj::resident_groups<hj::Cfg<T, NPL, 4, HJ_M_TANH, true>>(mode)      \
               : hj::resident_groups<hj::Cfg<T, NPL, 4, HJ_M_RAT, true>>(mode);
    HJ_FOR_EACH_DRIFT_NPL(HJ_DCASE)
#undef HJ_DCASE
    return 0;
  }
#define HJ_CASE(NPL, LPT)                                                 \
  if (s.npl == NPL && s.lpt == LPT)                                       \
    return mk == HJ_M_TANH                                                \
               ? hj::resident_groups<hj::Cfg<T, NPL, LPT, HJ_M_TANH>>(mode) \
               : hj::resident_groups<hj::Cfg<T, NPL, LPT, HJ_M_RAT>>(mode);
  HJ_FOR_EACH_SHAPE(HJ_CASE)
#undef HJ_CASE
  return 0;
}

// Lane groups of a persistent launch (0: one group per task).
template <typename T>
int64_t schedule_groups(const Shape& s, int mk, int mode, int sched, int64_t ntask,
                        int max_groups) {
  if (sched == HJ_SCHED_STATIC) return 0;
  int64_t res = dispatch_resident<T>(s, mk, mode);
  if (max_groups > 0) res = std::min<int64_t>(res, max_groups);
  if (res <= 0) return 0;
  if (sched == HJ_SCHED_PERSISTENT) return std::min(res, ntask);
  // automatic: persistent once the tasks fill the device twice over
  return ntask > 2 * res ? res : 0;
}

template <typename T>
hipError_t dispatch_eval(const Shape& s, int mk, const hj::EvalArgs<T>& A, hipStream_t st) {
  if (s.dr) {
#define HJ_DCASE(NPL)                                                                        \
  if (s.npl == NPL)                                                                          \
    return mk == HJ_M_TANH ? hj::launch_eval<hj::Cfg<T, NPL, 4, HJ_M_TANH, true>>(A, st)     \
                           : hj::launch_eval<hj::Cfg<T, NPL, 4, HJ_M_RAT, true>>(A, st);
    HJ_FOR_EACH_DRIFT_NPL(HJ_DCASE)
#undef HJ_DCASE
    return hipErrorInvalidValue;
  }
#define HJ_CASE(NPL, LPT)                                                               \
  if (s.npl == NPL && s.lpt == LPT)                                                     \
    return mk == HJ_M_TANH ? hj::launch_eval<hj::Cfg<T, NPL, LPT, HJ_M_TANH>>(A, st)    \
                           : hj::launch_eval<hj::Cfg<T, NPL, LPT, HJ_M_RAT>>(A, st);
  HJ_FOR_EACH_SHAPE(HJ_CASE)
#undef HJ_CASE
  return hipErrorInvalidValue;
}

// The FP64 continuation kernels of an FP32 lane shape.
hipError_t dispatch_continue(const Shape& s, int mk, const hj::ContArgs<float>& A, bool multi,
                             int64_t grid_groups, hipStream_t st) {
  if (s.dr) {
#define HJ_DCASE(NPL)                                                                        \
  if (s.npl == NPL)                                                                          \
    return mk == HJ_M_TANH                                                                   \
               ? hj::launch_continue<hj::Cfg<double, NPL, 4, HJ_M_TANH, true>>(A, multi,     \
                                                                             grid_groups, st) \
               : hj::launch_continue<hj::Cfg<double, NPL, 4, HJ_M_RAT, true>>(A, multi,      \
                                                                            grid_groups, st);
    HJ_FOR_EACH_DRIFT_NPL(HJ_DCASE)
#undef HJ_DCASE
    return hipErrorInvalidValue;
  }
#define HJ_CASE(NPL, LPT)                                                                      \
  if (s.npl == NPL && s.lpt == LPT)                                                            \
    return mk == HJ_M_TANH ? hj::launch_continue<hj::Cfg<double, NPL, LPT, HJ_M_TANH>>(        \
                                 A, multi, grid_groups, st)                                    \
                           : hj::launch_continue<hj::Cfg<double, NPL, LPT, HJ_M_RAT>>(         \
                                 A, multi, grid_groups, st);
  HJ_FOR_EACH_SHAPE(HJ_CASE)
#undef HJ_CASE
  return hipErrorInvalidValue;
}

int64_t dispatch_resident_continue(const Shape& s, int mk) {
  if (s.dr) {
#define HJ_DCASE(NPL)                                                                    \
  if (s.npl == NPL)                                                                      \
    return mk == HJ_M_TANH                                                               \
               ? hj::resident_continue_groups<hj::Cfg<double, NPL, 4, HJ_M_TANH, true>>() \
               : hj::resident_continue_groups<hj::Cfg<double, NPL, 4, HJ_M_RAT, true>>();
    HJ_FOR_EACH_DRIFT_NPL(HJ_DCASE)
#undef HJ_DCASE
    return 0;
  }
#define HJ_CASE(NPL, LPT)                                                          \
  if (s.npl == NPL && s.lpt == LPT)                                                \
    return mk == HJ_M_TANH                                                         \
               ? hj::resident_continue_groups<hj::Cfg<double, NPL, LPT, HJ_M_TANH>>() \
               : hj::resident_continue_groups<hj::Cfg<double, NPL, LPT, HJ_M_RAT>>();
  HJ_FOR_EACH_SHAPE(HJ_CASE)
#undef HJ_CASE
  return 0;
}

// The lane shape of the FP64 continuation: the descent's, or the compiled
// shape with the requested lanes per task and the descent shape's padded
// dimension (the parameter rows of the problem are laid out for that
// dimension, and the slot records are indexed by component, not by lane).
bool cont_shape_of(const Shape& s, int lpt, Shape& cs) {
  cs = s;
  if (lpt == 0 || lpt == s.lpt) return true;
  if (s.dr) return false;
  for (const Shape& t : hj::kShapes)
    if (t.lpt == lpt && t.npad() == s.npad()) {
      cs = t;
      return true;
    }
  return false;
}

int cont_shape_for(const Shape& s, int lpt, Shape& cs) {
  if (cont_shape_of(s, lpt, cs)) return HJ_OK;
  return fail(HJ_EUNSUPPORTED, "no continuation kernel with " + std::to_string(lpt) +
                                   " lanes per task for the " + std::to_string(s.npl) + "x" +
                                   std::to_string(s.lpt) + " descent shape");
}

// The tail-continuation kernels by shape and speed profile.
hipError_t dispatch_resume(const Shape& s, int mk, const hj::SolveArgs<double>& A,
                           int64_t grid_groups, hipStream_t st) {
#define HJ_CASE(NPL, LPT)                                                                 \
  if (s.npl == NPL && s.lpt == LPT)                                                       \
    return mk == HJ_M_TANH                                                                \
               ? hj::launch_resume<hj::Cfg<double, NPL, LPT, HJ_M_TANH>>(A, grid_groups, st) \
               : hj::launch_resume<hj::Cfg<double, NPL, LPT, HJ_M_RAT>>(A, grid_groups, st);
  HJ_FOR_EACH_RESUME_SHAPE(HJ_CASE)
#undef HJ_CASE
  return hipErrorInvalidValue;
}

int64_t dispatch_resident_resume(const Shape& s, int mk) {
#define HJ_CASE(NPL, LPT)                                                          \
  if (s.npl == NPL && s.lpt == LPT)                                                \
    return mk == HJ_M_TANH                                                         \
               ? hj::resident_resume_groups<hj::Cfg<double, NPL, LPT, HJ_M_TANH>>() \
               : hj::resident_resume_groups<hj::Cfg<double, NPL, LPT, HJ_M_RAT>>();
  HJ_FOR_EACH_RESUME_SHAPE(HJ_CASE)
#undef HJ_CASE
  return 0;
}

bool has_resume(const Shape& s) {
  bool found = false;
#define HJ_CASE(NPL, LPT) \
  if (!s.dr && s.npl == NPL && s.lpt == LPT) found = true;
  HJ_FOR_EACH_RESUME_SHAPE(HJ_CASE)
#undef HJ_CASE
  return found;
}

// Whether a solve hands its slow slots to a tail continuation, and the
// continuation's lane shape: the descent's with as many lanes per task, else
// the library's shape for n with tail_lanes_per_task lanes (default 2); a
// shape of another padded dimension gets parameter rows of its own.
bool tail_active(const Shape& s, bool f64, const hj_opts* o) {
  return f64 && o->tail_budget > 0 && o->mode == HJ_GD_ADJ && !s.dr;
}
int tail_lanes(const hj_opts* o) { return o->tail_lanes_per_task > 0 ? o->tail_lanes_per_task : 2; }
bool tail_shape_of(const Shape& s, int n, int lpt, Shape& ts) {
  if (lpt == s.lpt) {
    ts = s;
  } else if (!pick_shape(n, lpt, false, false, ts)) {
    return false;
  }
  return has_resume(ts);
}
int tail_shape_for(const Shape& s, int n, const hj_opts* o, Shape& ts) {
  if (!tail_shape_of(s, n, tail_lanes(o), ts))
    return fail(HJ_EUNSUPPORTED, "no tail-continuation kernel with " +
                                     std::to_string(tail_lanes(o)) + " lanes per task for the " +
                                     std::to_string(s.npl) + "x" + std::to_string(s.lpt) +
                                     " descent shape");
  return HJ_OK;
}

// Lane groups of the FP64 continuation launch of an FP32 GD solve over ntask
// slots (0: no continuation).
int64_t continue_groups(const Shape& s, int mk, const hj_opts* o, int64_t ntask) {
  if (o->dtype != HJ_F32 || o->mode != HJ_GD_ADJ || !o->cert_fp64 || !o->fp64_continue)
    return 0;
  int64_t g = dispatch_resident_continue(s, mk);
  if (o->max_groups > 0) g = std::min<int64_t>(g, o->max_groups);
  return std::max<int64_t>(1, std::min(g, ntask));
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ULL;
}

// The lane shape of a problem, or an error naming what is not compiled.
int shape_for(const hj_h_params* H, int n, int lpt, bool f32, Shape& s) {
  const bool drift = H->A != nullptr;
  if (pick_shape(n, lpt, drift, f32, s)) return HJ_OK;
  if (drift)
    return fail(HJ_EUNSUPPORTED, "the drift kernels take n <= " +
                                     std::to_string(HJ_MAX_N_DRIFT) +
                                     " and 4 lanes per task (n = " + std::to_string(n) +
                                     ", lanes_per_task = " + std::to_string(lpt) + ")");
  return fail(HJ_EUNSUPPORTED, "no kernel with " + std::to_string(lpt) +
                                   " lanes per task for n = " + std::to_string(n));
}

// The checkpoint interval a kernel of shape s runs with: the requested one,
// at most the step count, and for the kernels that keep the recomputed
// segment in LDS at most their capacity plus one (the interval trades memory
// for recomputation; results do not depend on it).
int eff_K(int K, const Shape& s, bool f64, int nsteps) {
  int k = std::max(1, std::min(K, nsteps));
  const int cap = hj::seg_lds_states(s.npl, s.lpt, f64 ? 8 : 4, s.dr);
  if (cap > 0) k = std::min(k, cap + 1);
  return k;
}

// Scratch layout of hj_solve with the schedule it will use: the lane groups
// of a persistent descent launch (0: one per task) and of the FP64
// continuation (0: none).  A persistent launch holds checkpoints for its
// resident lanes only.
template <typename T>
WsLayout solve_layout(const Shape& s, int mk, int n, int64_t B, int G, int nsteps,
                      const hj_opts* o, int64_t* groups, int64_t* cgroups) {
  const int K = eff_K(o->ckpt_K, s, sizeof(T) == 8, nsteps);
  const int64_t ntask = B * (int64_t)G;
  *groups = schedule_groups<T>(s, mk, o->mode, o->schedule, ntask, o->max_groups);
  Shape cs{};
  int tail_rec = 0;
  int tail_npad = 0;
  if (tail_active(s, sizeof(T) == 8, o)) {
    // the tail continuation takes the continuation's counters and checkpoints
    if (!tail_shape_of(s, n, tail_lanes(o), cs)) cs = s;  // rejected by the caller
    int64_t tg = has_resume(cs) ? dispatch_resident_resume(cs, mk) : 0;
    if (o->max_groups > 0) tg = std::min<int64_t>(tg, o->max_groups);
    *cgroups = std::max<int64_t>(1, std::min<int64_t>(tg, ntask));
    tail_rec = hj::kTailHead + 2 * n;
    if (cs.npad() != s.npad()) tail_npad = cs.npad();
  } else {
    if (!cont_shape_of(s, o->cont_lanes_per_task, cs)) cs = s;  // rejected by the caller
    *cgroups = continue_groups(cs, mk, o, ntask);
  }
  const size_t ck_lanes = *groups > 0 ? align_up((size_t)*groups * s.lpt, 256) : 0;
  const size_t cont_lanes = *cgroups > 0 ? align_up((size_t)*cgroups * cs.lpt, 256) : 0;
  return layout(s, n, B, G, nsteps, o->dtype, o->mode, K, false, true, ck_lanes, cont_lanes,
                cs.npl, eff_K(K, cs, true, nsteps), tail_rec, tail_npad);
}

template <typename T>
int solve_t(const hj_h_params* H, const hj_j_params* J, const void* x, int64_t B, int n,
            double t, int nsteps, const hj_guesses* gs, const hj_opts* o, double* out_u,
            void* out_argopt, int32_t* out_cert, const hj_slot_diag* diag) {
  Shape s{}, cs{};
  int rc = shape_for(H, n, o->lanes_per_task, sizeof(T) == 4, s);
  if (rc) return rc;
  const bool tail = tail_active(s, sizeof(T) == 8, o);
  if (tail) {
    rc = tail_shape_for(s, n, o, cs);
  } else {
    if (o->tail_budget > 0)
      return fail(HJ_EUNSUPPORTED, "tail hand-offs take the FP64 adjoint descent of a "
                                   "problem without a drift matrix");
    rc = cont_shape_for(s, o->cont_lanes_per_task, cs);
  }
  if (rc) return rc;
  const int npad = s.npad();
  const int K = eff_K(o->ckpt_K, s, sizeof(T) == 8, nsteps);
  const int64_t ntask = B * (int64_t)gs->G;
  int64_t groups = 0, cgroups = 0;
  WsLayout WL = solve_layout<T>(s, kernel_mk(H), n, B, gs->G, nsteps, o, &groups, &cgroups);
  if ((size_t)B * gs->G * s.lpt > (size_t)UINT32_MAX * 128)
    return fail(HJ_EINVAL, "B * G too large for one launch");
  void* ws = nullptr;
  rc = get_workspace(o, WL.total, &ws);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  const T *dT = nullptr, *aT = nullptr;
  const double *dD = nullptr, *aD = nullptr;
  rc = stage_params<T>(H, J, n, s, base + WL.params, st, &dT, &dD, &aT, &aD);
  if (rc) return rc;

  hj::SolveArgs<T> A;
  A.P = make_problem<T>(H, J, n, t, nsteps, o->formula, o->quad, dT, npad);
  A.P64 = make_problem<double>(H, J, n, t, nsteps, o->formula, o->quad, dD, npad);
  A.P.aop = aT;
  A.P64.aop = aD;
  A.x = static_cast<const T*>(x);
  A.guesses = static_cast<const T*>(gs->init);
  A.B = B;
  A.G = gs->G;
  A.R = gs->R_max;
  A.max_iter = o->max_iter;
  A.K = K;
  A.cert_fp64 = o->cert_fp64;
  A.alpha0 = (T)o->alpha0;
  A.sigma = (T)o->fd_sigma;
  A.eps_step = (T)o->eps_step;
  A.acc_rel = (T)o->acc_rel;
  A.armijo_c = (T)o->armijo_c;
  A.v_max = (T)o->v_max;
  A.cert_tol = o->cert_tol;
  A.stride = WL.stride;
  A.ck = WL.ck ? reinterpret_cast<T*>(base + WL.ck) : nullptr;
  A.seg = WL.seg ? reinterpret_cast<T*>(base + WL.seg) : nullptr;
  // per-slot records: the caller's diag arrays where given, else scratch
  const size_t BG = (size_t)B * gs->G;
  char* sp = base + WL.slots;
  double* w_phi = reinterpret_cast<double*>(sp);
  double* w_rho = w_phi + BG;
  int32_t* w_status = reinterpret_cast<int32_t*>(w_rho + BG);
  int32_t* w_cert = w_status + BG;
  int32_t* w_iters = w_cert + BG;
  int32_t* w_att = w_iters + BG;
  int64_t* w_fwd = reinterpret_cast<int64_t*>(w_att + BG);
  int64_t* w_bwd = w_fwd + BG;
  T* w_v = reinterpret_cast<T*>(sp + align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256));
  A.out.phi = (diag && diag->phi) ? diag->phi : w_phi;
  A.out.rho = (diag && diag->rho) ? diag->rho : w_rho;
  A.out.status = (diag && diag->status) ? diag->status : w_status;
  A.out.cert = (diag && diag->cert) ? diag->cert : w_cert;
  A.out.iters = (diag && diag->iters) ? diag->iters : w_iters;
  A.out.attempts = (diag && diag->attempts) ? diag->attempts : w_att;
  A.out.n_fwd = (diag && diag->n_fwd) ? diag->n_fwd : w_fwd;
  A.out.n_bwd = (diag && diag->n_bwd) ? diag->n_bwd : w_bwd;
  A.out.v = (diag && diag->v_final) ? static_cast<T*>(diag->v_final) : w_v;
  A.ntask = ntask;
  A.queue = groups > 0 ? reinterpret_cast<unsigned long long*>(base + WL.queue) : nullptr;
  A.inst = nullptr;
  A.n_inst = 0;
  A.handoff = nullptr;
  A.handoff_n = nullptr;
  A.tail_budget = 0;
  A.tail_stride = 0;
  A.tail = nullptr;
  A.tail_n = nullptr;
  unsigned long long* ctr = nullptr;
  if (cgroups > 0) {
    ctr = reinterpret_cast<unsigned long long*>(base + WL.cont_ctr);
    if (tail) {
      A.tail_budget = o->tail_budget;
      A.tail_stride = hj::kTailHead + 2 * n;
      A.tail = reinterpret_cast<double*>(base + WL.tail);
      A.tail_n = ctr;
    } else {
      A.handoff = reinterpret_cast<int64_t*>(base + WL.handoff);
      A.handoff_n = ctr;
    }
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, ctr, 16);
    HJ_HIP(hipGetLastError());
  }

  if (o->ev_begin) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_begin), st));
  HJ_HIP(dispatch_solve<T>(s, kernel_mk(H), A, o->mode, groups, st));
  if constexpr (sizeof(T) == 8) {
    if (tail && cgroups > 0) {
      // the continuation: the same problem and records, its own lane shape,
      // checkpoints and queue; no further hand-off
      hj::SolveArgs<double> R = A;
      if (cs.npad() != s.npad()) {
        const double *d2 = nullptr, *dd2 = nullptr, *a2 = nullptr, *ad2 = nullptr;
        rc = stage_params<double>(H, J, n, cs, base + WL.params2, st, &d2, &dd2, &a2, &ad2);
        if (rc) return rc;
        R.P = make_problem<double>(H, J, n, t, nsteps, o->formula, o->quad, dd2, cs.npad());
        R.P64 = R.P;
      }
      R.tail_budget = 0;
      R.K = eff_K(K, cs, true, nsteps);
      R.ck = reinterpret_cast<double*>(base + WL.ck64);
      R.seg = reinterpret_cast<double*>(base + WL.seg64);
      R.stride = WL.stride64;
      R.queue = ctr + 8;
      HJ_HIP(dispatch_resume(cs, kernel_mk(H), R, cgroups, st));
    }
  }
  if constexpr (sizeof(T) == 4) {
    if (cgroups > 0) {
      hj::ContArgs<float> CA;
      CA.S = A;
      CA.max_iter = o->max_iter;
      CA.K = eff_K(K, cs, true, nsteps);
      CA.alpha0 = o->alpha0;
      CA.eps_step = o->eps_step;
      CA.acc_rel = o->acc_rel;
      CA.armijo_c = o->armijo_c;
      CA.v_max = o->v_max;
      CA.ck = reinterpret_cast<double*>(base + WL.ck64);
      CA.seg = reinterpret_cast<double*>(base + WL.seg64);
      CA.stride = WL.stride64;
      CA.queue = ctr + 8;
      HJ_HIP(dispatch_continue(cs, kernel_mk(H), CA, false, cgroups, st));
    }
  }
  if (o->ev_end) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_end), st));
  HJ_HIP(hj::launch_select<T>(B, gs->G, n, o->formula, A.out.phi, A.out.cert, A.out.v, out_u,
                              static_cast<T*>(out_argopt), out_cert, st));
  return HJ_OK;
}

template <typename T>
int eval_t(const hj_h_params* H, const hj_j_params* J, const void* x, int64_t B, int n,
           double t, int nsteps, const void* v, int G, const hj_opts* o, double* out_phi,
           void* out_yN, double* out_rho, void* out_gv, void* out_gx) {
  Shape s{};
  int rc = shape_for(H, n, o->lanes_per_task, sizeof(T) == 4, s);
  if (rc) return rc;
  const int npad = s.npad();
  const int K = eff_K(o->ckpt_K, s, sizeof(T) == 8, nsteps);
  const bool grad = out_gv || out_gx;
  WsLayout WL = layout(s, n, B, G, nsteps, o->dtype, o->mode, K, grad, false);
  void* ws = nullptr;
  rc = get_workspace(o, WL.total, &ws);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  const T *dT = nullptr, *aT = nullptr;
  const double *dD = nullptr, *aD = nullptr;
  rc = stage_params<T>(H, J, n, s, base + WL.params, st, &dT, &dD, &aT, &aD);
  if (rc) return rc;
  hj::EvalArgs<T> A;
  A.P = make_problem<T>(H, J, n, t, nsteps, o->formula, o->quad, dT, npad);
  A.P.aop = aT;
  A.x = static_cast<const T*>(x);
  A.v = static_cast<const T*>(v);
  A.B = B;
  A.G = G;
  A.K = K;
  A.phi = out_phi;
  A.rho = out_rho;
  A.yN = static_cast<T*>(out_yN);
  A.gv = static_cast<T*>(out_gv);
  A.gx = static_cast<T*>(out_gx);
  A.stride = WL.stride;
  A.ck = grad ? reinterpret_cast<T*>(base + WL.ck) : nullptr;
  A.seg = grad ? reinterpret_cast<T*>(base + WL.seg) : nullptr;
  if (o->ev_begin) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_begin), st));
  HJ_HIP(dispatch_eval<T>(s, kernel_mk(H), A, st));
  if (o->ev_end) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_end), st));
  return HJ_OK;
}

hj_opts default_opts() {
  hj_opts o;
  std::memset(&o, 0, sizeof(o));
  o.dtype = HJ_F64;
  o.formula = HJ_LAX;
  o.mode = HJ_GD_ADJ;
  o.quad = HJ_RK4AUG;
  o.max_iter = 200;
  o.ckpt_K = 16;
  o.cert_fp64 = 1;
  o.alpha0 = 1.0 / 3.0;
  o.fd_sigma = 1e-4;
  o.eps_step = 0.5e-7;
  o.cert_tol = 1e-8;
  o.v_max = 1e6;
  o.acc_rel = 64 * 2.220446049250313e-16;
  o.armijo_c = 0.1;
  o.fp64_continue = 1;
  o.ode = HJ_RK4;
  o.M = 500;
  o.momentum = 0.9;
  return o;
}

int check_opts(const hj_opts* o) {
  if (o->dtype != HJ_F64 && o->dtype != HJ_F32) return fail(HJ_EDTYPE, "unknown dtype");
  if (o->formula < HJ_LAX || o->formula > HJ_LAX_MIN) return fail(HJ_EINVAL, "bad formula");
  if (o->mode < HJ_CD_FD || o->mode > HJ_MOMENTUM) return fail(HJ_EINVAL, "bad mode");
  if (o->ode != HJ_RK4 && o->ode != HJ_EULER && o->ode != HJ_STAGGERED)
    return fail(HJ_EINVAL, "bad ode scheme");
  if (o->mode == HJ_ALG1 && o->M < 1) return fail(HJ_EINVAL, "M must be >= 1");
  if ((o->mode == HJ_ALG1 || o->mode == HJ_MOMENTUM) && !(o->fd_sigma > 0.0))
    return fail(HJ_EINVAL, "fd_sigma must be > 0");
  if (o->mode == HJ_MOMENTUM && !(o->momentum >= 0.0 && o->momentum < 1.0))
    return fail(HJ_EINVAL, "momentum must be in [0, 1)");
  if (o->quad != HJ_TRAPZ && o->quad != HJ_RK4AUG) return fail(HJ_EINVAL, "bad quadrature");
  if (o->max_iter < 0) return fail(HJ_EINVAL, "max_iter must be >= 0");
  if (o->ckpt_K < 1) return fail(HJ_EINVAL, "ckpt_K must be >= 1");
  if (!(o->alpha0 > 0.0)) return fail(HJ_EINVAL, "alpha0 must be > 0");
  if (!(o->armijo_c >= 0.0 && o->armijo_c < 1.0))
    return fail(HJ_EINVAL, "armijo_c must be in [0, 1)");
  if (o->mode == HJ_CD_FD && !(o->fd_sigma > 0.0)) return fail(HJ_EINVAL, "fd_sigma must be > 0");
  if (o->lanes_per_task < 0) return fail(HJ_EINVAL, "lanes_per_task must be >= 0");
  if (o->schedule < HJ_SCHED_AUTO || o->schedule > HJ_SCHED_PERSISTENT)
    return fail(HJ_EINVAL, "bad schedule");
  if (o->max_groups < 0) return fail(HJ_EINVAL, "max_groups must be >= 0");
  if (o->cont_lanes_per_task < 0) return fail(HJ_EINVAL, "cont_lanes_per_task must be >= 0");
  if (o->tail_budget < 0) return fail(HJ_EINVAL, "tail_budget must be >= 0");
  if (o->tail_lanes_per_task < 0) return fail(HJ_EINVAL, "tail_lanes_per_task must be >= 0");
  if (o->n_group_cfg < 0 || (o->n_group_cfg > 0 && !o->group_cfg))
    return fail(HJ_EINVAL, "group_cfg must hold n_group_cfg entries");
  for (int c = 0; c < o->n_group_cfg; ++c) {
    const hj_group_cfg& g = o->group_cfg[c];
    if (g.lanes_per_task < 0 || g.ckpt_K < 0 || g.max_groups < 0 || g.cont_lanes_per_task < 0)
      return fail(HJ_EINVAL, "group_cfg entries must be >= 0");
  }
  return HJ_OK;
}

// ---------------------------------------------------------------------------
// the paper's scheme and families (hj_paper.hpp)
// ---------------------------------------------------------------------------
bool needs_paper(int H_kind, int J_kind, const hj_opts* o) {
  return o->mode == HJ_ALG1 || o->mode == HJ_MOMENTUM || H_kind == HJ_H_NORM ||
         J_kind == HJ_J_ROSENBROCK || o->formula == HJ_LAX_MIN || o->ode != HJ_RK4;
}

int check_paper(int H_kind, const hj_h_params* H, int J_kind, int n, const hj_opts* o,
                bool solve) {
  if (solve && o->mode != HJ_ALG1 && o->mode != HJ_MOMENTUM)
    return fail(HJ_EUNSUPPORTED, "these Hamiltonians, initial data, functionals and the "
                                 "Euler and staggered schemes descend with HJ_ALG1 or "
                                 "HJ_MOMENTUM");
  if (o->dtype != HJ_F64) return fail(HJ_EUNSUPPORTED, "the paper's scheme runs in FP64");
  if (H_kind == HJ_H_QUADRATIC && H->A)
    return fail(HJ_EUNSUPPORTED, "the paper's scheme takes no drift matrix");
  if (n > hj::kPaperMaxN)
    return fail(HJ_EUNSUPPORTED, "the paper's scheme takes n <= " +
                                     std::to_string(hj::kPaperMaxN));
  if (J_kind == HJ_J_ROSENBROCK && o->formula == HJ_HOPF)
    return fail(HJ_EUNSUPPORTED, "the Hopf functional needs the ellipsoid's conjugate");
  if (o->ode == HJ_RK4 && o->quad != HJ_RK4AUG)
    return fail(HJ_EUNSUPPORTED, "the paper's kernel pairs RK4 with the RK4-augmented rule");
  return HJ_OK;
}

hj::PaperProblem paper_problem(int H_kind, const hj_h_params* H, int J_kind,
                               const hj_j_params* J, int n, double t, int nsteps,
                               const hj_opts* o) {
  hj::PaperProblem P;
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  P.hkind = H_kind;
  P.jkind = J_kind;
  P.functional = o->formula;
  P.ode = o->ode;
  P.N = nsteps;
  P.h = t / nsteps;
  if (H_kind == HJ_H_QUADRATIC) {
    P.m_kind = H->m_kind;
    P.e = H->e;
    P.kappa = H->m_kind == HJ_M_CONST ? 0.0 : H->kappa;
    P.inv_s = H->m_kind == HJ_M_TANH ? 1.0 / H->s : 1.0;
    P.w = H->w;
    for (int i = 0; i < n; ++i) P.d[i] = H->d[i];
  } else {
    P.k = H->k;
    P.s1 = H->s1;
    P.s2 = H->s2;
    P.c0 = H->c0;
    P.beta = H->beta;
    P.gam = H->gam;
    for (int i = 0; i < n; ++i) P.mu[i] = H->mu[i];
  }
  for (int i = 0; i < hj::kPaperMaxN; ++i) {
    P.a2[i] = 1.0;
    P.ia2[i] = 1.0;
  }
  if (J_kind == HJ_J_ELLIPSOID)
    for (int i = 0; i < n; ++i) {
      P.a2[i] = J->a[i] * J->a[i];
      P.ia2[i] = 1.0 / (J->a[i] * J->a[i]);
    }
  P.j0 = J->j0;
  P.rscale = J->rscale;
  return P;
}

int paper_solve(int H_kind, const hj_h_params* H, int J_kind, const hj_j_params* J,
                const void* x, int64_t B, int n, double t, int nsteps, const hj_guesses* gs,
                const hj_opts* o, double* out_u, void* out_argopt, int32_t* out_cert,
                const hj_slot_diag* diag) {
  int rc = check_paper(H_kind, H, J_kind, n, o, true);
  if (rc) return rc;
  if (o->tail_budget > 0)
    return fail(HJ_EUNSUPPORTED, "tail hand-offs take the FP64 adjoint descent of a "
                                 "problem without a drift matrix");
  const size_t BG = (size_t)B * gs->G;
  const size_t need = align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256) + align_up(BG * n * 8, 256);
  void* ws = nullptr;
  rc = get_workspace(o, need, &ws);
  if (rc) return rc;
  char* sp = static_cast<char*>(ws);
  hj::PaperArgs A;
  std::memset(&A, 0, sizeof(A));
  A.P = paper_problem(H_kind, H, J_kind, J, n, t, nsteps, o);
  A.mode = o->mode;
  A.max_iter = o->max_iter;
  A.R = gs->R_max;
  A.G = gs->G;
  A.M = o->M;
  A.alpha0 = o->alpha0;
  A.sigma = o->fd_sigma;
  A.eps = o->eps_step;
  A.cert_tol = o->cert_tol;
  A.v_max = o->v_max;
  A.momentum = o->momentum;
  A.acc_rel = o->acc_rel;
  A.x = static_cast<const double*>(x);
  A.guesses = static_cast<const double*>(gs->init);
  A.ntask = (int64_t)BG;
  double* w_phi = reinterpret_cast<double*>(sp);
  double* w_rho = w_phi + BG;
  int32_t* w_status = reinterpret_cast<int32_t*>(w_rho + BG);
  int32_t* w_cert = w_status + BG;
  int32_t* w_iters = w_cert + BG;
  int32_t* w_att = w_iters + BG;
  int64_t* w_fwd = reinterpret_cast<int64_t*>(w_att + BG);
  int64_t* w_bwd = w_fwd + BG;
  double* w_v = reinterpret_cast<double*>(sp + align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256));
  A.out.phi = (diag && diag->phi) ? diag->phi : w_phi;
  A.out.rho = (diag && diag->rho) ? diag->rho : w_rho;
  A.out.status = (diag && diag->status) ? diag->status : w_status;
  A.out.cert = (diag && diag->cert) ? diag->cert : w_cert;
  A.out.iters = (diag && diag->iters) ? diag->iters : w_iters;
  A.out.attempts = (diag && diag->attempts) ? diag->attempts : w_att;
  A.out.n_fwd = (diag && diag->n_fwd) ? diag->n_fwd : w_fwd;
  A.out.n_bwd = (diag && diag->n_bwd) ? diag->n_bwd : w_bwd;
  A.out.v = (diag && diag->v_final) ? static_cast<double*>(diag->v_final) : w_v;
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  if (o->ev_begin) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_begin), st));
  HJ_HIP(hj::launch_solve_paper(A, st));
  if (o->ev_end) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_end), st));
  // selection over the guesses (u = min F1 / F2, or -min G)
  HJ_HIP(hj::launch_select<double>(B, gs->G, n, o->formula == HJ_HOPF ? HJ_HOPF : HJ_LAX,
                                   A.out.phi, A.out.cert, A.out.v, out_u,
                                   static_cast<double*>(out_argopt), out_cert, st));
  return HJ_OK;
}

int paper_eval(int H_kind, const hj_h_params* H, int J_kind, const hj_j_params* J,
               const void* x, int64_t B, int n, double t, int nsteps, const void* v, int G,
               const hj_opts* o, double* out_phi, void* out_yN, double* out_rho,
               void* out_gv, void* out_gx) {
  int rc = check_paper(H_kind, H, J_kind, n, o, false);
  if (rc) return rc;
  if (out_gv || out_gx || out_yN)
    return fail(HJ_EUNSUPPORTED, "the paper's scheme evaluates objectives and residuals only");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  const hj::PaperProblem P = paper_problem(H_kind, H, J_kind, J, n, t, nsteps, o);
  if (o->ev_begin) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_begin), st));
  HJ_HIP(hj::launch_eval_paper(P, static_cast<const double*>(x), static_cast<const double*>(v),
                               B, G, out_phi, out_rho, st));
  if (o->ev_end) HJ_HIP(hipEventRecord(static_cast<hipEvent_t>(o->ev_end), st));
  return HJ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// batched plans
// ---------------------------------------------------------------------------
struct hj_batch_plan_s {
  void* mem = nullptr;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> branch;  // capture streams of the launch groups after the first
  std::vector<hipEvent_t> ev;       // fork and join events of the capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t tasks = 0, groups = 0;
  int launches = 0;
  ~hj_batch_plan_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t b : branch) (void)hipStreamDestroy(b);
    if (cap) (void)hipStreamDestroy(cap);
    if (mem) (void)hipFree(mem);
  }
};

namespace {

// One launch of a plan: the instances that share a lane shape, profile and
// launch choices.
struct LaunchGroup {
  Shape s;
  int mk;
  int K = 0, maxg = 0;  // checkpoint interval, lane-group cap (0: the defaults)
  Shape cs{};           // lane shape of the FP64 continuation
  double work = 0.0;    // sum over tasks of n x steps (launch order)
  std::vector<int> inst;  // indices into the caller's array, longest first
  int64_t tasks = 0, points = 0, groups = 0;
  int max_steps = 0;
  // byte offsets in the plan memory
  size_t params = 0, table = 0, slots = 0, queue = 0, ck = 0, seg = 0, stride = 0;
  // FP64 continuation of FP32 slots (cgroups = 0: none)
  int64_t cgroups = 0;
  size_t handoff = 0, cont_ctr = 0, ck64 = 0, seg64 = 0, stride64 = 0;
};

template <typename T>
int plan_t(const hj_instance* inst, int n_inst, const hj_opts* o, hj_batch_plan_s* plan) {
  const size_t tsz = sizeof(T);
  // group by (shape, speed profile); within a group, longest instances first
  std::vector<LaunchGroup> lg;
  for (int i = 0; i < n_inst; ++i) {
    // the instance's launch choices: the first table entry covering its n
    int lpt = o->lanes_per_task, K = std::max(1, o->ckpt_K), maxg = o->max_groups;
    int clpt = o->cont_lanes_per_task;
    for (int c = 0; c < o->n_group_cfg; ++c) {
      const hj_group_cfg& gc = o->group_cfg[c];
      if (inst[i].n <= gc.n_max) {
        if (gc.lanes_per_task > 0) lpt = gc.lanes_per_task;
        if (gc.ckpt_K > 0) K = gc.ckpt_K;
        if (gc.max_groups > 0) maxg = gc.max_groups;
        if (gc.cont_lanes_per_task > 0) clpt = gc.cont_lanes_per_task;
        break;
      }
    }
    Shape s{}, cs{};
    if (!pick_shape(inst[i].n, lpt, false, sizeof(T) == 4, s))
      return fail(HJ_EUNSUPPORTED, "no kernel shape for instance " + std::to_string(i) +
                                       " with " + std::to_string(lpt) + " lanes per task");
    int rc2 = cont_shape_for(s, clpt, cs);
    if (rc2) return rc2;
    const int mk = kernel_mk(&inst[i].H);
    auto it = std::find_if(lg.begin(), lg.end(), [&](const LaunchGroup& g) {
      return g.s.npl == s.npl && g.s.lpt == s.lpt && g.mk == mk && g.K == K &&
             g.maxg == maxg && g.cs.lpt == cs.lpt;
    });
    if (it == lg.end()) {
      LaunchGroup g{s, mk};
      g.K = K;
      g.maxg = maxg;
      g.cs = cs;
      lg.push_back(g);
      it = lg.end() - 1;
    }
    it->inst.push_back(i);
  }
  for (LaunchGroup& g : lg) {
    std::stable_sort(g.inst.begin(), g.inst.end(), [&](int a, int b) {
      return (double)inst[a].nsteps * inst[a].n > (double)inst[b].nsteps * inst[b].n;
    });
    for (int i : g.inst) {
      g.tasks += inst[i].B * (int64_t)inst[i].guesses.G;
      g.points += inst[i].B;
      g.max_steps = std::max(g.max_steps, inst[i].nsteps);
      g.work += (double)inst[i].B * inst[i].guesses.G * inst[i].nsteps * inst[i].n;
    }
    int64_t res = dispatch_resident<T>(g.s, g.mk, HJ_GD_ADJ);
    if (g.maxg > 0) res = std::min<int64_t>(res > 0 ? res : g.tasks, g.maxg);
    g.groups = std::max<int64_t>(1, std::min(res > 0 ? res : g.tasks, g.tasks));
    hj_opts og = *o;
    og.max_groups = g.maxg;
    g.cgroups = continue_groups(g.cs, g.mk, &og, g.tasks);
  }
  // heaviest group first: the persistent launches take the chip in launch
  // order, and the heaviest group's tail (its longest tasks, then its FP64
  // continuation) then overlaps the lighter groups' work instead of
  // following it
  std::stable_sort(lg.begin(), lg.end(),
                   [](const LaunchGroup& a, const LaunchGroup& b) { return a.work > b.work; });
  // memory layout
  size_t off = 0;
  for (LaunchGroup& g : lg) {
    const int npad = g.s.npad();
    const int n = inst[g.inst[0]].n;  // the rows of every instance use its own n
    int nmax = 0;
    for (int i : g.inst) nmax = std::max(nmax, inst[i].n);
    g.params = off;
    off += align_up(g.inst.size() * (size_t)npad * 3 * (tsz + 8), 256);
    g.table = off;
    off += align_up(g.inst.size() * sizeof(hj::InstDesc<T>), 256);
    g.slots = off;
    off += align_up((size_t)g.tasks * (8 + 8 + 4 * 4 + 8 + 8), 256) +
           align_up((size_t)g.tasks * nmax * tsz, 256);
    g.queue = off;
    off += 256;
    const int K = eff_K(g.K, g.s, tsz == 8, g.max_steps);
    const int K64 = eff_K(K, g.cs, true, g.max_steps);
    g.stride = align_up((size_t)g.groups * g.s.lpt, 256);
    const size_t nck = (size_t)((g.max_steps + K - 1) / K) + 1;
    g.ck = off;
    off += align_up(nck * 2 * g.s.npl * g.stride * tsz, 256);
    g.seg = off;
    off += align_up((size_t)K * 2 * g.s.npl * g.stride * tsz, 256);
    if (g.cgroups > 0) {
      g.handoff = off;
      off += align_up((size_t)g.tasks * 8, 256);
      g.cont_ctr = off;
      off += 256;
      const size_t nck64 = (size_t)((g.max_steps + K64 - 1) / K64) + 1;
      g.stride64 = align_up((size_t)g.cgroups * g.cs.lpt, 256);
      g.ck64 = off;
      off += align_up(nck64 * 2 * g.cs.npl * g.stride64 * 8, 256);
      g.seg64 = off;
      off += align_up((size_t)K64 * 2 * g.cs.npl * g.stride64 * 8, 256);
    }
    (void)n;
  }
  if (hipMalloc(&plan->mem, std::max<size_t>(off, 256)) != hipSuccess) {
    plan->mem = nullptr;
    return fail(HJ_ENOMEM, "hipMalloc of " + std::to_string(off) + " bytes for the plan failed");
  }
  char* base = static_cast<char*>(plan->mem);
  // stage parameters and instance tables
  std::vector<hj::SolveArgs<T>> args;
  for (LaunchGroup& g : lg) {
    const int npad = g.s.npad();
    std::vector<char> pbuf(g.inst.size() * (size_t)npad * 3 * (tsz + 8));
    std::vector<hj::InstDesc<T>> table(g.inst.size());
    int64_t task0 = 0, point0 = 0;
    int nmax = 0;
    for (size_t j = 0; j < g.inst.size(); ++j) {
      const hj_instance& I = inst[g.inst[j]];
      nmax = std::max(nmax, I.n);
      char* q = pbuf.data() + j * (size_t)npad * 3 * (tsz + 8);
      HostParams<T> pt = host_params<T>(&I.H, &I.J, I.n, npad);
      HostParams<double> pd = host_params<double>(&I.H, &I.J, I.n, npad);
      std::memcpy(q, pt.d.data(), npad * tsz);
      std::memcpy(q + npad * tsz, pt.a2.data(), npad * tsz);
      std::memcpy(q + 2 * npad * tsz, pt.ia2.data(), npad * tsz);
      std::memcpy(q + 3 * npad * tsz, pd.d.data(), npad * 8);
      std::memcpy(q + 3 * npad * tsz + npad * 8, pd.a2.data(), npad * 8);
      std::memcpy(q + 3 * npad * tsz + 2 * npad * 8, pd.ia2.data(), npad * 8);
      char* dq = base + g.params + j * (size_t)npad * 3 * (tsz + 8);
      hj::InstDesc<T>& D = table[j];
      D.P = make_problem<T>(&I.H, &I.J, I.n, I.t, I.nsteps, o->formula, o->quad,
                            reinterpret_cast<const T*>(dq), npad);
      D.P64 = make_problem<double>(&I.H, &I.J, I.n, I.t, I.nsteps, o->formula, o->quad,
                                   reinterpret_cast<const double*>(dq + 3 * npad * tsz), npad);
      D.x = static_cast<const T*>(I.x);
      D.guesses = static_cast<const T*>(I.guesses.init);
      D.B = I.B;
      D.G = I.guesses.G;
      D.R = I.guesses.R_max;
      D.task0 = task0;
      D.point0 = point0;
      D.out_u = I.out_u;
      D.out_arg = static_cast<T*>(I.out_argopt);
      D.out_cert = I.out_cert;
      D.diag.phi = I.diag.phi;
      D.diag.rho = I.diag.rho;
      D.diag.status = I.diag.status;
      D.diag.cert = I.diag.cert;
      D.diag.iters = I.diag.iters;
      D.diag.attempts = I.diag.attempts;
      D.diag.n_fwd = I.diag.n_fwd;
      D.diag.n_bwd = I.diag.n_bwd;
      D.diag.v = static_cast<T*>(I.diag.v_final);
      task0 += I.B * (int64_t)I.guesses.G;
      point0 += I.B;
    }
    HJ_HIP(hipMemcpy(base + g.params, pbuf.data(), pbuf.size(), hipMemcpyHostToDevice));
    HJ_HIP(hipMemcpy(base + g.table, table.data(), table.size() * sizeof(hj::InstDesc<T>),
                     hipMemcpyHostToDevice));
    hj::SolveArgs<T> A;
    std::memset(&A, 0, sizeof(A));
    A.P = table[0].P;  // unused by the batched kernel except for n
    A.P.n = nmax;
    A.max_iter = o->max_iter;
    A.K = eff_K(g.K, g.s, tsz == 8, g.max_steps);
    A.cert_fp64 = o->cert_fp64;
    A.alpha0 = (T)o->alpha0;
    A.sigma = (T)o->fd_sigma;
    A.eps_step = (T)o->eps_step;
    A.acc_rel = (T)o->acc_rel;
    A.armijo_c = (T)o->armijo_c;
    A.v_max = (T)o->v_max;
    A.cert_tol = o->cert_tol;
    A.stride = g.stride;
    A.ck = reinterpret_cast<T*>(base + g.ck);
    A.seg = reinterpret_cast<T*>(base + g.seg);
    char* sp = base + g.slots;
    const size_t BG = (size_t)g.tasks;
    A.out.phi = reinterpret_cast<double*>(sp);
    A.out.rho = A.out.phi + BG;
    A.out.status = reinterpret_cast<int32_t*>(A.out.rho + BG);
    A.out.cert = A.out.status + BG;
    A.out.iters = A.out.cert + BG;
    A.out.attempts = A.out.iters + BG;
    A.out.n_fwd = reinterpret_cast<int64_t*>(A.out.attempts + BG);
    A.out.n_bwd = A.out.n_fwd + BG;
    A.out.v = reinterpret_cast<T*>(sp + align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256));
    A.ntask = g.tasks;
    A.queue = reinterpret_cast<unsigned long long*>(base + g.queue);
    A.inst = reinterpret_cast<const hj::InstDesc<T>*>(base + g.table);
    A.n_inst = (int)g.inst.size();
    A.handoff = g.cgroups > 0 ? reinterpret_cast<int64_t*>(base + g.handoff) : nullptr;
    A.handoff_n =
        g.cgroups > 0 ? reinterpret_cast<unsigned long long*>(base + g.cont_ctr) : nullptr;
    A.tail_budget = 0;
    A.tail_stride = 0;
    A.tail = nullptr;
    A.tail_n = nullptr;
    args.push_back(A);
  }
  // capture the launch groups into a graph as parallel branches (fork from
  // the capture stream, join back into it): the groups share no memory, and
  // a group's persistent launch ends with a tail of long tasks on few CUs
  // that the next group's work can fill.  Every stream has the default
  // priority.
  HJ_HIP(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking));
  for (size_t gi = 1; gi < lg.size(); ++gi) {
    hipStream_t b = nullptr;
    HJ_HIP(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    plan->branch.push_back(b);
  }
  for (size_t i = 0; i < lg.size(); ++i) {  // fork, then one join per branch
    hipEvent_t e = nullptr;
    HJ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    plan->ev.push_back(e);
  }
  HJ_HIP(hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipEventRecord(plan->ev[0], plan->cap);
  for (size_t gi = 1; gi < lg.size() && err == hipSuccess; ++gi)
    err = hipStreamWaitEvent(plan->branch[gi - 1], plan->ev[0], 0);
  for (size_t gi = 0; gi < lg.size() && err == hipSuccess; ++gi) {
    const LaunchGroup& g = lg[gi];
    const hj::SolveArgs<T>& A = args[gi];
    hipStream_t st = gi == 0 ? plan->cap : plan->branch[gi - 1];
    if (g.cgroups > 0) {
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, A.handoff_n, 16);
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = dispatch_solve<T>(g.s, g.mk, A, HJ_GD_ADJ, g.groups, st);
    if constexpr (sizeof(T) == 4) {
      if (err == hipSuccess && g.cgroups > 0) {
        hj::ContArgs<float> CA;
        CA.S = A;
        CA.max_iter = o->max_iter;
        CA.K = eff_K(A.K, g.cs, true, g.max_steps);
        CA.alpha0 = o->alpha0;
        CA.eps_step = o->eps_step;
        CA.acc_rel = o->acc_rel;
        CA.armijo_c = o->armijo_c;
        CA.v_max = o->v_max;
        CA.ck = reinterpret_cast<double*>(base + g.ck64);
        CA.seg = reinterpret_cast<double*>(base + g.seg64);
        CA.stride = g.stride64;
        CA.queue = A.handoff_n + 8;
        err = dispatch_continue(g.cs, g.mk, CA, true, g.cgroups, st);
      }
    }
    if (err == hipSuccess)
      err = hj::launch_select_batched<T>(A.inst, A.n_inst, g.points, A.P.n, o->formula,
                                         A.out.phi, A.out.cert, A.out.v, st);
    if (err == hipSuccess)
      err = hj::launch_scatter_diag<T>(A.inst, A.n_inst, g.tasks, A.P.n, A.out, st);
  }
  for (size_t gi = 1; gi < lg.size() && err == hipSuccess; ++gi) {
    err = hipEventRecord(plan->ev[gi], plan->branch[gi - 1]);
    if (err == hipSuccess) err = hipStreamWaitEvent(plan->cap, plan->ev[gi], 0);
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(plan->cap, &graph);
  if (err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(HJ_EDEVICE, std::string("launch during capture: ") + hipGetErrorString(err));
  }
  HJ_HIP(e2);
  plan->graph = graph;
  HJ_HIP(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
  plan->launches = (int)lg.size();
  for (const LaunchGroup& g : lg) {
    plan->tasks += g.tasks;
    plan->groups += g.groups;
  }
  return HJ_OK;
}

}  // namespace

extern "C" {

int32_t hj_solve(int32_t H_kind, const hj_h_params* H, int32_t J_kind, const hj_j_params* J,
                 const void* x, int64_t B, int32_t n, double t, int32_t nsteps,
                 const hj_guesses* guesses, const hj_opts* opts, double* out_u,
                 void* out_argopt, int32_t* out_cert, const hj_slot_diag* diag) {
  g_last_error.clear();
  int rc = check_problem(H_kind, H, J_kind, J, n, t, nsteps);
  if (rc) return rc;
  if (B < 0) return fail(HJ_EINVAL, "B must be >= 0");
  if (!guesses) return fail(HJ_EINVAL, "guesses are required");
  if (guesses->G < 1 || guesses->G > HJ_MAX_G) return fail(HJ_EINVAL, "G must be in [1, 64]");
  if (guesses->R_max < 0) return fail(HJ_EINVAL, "R_max must be >= 0");
  hj_opts o = opts ? *opts : default_opts();
  rc = check_opts(&o);
  if (rc) return rc;
  if (B == 0) return HJ_OK;
  if (!x || !guesses->init || !out_u || !out_argopt || !out_cert)
    return fail(HJ_EINVAL, "x, guesses->init and the outputs are required");
  if (needs_paper(H_kind, J_kind, &o))
    return paper_solve(H_kind, H, J_kind, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt,
                       out_cert, diag);
  if (o.dtype == HJ_F64)
    return solve_t<double>(H, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt, out_cert,
                           diag);
  return solve_t<float>(H, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt, out_cert, diag);
}

int32_t hj_solve_noalloc(int32_t H_kind, const hj_h_params* H, int32_t J_kind,
                         const hj_j_params* J, const void* x, int64_t B, int32_t n, double t,
                         int32_t nsteps, const hj_guesses* guesses, const hj_opts* opts,
                         double* out_u, void* out_argopt, int32_t* out_cert,
                         const hj_slot_diag* diag) {
  g_last_error.clear();
  int rc = check_problem(H_kind, H, J_kind, J, n, t, nsteps);
  if (rc) return rc;
  if (B < 0) return fail(HJ_EINVAL, "B must be >= 0");
  if (!guesses) return fail(HJ_EINVAL, "guesses are required");
  if (guesses->G < 1 || guesses->G > HJ_MAX_G) return fail(HJ_EINVAL, "G must be in [1, 64]");
  if (guesses->R_max < 0) return fail(HJ_EINVAL, "R_max must be >= 0");
  hj_opts o = opts ? *opts : default_opts();
  rc = check_opts(&o);
  if (rc) return rc;
  if (o.workspace)
    return fail(HJ_EINVAL, "hj_solve_noalloc uses the library's fixed scratch: "
                           "opts->workspace must be NULL");
  if (B == 0) return HJ_OK;
  if (!x || !guesses->init || !out_u || !out_argopt || !out_cert)
    return fail(HJ_EINVAL, "x, guesses->init and the outputs are required");
  if (needs_paper(H_kind, J_kind, &o)) {
    const size_t BG = (size_t)B * guesses->G;
    const size_t need = align_up(BG * (8 + 8 + 4 * 4 + 8 + 8), 256) + align_up(BG * n * 8, 256);
    if (need > HJ_NOALLOC_BYTES)
      return fail(HJ_ENOMEM, "hj_solve_noalloc: this solve needs " + std::to_string(need) +
                                 " bytes of scratch; the fixed scratch holds " +
                                 std::to_string((size_t)HJ_NOALLOC_BYTES) + " bytes");
    void* ptr = nullptr;
    rc = noalloc_scratch(&ptr);
    if (rc) return rc;
    o.workspace = ptr;
    o.ws_bytes = HJ_NOALLOC_BYTES;
    return paper_solve(H_kind, H, J_kind, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt,
                       out_cert, diag);
  }
  Shape s{};
  rc = shape_for(H, n, o.lanes_per_task, o.dtype == HJ_F32, s);
  if (rc) return rc;
  const int mk = kernel_mk(H);
  const int G = guesses->G;
  auto need_of = [&](const hj_opts& oo, int64_t* g) {
    int64_t cg = 0;
    return (oo.dtype == HJ_F64 ? solve_layout<double>(s, mk, n, B, G, nsteps, &oo, g, &cg)
                               : solve_layout<float>(s, mk, n, B, G, nsteps, &oo, g, &cg))
        .total;
  };
  int64_t groups = 0;
  size_t need = need_of(o, &groups);
  if (need > HJ_NOALLOC_BYTES) {
    // a persistent launch holds checkpoints for its lane groups only: halve
    // the groups until the layout fits (results do not depend on them)
    int64_t mg = groups;
    if (mg <= 0)
      mg = std::min<int64_t>(o.dtype == HJ_F64 ? dispatch_resident<double>(s, mk, o.mode)
                                               : dispatch_resident<float>(s, mk, o.mode),
                             B * (int64_t)G);
    o.schedule = HJ_SCHED_PERSISTENT;
    while (need > HJ_NOALLOC_BYTES && mg > 64) {
      mg = std::max<int64_t>(64, mg / 2);
      o.max_groups = (int32_t)mg;
      need = need_of(o, &groups);
    }
    if (need > HJ_NOALLOC_BYTES)
      return fail(HJ_ENOMEM, "hj_solve_noalloc: this solve needs " + std::to_string(need) +
                                 " bytes of scratch even with 64 lane groups; the fixed "
                                 "scratch holds " +
                                 std::to_string((size_t)HJ_NOALLOC_BYTES) +
                                 " bytes (use hj_solve, or fewer points)");
  }
  void* ptr = nullptr;
  rc = noalloc_scratch(&ptr);
  if (rc) return rc;
  o.workspace = ptr;
  o.ws_bytes = HJ_NOALLOC_BYTES;
  if (o.dtype == HJ_F64)
    return solve_t<double>(H, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt, out_cert,
                           diag);
  return solve_t<float>(H, J, x, B, n, t, nsteps, guesses, &o, out_u, out_argopt, out_cert, diag);
}

int32_t hj_lax_friedrichs(int32_t H_kind, const hj_h_params* H, int32_t J_kind,
                          const hj_j_params* J, double x0, double y0, double dx, double dy,
                          int32_t nx, int32_t ny, double dt, int32_t nt, double ax, double ay,
                          double* phi, double* work, void* stream) {
  g_last_error.clear();
  if (H_kind != HJ_H_QUADRATIC)
    return fail(HJ_EUNSUPPORTED, "the Lax-Friedrichs solver takes the quadratic family");
  int rc = check_problem(H_kind, H, J_kind, J, 2, 1.0, 1);
  if (rc) return rc;
  if (H->A) return fail(HJ_EUNSUPPORTED, "the Lax-Friedrichs solver takes no drift matrix");
  if (nx < 3 || ny < 3 || nt < 0 || !(dx > 0.0) || !(dy > 0.0) || !(dt > 0.0) ||
      !(ax >= 0.0) || !(ay >= 0.0) || !std::isfinite(x0) || !std::isfinite(y0))
    return fail(HJ_EINVAL, "need nx, ny >= 3, nt >= 0, dx, dy, dt > 0, ax, ay >= 0");
  if ((int64_t)nx * ny > ((int64_t)1 << 31))
    return fail(HJ_EINVAL, "the grid is limited to 2^31 cells");
  if (!phi) return fail(HJ_EINVAL, "phi is required");
  hj_opts o = default_opts();
  o.stream = stream;
  if (!work) {
    void* ws = nullptr;
    rc = get_workspace(&o, (size_t)nx * ny * sizeof(double), &ws);
    if (rc) return rc;
    work = static_cast<double*>(ws);
  }
  const hj::PaperProblem P = paper_problem(H_kind, H, J_kind, J, 2, 1.0, 1, &o);
  HJ_HIP(hj::launch_lax_friedrichs(P, x0, y0, dx, dy, nx, ny, dt, nt, ax, ay, phi, work,
                                   static_cast<hipStream_t>(stream)));
  return HJ_OK;
}

int32_t hj_eval(int32_t H_kind, const hj_h_params* H, int32_t J_kind, const hj_j_params* J,
                const void* x, int64_t B, int32_t n, double t, int32_t nsteps, const void* v,
                int32_t G, const hj_opts* opts, double* out_phi, void* out_yN, double* out_rho,
                void* out_grad_v, void* out_grad_x) {
  g_last_error.clear();
  int rc = check_problem(H_kind, H, J_kind, J, n, t, nsteps);
  if (rc) return rc;
  if (B < 0) return fail(HJ_EINVAL, "B must be >= 0");
  if (G < 1 || G > HJ_MAX_G) return fail(HJ_EINVAL, "G must be in [1, 64]");
  hj_opts o = opts ? *opts : default_opts();
  rc = check_opts(&o);
  if (rc) return rc;
  if (B == 0) return HJ_OK;
  if (!x || !v || !out_phi) return fail(HJ_EINVAL, "x, v and out_phi are required");
  if (needs_paper(H_kind, J_kind, &o))
    return paper_eval(H_kind, H, J_kind, J, x, B, n, t, nsteps, v, G, &o, out_phi, out_yN,
                      out_rho, out_grad_v, out_grad_x);
  if (o.dtype == HJ_F64)
    return eval_t<double>(H, J, x, B, n, t, nsteps, v, G, &o, out_phi, out_yN, out_rho,
                          out_grad_v, out_grad_x);
  return eval_t<float>(H, J, x, B, n, t, nsteps, v, G, &o, out_phi, out_yN, out_rho, out_grad_v,
                       out_grad_x);
}

size_t hj_workspace_size(int32_t n, int64_t B, int32_t G, int32_t nsteps, const hj_opts* opts) {
  if (n < 1 || n > HJ_MAX_N || B < 0 || G < 1 || nsteps < 1) return 0;
  hj_opts o = opts ? *opts : default_opts();
  // the largest of what hj_solve and hj_eval (with gradients) need, with or
  // without a drift matrix
  size_t need = 0;
  for (int drift = 0; drift < 2; ++drift) {
    Shape s{};
    if (!pick_shape(n, o.lanes_per_task, drift != 0, o.dtype == HJ_F32, s)) continue;
    for (int mk : {HJ_M_TANH, HJ_M_RAT}) {
      int64_t g = 0, cg = 0;
      WsLayout a = o.dtype == HJ_F64
                       ? solve_layout<double>(s, mk, n, B, G, nsteps, &o, &g, &cg)
                       : solve_layout<float>(s, mk, n, B, G, nsteps, &o, &g, &cg);
      need = std::max(need, a.total);
    }
    WsLayout b = layout(s, n, B, G, nsteps, o.dtype, o.mode,
                        eff_K(o.ckpt_K, s, o.dtype == HJ_F64, nsteps), true, false);
    need = std::max(need, b.total);
  }
  return need;
}

int32_t hj_batch_plan(int32_t H_kind, int32_t J_kind, const hj_instance* inst, int32_t n_inst,
                      const hj_opts* opts, hj_batch* out) {
  g_last_error.clear();
  if (!out) return fail(HJ_EINVAL, "out is required");
  *out = nullptr;
  if (!inst || n_inst < 1) return fail(HJ_EINVAL, "at least one instance is required");
  hj_opts o = opts ? *opts : default_opts();
  int rc = check_opts(&o);
  if (rc) return rc;
  if (o.mode != HJ_GD_ADJ) return fail(HJ_EUNSUPPORTED, "batched solves use HJ_GD_ADJ");
  if (o.tail_budget > 0)
    return fail(HJ_EUNSUPPORTED, "tail hand-offs are for single solves, not batch plans");
  if (needs_paper(H_kind, J_kind, &o))
    return fail(HJ_EUNSUPPORTED, "batched plans take the quadratic family, ellipsoid data, "
                                 "the F1 / G functionals and RK4");
  for (int i = 0; i < n_inst; ++i) {
    const hj_instance& I = inst[i];
    rc = check_problem(H_kind, &I.H, J_kind, &I.J, I.n, I.t, I.nsteps);
    if (rc) return fail(rc, "instance " + std::to_string(i) + ": " + g_last_error);
    if (I.B < 1) return fail(HJ_EINVAL, "instance " + std::to_string(i) + ": B must be >= 1");
    if (I.guesses.G < 1 || I.guesses.G > HJ_MAX_G || I.guesses.R_max < 0)
      return fail(HJ_EINVAL, "instance " + std::to_string(i) + ": bad G or R_max");
    if (!I.x || !I.guesses.init || !I.out_u || !I.out_argopt || !I.out_cert)
      return fail(HJ_EINVAL, "instance " + std::to_string(i) + ": missing arrays");
    if (I.H.A)
      return fail(HJ_EUNSUPPORTED,
                  "instance " + std::to_string(i) + ": batched plans take no drift matrix");
  }
  hj_batch_plan_s* plan = new hj_batch_plan_s();
  rc = o.dtype == HJ_F64 ? plan_t<double>(inst, n_inst, &o, plan)
                         : plan_t<float>(inst, n_inst, &o, plan);
  if (rc) {
    delete plan;
    return rc;
  }
  *out = plan;
  return HJ_OK;
}

int32_t hj_batch_run(hj_batch plan, void* stream) {
  g_last_error.clear();
  if (!plan || !plan->exec) return fail(HJ_EINVAL, "invalid plan");
  HJ_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  return HJ_OK;
}

int32_t hj_batch_info(hj_batch plan, int64_t* tasks, int64_t* groups, int32_t* launches) {
  if (!plan) return fail(HJ_EINVAL, "invalid plan");
  if (tasks) *tasks = plan->tasks;
  if (groups) *groups = plan->groups;
  if (launches) *launches = plan->launches;
  return HJ_OK;
}

int32_t hj_batch_free(hj_batch plan) {
  if (!plan) return HJ_OK;
  HJ_HIP(hipDeviceSynchronize());
  delete plan;
  return HJ_OK;
}

const char* hj_last_error(void) { return g_last_error.c_str(); }

int32_t hj_version(void) { return HJ_VERSION; }

}  // extern "C"
