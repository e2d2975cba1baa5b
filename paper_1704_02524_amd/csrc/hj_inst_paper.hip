// Kernel instances and launchers of the paper's scheme and families: one
// lane per (point, guess) task, 2, 4, 8 or 16 components per lane, both
// Hamiltonian families.
#include "hj_paper.hpp"

namespace hj {

namespace {
template <int NPL> hipError_t solve_npl(const PaperArgs& A, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (A.ntask + block - 1) / block;
  if (A.P.hkind == HJ_H_NORM)
    hipLaunchKernelGGL((k_solve_paper<NPL, HJ_H_NORM>), dim3((unsigned)grid), dim3(block), 0,
                       st, A);
  else
    hipLaunchKernelGGL((k_solve_paper<NPL, HJ_H_QUADRATIC>), dim3((unsigned)grid), dim3(block),
                       0, st, A);
  return hipGetLastError();
}
template <int NPL>
hipError_t eval_npl(const PaperProblem& P, const double* x, const double* v, int64_t B, int G,
                    double* phi, double* rho, hipStream_t st) {
  const int block = 256;
  const int64_t grid = (B * G + block - 1) / block;
  if (P.hkind == HJ_H_NORM)
    hipLaunchKernelGGL((k_eval_paper<NPL, HJ_H_NORM>), dim3((unsigned)grid), dim3(block), 0, st,
                       P, x, v, B, G, phi, rho);
  else
    hipLaunchKernelGGL((k_eval_paper<NPL, HJ_H_QUADRATIC>), dim3((unsigned)grid), dim3(block), 0,
                       st, P, x, v, B, G, phi, rho);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_solve_paper(const PaperArgs& A, hipStream_t st) {
  const int n = A.P.n;
  if (n <= 2) return solve_npl<2>(A, st);
  if (n <= 4) return solve_npl<4>(A, st);
  if (n <= 8) return solve_npl<8>(A, st);
  if (n <= kPaperMaxN) return solve_npl<16>(A, st);
  return hipErrorInvalidValue;
}

hipError_t launch_eval_paper(const PaperProblem& P, const double* x, const double* v, int64_t B,
                             int G, double* phi, double* rho, hipStream_t st) {
  const int n = P.n;
  if (n <= 2) return eval_npl<2>(P, x, v, B, G, phi, rho, st);
  if (n <= 4) return eval_npl<4>(P, x, v, B, G, phi, rho, st);
  if (n <= 8) return eval_npl<8>(P, x, v, B, G, phi, rho, st);
  if (n <= kPaperMaxN) return eval_npl<16>(P, x, v, B, G, phi, rho, st);
  return hipErrorInvalidValue;
}

hipError_t launch_lax_friedrichs(const PaperProblem& P, double x0, double y0, double dx,
                                 double dy, int nx, int ny, double dt, int nt, double ax,
                                 double ay, double* phi, double* work, hipStream_t st) {
  const int block = 256;
  const int64_t cells = (int64_t)nx * ny;
  const unsigned grid = (unsigned)((cells + block - 1) / block);
  // kLfT steps per launch; an even number of ping-pong launches ends in the
  // array the caller reads
  const int launches = (nt + kLfT - 1) / kLfT;
  double* a = (launches % 2 == 0) ? phi : work;
  double* b = (launches % 2 == 0) ? work : phi;
  hipLaunchKernelGGL(k_lf_init, dim3(grid), dim3(block), 0, st, P, x0, y0, dx, dy, nx, ny, a);
  hipError_t e = hipGetLastError();
  const dim3 tiles((unsigned)((nx + kLfTX - 1) / kLfTX), (unsigned)((ny + kLfTY - 1) / kLfTY));
  for (int s = 0; s < nt && e == hipSuccess; s += kLfT) {
    const int nsub = nt - s < kLfT ? nt - s : kLfT;
    hipLaunchKernelGGL(k_lf_steps, tiles, dim3(block), 0, st, P, x0, y0, dx, dy, nx, ny, dt, ax,
                       ay, nsub, a, b);
    e = hipGetLastError();
    double* tmp = a;
    a = b;
    b = tmp;
  }
  return e;
}

}  // namespace hj
