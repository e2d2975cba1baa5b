// hj_paper.hpp -- the paper's own scheme and its further problem families on
// gfx950: forward Euler characteristics with the rectangle rule (section
// 4.2, eq. num_int), the staggered discrete Lax and Hopf forms of section 3
// (implicit half-steps by fixed-point iteration) or RK4 with the
// RK4-augmented rule, forward-difference
// derivatives (eq. num_diff) driving Algorithm 1 (section 4.1: cyclic
// coordinate descent, alpha = 1/L halved every M updates, stopped after d
// consecutive moves below epsilon) or heavy-ball descent, for
//  - the quadratic family H = 1/2 m(|x|^2) sum d p^2 + 1/2 w |x|^2 (section
//    5 Example 2 is m = 1, d = w = +-1),
//  - the degree-1 family H = s1 c1(x)|p_A| + s2 c2(x)|p_B|, A the first k
//    components, c_i(x) = c0 (1 + beta exp(-gam |x -+ mu|^2)) (section 5
//    Examples 3 and 5; the zero subgradient where a block of p vanishes),
// with ellipsoid or Rosenbrock (eq. weird) initial data, and the functionals
// F1 (Lax), G (Hopf) and F2 = min_k g(gamma_k) (eq. num_min).
//
// One lane per (point, guess) task; the problem (n <= 16 components) travels
// by value in the kernel arguments.  Vector components live in registers and
// are indexed with compile-time indices only (a runtime coordinate j is
// selected by comparison), so nothing spills to private memory.
#pragma once

#include "hj_device.hpp"
#include "hj_launch.hpp"

namespace hj {

// H, H_x and H_p at (x, p).
template <int NPL, int HK>
__device__ __forceinline__ double paper_grads(const PaperProblem& P, const double (&x)[NPL],
                                              const double (&p)[NPL], double (&Hx)[NPL],
                                              double (&Hp)[NPL]) {
  if constexpr (HK == HJ_H_NORM) {
    double r1 = 0.0, r2 = 0.0, nA2 = 0.0, nB2 = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const double a = x[i] - P.mu[i], b = x[i] + P.mu[i];
      r1 = fmaT(a, a, r1);
      r2 = fmaT(b, b, r2);
      if (i < P.k)
        nA2 = fmaT(p[i], p[i], nA2);
      else
        nB2 = fmaT(p[i], p[i], nB2);
    }
    const double E1 = exp(-P.gam * r1), E2 = exp(-P.gam * r2);
    const double c1 = P.c0 * (1.0 + P.beta * E1), c2 = P.c0 * (1.0 + P.beta * E2);
    const double nA = sqrt(nA2), nB = sqrt(nB2);
    const double gx1 = P.c0 * P.beta * E1 * (-2.0 * P.gam);  // grad c1 = gx1 (x - mu)
    const double gx2 = P.c0 * P.beta * E2 * (-2.0 * P.gam);  // grad c2 = gx2 (x + mu)
    const double fA = nA > 0.0 ? P.s1 * c1 / nA : 0.0, fB = nB > 0.0 ? P.s2 * c2 / nB : 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      Hx[i] = P.s1 * nA * (gx1 * (x[i] - P.mu[i])) + P.s2 * nB * (gx2 * (x[i] + P.mu[i]));
      Hp[i] = (i < P.k ? fA : fB) * p[i];
    }
    return P.s1 * c1 * nA + P.s2 * c2 * nB;
  } else {
    double r = 0.0, q = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      r = fmaT(x[i], x[i], r);
      q = fmaT(P.d[i] * p[i], p[i], q);
    }
    double c = 1.0, c1 = 0.0;
    if (P.m_kind == HJ_M_RAT) {
      const double iv = 1.0 / (1.0 + r);
      c = 1.0 + P.kappa * r * iv;
      c1 = P.kappa * iv * iv;
    } else if (P.m_kind == HJ_M_TANH) {
      const double th = dtanh(r * P.inv_s);
      c = 1.0 + P.kappa * th;
      c1 = P.kappa * P.inv_s * (1.0 - th * th);
    }
    const double m = P.e == 2 ? c * c : c, m1 = P.e == 2 ? 2.0 * c * c1 : c1;
    const double cx = q * m1 + P.w;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      Hp[i] = m * P.d[i] * p[i];
      Hx[i] = cx * x[i];
    }
    return 0.5 * m * q + 0.5 * P.w * r;
  }
}

// Integrand of the action: Lax <p, H_p> - H, Hopf H - <H_x, gamma>.
template <int NPL>
__device__ __forceinline__ double paper_integrand(const PaperProblem& P, const double (&x)[NPL],
                                                  const double (&p)[NPL], double H,
                                                  const double (&Hx)[NPL],
                                                  const double (&Hp)[NPL]) {
  double s = 0.0;
  if (P.functional == HJ_HOPF) {
#pragma unroll
    for (int i = 0; i < NPL; ++i) s = fmaT(Hx[i], x[i], s);
    return H - s;
  }
#pragma unroll
  for (int i = 0; i < NPL; ++i) s = fmaT(p[i], Hp[i], s);
  return s - H;
}

template <int NPL>
__device__ __forceinline__ double paper_g(const PaperProblem& P, const double (&x)[NPL]) {
  if (P.jkind == HJ_J_ROSENBROCK) {
    const double a = 1.0 - x[0], b = 1.0 + x[1] - x[0] * x[0];
    return P.rscale * (-100.0 + a * a + 100.0 * b * b);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NPL; ++i) s = fmaT(x[i] * x[i], P.ia2[i], s);
  return 0.5 * s + P.j0;
}

template <int NPL>
__device__ __forceinline__ void paper_grad_g(const PaperProblem& P, const double (&x)[NPL],
                                             double (&out)[NPL]) {
  if (P.jkind == HJ_J_ROSENBROCK) {
    const double b = 1.0 + x[1] - x[0] * x[0];
#pragma unroll
    for (int i = 0; i < NPL; ++i) out[i] = 0.0;
    out[0] = P.rscale * (-2.0 * (1.0 - x[0]) - 400.0 * x[0] * b);
    out[1] = P.rscale * 200.0 * b;
    return;
  }
#pragma unroll
  for (int i = 0; i < NPL; ++i) out[i] = x[i] * P.ia2[i];
}

// Certificate of the Lax functionals at (gamma, p): p = grad g(gamma), on
// directions for the degree-1 family (the scale of p is free there).
template <int NPL, int HK>
__device__ __forceinline__ double paper_lax_residual(const PaperProblem& P,
                                                     const double (&x)[NPL],
                                                     const double (&p)[NPL]) {
  double gg[NPL];
  paper_grad_g<NPL>(P, x, gg);
  double sp = 1.0, sg = 1.0;
  if constexpr (HK == HJ_H_NORM) {
    double np2 = 0.0, ng2 = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      np2 = fmaT(p[i], p[i], np2);
      ng2 = fmaT(gg[i], gg[i], ng2);
    }
    sp = np2 > 0.0 ? 1.0 / sqrt(np2) : 0.0;
    sg = ng2 > 0.0 ? 1.0 / sqrt(ng2) : 0.0;
  }
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NPL; ++i) r = nanmax(r, dabs(p[i] * sp - gg[i] * sg));
  return r;
}

// One implicit half-step of the staggered schemes, solved by fixed-point
// iteration from z (its initial guess) until a sweep moves z by at most
// 1e-14 (1 + |z|) in the max norm, or for 60 sweeps:
//   IX (Lax):   z = rhs - delta H_p(z, o), the new x with the new p = o;
//   else (Hopf): z = rhs + delta H_x(o, z), the new p at the new x = o.
template <int NPL, int HK, bool IX>
__device__ __forceinline__ void stagger_fixed_point(const PaperProblem& P,
                                                    const double (&rhs)[NPL],
                                                    const double (&o)[NPL], double (&z)[NPL]) {
  double Hx[NPL], Hp[NPL];
  for (int it = 0; it < 60; ++it) {
    if constexpr (IX)
      paper_grads<NPL, HK>(P, z, o, Hx, Hp);
    else
      paper_grads<NPL, HK>(P, o, z, Hx, Hp);
    double dz = 0.0, nz = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const double zn = IX ? rhs[i] - P.h * Hp[i] : rhs[i] + P.h * Hx[i];
      dz = nanmax(dz, dabs(zn - z[i]));
      nz = dabs(zn) > nz ? dabs(zn) : nz;
      z[i] = zn;
    }
    if (!(dz > 1e-14 * (1.0 + nz))) break;
  }
}

// The staggered discrete functionals of section 3 (eqs. hahalolXDform and
// hahalolXDform2), evaluated on the fly from n = N (x_N = x, p_N = v) down
// to n = 0 with delta = t / N:
//   Lax dynamics: p_{n-1} = p_n + delta H_x(x_n, p_n), then x_{n-1} from
//     x_n - x_{n-1} = delta H_p(x_{n-1}, p_{n-1});
//     F1 = g(x_0) + sum_{n<N} (<p_n, x_{n+1} - x_n> - delta H(x_n, p_n)),
//     certified by grad g(x_0) = p_0 + delta H_x(x_0, p_0) (stationarity in
//     x_0); F2 = min over n of g(x_n), first minimiser from n = N down;
//   Hopf dynamics: x_{n-1} = x_n - delta H_p(x_n, p_n), then for n - 1 >= 1
//     p_{n-1} from p_{n-1} - p_n = delta H_x(x_{n-1}, p_{n-1});
//     -G = g*(p_1) - <x, v> + delta sum_{n>=1} H(x_n, p_n)
//          - sum_{1<=n<N} <p_n - p_{n+1}, x_n>, certified by x_0 = a^2 p_1.
// Every grads evaluation at a node (x_n, p_n) serves both its H term and the
// explicit half of the next step.
template <int NPL, int HK>
__device__ double paper_stagger_eval(const PaperProblem& P, const double (&x0)[NPL],
                                     const double (&v)[NPL], double& rho) {
  double x[NPL], p[NPL], Hx[NPL], Hp[NPL], rhs[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    x[i] = x0[i];
    p[i] = v[i];
  }
  const double h = P.h;
  double q = 0.0;
  if (P.functional == HJ_HOPF) {
    for (int m = P.N; m >= 1; --m) {
      const double H = paper_grads<NPL, HK>(P, x, p, Hx, Hp);
      q = fmaT(h, H, q);
#pragma unroll
      for (int i = 0; i < NPL; ++i) x[i] = x[i] - h * Hp[i];
      if (m >= 2) {
#pragma unroll
        for (int i = 0; i < NPL; ++i) rhs[i] = p[i];
        stagger_fixed_point<NPL, HK, false>(P, rhs, x, p);
        // -<p_{m-1} - p_m, x_{m-1}>
#pragma unroll
        for (int i = 0; i < NPL; ++i) q -= (p[i] - rhs[i]) * x[i];
      }
    }
    double gs = 0.0, xv = 0.0, r = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      gs = fmaT(P.a2[i] * p[i], p[i], gs);
      xv = fmaT(x0[i], v[i], xv);
      r = nanmax(r, dabs(x[i] - P.a2[i] * p[i]));
    }
    rho = r;
    return 0.5 * gs - P.j0 - xv + q;
  }
  const bool fmin = P.functional == HJ_LAX_MIN;
  double gmin = 0.0, xm[NPL], pm[NPL];
  if (fmin) {
    gmin = paper_g<NPL>(P, x);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      xm[i] = x[i];
      pm[i] = p[i];
    }
  }
  for (int m = P.N; m >= 1; --m) {
    const double H = paper_grads<NPL, HK>(P, x, p, Hx, Hp);
    if (m < P.N) q = fmaT(-h, H, q);  // the H term of node m < N
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      rhs[i] = x[i];
      p[i] = p[i] + h * Hx[i];
      x[i] = x[i] - h * Hp[i];
    }
    stagger_fixed_point<NPL, HK, true>(P, rhs, p, x);
#pragma unroll
    for (int i = 0; i < NPL; ++i) q = fmaT(p[i], rhs[i] - x[i], q);
    if (fmin) {
      const double gk = paper_g<NPL>(P, x);
      if (gk < gmin || (gk != gk && gmin == gmin)) {
        gmin = gk;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          xm[i] = x[i];
          pm[i] = p[i];
        }
      }
    }
  }
  if (fmin) {
    rho = paper_lax_residual<NPL, HK>(P, xm, pm);
    return gmin;
  }
  const double H0 = paper_grads<NPL, HK>(P, x, p, Hx, Hp);
  q = fmaT(-h, H0, q);
#pragma unroll
  for (int i = 0; i < NPL; ++i) p[i] = p[i] + h * Hx[i];
  rho = paper_lax_residual<NPL, HK>(P, x, p);
  return paper_g<NPL>(P, x) + q;
}

// The discrete functional at v (F1, G or F2) and its certificate residual.
template <int NPL, int HK>
__device__ double paper_eval(const PaperProblem& P, const double (&x0)[NPL],
                             const double (&v)[NPL], double& rho) {
  if (P.ode == HJ_STAGGERED) return paper_stagger_eval<NPL, HK>(P, x0, v, rho);
  double x[NPL], p[NPL], Hx[NPL], Hp[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    x[i] = x0[i];
    p[i] = v[i];
  }
  const bool fmin = P.functional == HJ_LAX_MIN;
  double q = 0.0, gmin = 0.0, xm[NPL], pm[NPL];
  if (fmin) {
    gmin = paper_g<NPL>(P, x);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      xm[i] = x[i];
      pm[i] = p[i];
    }
  }
  const double h = P.h;
  for (int s = 0; s < P.N; ++s) {
    if (P.ode == HJ_EULER) {
      const double H = paper_grads<NPL, HK>(P, x, p, Hx, Hp);
      if (!fmin) q += h * paper_integrand<NPL>(P, x, p, H, Hx, Hp);
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        x[i] = x[i] + h * (-Hp[i]);
        p[i] = p[i] + h * Hx[i];
      }
    } else {
      // RK4 with the RK4-augmented rule: K = (-H_p, H_x) at the four stages
      double Kx[4][NPL], Kp[4][NPL], it[4], Yx[NPL], Yp[NPL];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const double c = st == 0 ? 0.0 : (st == 3 ? h : 0.5 * h);
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          Yx[i] = st == 0 ? x[i] : x[i] + c * Kx[st - 1 < 0 ? 0 : st - 1][i];
          Yp[i] = st == 0 ? p[i] : p[i] + c * Kp[st - 1 < 0 ? 0 : st - 1][i];
        }
        const double H = paper_grads<NPL, HK>(P, Yx, Yp, Hx, Hp);
        it[st] = fmin ? 0.0 : paper_integrand<NPL>(P, Yx, Yp, H, Hx, Hp);
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          Kx[st][i] = -Hp[i];
          Kp[st][i] = Hx[i];
        }
      }
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        x[i] = x[i] + h / 6.0 * (Kx[0][i] + 2.0 * Kx[1][i] + 2.0 * Kx[2][i] + Kx[3][i]);
        p[i] = p[i] + h / 6.0 * (Kp[0][i] + 2.0 * Kp[1][i] + 2.0 * Kp[2][i] + Kp[3][i]);
      }
      q += h / 6.0 * (it[0] + 2.0 * it[1] + 2.0 * it[2] + it[3]);
    }
    if (fmin) {
      const double gk = paper_g<NPL>(P, x);
      if (gk < gmin || (gk != gk && gmin == gmin)) {
        gmin = gk;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          xm[i] = x[i];
          pm[i] = p[i];
        }
      }
    }
  }
  if (fmin) {
    rho = paper_lax_residual<NPL, HK>(P, xm, pm);
    return gmin;
  }
  if (P.functional == HJ_HOPF) {
    double gs = 0.0, xv = 0.0, r = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      gs = fmaT(P.a2[i] * p[i], p[i], gs);
      xv = fmaT(x0[i], v[i], xv);
      r = nanmax(r, dabs(x[i] - P.a2[i] * p[i]));
    }
    rho = r;
    return 0.5 * gs - P.j0 + q - xv;
  }
  rho = paper_lax_residual<NPL, HK>(P, x, p);
  return paper_g<NPL>(P, x) + q;
}

template <int NPL>
__device__ __forceinline__ double paper_vmax(const PaperProblem& P, const double (&v)[NPL]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NPL; ++i) s = nanmax(s, dabs(v[i]));
  (void)P;
  return s;
}

// Algorithm 1 from v (in/out): two evaluations per coordinate update.
template <int NPL, int HK>
__device__ int paper_alg1(const PaperArgs& A, const double (&x)[NPL], double (&v)[NPL],
                          double& phi, double& rho, int& iters, int64_t& n_eval) {
  const PaperProblem& P = A.P;
  const int n = P.n;
  double alpha = A.alpha0;
  phi = paper_eval<NPL, HK>(P, x, v, rho);
  n_eval += 1;
  int count = 0, kM = 0, upd = 0, j = 0;
  int status = isfinite(phi) ? HJ_ST_MAXITER : HJ_ST_DIVERGED;
  const int cap = A.max_iter * n;
  while (status == HJ_ST_MAXITER && upd < cap) {
    double vt[NPL], vj = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      if (i == j) vj = v[i];
      vt[i] = (i == j) ? v[i] + A.sigma : v[i];
    }
    double rt;
    const double fp = paper_eval<NPL, HK>(P, x, vt, rt);
    const double gj = (fp - phi) / A.sigma;
    const double step = alpha * gj;
#pragma unroll
    for (int i = 0; i < NPL; ++i)
      if (i == j) v[i] = vj - step;
    phi = paper_eval<NPL, HK>(P, x, v, rho);
    n_eval += 2;
    ++upd;
    if (++kM == A.M) {
      kM = 0;
      alpha *= 0.5;
    }
    const double as = dabs(step);
    if (as > A.eps)
      count = 0;
    else if (as < A.eps)
      ++count;
    j = (j + 1 == n) ? 0 : j + 1;
    if (!isfinite(phi) || !(paper_vmax<NPL>(P, v) <= A.v_max))
      status = HJ_ST_DIVERGED;
    else if (count == n)
      status = HJ_ST_CONVERGED;
  }
  iters = upd;
  if (status == HJ_ST_DIVERGED) rho = __builtin_nan("");
  return status;
}

// Heavy-ball descent with a forward-difference gradient (n + 1 evaluations
// per iteration); a trial that raises the objective beyond the rounding
// allowance is rejected, the momentum dropped and alpha halved.
template <int NPL, int HK>
__device__ int paper_momentum(const PaperArgs& A, const double (&x)[NPL], double (&v)[NPL],
                              double& phi, double& rho, int& iters, int64_t& n_eval) {
  const PaperProblem& P = A.P;
  const int n = P.n;
  double alpha = A.alpha0;
  const double floor_a = A.alpha0 * 9.094947017729282e-13;  // alpha0 2^-40
  phi = paper_eval<NPL, HK>(P, x, v, rho);
  n_eval += 1;
  double vp[NPL], g[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) vp[i] = v[i];
  int it = 0;
  int status = isfinite(phi) ? HJ_ST_MAXITER : HJ_ST_DIVERGED;
  while (status == HJ_ST_MAXITER && it < A.max_iter) {
    ++it;
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      g[j] = 0.0;
      if (j < n) {
        double vt[NPL], rt;
#pragma unroll
        for (int i = 0; i < NPL; ++i) vt[i] = (i == j) ? v[i] + A.sigma : v[i];
        g[j] = (paper_eval<NPL, HK>(P, x, vt, rt) - phi) / A.sigma;
      }
    }
    double vt[NPL], smax = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      vt[i] = v[i] - alpha * g[i] + A.momentum * (v[i] - vp[i]);
      smax = nanmax(smax, dabs(vt[i] - v[i]));
    }
    double rt;
    const double ft = paper_eval<NPL, HK>(P, x, vt, rt);
    n_eval += n + 1;
#pragma unroll
    for (int i = 0; i < NPL; ++i) vp[i] = v[i];
    if (ft <= phi + A.acc_rel * dabs(phi)) {
#pragma unroll
      for (int i = 0; i < NPL; ++i) v[i] = vt[i];
      phi = ft;
      rho = rt;
    } else {
      alpha *= 0.5;
    }
    if (!isfinite(phi) || !(paper_vmax<NPL>(P, v) <= A.v_max))
      status = HJ_ST_DIVERGED;
    else if (smax < A.eps)
      status = HJ_ST_CONVERGED;
    else if (alpha < floor_a)
      status = HJ_ST_STALLED;
  }
  iters = it;
  if (status == HJ_ST_DIVERGED) rho = __builtin_nan("");
  return status;
}

// One lane per (point, guess) slot: attempts from the slot's guesses until
// one is certified, the slot's record as in the adjoint-descent kernels.
template <int NPL, int HK>
__global__ __launch_bounds__(256) void k_solve_paper(PaperArgs A) {
  const int64_t task = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (task >= A.ntask) return;
  const int n = A.P.n;
  const int64_t b = task / A.G;
  double x[NPL], v[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) x[i] = i < n ? A.x[b * n + i] : 0.0;
  double bphi = __builtin_nan(""), brho = __builtin_nan("");
  int bcert = -1, bstatus = HJ_ST_DIVERGED, iters = 0, att = 0;
  int64_t n_eval = 0;
  double bv[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) bv[i] = __builtin_nan("");
  for (int r = 0; r <= A.R; ++r) {
    const double* g0 = A.guesses + (task * (A.R + 1) + r) * n;
#pragma unroll
    for (int i = 0; i < NPL; ++i) v[i] = i < n ? g0[i] : 0.0;
    double phi, rho;
    int it = 0;
    const int st = A.mode == HJ_MOMENTUM ? paper_momentum<NPL, HK>(A, x, v, phi, rho, it, n_eval)
                                         : paper_alg1<NPL, HK>(A, x, v, phi, rho, it, n_eval);
    iters += it;
    att = r + 1;
    const bool fin = st != HJ_ST_DIVERGED && isfinite(phi);
    const bool cert = fin && rho <= A.cert_tol;
    if (cert || (fin && (bcert < 0 || phi < bphi))) {
      bphi = phi;
      brho = rho;
      bcert = cert ? 1 : 0;
      bstatus = st;
#pragma unroll
      for (int i = 0; i < NPL; ++i) bv[i] = v[i];
    }
    if (cert) break;
  }
  if (A.out.phi) A.out.phi[task] = bphi;
  if (A.out.rho) A.out.rho[task] = brho;
  if (A.out.status) A.out.status[task] = bstatus;
  if (A.out.cert) A.out.cert[task] = bcert;
  if (A.out.iters) A.out.iters[task] = iters;
  if (A.out.attempts) A.out.attempts[task] = att;
  if (A.out.n_fwd) A.out.n_fwd[task] = n_eval;
  if (A.out.n_bwd) A.out.n_bwd[task] = 0;
#pragma unroll
  for (int i = 0; i < NPL; ++i)
    if (i < n) A.out.v[task * n + i] = bv[i];
}

// The functional at given v: phi [B*G], rho [B*G].
template <int NPL, int HK>
__global__ __launch_bounds__(256) void k_eval_paper(PaperProblem P, const double* x,
                                                    const double* v, int64_t B, int G,
                                                    double* phi, double* rho) {
  const int64_t task = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (task >= B * G) return;
  const int n = P.n;
  const int64_t b = task / G;
  double xx[NPL], vv[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    xx[i] = i < n ? x[b * n + i] : 0.0;
    vv[i] = i < n ? v[task * n + i] : 0.0;
  }
  double r;
  const double f = paper_eval<NPL, HK>(P, xx, vv, r);
  phi[task] = f;
  if (rho) rho[task] = r;
}

// ---------------------------------------------------------------------------
// Lax-Friedrichs grid solver of phi_t + H(x, grad phi) = 0 in two space
// dimensions (the independent check of section 5), H of the quadratic
// family: phi^{k+1} = phi^k - dt [H(x, (D+x + D-x)/2, (D+y + D-y)/2)
//   - ax (D+x - D-x)/2 - ay (D+y - D-y)/2], one-sided differences D+-,
// linear extrapolation across the boundary; row j of phi is y_j = y0 + j dy,
// column i is x_i = x0 + i dx.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lf_hamiltonian(const PaperProblem& P, double x, double y,
                                                 double p1, double p2) {
  const double r = x * x + y * y;
  double c = 1.0;
  if (P.m_kind == HJ_M_RAT)
    c = 1.0 + P.kappa * r / (1.0 + r);
  else if (P.m_kind == HJ_M_TANH)
    c = 1.0 + P.kappa * dtanh(r * P.inv_s);
  const double m = P.e == 2 ? c * c : c;
  const double q = P.d[0] * p1 * p1 + P.d[1] * p2 * p2;
  return 0.5 * m * q + 0.5 * P.w * r;
}

__global__ __launch_bounds__(256) void k_lf_init(PaperProblem P, double x0, double y0, double dx,
                                                 double dy, int nx, int ny, double* phi) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= (int64_t)nx * ny) return;
  const int i = (int)(c % nx), j = (int)(c / nx);
  double xy[2] = {x0 + i * dx, y0 + j * dy};
  phi[c] = paper_g<2>(P, xy);
}

// One Lax-Friedrichs update of a cell from its value c and its four
// neighbours (left, right, down, up) at the previous level.
// idx, idy: 1 / dx, 1 / dy.
__device__ __forceinline__ double lf_update(const PaperProblem& P, double x, double y, double c,
                                            double l, double r, double d, double u, double idx,
                                            double idy, double dt, double ax, double ay) {
  const double pp = (r - c) * idx, pm = (c - l) * idx;
  const double qp = (u - c) * idy, qm = (c - d) * idy;
  const double Hn = lf_hamiltonian(P, x, y, 0.5 * (pp + pm), 0.5 * (qp + qm)) -
                    0.5 * ax * (pp - pm) - 0.5 * ay * (qp - qm);
  return c - dt * Hn;
}

// The Lax-Friedrichs solver, several steps per launch (temporal blocking).
// A block owns a tile of kLfTX x kLfTY cells; it loads the tile with a halo
// of kLfT cells into LDS, advances the whole region nsub <= kLfT steps
// there, and writes back its own cells.  Each step's valid region shrinks
// by one cell on every side that borders another tile's cells; a side on
// the domain boundary keeps its edge cells, which extrapolate their missing
// neighbour linearly from the in-tile one.  Every cell takes lf_update
// whatever the tiling, so the result does not depend on it; the grid makes
// a round trip through the cache hierarchy, and the device a launch, per
// kLfT steps instead of per step.  A block's 256 lanes walk a rectangle 4
// rows of 64 columns at a time (no integer division per cell).
constexpr int kLfTX = 64, kLfTY = 32, kLfT = 4;
constexpr int kLfRW = kLfTX + 2 * kLfT, kLfRH = kLfTY + 2 * kLfT;

__global__ __launch_bounds__(256) void k_lf_steps(PaperProblem P, double x0, double y0,
                                                  double dx, double dy, int nx, int ny,
                                                  double dt, double ax, double ay, int nsub,
                                                  const double* __restrict__ in,
                                                  double* __restrict__ out) {
  __shared__ double buf[2][kLfRH * kLfRW];
  // the block walks a rectangle as 4 rows of 64 columns at a time
  const int tc = threadIdx.x & 63, tr = threadIdx.x >> 6;
  const double idx = 1.0 / dx, idy = 1.0 / dy;
  const int tx0 = blockIdx.x * kLfTX, ty0 = blockIdx.y * kLfTY;  // tile origin
  const int gx0 = tx0 - kLfT, gy0 = ty0 - kLfT;                  // region origin
  // the region clipped to the domain
  const int rxl = gx0 > 0 ? gx0 : 0, rxh = gx0 + kLfRW < nx ? gx0 + kLfRW : nx;
  const int ryl = gy0 > 0 ? gy0 : 0, ryh = gy0 + kLfRH < ny ? gy0 + kLfRH : ny;
  for (int gy = ryl + tr; gy < ryh; gy += 4)
    for (int gx = rxl + tc; gx < rxh; gx += 64)
      buf[0][(gy - gy0) * kLfRW + (gx - gx0)] = in[(int64_t)gy * nx + gx];
  __syncthreads();
  int cur = 0;
  for (int s = 1; s <= nsub; ++s) {
    const int xl = rxl == 0 ? 0 : rxl + s, xh = rxh == nx ? nx : rxh - s;
    const int yl = ryl == 0 ? 0 : ryl + s, yh = ryh == ny ? ny : ryh - s;
    const double* B = buf[cur];
    double* Nw = buf[cur ^ 1];
    for (int gy = yl + tr; gy < yh; gy += 4)
      for (int gx = xl + tc; gx < xh; gx += 64) {
        const int L = (gy - gy0) * kLfRW + (gx - gx0);
        const double ce = B[L];
        const double l = gx > 0 ? B[L - 1] : 2.0 * ce - B[L + 1];
        const double r = gx < nx - 1 ? B[L + 1] : 2.0 * ce - B[L - 1];
        const double d = gy > 0 ? B[L - kLfRW] : 2.0 * ce - B[L + kLfRW];
        const double u = gy < ny - 1 ? B[L + kLfRW] : 2.0 * ce - B[L - kLfRW];
        Nw[L] = lf_update(P, x0 + gx * dx, y0 + gy * dy, ce, l, r, d, u, idx, idy, dt, ax, ay);
      }
    __syncthreads();
    cur ^= 1;
  }
  const int xe = tx0 + kLfTX < nx ? tx0 + kLfTX : nx, ye = ty0 + kLfTY < ny ? ty0 + kLfTY : ny;
  for (int gy = ty0 + tr; gy < ye; gy += 4)
    for (int gx = tx0 + tc; gx < xe; gx += 64)
      out[(int64_t)gy * nx + gx] = buf[cur][(gy - gy0) * kLfRW + (gx - gx0)];
}

}  // namespace hj
