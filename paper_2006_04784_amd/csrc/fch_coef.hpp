// fch_coef.hpp -- per-step scalars of the schemes, shared by the host-side
// orchestration and the device-side controllers (one definition, so a step
// driven from the host and one driven from device memory use the same
// arithmetic).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "fch_kernels.hpp"

namespace fch {

// eq. BDF2Coef; k_n <= 0 selects the first-order startup step (u* = u^n)
__host__ __device__ inline void set_bdf2(StepCtl& v, double k_np1, double k_n) {
  v.k_np1 = k_np1;
  v.k_n = k_n;
  if (k_n <= 0.0) {
    v.a = 1.0 / k_np1;
    v.b = -1.0 / k_np1;
    v.c = 0.0;
    v.gamma = 0.0;
  } else {
    v.a = 1.0 / k_np1 + 1.0 / (k_np1 + k_n);
    v.b = -1.0 / k_np1 - 1.0 / k_n;
    v.c = 1.0 / k_n - 1.0 / (k_np1 + k_n);
    v.gamma = k_np1 / k_n;
  }
}

// eq. Predictor: AM3 weights of F(u~), F^n, F^{n-1}
__host__ __device__ inline void set_am3(StepCtl& v, double k_np1, double k_n) {
  const double g = k_np1 / k_n;
  v.w1 = k_np1 / 6.0 * (3.0 + 2.0 * g) / (1.0 + g);
  v.w2 = k_np1 / 6.0 * (3.0 + g);
  v.w3 = -k_np1 / 6.0 * g * g / (1.0 + g);
}

// Table SearchSize: lambda(q, k) linear in k between the printed columns,
// constant outside; -1 when q is not one of the tabulated rows
__host__ __device__ inline double lambda_table(double q, double k) {
  const double ks[10] = {1e-6, 1e-5, 5e-5, 1e-4, 5e-4, 1e-3, 5e-3, 0.01, 0.02, 0.03};
  const double qs[3] = {0.0, 0.2, 0.5};
  const double lam[3][10] = {{1.0, 1.07, 1.11, 1.14, 1.24, 1.34, 1.60, 1.738, 1.804, 1.855},
                             {1.0, 1.04, 1.15, 1.28, 1.50, 1.70, 1.87, 1.92, 1.95, 1.97},
                             {1.0, 1.20, 1.32, 1.45, 1.72, 1.83, 1.965, 1.97, 1.985, 1.99}};
  int row = -1;
  for (int i = 0; i < 3; ++i)
    if (fabs(q - qs[i]) < 1e-12) row = i;
  if (row < 0) return -1.0;
  if (k <= ks[0]) return lam[row][0];
  if (k >= ks[9]) return lam[row][9];
  int j = 0;
  while (k > ks[j + 1]) ++j;
  const double t = (k - ks[j]) / (ks[j + 1] - ks[j]);
  return lam[row][j] + t * (lam[row][j + 1] - lam[row][j]);
}

// Sec. 3.2 Steps 3-4: from the relative AM3 error e of the trial step
// k_np1, the acceptance and the next trial step (rho_s (sigma/e)^{1/3} k,
// capped, clamped to [k_min, k_max]); returns accept
__host__ __device__ inline int am3_decide(StepCtl& v, double e) {
  const double kt = v.k_np1;
  const double ee = e > 1e-300 ? e : 1e-300;
  double kn = v.rho_s * cbrt(v.sigma_tol / ee) * kt;
  if (v.cap > 0.0 && kn > v.cap * kt) kn = v.cap * kt;
  if (kn > v.k_max) kn = v.k_max;
  if (kn < v.k_min) kn = v.k_min;
  v.err = e;
  v.k_next = kn;
  v.accept = (e <= v.sigma_tol) || (kt <= v.k_min);
  return v.accept;
}

// SAV auxiliary scalar at the extrapolated state (eqs. 4.5-4.6):
// s* = sqrt(E_1(u*) + D0).  Returns 0, 1 (non-finite) or 2 (E_1 + D0 <= 0);
// s is 1 when unusable.
__host__ __device__ inline int sav_sstar(double E1, double D0, double& s) {
  const double s2 = E1 + D0;
  s = 1.0;
  if (!isfinite(s2)) return 1;
  if (!(s2 > 0.0)) return 2;
  s = sqrt(s2);
  return 0;
}

// SAV scalar solve (eq. 4.8) from g_p = (X, a p + b u^n + c u^{n-1}) and
// g_q = (X, q): r^{n+1} = (-b r^n - c r^{n-1} + g_p / 2) / (a - a g_q / 2)
__host__ __device__ inline double sav_r_solve(const StepCtl& v, double r_n, double r_nm1,
                                              double gp, double gq) {
  return (-v.b * r_n - v.c * r_nm1 + 0.5 * gp) / (v.a - 0.5 * v.a * gq);
}
__host__ __device__ inline double sav_r_solve(const StepCtl& v, double gp, double gq) {
  return sav_r_solve(v, v.r_n, v.r_nm1, gp, gq);
}

// Sec. 3.3 stopping test after `iters` iterations whose last step ratio is
// ||d|| / ||u_{s+1}||: 0 continue, 1 converged (or the fixed count reached),
// 2 iteration limit, 3 non-finite
__host__ __device__ inline int psd_done_code(int fixed_iters, double tol, int max_iter,
                                             double ratio, int iters) {
  if (!isfinite(ratio)) return 3;
  if (fixed_iters > 0) return iters >= fixed_iters ? 1 : 0;
  if (ratio < tol) return 1;
  if (iters >= max_iter) return 2;
  return 0;
}
__host__ __device__ inline int psd_done_code(const StepCtl& v, double ratio, int iters) {
  return psd_done_code(v.fixed_iters, v.tol, v.max_iter, ratio, iters);
}

// Device-controlled adaptive BDF2-PSD: the solve's control block for the
// attempt at the run's current trial step (the BDF2 coefficients of the
// run's control block, lambda fixed or from Table SearchSize), and the
// stages of the new attempt armed.  False when there is no lambda.
__host__ __device__ inline bool psd_arm(EnsMember* m) {
  StepCtl& s = m->sctl;
  const StepCtl& c = m->ctl;
  s.k_np1 = c.k_np1;
  s.k_n = c.k_n;
  s.a = c.a;
  s.b = c.b;
  s.c = c.c;
  s.gamma = c.gamma;
  s.lambda = m->psd_lambda > 0.0 ? m->psd_lambda : lambda_table(m->c.q, c.k_np1);
  s.iters = 0;
  s.done = 0;
  s.ratio = 0.0;
  m->psd_init_skip = 0;
  m->psd_eval_skip = 1;
  return s.lambda > 0.0;
}

}  // namespace fch
