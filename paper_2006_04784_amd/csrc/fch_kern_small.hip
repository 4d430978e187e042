// fch_kern_small.hip -- single-workgroup kernels: control block writes,
// deterministic reductions of per-workgroup partial sums into the scalars of
// the schemes (SAV s* and r, PSD stopping ratio, AM3 error and next step,
// energy), and the SAV combine u^{n+1} = p + r q.
#include <hip/hip_runtime.h>

#include "fch_kernels_impl.hpp"

namespace fch {

// ===========================================================================
// Small kernels: control block, reductions, SAV combine
// ===========================================================================
__global__ void k_ctl_set(StepCtl* ctl, StepCtl v) { *ctl = v; }

__device__ __forceinline__ double sum_strided(const double* p, int n, int stride, int off,
                                              double* red) {
  constexpr int NT = 256;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += p[(size_t)i * stride + off];
  double v[1] = {s};
  __shared__ double tot;
  block_reduce<NT, 1>(v, red, &tot);
  __syncthreads();
  return tot;
}

__global__ __launch_bounds__(256) void k_finalize(FinArgs a) {
  __shared__ double red[256];
  StepCtl* ctl = a.ctl;
  const Consts& c = a.c;
  if (a.mode == FIN_PSD && ctl->done) return;
  double r0 = 0, r1 = 0, c0 = 0, c1 = 0;
  if (a.rpart) {
    r0 = sum_strided(a.rpart, a.nrow, 2, 0, red);
    r1 = sum_strided(a.rpart, a.nrow, 2, 1, red);
  }
  if (a.cpart) {
    c0 = sum_strided(a.cpart, a.ncol, 2, 0, red);
    c1 = sum_strided(a.cpart, a.ncol, 2, 1, red);
  }
  if (threadIdx.x != 0) return;
  switch (a.mode) {
    case FIN_SAV_S: {
      const double E1 = c.h2 * r0;
      const double s2 = E1 + c.D0;
      ctl->E1 = E1;
      if (!isfinite(s2)) {
        ctl->nonfinite = 1;
        ctl->s_star = 1.0;
      } else if (!(s2 > 0.0)) {
        ctl->invalid = 1;
        ctl->s_star = 1.0;
      } else {
        ctl->s_star = sqrt(s2);
      }
      break;
    }
    case FIN_SAV_R: {
      const double gp = c.pars * c0, gq = c.pars * c1;
      const double r = (-ctl->b * ctl->r_n - ctl->c * ctl->r_nm1 + 0.5 * gp) /
                       (ctl->a - 0.5 * ctl->a * gq);
      ctl->r_np1 = r;
      if (!isfinite(r)) ctl->nonfinite = 1;
      break;
    }
    case FIN_PSD: {
      const double ratio = sqrt(c0 / c1);
      ctl->ratio = ratio;
      ctl->iters += 1;
      if (!isfinite(ratio)) {
        ctl->nonfinite = 1;
        ctl->done = 3;
      } else if (ctl->fixed_iters > 0) {
        if (ctl->iters >= ctl->fixed_iters) ctl->done = 1;
      } else if (ratio < ctl->tol) {
        ctl->done = 1;
      } else if (ctl->iters >= ctl->max_iter) {
        ctl->done = 2;
      }
      break;
    }
    case FIN_AM3: {
      const double e = sqrt(c0 / c1);
      const double ee = e > 1e-300 ? e : 1e-300;
      double kn = ctl->rho_s * cbrt(ctl->sigma_tol / ee) * ctl->k_np1;
      if (ctl->cap > 0.0 && kn > ctl->cap * ctl->k_np1) kn = ctl->cap * ctl->k_np1;
      if (kn > ctl->k_max) kn = ctl->k_max;
      if (kn < ctl->k_min) kn = ctl->k_min;
      ctl->err = e;
      ctl->k_next = kn;
      ctl->accept = (e <= ctl->sigma_tol) || (ctl->k_np1 <= ctl->k_min);
      if (!isfinite(e)) ctl->nonfinite = 1;
      break;
    }
    case FIN_ENERGY: {
      ctl->energy = c.h2 * r1 - 0.5 * c.eps2 * c.eta1 * c.pars * c0;
      if (!isfinite(ctl->energy)) ctl->nonfinite = 1;
      break;
    }
  }
}

__global__ void k_axpy_r(cd* out, const cd* q, const StepCtl* ctl, size_t n) {
  const double r = ctl->r_np1;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const cd o = out[i], qq = q[i];
    out[i] = cd{fma(r, qq.x, o.x), fma(r, qq.y, o.y)};
  }
}

// Per-member controller of a batched adaptive BDF2-IMEX attempt (Sec. 3.2,
// Steps 3-4 and Step 0 of the next step): relative AM3 error from the
// column partial sums, accept / reject, the next trial step, slot rotation,
// and the BDF2 / AM3 scalars of the next attempt.
__global__ __launch_bounds__(256) void k_ens_control(EnsMember* mem, int first) {
  __shared__ double red[256];
  EnsMember* m = mem + first + blockIdx.x;
  if (m->ctl.done) return;
  const double c0 = sum_strided(m->cpart, m->H, 2, 0, red);
  const double c1 = sum_strided(m->cpart, m->H, 2, 1, red);
  if (threadIdx.x != 0) return;
  StepCtl& ctl = m->ctl;
  const double kt = ctl.k_np1;
  const double e = sqrt(c0 / c1);
  const double ee = e > 1e-300 ? e : 1e-300;
  double kn = ctl.rho_s * cbrt(ctl.sigma_tol / ee) * kt;
  if (ctl.cap > 0.0 && kn > ctl.cap * kt) kn = ctl.cap * kt;
  if (kn > ctl.k_max) kn = ctl.k_max;
  if (kn < ctl.k_min) kn = ctl.k_min;
  const int accept = (e <= ctl.sigma_tol) || (kt <= ctl.k_min);
  ctl.err = e;
  ctl.k_next = kn;
  ctl.accept = accept;
  if (!isfinite(e)) {
    ctl.nonfinite = 1;
    ctl.done = 1;
    return;
  }
  if (accept) {
    const int op = m->prev;
    m->prev = m->cur;
    m->cur = m->trial;
    m->trial = op;
    const int ofm = m->fm;
    m->fm = m->fn;
    m->fn = m->ft;
    m->ft = ofm;
    m->t += kt;
    if (m->accepted < m->klog_cap) m->klog[m->accepted] = kt;
    m->accepted += 1;
    ctl.k_n = kt;
  } else {
    m->rejected += 1;
  }
  if (m->t >= m->t_end * (1.0 - 1e-14) || m->accepted >= m->max_accepted) {
    ctl.done = 1;
    return;
  }
  double k1 = kn;
  if (k1 > m->t_end - m->t) k1 = m->t_end - m->t;
  const double k0 = ctl.k_n;
  ctl.k_np1 = k1;
  ctl.a = 1.0 / k1 + 1.0 / (k1 + k0);
  ctl.b = -1.0 / k1 - 1.0 / k0;
  ctl.c = 1.0 / k0 - 1.0 / (k1 + k0);
  const double g = k1 / k0;
  ctl.gamma = g;
  ctl.w1 = k1 / 6.0 * (3.0 + 2.0 * g) / (1.0 + g);
  ctl.w2 = k1 / 6.0 * (3.0 + g);
  ctl.w3 = -k1 / 6.0 * g * g / (1.0 + g);
}

hipError_t launch_ens_control(EnsMember* m, int first, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_control, dim3(count), dim3(256), 0, s, m, first);
  return hipGetLastError();
}

hipError_t launch_ctl_set(StepCtl* ctl, const StepCtl& v, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(1), 0, s, ctl, v);
  return hipGetLastError();
}
hipError_t launch_finalize(const FinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_axpy_r(cd* out, const cd* q, const StepCtl* ctl, size_t n, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_axpy_r, dim3((unsigned)blocks), dim3(256), 0, s, out, q, ctl, n);
  return hipGetLastError();
}

}  // namespace fch
