// fch_kern_small.hip -- single-workgroup kernels: control block writes,
// deterministic reductions of per-workgroup partial sums into the scalars of
// the schemes (SAV s* and r, PSD stopping ratio, AM3 error and next step,
// energy), and the SAV combine u^{n+1} = p + r q.
#include <hip/hip_runtime.h>

#include "fch_coef.hpp"
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
    if (a.mode == FIN_PSD) {
      // the same summation as the stopping test folded into the row pass
      fixed_sum2<256, 4096 / 2 + 1, 32>(a.cpart, a.ncol, c0, c1);
    } else {
      c0 = sum_strided(a.cpart, a.ncol, 2, 0, red);
      c1 = sum_strided(a.cpart, a.ncol, 2, 1, red);
    }
  }
  if (threadIdx.x != 0) return;
  switch (a.mode) {
    case FIN_SAV_S: {
      const double E1 = c.h2 * r0;
      double sst;
      const int st = sav_sstar(E1, c.D0, sst);
      ctl->E1 = E1;
      ctl->s_star = sst;
      if (st == 1) ctl->nonfinite = 1;
      if (st == 2) ctl->invalid = 1;
      break;
    }
    case FIN_PSD: {
      const double ratio = sqrt(c0 / c1);
      const int it = ctl->iters + 1;
      const int code = psd_done_code(*ctl, ratio, it);
      ctl->ratio = ratio;
      ctl->iters = it;
      if (code) ctl->done = code;
      if (code == 3) ctl->nonfinite = 1;
      break;
    }
    case FIN_AM3: {
      const double e = sqrt(c0 / c1);
      am3_decide(*ctl, e);
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

// u^{n+1} = p + r^{n+1} q (eq. 4.8).  Every workgroup solves for r^{n+1} from
// the column partial sums (g_p, g_q) in the same order; workgroup 0 records it.
__global__ __launch_bounds__(256) void k_sav_combine(cd* out, const cd* q, StepCtl* ctl, size_t n,
                                                     const double* cpart, int ncol, double pars) {
  __shared__ double rs;
  double c0 = 0.0, c1 = 0.0;
  fixed_sum2<256, 4096 / 2 + 1, 32>(cpart, ncol, c0, c1);
  if (threadIdx.x == 0) {
    const double r = sav_r_solve(*ctl, pars * c0, pars * c1);
    rs = r;
    if (blockIdx.x == 0) {
      ctl->r_np1 = r;
      if (!isfinite(r)) ctl->nonfinite = 1;
    }
  }
  __syncthreads();
  const double r = rs;
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
// the run has ended: every stage of a PSD member stands still from now on
__device__ __forceinline__ void ens_finish(EnsMember* m) {
  m->ctl.done = 1;
  m->psd_init_skip = 1;
  m->psd_eval_skip = 1;
  m->sctl.done = 4;
}

// The controller's decisions, on the workgroup's copy of the member block m
// (thread 0): from the AM3 sums c0, c1 and the trial's largest u.
__device__ void ens_decide(EnsMember* m, double c0, double c1, double um) {
  StepCtl& ctl = m->ctl;
  if (m->psd) {
    // the solve stopped: converged (1), at max_iter (2) or non-finite (3)
    m->psd_iters += m->sctl.iters;
    m->psd_last_iters = m->sctl.iters;
    if (m->sctl.done == 2) m->psd_noconv = 1;
    if (m->sctl.done == 3 || m->sctl.nonfinite) ctl.nonfinite = 1;
    if (m->sctl.done != 1) {
      ens_finish(m);
      return;
    }
  }
  const double kt = ctl.k_np1;
  const double e = sqrt(c0 / c1);
  const int accept = am3_decide(ctl, e);
  const double kn = ctl.k_next;
  if (!isfinite(e) || ctl.invalid) {  // invalid: SAV's E_1 + D_0 <= 0
    if (!ctl.invalid) ctl.nonfinite = 1;
    ens_finish(m);
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
    if (m->t >= m->umax_t0) m->umax = fmax(m->umax, um);
    if (m->sav) m->rslot = (m->rslot + 1) % 3;  // r^{n+1} becomes r^n
    ctl.k_n = kt;
  } else {
    m->rejected += 1;
  }
  if (m->t >= m->t_end * (1.0 - 1e-14) || m->accepted >= m->max_accepted) {
    ens_finish(m);
    return;
  }
  double k1 = kn;
  if (k1 > m->t_end - m->t) k1 = m->t_end - m->t;
  const double k0 = ctl.k_n;
  set_bdf2(ctl, k1, k0);
  set_am3(ctl, k1, k0);
  if (m->psd && !psd_arm(m)) {  // no lambda for this q
    ctl.invalid = 1;
    ens_finish(m);
  }
}

// The member block is copied into LDS with one round of coalesced loads, the
// decisions run on that copy (each field read then costs LDS latency, not a
// dependent global load), and the block is written back whole: no other
// launch touches the member while its controller runs (a member's stages run
// in order on its class's stream).
__global__ __launch_bounds__(256) void k_ens_control(EnsMember* mem, int first) {
  __shared__ double red[2 * 4];
  constexpr int NWORD = sizeof(EnsMember) / 8;
  static_assert(sizeof(EnsMember) % 8 == 0 && alignof(EnsMember) >= 8, "8-byte words");
  __shared__ unsigned long long words[NWORD];
  EnsMember* gm = mem + first + blockIdx.x;
  unsigned long long* gw = reinterpret_cast<unsigned long long*>(gm);
  for (int i = threadIdx.x; i < NWORD; i += 256) words[i] = gw[i];
  __syncthreads();
  EnsMember* m = reinterpret_cast<EnsMember*>(words);
  if (m->ctl.done) return;
  if (m->psd && m->psd_eval_skip) return;  // the PSD solve of the attempt still runs
  // the AM3 sums: both columns of the partials in one pass, each in the
  // order of the single-column sum (per thread i = tid, tid + 256, ...,
  // then the fixed block reduction)
  double acc[2] = {0.0, 0.0};
  const double* cp = m->cpart;
  for (int i = threadIdx.x; i < m->H; i += 256) {
    acc[0] += cp[2 * (size_t)i];
    acc[1] += cp[2 * (size_t)i + 1];
  }
  __shared__ double sums[2];
  block_reduce<256, 2>(acc, red, sums);
  // largest u of the trial state: one value per workgroup of the trial
  // evaluation's row pass (the other slots hold -inf); the slots are reset
  double um = -INFINITY;
  for (int i = threadIdx.x; i < m->c.N; i += 256) {
    um = fmax(um, m->umaxpart[i]);
    m->umaxpart[i] = -INFINITY;
  }
  __shared__ double umx[256];
  umx[threadIdx.x] = um;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) umx[threadIdx.x] = fmax(umx[threadIdx.x], umx[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) ens_decide(m, sums[0], sums[1], umx[0]);
  __syncthreads();
  for (int i = threadIdx.x; i < NWORD; i += 256) gw[i] = words[i];
}

hipError_t launch_ens_control(EnsMember* m, int first, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_control, dim3(count), dim3(256), 0, s, m, first);
  return hipGetLastError();
}

// Control block of one step whose step sizes (and SAV scalars) live in device
// memory: v carries the constant fields (tolerances, step-control options,
// iteration limits, a fixed lambda); k_dev = (k_{n+1}, k_n) and r_dev =
// (r^n, r^{n-1}) are read when the step runs.  An unusable k (or an
// untabulated q when lambda comes from Table SearchSize) marks the block
// invalid; the PSD kernels then do nothing.
__global__ void k_ctl_dev(StepCtl* ctl, StepCtl v, const double* k_dev, const double* r_dev,
                          double q, int flags) {
  // CTL_K1_ONLY: a one-step method reads only k_dev[0]
  const double k1 = k_dev[0], k0 = (flags & CTL_K1_ONLY) ? 0.0 : k_dev[1];
  set_bdf2(v, k1, k0);
  if (flags & CTL_AM3) set_am3(v, k1, k0);
  if (flags & CTL_SAV) {
    v.r_n = r_dev[0];
    v.r_nm1 = (k0 > 0.0) ? r_dev[1] : 0.0;
  }
  if (flags & CTL_LAMBDA) v.lambda = lambda_table(q, k1);
  bool bad = !(k1 > 0.0) || !isfinite(k1) || !isfinite(k0);
  if (flags & CTL_AM3) bad = bad || !(k0 > 0.0);
  if (flags & CTL_LAMBDA) bad = bad || !(v.lambda > 0.0);
  if (flags & CTL_SAV) bad = bad || !isfinite(v.r_n) || !isfinite(v.r_nm1);
  if (bad) {
    v.invalid = 1;
    v.done = 4;
  }
  *ctl = v;
}

// Scalar results and status of the last step, written to caller memory:
// SAV r^{n+1}; PSD iterations; adaptivity (accept, k_next, err); the
// finalized energy of a chemical-potential evaluation.  status:
// 0 ok, -1 invalid scalars, -3 the one-launch PSD solve gave up at a grid
// barrier, -5 PSD not converged, -6 non-finite values.
__global__ void k_ctl_out(const StepCtl* ctl, int what, double* d_out, int* i_out, int* status) {
  const StepCtl& c = *ctl;
  int st = 0;
  if (c.invalid)
    st = -1;
  else if (c.nonfinite || (what == OUT_PSD && c.done == 3))
    st = -6;
  else if (what == OUT_PSD && c.done == 2)
    st = -5;
  else if (what == OUT_PSD && c.done == 5)
    st = -3;  // the one-launch solve's grid barrier gave up
  if (what == OUT_SAV && d_out) d_out[0] = c.r_np1;
  if (what == OUT_ENERGY && d_out) d_out[0] = c.energy;
  if (what == OUT_PSD && i_out) i_out[0] = c.iters;
  if (what == OUT_ADAPT && d_out) {
    d_out[0] = c.accept ? 1.0 : 0.0;
    d_out[1] = c.k_next;
    d_out[2] = c.err;
  }
  if (status) *status = st;
}

hipError_t launch_ctl_dev(StepCtl* ctl, const StepCtl& v, const double* k_dev,
                          const double* r_dev, double q, int flags, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_dev, dim3(1), dim3(1), 0, s, ctl, v, k_dev, r_dev, q, flags);
  return hipGetLastError();
}
hipError_t launch_ctl_out(const StepCtl* ctl, int what, double* d_out, int* i_out, int* status,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_out, dim3(1), dim3(1), 0, s, ctl, what, d_out, i_out, status);
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
hipError_t launch_sav_combine(cd* out, const cd* q, StepCtl* ctl, size_t n, const double* cpart,
                              int ncol, double pars, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 512) blocks = 512;  // each workgroup also reads the 2 ncol partial sums
  hipLaunchKernelGGL(k_sav_combine, dim3((unsigned)blocks), dim3(256), 0, s, out, q, ctl, n, cpart,
                     ncol, pars);
  return hipGetLastError();
}

}  // namespace fch
