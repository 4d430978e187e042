// fch_capi.hip -- host side of the C ABI declared in include/fch.h: plan and
// workspace management, argument validation, and the launch sequences of
// each call (which kernels run, in which order, on which buffers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "fch.h"
#include "fch_coef.hpp"
#include "fch_kernels.hpp"
#include "fch_plan.hpp"

using fch::cd;
using fch::ColArgs;
using fch::FinArgs;
using fch::RowArgs;
using fch::StepCtl;

namespace {

#define HIPCHK(x)                                 \
  do {                                            \
    if ((x) != hipSuccess) return FCH_E_HIP;      \
  } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// host evaluation of W_q and its derivatives (eq. e:Wq-def), used for the
// plan constants alpha_m and the default SAV constants
void well_host(const fch_params& p, double u, double* W, double* W1, double* W2) {
  const double dm = u - p.b_minus, dp = u - p.b_plus;
  double A = 0.5 * dm * dm, A1 = dm, A2 = 1.0;
  if (p.q != 0.0) {
    const double z = dm / p.eps;
    const double e = std::exp(-std::fabs(z));
    const double den = 1.0 / (1.0 + e * e);
    const double sech = 2.0 * e * den;
    const double th = std::copysign((1.0 - e * e) * den, z);
    A += p.q * p.eps * (1.0 - sech);
    A1 += p.q * sech * th;
    A2 += (p.q / p.eps) * sech * (sech * sech - th * th);
  }
  const double g3 = p.gamma_w / 3.0;
  const double B = 0.5 * dp * dp + g3 * (u - 0.5 * (3.0 * p.b_plus - p.b_minus));
  const double B1 = dp + g3;
  if (W) *W = A * B;
  if (W1) *W1 = A1 * B + A * B1;
  if (W2) *W2 = A2 * B + 2.0 * A1 * B1 + A;
}

double eff_eta(const fch_params& p, double eta) { return eta * std::pow(p.eps, p.p); }

fch_status validate_params(const fch_params* p) {
  if (!p) return FCH_E_INVALID;
  if (!finite_pos(p->L) || !finite_pos(p->eps)) return FCH_E_INVALID;
  if (!std::isfinite(p->eta1) || !std::isfinite(p->eta2) || !std::isfinite(p->q) || p->q < 0.0)
    return FCH_E_INVALID;
  if (!std::isfinite(p->gamma_w) || !std::isfinite(p->b_minus) || !std::isfinite(p->b_plus))
    return FCH_E_INVALID;
  if (!std::isfinite(p->beta1) || !std::isfinite(p->beta2) || !std::isfinite(p->zeta) ||
      !std::isfinite(p->D0))
    return FCH_E_INVALID;
  if (!is_pow2(p->N) || p->N < 16) return p->N > 0 && p->N < 16 ? FCH_E_UNSUPPORTED : FCH_E_INVALID;
  if (fch::row_variant_count(p->N) == 0 || fch::col_variant_count(p->N) == 0)
    return FCH_E_UNSUPPORTED;
  return FCH_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t spec_bytes(int N) { return (size_t)(N / 2 + 1) * (size_t)N * sizeof(cd); }

size_t workspace_layout(int N, fch_plan_s* p) {
  const size_t S = align256(spec_bytes(N));
  const size_t R = align256(sizeof(double) * 2 * (size_t)N);
  const size_t C = align256(sizeof(double) * 2 * (size_t)(N / 2 + 1));
  if (p) {
    char* b = p->ws;
    p->P0 = (cd*)b; b += S;
    p->P1 = (cd*)b; b += S;
    p->aux = (cd*)b; b += S;
    p->st = (cd*)b; b += S;
    for (int i = 0; i < 3; ++i) { p->Fc[i] = (cd*)b; b += S; }
    p->rpart = (double*)b; b += R;
    p->cpart = (double*)b; b += C;
  }
  return 7 * S + R + C;
}

StepCtl ctl_zero() {
  StepCtl v;
  std::memset(&v, 0, sizeof(v));
  return v;
}

using fch::set_bdf2;
using fch::set_am3;
using fch::lambda_table;

RowArgs row_args(fch_plan_s* p) {
  RowArgs a;
  std::memset(&a, 0, sizeof(a));
  a.c = p->c;
  a.P0 = p->P0;
  a.P1 = p->P1;
  a.ctl = p->ctl;
  a.tw = p->tw;
  a.check_done = p->check_done;
  return a;
}

ColArgs col_args(fch_plan_s* p) {
  ColArgs a;
  std::memset(&a, 0, sizeof(a));
  a.c = p->c;
  a.P0 = p->P0;
  a.P1 = p->P1;
  a.ctl = p->ctl;
  a.tw = p->tw;
  a.check_done = p->check_done;
  return a;
}

// the launches made while it lives read the control block's done code
struct CheckDone {
  fch_plan_s* p;
  int keep;
  explicit CheckDone(fch_plan_s* q) : p(q), keep(q->check_done) { p->check_done = 1; }
  ~CheckDone() { p->check_done = keep; }
};

fch_status need_ws(fch_plan_s* p) { return p->ws ? FCH_OK : FCH_E_NOMEM; }

// kernel timing (mode 2, below): the stream gets work that is not a timed launch
void prof_break(fch_plan_s* p) { p->prof_last = -1; }

fch_status ctl_set(fch_plan_s* p, const StepCtl& v) {
  prof_break(p);
  HIPCHK(fch::launch_ctl_set(p->ctl, v, p->stream));
  p->stats.launches += 1;
  return FCH_OK;
}

fch_status readback(fch_plan_s* p) {
  prof_break(p);
  HIPCHK(hipMemcpyAsync(p->hctl, p->ctl, sizeof(StepCtl), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return FCH_OK;
}

constexpr int kProfCap = 16384;

// kernel timing: an event pair recorded on the plan's stream around the
// next launch when timing is on
// Kernel timing of the row and column passes.  prof_on = 1: event records
// bracket each launch on the stream.  prof_on = 2: nothing enters the stream;
// each launch folds its earliest workgroup start (device wall clock) into its
// own slot of prof_ts, and its time is the interval to the next launch's
// start, counted only when that next launch follows it directly on the stream
// (prof_break marks any other work: small kernels, copies, host waits, a new
// call).  In a back-to-back chain that interval is the kernel's share of the
// chain, start to start.
int prof_begin(fch_plan_s* p, int kind) {
  if (!p->prof_on || p->prof_n >= kProfCap) return -1;
  const int i = p->prof_n++;
  p->prof_kind[i] = kind;
  p->prof_prev[i] = p->prof_last;
  p->prof_last = i;
  if (p->prof_on == 1) (void)hipEventRecord(p->prof_ev[2 * i], p->stream);
  return i;
}
void prof_end(fch_plan_s* p, int i) {
  if (i >= 0 && p->prof_on == 1) (void)hipEventRecord(p->prof_ev[2 * i + 1], p->stream);
}
unsigned long long* prof_slot(fch_plan_s* p, int i) {
  return (i >= 0 && p->prof_on == 2) ? p->prof_ts + i : nullptr;
}

fch_status col(fch_plan_s* p, int epi, int pro, const ColArgs& a) {
  const int kind = (epi != fch::EPI_NONE && pro != fch::PRO_NONE) ? 1 : 2;
  const int r = prof_begin(p, kind);
  ColArgs b = a;
  b.tstart = prof_slot(p, r);
  HIPCHK(p->cv->col(epi, pro, b, p->stream, nullptr, nullptr, &p->lane));
  prof_end(p, r);
  p->stats.launches += 1;
  return FCH_OK;
}

fch_status row_mu(fch_plan_s* p, double* partial, cd* pair0 = nullptr, cd* pair1 = nullptr) {
  RowArgs a = row_args(p);
  a.partial = partial;
  if (pair0) {
    a.P0 = pair0;
    a.P1 = pair1;
  }
  const int r = prof_begin(p, 0);
  a.tstart = prof_slot(p, r);
  HIPCHK(p->rv->row(fch::ROW_MU, a, p->stream, nullptr, nullptr));
  prof_end(p, r);
  p->stats.launches += 1;
  return FCH_OK;
}

// n PSD iterations (Sec. 3.3) after `done_before` iterations of the solve:
// each is a row pass (chemical-potential pieces of the iterate) and a column
// pass (step, partial sums, next iterate's inverse transform).  From the
// second iteration on, the row pass first evaluates the previous iteration's
// stopping test; the last one is evaluated by one finalize launch.  Once the
// test has stopped the solve, the remaining launches return at once.
fch_status psd_iterations(fch_plan_s* p, const ColArgs& a, int done_before, int n);

fch_status finalize(fch_plan_s* p, int mode, bool rows, bool cols) {
  FinArgs f;
  std::memset(&f, 0, sizeof(f));
  f.c = p->c;
  f.rpart = rows ? p->rpart : nullptr;
  f.nrow = p->N / p->rv->R;
  f.cpart = cols ? p->cpart : nullptr;
  f.ncol = p->H;
  f.ctl = p->ctl;
  f.mode = mode;
  prof_break(p);
  HIPCHK(fch::launch_finalize(f, p->stream));
  p->stats.launches += 1;
  return FCH_OK;
}

#define CHK(x)                         \
  do {                                 \
    fch_status s_ = (x);               \
    if (s_ != FCH_OK) return s_;       \
  } while (0)

fch_status psd_iterations(fch_plan_s* p, const ColArgs& a, int done_before, int n) {
  for (int i = 0; i < n; ++i) {
    RowArgs r = row_args(p);
    r.check_done = 1;  // a stopped solve's remaining launches return at once
    if (i > 0) {
      r.psd_part = p->cpart;
      r.psd_ncol = p->H;
      r.psd_iter = done_before + i;
    }
    const int pr = prof_begin(p, 0);
    r.tstart = prof_slot(p, pr);
    HIPCHK(p->rv->row(fch::ROW_MU, r, p->stream, nullptr, nullptr));
    prof_end(p, pr);
    p->stats.launches += 1;
    CHK(col(p, fch::EPI_PSD, fch::PRO_NEXT_FIELD, a));
  }
  if (n > 0) CHK(finalize(p, fch::FIN_PSD, false, true));
  return FCH_OK;
}


// one BDF2-IMEX step: inverse column pass of (u*, Lap u*), row pass, forward
// column pass with the IMEX epilogue.  pair0/pair1 (nullable) replace the
// workspace's pair buffer.
fch_status imex_attempt(fch_plan_s* p, const cd* un, const cd* um, double k_np1, double k_n,
                        cd* out, cd* pair0 = nullptr, cd* pair1 = nullptr) {
  StepCtl v = ctl_zero();
  set_bdf2(v, k_np1, k_n);
  CHK(ctl_set(p, v));
  ColArgs a = col_args(p);
  if (pair0) {
    a.P0 = pair0;
    a.P1 = pair1;
  }
  a.s0 = un;
  a.s1 = um ? um : un;
  CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
  CHK(row_mu(p, nullptr, pair0, pair1));
  a.out = out;
  CHK(col(p, fch::EPI_IMEX, fch::PRO_NONE, a));
  p->stats.fft_calls += 4;
  p->stats.steps += 1;
  return FCH_OK;
}

fch_status status_from_ctl(fch_plan_s* p) {
  if (p->hctl->nonfinite) return FCH_E_NONFINITE;
  if (p->hctl->invalid) return FCH_E_INVALID;
  return FCH_OK;
}

}  // namespace

namespace fch {
Consts consts_from_params(const fch_params& prm) {
  Consts c;
  c.N = prm.N;
  c.L = prm.L;
  c.eps = prm.eps;
  c.inv_eps = 1.0 / prm.eps;
  c.eps2 = prm.eps * prm.eps;
  c.eta1 = eff_eta(prm, prm.eta1);
  c.eta2 = eff_eta(prm, prm.eta2);
  c.q = prm.q;
  c.gw3 = prm.gamma_w / 3.0;
  c.bm = prm.b_minus;
  c.bp = prm.b_plus;
  c.bshift = 0.5 * (3.0 * prm.b_plus - prm.b_minus);
  c.alpha = fch_alpha_m(&prm);
  c.beta1 = prm.beta1;
  c.beta2 = prm.beta2;
  c.zeta = prm.zeta;
  c.D0 = prm.D0;
  const double tk = 2.0 * M_PI / prm.L;
  c.kscale = tk * tk;
  c.invN2 = 1.0 / ((double)prm.N * (double)prm.N);
  const double h = prm.L / prm.N;
  c.h2 = h * h;
  c.pars = prm.L * prm.L / ((double)prm.N * prm.N * (double)prm.N * prm.N);
  return c;
}

fch_status validate_params_internal(const fch_params* p) { return validate_params(p); }
}  // namespace fch

static fch_status copy_spec(fch_plan_t p, cd* dst, const cd* src);

// ---- scratch of the no-allocation IMEX step ----------------------------------
// fch_step_imex_static keeps its pair buffer (the two half spectra that the
// row and column passes hand to each other) in this file-scope device array
// instead of the caller's workspace.  Each GPU holds its own copy for the
// life of the process.  In host code `scratch` names a host-side stand-in, not
// a device address: the device address is taken once per device with
// hipGetSymbolAddress (scratch_resolve) and only that pointer is ever handed
// to kernels.
namespace {
constexpr int kStaticMaxN = FCH_STATIC_MAX_N;
constexpr size_t kStaticSpec = (size_t)(kStaticMaxN / 2 + 1) * kStaticMaxN * sizeof(cd);
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) char scratch[2 * kStaticSpec];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// device address of `scratch` on device dev, resolved on first use with that
// device current (the caller's current device is restored)
fch_status scratch_resolve(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return FCH_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return FCH_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return FCH_OK;
}
}  // namespace

// ===========================================================================
extern "C" {

const char* fch_status_string(fch_status s) {
  switch (s) {
    case FCH_OK: return "ok";
    case FCH_E_INVALID: return "invalid argument";
    case FCH_E_UNSUPPORTED: return "unsupported grid size or configuration";
    case FCH_E_HIP: return "HIP runtime error";
    case FCH_E_NOMEM: return "workspace missing or too small";
    case FCH_E_NOCONV: return "PSD did not converge within max_iter";
    case FCH_E_NONFINITE: return "non-finite value in the state";
  }
  return "unknown status";
}

double fch_alpha_m(const fch_params* prm) {
  if (!prm) return NAN;
  double w2 = 0.0;
  well_host(*prm, prm->b_minus, nullptr, nullptr, &w2);
  return w2;
}

fch_status fch_sav_constants(const fch_params* prm, double* zeta, double* D0) {
  if (!prm || !zeta || !D0 || !finite_pos(prm->L) || !finite_pos(prm->eps)) return FCH_E_INVALID;
  const double eta2 = eff_eta(*prm, prm->eta2);
  double min_w2 = INFINITY, min_g = INFINITY;
  const int n = 60001;
  for (int i = 0; i < n; ++i) {
    const double u = -3.0 + 6.0 * i / (n - 1);
    double W, W1, W2;
    well_host(*prm, u, &W, &W1, &W2);
    min_w2 = std::fmin(min_w2, W2);
    min_g = std::fmin(min_g, 0.5 * W1 * W1 - eta2 * W);
  }
  *zeta = std::ceil(10.0 * std::fmax(0.0, -min_w2)) / 10.0;
  *D0 = prm->L * prm->L * (std::fmax(0.0, -min_g) + 1.0);
  return FCH_OK;
}

// The one-launch PSD solve needs all of its workgroups resident at once: at
// most what the occupancy of the kernel allows on this device's CUs, by
// default one workgroup per CU (or fewer when a phase has fewer tasks: each
// grid barrier costs one agent-scope release and acquire per workgroup, so
// fewer, busier workgroups are faster).  It starts switched off; without a
// compiled pair for N it cannot be switched on.
static void psd1_setup(fch_plan_s* p) {
  p->psd1 = nullptr;
  p->psd1_grid = 0;
  p->psd1_on = 0;
  const fch::PsdSolveVT* vt = fch::psd_solve_variant(p->N);
  if (!vt) return;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, vt->func, vt->threads, 0) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess ||
      per_cu < 1 || cus < 1) {
    (void)hipGetLastError();
    return;
  }
  const int tasks = std::max(p->N / vt->R, p->N / 2);
  p->psd1 = vt;
  p->psd1_max_grid = per_cu * cus;
  p->psd1_def_grid = std::min(cus, tasks);
  p->psd1_grid = p->psd1_def_grid;
  p->psd1_on = 0;
}

// the iterations of a PSD solve after its PRO_PSD_INIT column pass: one
// k_psd_solve launch (the plan's one-launch pair) or, when that is off or not
// compiled for N, `limit` row and column passes and the final test
static fch_status psd_solve_launch(fch_plan_s* p, const ColArgs& a, int limit) {
  if (!(p->psd1 && p->psd1_on)) {
    CHK(psd_iterations(p, a, 0, limit));
    return FCH_OK;
  }
  RowArgs ra = row_args(p);
  ra.check_done = 0;
  ColArgs ca = a;
  ca.check_done = 0;
  ca.partial = p->cpart;
  prof_break(p);
  HIPCHK(p->psd1->launch(ra, ca, limit, p->psd1_grid, p->stream));
  p->stats.launches += 1;
  return FCH_OK;
}

fch_status fch_plan_create(const fch_params* prm, fch_plan_t* out) {
  if (!out) return FCH_E_INVALID;
  CHK(validate_params(prm));
  fch_plan_s* p = new (std::nothrow) fch_plan_s;
  if (!p) return FCH_E_NOMEM;
  std::memset(p, 0, sizeof(*p));
  p->prm = *prm;
  p->N = prm->N;
  p->H = prm->N / 2 + 1;
  p->rv = fch::row_variant(prm->N, 0);
  p->cv = fch::col_variant(prm->N, 0);
  p->psd_hint = 4;
  p->c = fch::consts_from_params(*prm);

  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return FCH_E_HIP; }
  // twiddles exp(-2 pi i m / N), evaluated in extended precision
  const int N = prm->N;
  cd* htw = new (std::nothrow) cd[N];
  if (!htw) { delete p; return FCH_E_NOMEM; }
  for (int m = 0; m < N; ++m) {
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / N;
    htw[m].x = (double)cosl(ang);
    htw[m].y = (double)-sinl(ang);
  }
  bool ok = hipMalloc((void**)&p->tw, sizeof(cd) * N) == hipSuccess &&
            hipMalloc((void**)&p->ctl, sizeof(StepCtl)) == hipSuccess &&
            hipHostMalloc((void**)&p->hctl, sizeof(StepCtl), hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&p->dmem, sizeof(fch::EnsMember)) == hipSuccess &&
            hipHostMalloc((void**)&p->hmem, sizeof(fch::EnsMember), hipHostMallocDefault) ==
                hipSuccess &&
            hipMemcpy(p->tw, htw, sizeof(cd) * N, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemset(p->ctl, 0, sizeof(StepCtl)) == hipSuccess;
  delete[] htw;
  if (!ok) {
    fch_plan_destroy(p);
    return FCH_E_HIP;
  }
  std::memset(p->hctl, 0, sizeof(StepCtl));
  char* sp = nullptr;
  if (scratch_resolve(p->device, &sp) != FCH_OK) {
    fch_plan_destroy(p);
    return FCH_E_HIP;
  }
  if (p->N >= 4096 &&
      (hipStreamCreateWithFlags(&p->lane.stream, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&p->lane.fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&p->lane.join, hipEventDisableTiming) != hipSuccess)) {
    fch_plan_destroy(p);
    return FCH_E_HIP;
  }
  psd1_setup(p);
  *out = p;
  return FCH_OK;
}

fch_status fch_plan_profile(fch_plan_t p, int32_t enable) {
  if (!p) return FCH_E_INVALID;
  if (enable && !p->prof_ev) {
    p->prof_ev = new (std::nothrow) hipEvent_t[2 * kProfCap];
    p->prof_kind = new (std::nothrow) int[kProfCap];
    p->prof_prev = new (std::nothrow) int[kProfCap];
    if (!p->prof_ev || !p->prof_kind || !p->prof_prev) return FCH_E_NOMEM;
    for (int i = 0; i < 2 * kProfCap; ++i) HIPCHK(hipEventCreate(&p->prof_ev[i]));
  }
  if (enable == 2 && !p->prof_ts) {
    HIPCHK(hipMalloc((void**)&p->prof_ts, sizeof(unsigned long long) * kProfCap));
    HIPCHK(hipMemsetAsync(p->prof_ts, 0xff, sizeof(unsigned long long) * kProfCap, p->stream));
  }
  p->prof_on = (enable == 2) ? 2 : (enable ? 1 : 0);
  p->prof_last = -1;
  return FCH_OK;
}

fch_status fch_plan_profile_read(fch_plan_t p, fch_profile* out) {
  if (!p || !out) return FCH_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (p->prof_on == 2) {
    const int n = p->prof_n;
    unsigned long long* ts = new (std::nothrow) unsigned long long[n > 0 ? n : 1];
    if (!ts) return FCH_E_NOMEM;
    int khz = 0;
    if (hipMemcpy(ts, p->prof_ts, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) != hipSuccess ||
        khz <= 0) {
      delete[] ts;
      return FCH_E_HIP;
    }
    for (int i = 0; i + 1 < n; ++i) {
      if (p->prof_prev[i + 1] != i || ts[i + 1] < ts[i] || ts[i + 1] == ~0ULL) continue;
      out->count[p->prof_kind[i]] += 1;
      out->ms[p->prof_kind[i]] += (double)(ts[i + 1] - ts[i]) / (double)khz;
    }
    delete[] ts;
    HIPCHK(hipMemsetAsync(p->prof_ts, 0xff, sizeof(unsigned long long) * kProfCap, p->stream));
  } else {
    for (int i = 0; i < p->prof_n; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]));
      out->count[p->prof_kind[i]] += 1;
      out->ms[p->prof_kind[i]] += ms;
    }
  }
  p->prof_n = 0;
  p->prof_last = -1;
  return FCH_OK;
}

namespace {
void drop_chain(fch_plan_s* p) {
  if (p->chain_exec) (void)hipGraphExecDestroy(p->chain_exec);
  p->chain_exec = nullptr;
  std::memset(p->chain_key, 0, sizeof(p->chain_key));
}
}  // namespace

fch_status fch_plan_set_graph(fch_plan_t p, int32_t steps) {
  if (!p || steps < 0 || steps > 256 || (steps & 1)) return FCH_E_INVALID;
  if (steps > 0 && !p->gstream) {
    if (hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) != hipSuccess) {
      p->gstream = nullptr;
      return FCH_E_HIP;
    }
    if (hipEventCreateWithFlags(&p->gfork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->gjoin, hipEventDisableTiming) != hipSuccess)
      return FCH_E_HIP;
  }
  if (steps != p->graph_steps) drop_chain(p);
  p->graph_steps = steps;
  return FCH_OK;
}

fch_status fch_plan_destroy(fch_plan_t p) {
  if (!p) return FCH_E_INVALID;
  drop_chain(p);
  if (p->gstream) {
    (void)hipStreamSynchronize(p->gstream);
    (void)hipStreamDestroy(p->gstream);
  }
  if (p->gfork) (void)hipEventDestroy(p->gfork);
  if (p->gjoin) (void)hipEventDestroy(p->gjoin);
  if (p->lane.stream) {
    (void)hipStreamSynchronize(p->lane.stream);
    (void)hipStreamDestroy(p->lane.stream);
  }
  if (p->lane.fork) (void)hipEventDestroy(p->lane.fork);
  if (p->lane.join) (void)hipEventDestroy(p->lane.join);
  if (p->prof_ev) {
    for (int i = 0; i < 2 * kProfCap; ++i) (void)hipEventDestroy(p->prof_ev[i]);
    delete[] p->prof_ev;
    delete[] p->prof_kind;
    delete[] p->prof_prev;
  }
  if (p->prof_ts) {
    (void)hipFree(p->prof_ts);
  }
  if (p->tw) (void)hipFree(p->tw);
  if (p->ctl) (void)hipFree(p->ctl);
  if (p->hctl) (void)hipHostFree(p->hctl);
  if (p->dmem) (void)hipFree(p->dmem);
  if (p->hmem) (void)hipHostFree(p->hmem);
  delete p;
  return FCH_OK;
}

fch_status fch_plan_set_stream(fch_plan_t p, void* stream) {
  if (!p) return FCH_E_INVALID;
  p->stream = (hipStream_t)stream;
  return FCH_OK;
}

size_t fch_plan_workspace_bytes(fch_plan_t p) {
  if (!p) return 0;
  return workspace_layout(p->N, nullptr);
}

fch_status fch_plan_set_workspace(fch_plan_t p, void* dptr, size_t bytes) {
  if (!p || !dptr) return FCH_E_INVALID;
  if (((uintptr_t)dptr & 255) != 0) return FCH_E_INVALID;
  if (bytes < workspace_layout(p->N, nullptr)) return FCH_E_NOMEM;
  p->ws = (char*)dptr;
  p->ws_bytes = bytes;
  workspace_layout(p->N, p);
  return FCH_OK;
}

int32_t fch_row_config_count(int32_t N) { return fch::row_variant_count(N); }
int32_t fch_col_config_count(int32_t N) { return fch::col_variant_count(N); }

static void fill_cfg(const fch::RowVT* r, const fch::ColVT* c, fch_launch_cfg* cfg) {
  cfg->row_R = r->R;
  cfg->row_E = r->E;
  cfg->row_twl = r->twl;
  cfg->col_E = c->E;
  cfg->col_twl = c->twl;
}

fch_status fch_config_get(int32_t N, int32_t ri, int32_t ci, fch_launch_cfg* cfg) {
  const fch::RowVT* r = fch::row_variant(N, ri);
  const fch::ColVT* c = fch::col_variant(N, ci);
  if (!r || !c || !cfg) return FCH_E_UNSUPPORTED;
  fill_cfg(r, c, cfg);
  return FCH_OK;
}

fch_status fch_plan_set_config(fch_plan_t p, const fch_launch_cfg* cfg) {
  if (!p) return FCH_E_INVALID;
  if (!cfg) {
    p->rv = fch::row_variant(p->N, 0);
    p->cv = fch::col_variant(p->N, 0);
    return FCH_OK;
  }
  const fch::RowVT* r = nullptr;
  const fch::ColVT* c = nullptr;
  for (int i = 0; i < fch::row_variant_count(p->N); ++i) {
    const fch::RowVT* v = fch::row_variant(p->N, i);
    if (v->R == cfg->row_R && v->E == cfg->row_E && v->twl == cfg->row_twl) r = v;
  }
  for (int i = 0; i < fch::col_variant_count(p->N); ++i) {
    const fch::ColVT* v = fch::col_variant(p->N, i);
    if (v->E == cfg->col_E && v->twl == cfg->col_twl) c = v;
  }
  if (!r || !c) return FCH_E_UNSUPPORTED;
  p->rv = r;
  p->cv = c;
  return FCH_OK;
}

fch_status fch_plan_set_psd_solve(fch_plan_t p, int32_t on, int32_t grid) {
  if (!p || (on != 0 && on != 1)) return FCH_E_INVALID;
  if (on && !p->psd1) return FCH_E_UNSUPPORTED;
  if (on && grid > 0) {
    if (grid > p->psd1_max_grid) return FCH_E_INVALID;
    p->psd1_grid = grid;
  } else if (on) {
    p->psd1_grid = p->psd1_def_grid;
  }
  p->psd1_on = on;
  return FCH_OK;
}

fch_status fch_plan_get_psd_solve(fch_plan_t p, int32_t* on, int32_t* grid) {
  if (!p || !on) return FCH_E_INVALID;
  *on = p->psd1 ? p->psd1_on : 0;
  if (grid) *grid = p->psd1 ? p->psd1_grid : 0;
  return FCH_OK;
}

fch_status fch_plan_get_config(fch_plan_t p, fch_launch_cfg* cfg) {
  if (!p || !cfg) return FCH_E_INVALID;
  fill_cfg(p->rv, p->cv, cfg);
  return FCH_OK;
}

fch_status fch_autotune(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1, double k,
                        int32_t reps, fch_launch_cfg* best, double* us) {
  if (!p || !uh_n || !uh_nm1 || !finite_pos(k) || reps < 1) return FCH_E_INVALID;
  CHK(need_ws(p));
  const int nr = fch::row_variant_count(p->N), nc = fch::col_variant_count(p->N);
  const int npair = nr * nc;
  // per pair: the best chain time per step over the sweeps, and the row and
  // column shares of that chain (device clock, launch start to launch start)
  double* tbest = new (std::nothrow) double[3 * npair];
  if (!tbest) return FCH_E_NOMEM;
  double* rbest = tbest + npair;
  double* cbest = rbest + npair;
  for (int i = 0; i < npair; ++i) tbest[i] = rbest[i] = cbest[i] = 1e30;
  // steps per timed chain; the launch starts land in the row partial-sum
  // area of the workspace (2N doubles: one slot per launch)
  const int K = std::max(2, std::min(reps, p->N - 1));
  const int nslot = 2 * K + 1;
  unsigned long long* slots = (unsigned long long*)p->rpart;
  unsigned long long* hs = new (std::nothrow) unsigned long long[nslot];
  if (!hs) { delete[] tbest; return FCH_E_NOMEM; }
  int khz = 0;
  hipEvent_t ev[2];
  for (int i = 0; i < 2; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) { delete[] tbest; delete[] hs; return FCH_E_HIP; }
  const fch::RowVT* keep_r = p->rv;
  const fch::ColVT* keep_c = p->cv;
  const int keep_prof = p->prof_on;
  p->prof_on = 0;
  fch_status st = FCH_OK;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) != hipSuccess ||
      khz <= 0)
    st = FCH_E_HIP;
  // scratch copies of the state: the fused chain runs on Fc[0..1]
  cd *cur = p->Fc[0], *prev = p->Fc[1];
  if (st == FCH_OK && (copy_spec(p, cur, (const cd*)uh_n) != FCH_OK ||
                       copy_spec(p, prev, (const cd*)uh_nm1) != FCH_OK))
    st = FCH_E_HIP;
  StepCtl v = ctl_zero();
  set_bdf2(v, k, k);
  if (st == FCH_OK) st = ctl_set(p, v);
  // sweep 0 warms code objects and caches; sweeps 1..3 are timed
  for (int sweep = 0; sweep < 4 && st == FCH_OK; ++sweep) {
    for (int pi = 0; pi < npair && st == FCH_OK; ++pi) {
      p->rv = fch::row_variant(p->N, pi / nc);
      p->cv = fch::col_variant(p->N, pi % nc);
      if (hipMemsetAsync(slots, 0xff, sizeof(unsigned long long) * nslot, p->stream) !=
          hipSuccess) {
        st = FCH_E_HIP;
        break;
      }
      ColArgs a = col_args(p);
      a.s0 = cur;
      a.s1 = prev;
      a.tstart = slots;
      if (p->cv->col(fch::EPI_NONE, fch::PRO_EXTRAP, a, p->stream, nullptr, nullptr, &p->lane) !=
              hipSuccess ||
          hipEventRecord(ev[0], p->stream) != hipSuccess) {
        st = FCH_E_HIP;
        break;
      }
      for (int s = 0; s < K && st == FCH_OK; ++s) {
        RowArgs r = row_args(p);
        r.tstart = slots + 1 + 2 * s;
        a.s0 = cur;
        a.s1 = prev;
        a.out = prev;
        a.tstart = slots + 2 + 2 * s;
        if (p->rv->row(fch::ROW_MU, r, p->stream, nullptr, nullptr) != hipSuccess ||
            p->cv->col(fch::EPI_IMEX, s + 1 < K ? fch::PRO_NEXT_EXTRAP : fch::PRO_NONE, a,
                       p->stream, nullptr, nullptr, &p->lane) != hipSuccess)
          st = FCH_E_HIP;
        std::swap(cur, prev);
      }
      if (st != FCH_OK || hipEventRecord(ev[1], p->stream) != hipSuccess ||
          hipMemcpyAsync(hs, slots, sizeof(unsigned long long) * nslot, hipMemcpyDeviceToHost,
                         p->stream) != hipSuccess ||
          hipStreamSynchronize(p->stream) != hipSuccess) {
        st = FCH_E_HIP;
        break;
      }
      if (sweep == 0) continue;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
      const double per_step = 1e3 * ms / K;  // microseconds
      if (per_step < tbest[pi]) {
        // row s spans slots 1+2s -> 2+2s, its column pass 2+2s -> 3+2s (the
        // last column pass has no successor and is left out)
        double rs = 0.0, cs = 0.0;
        for (int s = 0; s < K; ++s) rs += (double)(hs[2 + 2 * s] - hs[1 + 2 * s]);
        for (int s = 0; s + 1 < K; ++s) cs += (double)(hs[3 + 2 * s] - hs[2 + 2 * s]);
        tbest[pi] = per_step;
        rbest[pi] = 1e3 * rs / K / khz;
        cbest[pi] = 1e3 * cs / (K - 1) / khz;
      }
    }
  }
  for (int i = 0; i < 2; ++i) (void)hipEventDestroy(ev[i]);
  delete[] hs;
  p->prof_on = keep_prof;
  if (st != FCH_OK) {
    p->rv = keep_r;
    p->cv = keep_c;
    delete[] tbest;
    return st;
  }
  // the fastest pair; pairs within 1% of it count as ties, resolved by list
  // order (the first listed variants are the defaults), so that timing noise
  // does not change the choice between near-equal variants from run to run
  int bp = 0;
  for (int i = 1; i < npair; ++i)
    if (tbest[i] < tbest[bp]) bp = i;
  const double tmin = tbest[bp];
  for (int i = 0; i < npair; ++i)
    if (tbest[i] <= 1.01 * tmin) { bp = i; break; }
  p->rv = fch::row_variant(p->N, bp / nc);
  p->cv = fch::col_variant(p->N, bp % nc);
  if (best) fill_cfg(p->rv, p->cv, best);
  if (us) {
    us[0] = rbest[bp];
    us[1] = cbest[bp];
  }
  delete[] tbest;
  return FCH_OK;
}

fch_status fch_plan_stats(fch_plan_t p, fch_stats* out) {
  if (!p || !out) return FCH_E_INVALID;
  *out = p->stats;
  return FCH_OK;
}

fch_status fch_plan_reset_stats(fch_plan_t p) {
  if (!p) return FCH_E_INVALID;
  std::memset(&p->stats, 0, sizeof(p->stats));
  return FCH_OK;
}

// ---- transforms -----------------------------------------------------------
fch_status fch_forward(fch_plan_t p, const double* u, fch_c128* uh) {
  if (!p || !u || !uh) return FCH_E_INVALID;
  CHK(need_ws(p));
  prof_break(p);
  RowArgs r = row_args(p);
  r.u_in = u;
  r.X_out = p->P0;
  int pr = prof_begin(p, 3);
  HIPCHK(p->rv->row(fch::ROW_FWD, r, p->stream, nullptr, nullptr));
  prof_end(p, pr);
  ColArgs a = col_args(p);
  a.X_in = p->P0;
  a.X_out = (cd*)uh;
  pr = prof_begin(p, 3);
  HIPCHK(p->cv->col_fwd1(a, p->stream, nullptr, nullptr));
  prof_end(p, pr);
  p->stats.launches += 2;
  p->stats.fft_calls += 1;
  return FCH_OK;
}

fch_status fch_inverse(fch_plan_t p, const fch_c128* uh, double* u) {
  if (!p || !u || !uh) return FCH_E_INVALID;
  CHK(need_ws(p));
  prof_break(p);
  ColArgs a = col_args(p);
  a.X_in = (const cd*)uh;
  a.X_out = p->P0;
  int pr = prof_begin(p, 3);
  HIPCHK(p->cv->col_inv1(a, p->stream, nullptr, nullptr));
  prof_end(p, pr);
  RowArgs r = row_args(p);
  r.X_in = p->P0;
  r.u_out = u;
  pr = prof_begin(p, 3);
  HIPCHK(p->rv->row(fch::ROW_INV, r, p->stream, nullptr, nullptr));
  prof_end(p, pr);
  p->stats.launches += 2;
  p->stats.fft_calls += 1;
  return FCH_OK;
}

fch_status fch_forward_batch(fch_plan_t p, int32_t batch, const double* u, fch_c128* uh) {
  if (!p || !u || !uh || batch < 1 || batch > 65535) return FCH_E_INVALID;
  const size_t ps = (size_t)p->N * p->N, ss = (size_t)p->N * p->H;
  RowArgs r = row_args(p);
  r.u_in = u;
  r.X_out = (cd*)uh;
  HIPCHK(p->rv->row_batch(fch::ROW_FWD, r, batch, ps, ss, p->stream));
  ColArgs a = col_args(p);
  a.X_in = (const cd*)uh;
  a.X_out = (cd*)uh;
  HIPCHK(p->cv->col1_batch(-1, a, batch, ss, p->stream));
  p->stats.launches += 2;
  p->stats.fft_calls += batch;
  return FCH_OK;
}

size_t fch_inverse_batch_ws_bytes(fch_plan_t p, int32_t batch) {
  if (!p || batch < 1) return 0;
  return (size_t)batch * p->H * p->N * sizeof(cd);
}

fch_status fch_inverse_batch(fch_plan_t p, int32_t batch, const fch_c128* uh, double* u,
                             void* ws, size_t ws_bytes) {
  if (!p || !u || !uh || !ws || batch < 1 || batch > 65535) return FCH_E_INVALID;
  if (ws_bytes < fch_inverse_batch_ws_bytes(p, batch)) return FCH_E_INVALID;
  const size_t ps = (size_t)p->N * p->N, ss = (size_t)p->N * p->H;
  ColArgs a = col_args(p);
  a.X_in = (const cd*)uh;
  a.X_out = (cd*)ws;
  HIPCHK(p->cv->col1_batch(+1, a, batch, ss, p->stream));
  RowArgs r = row_args(p);
  r.X_in = (const cd*)ws;
  r.u_out = u;
  HIPCHK(p->rv->row_batch(fch::ROW_INV, r, batch, ps, ss, p->stream));
  p->stats.launches += 2;
  p->stats.fft_calls += batch;
  return FCH_OK;
}

// ---- chemical potential ---------------------------------------------------
fch_status fch_chem_potential(fch_plan_t p, const fch_c128* uh, fch_c128* muh, double* energy) {
  if (!p || !uh || !muh || (const void*)uh == (const void*)muh) return FCH_E_INVALID;
  CHK(need_ws(p));
  CHK(ctl_set(p, ctl_zero()));
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, p->rpart));
  a.out = (cd*)muh;
  a.partial = p->cpart;
  CHK(col(p, fch::EPI_MU, fch::PRO_NONE, a));
  p->stats.fft_calls += 4;
  if (energy) {
    CHK(finalize(p, fch::FIN_ENERGY, true, true));
    CHK(readback(p));
    *energy = p->hctl->energy;
    CHK(status_from_ctl(p));
  }
  return FCH_OK;
}

fch_status fch_chem_potential_dev(fch_plan_t p, const fch_c128* uh, fch_c128* muh,
                                  double* mu_phys, double* energy_dev, int32_t* status_dev) {
  if (!p || !uh || !muh || (const void*)uh == (const void*)muh) return FCH_E_INVALID;
  const void* mp = mu_phys;
  if (mp && (mp == (const void*)uh || mp == (const void*)muh)) return FCH_E_INVALID;
  CHK(need_ws(p));
  CHK(ctl_set(p, ctl_zero()));
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, p->rpart));
  a.out = (cd*)muh;
  a.partial = p->cpart;
  CHK(col(p, fch::EPI_MU, fch::PRO_NONE, a));
  p->stats.fft_calls += 4;
  if (energy_dev || status_dev) {
    CHK(finalize(p, fch::FIN_ENERGY, true, true));
    HIPCHK(fch::launch_ctl_out(p->ctl, fch::OUT_ENERGY, energy_dev, nullptr, status_dev,
                               p->stream));
    p->stats.launches += 1;
  }
  if (mu_phys) CHK(fch_inverse(p, muh, (double*)mu_phys));
  return FCH_OK;
}

fch_status fch_rhs(fch_plan_t p, const fch_c128* uh, fch_c128* Fh) {
  if (!p || !uh || !Fh || (const void*)uh == (const void*)Fh) return FCH_E_INVALID;
  CHK(need_ws(p));
  CHK(ctl_set(p, ctl_zero()));
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, nullptr));
  a.out = (cd*)Fh;
  CHK(col(p, fch::EPI_F, fch::PRO_NONE, a));
  p->stats.fft_calls += 4;
  return FCH_OK;
}

// ---- steps ----------------------------------------------------------------
static fch_status check_step(fch_plan_t p, const fch_c128* un, const fch_c128* um, double k_np1,
                             double k_n, const fch_c128* out) {
  if (!p || !un || !out) return FCH_E_INVALID;
  if (!finite_pos(k_np1) || !std::isfinite(k_n)) return FCH_E_INVALID;
  if (k_n > 0.0 && !um) return FCH_E_INVALID;
  if ((const void*)out == (const void*)un) return FCH_E_INVALID;
  return need_ws(p);
}

fch_status fch_step_imex(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1,
                         double k_np1, double k_n, fch_c128* uh_np1) {
  CHK(check_step(p, uh_n, uh_nm1, k_np1, k_n, uh_np1));
  const cd* um = (k_n > 0.0) ? (const cd*)uh_nm1 : (const cd*)uh_n;
  return imex_attempt(p, (const cd*)uh_n, um, k_np1, k_n, (cd*)uh_np1);
}

fch_status fch_step_imex_static(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1,
                                double k_np1, double k_n, fch_c128* uh_np1) {
  if (!p || !uh_n || !uh_np1) return FCH_E_INVALID;
  if (p->N > kStaticMaxN) return FCH_E_UNSUPPORTED;
  if (!finite_pos(k_np1) || !std::isfinite(k_n)) return FCH_E_INVALID;
  if (k_n > 0.0 && !uh_nm1) return FCH_E_INVALID;
  if ((const void*)uh_np1 == (const void*)uh_n) return FCH_E_INVALID;
  char* sp = nullptr;
  CHK(scratch_resolve(p->device, &sp));
  cd* pair0 = (cd*)sp;
  cd* pair1 = (cd*)(sp + align256(spec_bytes(p->N)));
  const cd* um = (k_n > 0.0) ? (const cd*)uh_nm1 : (const cd*)uh_n;
  return imex_attempt(p, (const cd*)uh_n, um, k_np1, k_n, (cd*)uh_np1, pair0, pair1);
}

fch_status fch_sav_r(fch_plan_t p, const fch_c128* uh, double* r) {
  if (!p || !uh || !r) return FCH_E_INVALID;
  CHK(need_ws(p));
  CHK(ctl_set(p, ctl_zero()));
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, p->rpart));
  CHK(finalize(p, fch::FIN_SAV_S, true, false));
  CHK(readback(p));
  CHK(status_from_ctl(p));
  *r = p->hctl->s_star;
  return FCH_OK;
}

fch_status fch_step_sav(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1, double r_n,
                        double r_nm1, double k_np1, double k_n, fch_c128* uh_np1, double* r_np1) {
  CHK(check_step(p, uh_n, uh_nm1, k_np1, k_n, uh_np1));
  if (!r_np1 || !std::isfinite(r_n) || !std::isfinite(r_nm1)) return FCH_E_INVALID;
  const cd* un = (const cd*)uh_n;
  const cd* um = (k_n > 0.0) ? (const cd*)uh_nm1 : un;
  StepCtl v = ctl_zero();
  set_bdf2(v, k_np1, k_n);
  v.r_n = r_n;
  v.r_nm1 = (k_n > 0.0) ? r_nm1 : 0.0;
  CHK(ctl_set(p, v));
  ColArgs a = col_args(p);
  a.s0 = un;
  a.s1 = um;
  CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
  CHK(row_mu(p, p->rpart));
  a.out = (cd*)uh_np1;
  a.aux = p->aux;
  a.partial = p->cpart;
  a.sav_rpart = p->rpart;
  a.sav_nrow = p->N / p->rv->R;
  CHK(col(p, fch::EPI_SAV, fch::PRO_NONE, a));
  prof_break(p);
  HIPCHK(fch::launch_sav_combine((cd*)uh_np1, p->aux, p->ctl, (size_t)p->H * p->N, p->cpart, p->H,
                                 p->c.pars, p->stream));
  p->stats.launches += 1;
  p->stats.fft_calls += 4;
  p->stats.steps += 1;
  CHK(readback(p));
  CHK(status_from_ctl(p));
  *r_np1 = p->hctl->r_np1;
  return FCH_OK;
}

fch_status fch_step_psd(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1, double k_np1,
                        double k_n, const fch_c128* guess, const fch_psd_opts* opts,
                        fch_c128* uh_np1, fch_psd_stats* stats) {
  CHK(check_step(p, uh_n, uh_nm1, k_np1, k_n, uh_np1));
  if (!opts || opts->max_iter < 1 || !(opts->tol > 0.0 || opts->fixed_iters > 0))
    return FCH_E_INVALID;
  if ((const void*)guess == (const void*)uh_np1 && guess) return FCH_E_INVALID;
  const double lam = opts->lambda > 0.0 ? opts->lambda : lambda_table(p->prm.q, k_np1);
  if (!(lam > 0.0)) return FCH_E_INVALID;
  const cd* un = (const cd*)uh_n;
  const cd* um = (k_n > 0.0) ? (const cd*)uh_nm1 : un;
  StepCtl v = ctl_zero();
  set_bdf2(v, k_np1, k_n);
  v.lambda = lam;
  v.tol = opts->tol;
  v.max_iter = opts->max_iter;
  v.fixed_iters = opts->fixed_iters;
  CHK(ctl_set(p, v));
  CheckDone cd_guard(p);
  ColArgs a = col_args(p);
  a.s0 = un;
  a.s1 = um;
  a.guess = (const cd*)guess;
  a.out = (cd*)uh_np1;
  a.aux = p->aux;
  CHK(col(p, fch::EPI_NONE, fch::PRO_PSD_INIT, a));
  a.partial = p->cpart;
  const int limit = opts->fixed_iters > 0 ? opts->fixed_iters : opts->max_iter;
  if (p->psd1 && p->psd1_on) {
    CHK(psd_solve_launch(p, a, limit));
    CHK(readback(p));
  } else {
    int queued = 0;
    int chunk = p->psd_hint > 0 ? p->psd_hint : 4;
    for (;;) {
      const int n = (chunk < limit - queued) ? chunk : (limit - queued);
      CHK(psd_iterations(p, a, queued, n));
      queued += n;
      CHK(readback(p));
      if (p->hctl->done || queued >= limit) break;
      chunk = 4;
    }
  }
  if (p->hctl->done == 5) return FCH_E_HIP;
  const int iters = p->hctl->iters;
  p->psd_hint = iters > 0 ? iters : 4;
  p->stats.psd_iters += iters;
  p->stats.fft_calls += 4LL * iters;
  p->stats.steps += 1;
  if (stats) {
    stats->iters = iters;
    stats->fft_calls = 4LL * iters;
    stats->last_ratio = p->hctl->ratio;
  }
  if (p->hctl->nonfinite || p->hctl->done == 3) return FCH_E_NONFINITE;
  if (p->hctl->done == 2) return FCH_E_NOCONV;
  return FCH_OK;
}

// ---- ETDRK2 ----------------------------------------------------------------
static fch_status etd_opts(const fch_etd_opts* o, double* k0, double* k2) {
  *k0 = o ? o->kappa0 : 1e-2;  // the values of Sec. 3.6
  *k2 = o ? o->kappa2 : 15.0;
  if (!(*k0 >= 0.0) || !(*k2 >= 0.0) || !std::isfinite(*k0) || !std::isfinite(*k2))
    return FCH_E_INVALID;
  return FCH_OK;
}

namespace {
// the second stage from u~ (in st) and w (in aux): its evaluation then
// u^{n+1} = w + k phi2 N(u~), optionally followed by the inverse column
// transforms of (u^{n+1}, Lap u^{n+1}) for the next evaluation
fch_status etd_second(fch_plan_s* p, cd* ut, cd* out, bool next) {
  CHK(row_mu(p, nullptr));
  ColArgs b = col_args(p);
  b.s0 = ut;
  b.s1 = p->aux;
  b.out = out;
  CHK(col(p, fch::EPI_ETD2, next ? fch::PRO_NEXT_FIELD : fch::PRO_NONE, b));
  p->stats.fft_calls += 4;
  return FCH_OK;
}
// the first stage from the cached F(u^n): u~ into ut and w into aux, and the
// inverse column transforms of (u~, Lap u~)
fch_status etd_first_cached(fch_plan_s* p, const cd* un, const cd* Fn, cd* ut) {
  ColArgs a = col_args(p);
  a.s0 = un;
  a.f_n = Fn;
  a.out = ut;
  a.aux = p->aux;
  return col(p, fch::EPI_NONE, fch::PRO_ETD1, a);
}
// the first stage with its own evaluation of mu(u^n), whose (u^n, Lap u^n)
// the pair buffer already holds column-inverted
fch_status etd_first_eval(fch_plan_s* p, const cd* un, cd* ut) {
  CHK(row_mu(p, nullptr));
  ColArgs a = col_args(p);
  a.s0 = un;
  a.out = ut;
  a.aux = p->aux;
  CHK(col(p, fch::EPI_ETD1, fch::PRO_NEXT_FIELD, a));
  p->stats.fft_calls += 4;
  return FCH_OK;
}
StepCtl etd_ctl(double k, double kappa0, double kappa2) {
  StepCtl v = ctl_zero();
  v.k_np1 = k;
  v.kappa0 = kappa0;
  v.kappa2 = kappa2;
  return v;
}
}  // namespace

namespace {
// the launches of one step once the control block holds k, kappa0, kappa2
fch_status etd_step_launch(fch_plan_s* p, const fch_c128* uh_n, const fch_c128* F_n,
                           fch_c128* uh_np1) {
  const cd* un = (const cd*)uh_n;
  if (F_n) {
    CHK(etd_first_cached(p, un, (const cd*)F_n, p->st));
  } else {
    ColArgs a = col_args(p);
    a.s0 = un;
    CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
    CHK(etd_first_eval(p, un, p->st));
  }
  CHK(etd_second(p, p->st, (cd*)uh_np1, false));
  p->stats.steps += 1;
  return FCH_OK;
}
}  // namespace

fch_status fch_step_etd(fch_plan_t p, const fch_c128* uh_n, const fch_c128* F_n, double k,
                        const fch_etd_opts* opts, fch_c128* uh_np1) {
  if (!p || !uh_n || !uh_np1 || !finite_pos(k)) return FCH_E_INVALID;
  double k0, k2;
  CHK(etd_opts(opts, &k0, &k2));
  CHK(need_ws(p));
  CHK(ctl_set(p, etd_ctl(k, k0, k2)));
  return etd_step_launch(p, uh_n, F_n, uh_np1);
}

// ---- adaptivity -----------------------------------------------------------
static fch_status check_adapt(const fch_adapt_opts* o) {
  if (!o || !finite_pos(o->sigma_tol) || !finite_pos(o->k_min) || !(o->k_max >= o->k_min) ||
      !finite_pos(o->rho_s) || std::isnan(o->cap))
    return FCH_E_INVALID;
  return FCH_OK;
}

static void set_adapt(StepCtl& v, const fch_adapt_opts* o) {
  v.sigma_tol = o->sigma_tol;
  v.k_min = o->k_min;
  v.k_max = o->k_max;
  v.rho_s = o->rho_s;
  v.cap = o->cap;
}

fch_status fch_adapt_dt(fch_plan_t p, const fch_c128* uh_trial, const fch_c128* uh_n,
                        const fch_c128* F_n, const fch_c128* F_nm1, double k_trial, double k_n,
                        const fch_adapt_opts* opts, fch_c128* F_trial, int32_t* accept,
                        double* k_next, double* err) {
  if (!p || !uh_trial || !uh_n || !F_n || !F_nm1 || !F_trial) return FCH_E_INVALID;
  if (!finite_pos(k_trial) || !finite_pos(k_n)) return FCH_E_INVALID;
  const void* outs = F_trial;
  if (outs == uh_trial || outs == uh_n || outs == F_n || outs == F_nm1) return FCH_E_INVALID;
  CHK(check_adapt(opts));
  CHK(need_ws(p));
  StepCtl v = ctl_zero();
  set_bdf2(v, k_trial, k_n);
  set_am3(v, k_trial, k_n);
  set_adapt(v, opts);
  CHK(ctl_set(p, v));
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh_trial;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, nullptr));
  a.s1 = (const cd*)uh_n;
  a.f_n = (const cd*)F_n;
  a.f_nm1 = (const cd*)F_nm1;
  a.out = (cd*)F_trial;
  a.partial = p->cpart;
  CHK(col(p, fch::EPI_AM3, fch::PRO_NONE, a));
  CHK(finalize(p, fch::FIN_AM3, false, true));
  p->stats.fft_calls += 4;
  CHK(readback(p));
  if (accept) *accept = p->hctl->accept;
  if (k_next) *k_next = p->hctl->k_next;
  if (err) *err = p->hctl->err;
  return status_from_ctl(p);
}

// ---- steps with device-resident scalars (graph-capturable) ----------------
namespace {
fch_status ctl_dev(fch_plan_s* p, const StepCtl& v, const double* k_dev, const double* r_dev,
                   int flags) {
  prof_break(p);
  HIPCHK(fch::launch_ctl_dev(p->ctl, v, k_dev, r_dev, p->prm.q, flags, p->stream));
  p->stats.launches += 1;
  return FCH_OK;
}
fch_status ctl_out(fch_plan_s* p, int what, double* d_out, int32_t* i_out, int32_t* status) {
  prof_break(p);
  if (!d_out && !i_out && !status) return FCH_OK;
  HIPCHK(fch::launch_ctl_out(p->ctl, what, d_out, i_out, status, p->stream));
  p->stats.launches += 1;
  return FCH_OK;
}
fch_status check_step_dev(fch_plan_s* p, const fch_c128* un, const fch_c128* um,
                          const double* k_dev, const fch_c128* out) {
  if (!p || !un || !um || !k_dev || !out) return FCH_E_INVALID;
  if ((const void*)out == (const void*)un) return FCH_E_INVALID;
  return need_ws(p);
}
}  // namespace

fch_status fch_step_imex_dev(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1,
                             const double* k_dev, fch_c128* uh_np1, int32_t* status_dev) {
  CHK(check_step_dev(p, uh_n, uh_nm1, k_dev, uh_np1));
  CHK(ctl_dev(p, ctl_zero(), k_dev, nullptr, 0));
  CheckDone cd_guard(p);
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh_n;
  a.s1 = (const cd*)uh_nm1;
  CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
  CHK(row_mu(p, nullptr));
  a.out = (cd*)uh_np1;
  CHK(col(p, fch::EPI_IMEX, fch::PRO_NONE, a));
  p->stats.fft_calls += 4;
  p->stats.steps += 1;
  return ctl_out(p, fch::OUT_STATUS, nullptr, nullptr, status_dev);
}

fch_status fch_step_sav_dev(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1,
                            const double* r_dev, const double* k_dev, fch_c128* uh_np1,
                            double* r_np1_dev, int32_t* status_dev) {
  CHK(check_step_dev(p, uh_n, uh_nm1, k_dev, uh_np1));
  if (!r_dev || !r_np1_dev) return FCH_E_INVALID;
  CHK(ctl_dev(p, ctl_zero(), k_dev, r_dev, fch::CTL_SAV));
  CheckDone cd_guard(p);
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh_n;
  a.s1 = (const cd*)uh_nm1;
  CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
  CHK(row_mu(p, p->rpart));
  a.out = (cd*)uh_np1;
  a.aux = p->aux;
  a.partial = p->cpart;
  a.sav_rpart = p->rpart;
  a.sav_nrow = p->N / p->rv->R;
  CHK(col(p, fch::EPI_SAV, fch::PRO_NONE, a));
  prof_break(p);
  HIPCHK(fch::launch_sav_combine((cd*)uh_np1, p->aux, p->ctl, (size_t)p->H * p->N, p->cpart, p->H,
                                 p->c.pars, p->stream));
  p->stats.launches += 1;
  p->stats.fft_calls += 4;
  p->stats.steps += 1;
  return ctl_out(p, fch::OUT_SAV, r_np1_dev, nullptr, status_dev);
}

fch_status fch_step_psd_dev(fch_plan_t p, const fch_c128* uh_n, const fch_c128* uh_nm1,
                            const double* k_dev, const fch_c128* guess,
                            const fch_psd_opts* opts, fch_c128* uh_np1, int32_t* iters_dev,
                            int32_t* status_dev) {
  CHK(check_step_dev(p, uh_n, uh_nm1, k_dev, uh_np1));
  if (!opts || opts->max_iter < 1 || !(opts->tol > 0.0 || opts->fixed_iters > 0))
    return FCH_E_INVALID;
  if (guess && (const void*)guess == (const void*)uh_np1) return FCH_E_INVALID;
  int flags = 0;
  StepCtl v = ctl_zero();
  if (opts->lambda > 0.0) {
    v.lambda = opts->lambda;
  } else {
    if (!(lambda_table(p->prm.q, 1e-3) > 0.0)) return FCH_E_INVALID;
    flags |= fch::CTL_LAMBDA;
  }
  v.tol = opts->tol;
  v.max_iter = opts->max_iter;
  v.fixed_iters = opts->fixed_iters;
  CHK(ctl_dev(p, v, k_dev, nullptr, flags));
  CheckDone cd_guard(p);
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh_n;
  a.s1 = (const cd*)uh_nm1;
  a.guess = (const cd*)guess;
  a.out = (cd*)uh_np1;
  a.aux = p->aux;
  CHK(col(p, fch::EPI_NONE, fch::PRO_PSD_INIT, a));
  a.partial = p->cpart;
  // one k_psd_solve launch, or (without it) every iteration up to the limit,
  // whose launches return at once after the device flag is set (converged,
  // limit, non-finite)
  const int limit = opts->fixed_iters > 0 ? opts->fixed_iters : opts->max_iter;
  CHK(psd_solve_launch(p, a, limit));
  p->stats.steps += 1;
  return ctl_out(p, fch::OUT_PSD, nullptr, iters_dev, status_dev);
}

fch_status fch_step_etd_dev(fch_plan_t p, const fch_c128* uh_n, const fch_c128* F_n,
                            const double* k_dev, const fch_etd_opts* opts, fch_c128* uh_np1,
                            int32_t* status_dev) {
  if (!p || !uh_n || !uh_np1 || !k_dev) return FCH_E_INVALID;
  double k0, k2;
  CHK(etd_opts(opts, &k0, &k2));
  CHK(need_ws(p));
  StepCtl v = ctl_zero();
  v.kappa0 = k0;
  v.kappa2 = k2;
  CHK(ctl_dev(p, v, k_dev, nullptr, fch::CTL_K1_ONLY));
  CheckDone cd_guard(p);
  CHK(etd_step_launch(p, uh_n, F_n, uh_np1));
  return ctl_out(p, fch::OUT_STATUS, nullptr, nullptr, status_dev);
}

fch_status fch_adapt_dt_dev(fch_plan_t p, const fch_c128* uh_trial, const fch_c128* uh_n,
                            const fch_c128* F_n, const fch_c128* F_nm1, const double* k_dev,
                            const fch_adapt_opts* opts, fch_c128* F_trial, double* out_dev,
                            int32_t* status_dev) {
  if (!p || !uh_trial || !uh_n || !F_n || !F_nm1 || !F_trial || !k_dev || !out_dev)
    return FCH_E_INVALID;
  const void* outs = F_trial;
  if (outs == uh_trial || outs == uh_n || outs == F_n || outs == F_nm1) return FCH_E_INVALID;
  CHK(check_adapt(opts));
  CHK(need_ws(p));
  StepCtl v = ctl_zero();
  set_adapt(v, opts);
  CHK(ctl_dev(p, v, k_dev, nullptr, fch::CTL_AM3));
  CheckDone cd_guard(p);
  ColArgs a = col_args(p);
  a.s0 = (const cd*)uh_trial;
  CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
  CHK(row_mu(p, nullptr));
  a.s1 = (const cd*)uh_n;
  a.f_n = (const cd*)F_n;
  a.f_nm1 = (const cd*)F_nm1;
  a.out = (cd*)F_trial;
  a.partial = p->cpart;
  CHK(col(p, fch::EPI_AM3, fch::PRO_NONE, a));
  CHK(finalize(p, fch::FIN_AM3, false, true));
  p->stats.fft_calls += 4;
  return ctl_out(p, fch::OUT_ADAPT, out_dev, nullptr, status_dev);
}

// ---- trajectories ---------------------------------------------------------
static fch_status copy_spec(fch_plan_t p, cd* dst, const cd* src) {
  if (dst == src) return FCH_OK;
  prof_break(p);
  HIPCHK(hipMemcpyAsync(dst, src, spec_bytes(p->N), hipMemcpyDeviceToDevice, p->stream));
  return FCH_OK;
}

// put (cur, prev) back into the caller's (uh_n, uh_nm1)
static fch_status settle(fch_plan_t p, cd* B0, cd* B1, cd* cur, cd* prev) {
  if (cur == B0 && prev == B1) return FCH_OK;
  if (cur == B1 && prev == B0) {
    CHK(copy_spec(p, p->st, B1));
    CHK(copy_spec(p, B1, B0));
    return copy_spec(p, B0, p->st);
  }
  // one of them lives in the spare buffer
  if (cur == B0) return copy_spec(p, B1, prev);
  if (prev == B1) return copy_spec(p, B0, cur);
  if (cur == B1) {  // prev is the spare
    CHK(copy_spec(p, B0, B1));
    return copy_spec(p, B1, prev);
  }
  // cur is the spare, prev == B0
  CHK(copy_spec(p, B1, B0));
  return copy_spec(p, B0, cur);
}

static fch_status sav_or_psd_step(fch_plan_t p, const fch_run_opts* o, const cd* un, const cd* um,
                                  double k1, double k0, cd* out, double* rs, double* r_new,
                                  int64_t* iters) {
  if (o->scheme == FCH_SAV) {
    return fch_step_sav(p, (const fch_c128*)un, (const fch_c128*)um, rs[0], rs[1], k1, k0,
                        (fch_c128*)out, r_new);
  }
  fch_psd_stats st;
  fch_status s = fch_step_psd(p, (const fch_c128*)un, (const fch_c128*)um, k1, k0, nullptr,
                              &o->psd, (fch_c128*)out, &st);
  *iters += st.iters;
  return s;
}

namespace {
// Launches graph_steps fused IMEX steps (row pass, then column pass with the
// next step's prologue) from (cur, prev); graph_steps is even, so the buffer
// roles are the same afterwards.  The graph is captured on the internal
// stream on first use for this buffer pair, workspace and launch variants.
fch_status chain_replay(fch_plan_s* p, cd* cur, cd* prev) {
  const void* key[6] = {cur, prev, p->P0, p->rv, p->cv, (const void*)(intptr_t)p->graph_steps};
  if (p->chain_exec && std::memcmp(key, p->chain_key, sizeof(key)) != 0) drop_chain(p);
  if (!p->chain_exec) {
    hipStream_t user = p->stream;
    p->stream = p->gstream;
    if (hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      p->stream = user;
      return FCH_E_HIP;
    }
    const fch_stats saved = p->stats;
    fch_status st = FCH_OK;
    cd *c = cur, *pv = prev;
    ColArgs a = col_args(p);
    for (int i = 0; i < p->graph_steps && st == FCH_OK; ++i) {
      st = row_mu(p, nullptr);
      if (st != FCH_OK) break;
      a.s0 = c;
      a.s1 = pv;
      a.out = pv;
      st = col(p, fch::EPI_IMEX, fch::PRO_NEXT_EXTRAP, a);
      std::swap(c, pv);
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->gstream, &g);
    p->stream = user;
    p->stats = saved;
    if (st == FCH_OK && (ec != hipSuccess || !g)) st = FCH_E_HIP;
    if (st == FCH_OK && hipGraphInstantiate(&p->chain_exec, g, nullptr, nullptr, 0) != hipSuccess) {
      p->chain_exec = nullptr;
      st = FCH_E_HIP;
    }
    if (g) (void)hipGraphDestroy(g);
    if (st != FCH_OK) return st;
    std::memcpy(p->chain_key, key, sizeof(key));
  }
  HIPCHK(hipEventRecord(p->gfork, p->stream));
  HIPCHK(hipStreamWaitEvent(p->gstream, p->gfork, 0));
  HIPCHK(hipGraphLaunch(p->chain_exec, p->gstream));
  HIPCHK(hipEventRecord(p->gjoin, p->gstream));
  HIPCHK(hipStreamWaitEvent(p->stream, p->gjoin, 0));
  p->stats.launches += 2 * p->graph_steps;
  p->stats.fft_calls += 4 * p->graph_steps;
  p->stats.steps += p->graph_steps;
  return FCH_OK;
}
}  // namespace

fch_status fch_run(fch_plan_t p, const fch_run_opts* o, fch_c128* uh_n, fch_c128* uh_nm1,
                   double* rs, fch_run_info* info) {
  if (!p || !o || !uh_n || !uh_nm1 || uh_n == uh_nm1) return FCH_E_INVALID;
  if (o->scheme < FCH_IMEX || o->scheme > FCH_ETD) return FCH_E_INVALID;
  double ka0 = 0.0, ka2 = 0.0;
  if (o->scheme == FCH_ETD) CHK(etd_opts(&o->etd, &ka0, &ka2));
  if (o->scheme == FCH_SAV && !rs) return FCH_E_INVALID;
  CHK(need_ws(p));
  cd* B0 = (cd*)uh_n;
  cd* B1 = (cd*)uh_nm1;
  cd *cur = B0, *prev = B1, *spare = p->st;
  fch_run_info inf;
  std::memset(&inf, 0, sizeof(inf));
  double r0 = 0.0;
  if (o->scheme == FCH_SAV && o->startup) {
    CHK(fch_sav_r(p, uh_n, &r0));
    rs[0] = r0;
    rs[1] = r0;
  }

  if (!o->adaptive && o->scheme == FCH_ETD) {
    // one-step method: nsteps steps of size k; each first stage evaluates
    // mu(u^n) and hands u~ to the second, whose column pass starts the next
    // step's evaluation.  u^{n+1} overwrites u^{n-1}.
    if (!finite_pos(o->k) || o->nsteps < 0) return FCH_E_INVALID;
    if (o->nsteps > 0) {
      CHK(ctl_set(p, etd_ctl(o->k, ka0, ka2)));
      ColArgs a = col_args(p);
      a.s0 = cur;
      CHK(col(p, fch::EPI_NONE, fch::PRO_FIELD, a));
    }
    for (int64_t n = 0; n < o->nsteps; ++n) {
      CHK(etd_first_eval(p, cur, spare));
      CHK(etd_second(p, spare, prev, n + 1 < o->nsteps));
      std::swap(cur, prev);
      p->stats.steps += 1;
    }
    inf.accepted = o->nsteps;
    inf.t = o->nsteps * o->k;
    inf.k_last = o->k;
    inf.k_next = o->k;
    CHK(settle(p, B0, B1, cur, prev));
    if (info) {
      inf.fft_calls = p->stats.fft_calls;
      *info = inf;
    }
    return FCH_OK;
  }

  if (!o->adaptive) {
    if (!finite_pos(o->k) || o->nsteps < 0) return FCH_E_INVALID;
    int64_t done = 0;
    double k_n = o->k_prev;
    if (o->startup && o->nsteps > 0) {
      // first-order step from u^0
      if (o->scheme == FCH_IMEX) {
        CHK(imex_attempt(p, cur, cur, o->k, -1.0, prev));
      } else {
        double rn = 0;
        int64_t it = 0;
        CHK(sav_or_psd_step(p, o, cur, cur, o->k, -1.0, prev, rs, &rn, &it));
        inf.psd_iters += it;
        if (o->scheme == FCH_SAV) { rs[1] = rs[0]; rs[0] = rn; }
      }
      std::swap(cur, prev);
      k_n = o->k;
      done = 1;
    }
    if (done < o->nsteps && !finite_pos(k_n)) return FCH_E_INVALID;
    if (o->scheme == FCH_IMEX && done < o->nsteps) {
      if (k_n != o->k) {  // a step-ratio change: one unfused step first
        CHK(imex_attempt(p, cur, prev, o->k, k_n, prev));
        std::swap(cur, prev);
        k_n = o->k;
        ++done;
      }
      if (done < o->nsteps) {
        // fused chain at gamma = 1: each column pass ends one step and
        // starts the next; u^{n+1} overwrites u^{n-1}
        StepCtl v = ctl_zero();
        set_bdf2(v, o->k, o->k);
        CHK(ctl_set(p, v));
        ColArgs a = col_args(p);
        a.s0 = cur;
        a.s1 = prev;
        CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
        while (done < o->nsteps) {
          // the last step (no next prologue) always runs outside the graph
          if (p->graph_steps > 0 && !p->prof_on && o->nsteps - done > p->graph_steps) {
            CHK(chain_replay(p, cur, prev));
            done += p->graph_steps;
            continue;
          }
          CHK(row_mu(p, nullptr));
          const bool last = (done + 1 == o->nsteps);
          a.s0 = cur;
          a.s1 = prev;
          a.out = prev;
          CHK(col(p, fch::EPI_IMEX, last ? fch::PRO_NONE : fch::PRO_NEXT_EXTRAP, a));
          std::swap(cur, prev);
          ++done;
          p->stats.fft_calls += 4;
          p->stats.steps += 1;
        }
      }
    } else {
      // SAV: steps at a changed ratio one at a time, then the fused chain
      while (done < o->nsteps && (o->scheme != FCH_SAV || k_n != o->k)) {
        double rn = 0;
        int64_t it = 0;
        CHK(sav_or_psd_step(p, o, cur, prev, o->k, k_n, prev, rs, &rn, &it));
        inf.psd_iters += it;
        if (o->scheme == FCH_SAV) { rs[1] = rs[0]; rs[0] = rn; }
        std::swap(cur, prev);
        k_n = o->k;
        ++done;
      }
      if (o->scheme == FCH_SAV && done < o->nsteps) {
        // fused SAV chain at gamma = 1 with r on the device: row pass (E_1
        // partials), SAV column pass (p over u^{n-1}, q, the (g_p, g_q)
        // partials), then a column pass that solves for r^{n+1} in every
        // workgroup, writes u^{n+1} = p + r^{n+1} q and starts the next step's
        // evaluation.  No host synchronization until the end.
        StepCtl v = ctl_zero();
        set_bdf2(v, o->k, o->k);
        v.rring[0] = rs[0];
        v.rring[2] = rs[1];
        CHK(ctl_set(p, v));
        ColArgs a = col_args(p);
        a.s0 = cur;
        a.s1 = prev;
        CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
        int slot = 0;
        while (done < o->nsteps) {
          CHK(row_mu(p, p->rpart));
          ColArgs b = col_args(p);
          b.s0 = cur;
          b.s1 = prev;
          b.out = prev;
          b.aux = p->aux;
          b.partial = p->cpart;
          b.sav_rpart = p->rpart;
          b.sav_nrow = p->N / p->rv->R;
          CHK(col(p, fch::EPI_SAV, fch::PRO_NONE, b));
          ColArgs c = col_args(p);
          c.s0 = cur;
          c.out = prev;
          c.aux = p->aux;
          c.sav_cpart = p->cpart;
          c.sav_ncol = p->H;
          c.rslot = slot;
          CHK(col(p, fch::EPI_NONE, fch::PRO_SAV_NEXT, c));
          slot = (slot + 1) % 3;
          std::swap(cur, prev);
          ++done;
          p->stats.fft_calls += 4;
          p->stats.steps += 1;
        }
        CHK(readback(p));
        CHK(status_from_ctl(p));
        rs[0] = p->hctl->rring[slot];
        rs[1] = p->hctl->rring[(slot + 2) % 3];
      }
    }
    inf.accepted = done;
    inf.t = done * o->k;
    inf.k_last = o->k;
    inf.k_next = o->k;
    CHK(settle(p, B0, B1, cur, prev));
    if (info) {
      inf.fft_calls = p->stats.fft_calls;
      *info = inf;
    }
    return FCH_OK;
  }

  // ---- adaptive (Sec. 3.2) ----
  CHK(check_adapt(&o->adapt));
  const fch_adapt_opts* ad = &o->adapt;
  if (!(o->t_end > 0.0)) return FCH_E_INVALID;
  if (o->scheme == FCH_PSD &&
      (o->psd.max_iter < 1 || !(o->psd.tol > 0.0 || o->psd.fixed_iters > 0)))
    return FCH_E_INVALID;
  cd* Fn = p->Fc[0];
  cd* Fm = p->Fc[1];
  cd* Ft = p->Fc[2];
  double t = 0.0, k_n = o->k_prev, kt = o->k;
  if (o->startup) {
    // the startup step is clamped to the run like the last step (t_end > 0)
    const double k1 = std::min(o->k_first > 0.0 ? o->k_first : ad->k_min, o->t_end);
    CHK(fch_rhs(p, (const fch_c128*)cur, (fch_c128*)Fm));
    if (o->scheme == FCH_IMEX) {
      CHK(imex_attempt(p, cur, cur, k1, -1.0, prev));
    } else if (o->scheme == FCH_ETD) {
      CHK(ctl_set(p, etd_ctl(k1, ka0, ka2)));
      CHK(etd_first_cached(p, cur, Fm, Ft));
      CHK(etd_second(p, Ft, prev, false));
      p->stats.steps += 1;
    } else {
      double rn = 0;
      int64_t it = 0;
      CHK(sav_or_psd_step(p, o, cur, cur, k1, -1.0, prev, rs, &rn, &it));
      inf.psd_iters += it;
      if (o->scheme == FCH_SAV) { rs[1] = rs[0]; rs[0] = rn; }
    }
    std::swap(cur, prev);
    CHK(fch_rhs(p, (const fch_c128*)cur, (fch_c128*)Fn));
    t = k1;
    k_n = k1;
    kt = k1;  // Step 0: the first trial step equals the last step
    inf.accepted = 1;
  } else {
    if (!finite_pos(k_n) || !finite_pos(kt)) return FCH_E_INVALID;
    CHK(fch_rhs(p, (const fch_c128*)cur, (fch_c128*)Fn));
    CHK(fch_rhs(p, (const fch_c128*)prev, (fch_c128*)Fm));
  }
  const double t_end = o->t_end;
  const int64_t max_acc = o->nsteps > 0 ? o->nsteps : INT64_MAX;
  if (!p->prof_on && !o->dyadic) {
    // Attempts under device control: the run is described as one ensemble
    // member (state and F slots, time, step scalars) and each attempt is the
    // batched kernels' sequence with the per-member controller, which accepts
    // or rejects, rotates the slots and sets the next attempt's scalars.  The
    // host only reads the member back between chunks of queued attempts
    // (attempts queued after the run ended return at once).
    fch::EnsMember& m = *p->hmem;
    std::memset(&m, 0, sizeof(m));
    m.c = p->c;
    m.tw = p->tw;
    m.ring[0] = cur;
    m.ring[1] = prev;
    m.ring[2] = spare;
    m.fring[0] = Fn;
    m.fring[1] = Fm;
    m.fring[2] = Ft;
    m.P0 = p->P0;
    m.P1 = p->P1;
    m.aux = p->aux;
    m.cpart = p->cpart;
    // rpart serves twice, in stream order: SAV's E_1 partials (first row pass,
    // read by the SAV column pass), then the trial row pass's largest u per
    // workgroup (reset by the controller; never folded into umax here)
    m.rpart = p->rpart;
    m.umaxpart = p->rpart;
    m.sav = (o->scheme == FCH_SAV) ? 1 : 0;
    m.psd = (o->scheme == FCH_PSD) ? 1 : 0;
    m.rslot = 0;
    m.nrow = p->N / p->rv->R;
    m.umax = -INFINITY;
    m.umax_t0 = INFINITY;
    m.klog = nullptr;
    m.klog_cap = 0;
    m.cur = 0;
    m.prev = 1;
    m.trial = 2;
    m.fn = 0;
    m.fm = 1;
    m.ft = 2;
    m.t = t;
    m.t_end = t_end;
    m.accepted = inf.accepted;
    m.rejected = 0;
    m.max_accepted = max_acc;
    m.H = p->H;
    StepCtl& v = m.ctl;
    set_adapt(v, ad);
    const double kt_first = kt;  // reported as the next trial if no attempt runs
    if (kt > t_end - t) kt = t_end - t;
    set_bdf2(v, kt, k_n);
    set_am3(v, kt, k_n);
    v.kappa0 = ka0;
    v.kappa2 = ka2;
    if (m.sav) {
      v.rring[0] = rs[0];  // r^n
      v.rring[2] = rs[1];  // r^{n-1}
    }
    v.done = (t >= t_end * (1.0 - 1e-14) || inf.accepted >= max_acc) ? 1 : 0;
    const bool etd = (o->scheme == FCH_ETD);
    if (m.psd) {
      // the solve's options; the first attempt's control block and stages
      m.sctl = ctl_zero();
      m.sctl.tol = o->psd.tol;
      m.sctl.max_iter = o->psd.max_iter;
      m.sctl.fixed_iters = o->psd.fixed_iters;
      m.psd_lambda = o->psd.lambda;
      if (!fch::psd_arm(&m)) return FCH_E_INVALID;
      if (v.done) {
        m.psd_init_skip = 1;
        m.psd_eval_skip = 1;
        m.sctl.done = 4;
      }
    }
    HIPCHK(hipMemcpyAsync(p->dmem, &m, sizeof(m), hipMemcpyHostToDevice, p->stream));
    int64_t before = m.accepted + m.rejected;
    // PSD: iterations queued per round, from the iterations per attempt so far
    int psd_c = std::max(2, std::min(64, p->psd_hint + 1));
    while (!m.ctl.done) {
      const int64_t left = max_acc - m.accepted;
      if (m.psd) {
        // rounds of PSD_INIT, psd_c iterations, the F(u~) evaluation (row pass
        // and AM3 column pass) and the controller; each stage runs only in its
        // phase of the attempt
        const int rounds = (int)std::max<int64_t>(1, std::min<int64_t>(8, left));
        for (int i = 0; i < rounds; ++i) {
          HIPCHK(p->cv->col_ens(fch::ENS_PSD_INIT, p->dmem, 0, 1, p->stream));
          for (int j = 0; j < psd_c; ++j) {
            HIPCHK(p->rv->row_ens(p->dmem, 0, 1, fch::ENS_ROW_PSD, p->stream));
            HIPCHK(p->cv->col_ens(fch::ENS_PSD, p->dmem, 0, 1, p->stream));
          }
          // the row pass that stopped the solve left the column-inverted
          // (u, Lap u) of the final iterate in the pair buffer: F(u~) starts there
          HIPCHK(p->rv->row_ens(p->dmem, 0, 1, fch::ENS_ROW_TRACK, p->stream));
          HIPCHK(p->cv->col_ens(fch::ENS_AM3, p->dmem, 0, 1, p->stream));
          HIPCHK(fch::launch_ens_control(p->dmem, 0, 1, p->stream));
        }
        p->stats.launches += (4LL + 2LL * psd_c) * rounds;
        HIPCHK(hipMemcpyAsync(&m, p->dmem, sizeof(m), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        if (m.ctl.nonfinite) return FCH_E_NONFINITE;
        if (m.ctl.invalid) return FCH_E_INVALID;
        // the next rounds queue as many iterations as the latest attempt took,
        // plus one: counts change slowly from attempt to attempt, and an
        // attempt that needs more continues in the next round
        if (m.psd_last_iters > 0) psd_c = std::max(2, std::min(64, m.psd_last_iters + 1));
        continue;
      }
      const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(32, left));
      for (int i = 0; i < chunk; ++i) {
        HIPCHK(p->cv->col_ens(etd ? fch::ENS_ETD_PRO : fch::ENS_PRO, p->dmem, 0, 1, p->stream));
        HIPCHK(p->rv->row_ens(p->dmem, 0, 1, fch::ENS_ROW, p->stream));
        if (m.sav) {
          HIPCHK(p->cv->col_ens(fch::ENS_SAV, p->dmem, 0, 1, p->stream));
          HIPCHK(p->cv->col_ens(fch::ENS_SAV_FIELD, p->dmem, 0, 1, p->stream));
        } else {
          HIPCHK(p->cv->col_ens(etd ? fch::ENS_ETD2 : fch::ENS_IMEX, p->dmem, 0, 1, p->stream));
        }
        HIPCHK(p->rv->row_ens(p->dmem, 0, 1, fch::ENS_ROW_TRACK, p->stream));
        HIPCHK(p->cv->col_ens(fch::ENS_AM3, p->dmem, 0, 1, p->stream));
        HIPCHK(fch::launch_ens_control(p->dmem, 0, 1, p->stream));
      }
      p->stats.launches += (m.sav ? 7LL : 6LL) * chunk;
      HIPCHK(hipMemcpyAsync(&m, p->dmem, sizeof(m), hipMemcpyDeviceToHost, p->stream));
      HIPCHK(hipStreamSynchronize(p->stream));
      if (m.ctl.nonfinite) return FCH_E_NONFINITE;
      if (m.ctl.invalid) return FCH_E_INVALID;
    }
    if (m.sav) {
      rs[0] = m.ctl.rring[m.rslot];
      rs[1] = m.ctl.rring[(m.rslot + 2) % 3];
    }
    const int64_t attempts = m.accepted + m.rejected - before;
    if (m.psd) {
      // 4 FFT calls per PSD iteration and per F(u~) evaluation
      p->stats.fft_calls += 4 * (m.psd_iters + attempts);
      p->stats.psd_iters += m.psd_iters;
      inf.psd_iters += m.psd_iters;
      if (attempts > 0) p->psd_hint = (int)((m.psd_iters + attempts - 1) / attempts);
    } else {
      p->stats.fft_calls += 8 * attempts;
    }
    p->stats.rejected += m.rejected;
    cur = m.ring[m.cur];
    prev = m.ring[m.prev];
    inf.accepted = m.accepted;
    inf.rejected = m.rejected;
    inf.t = m.t;
    inf.k_last = m.ctl.k_n;
    inf.k_next = attempts > 0 ? m.ctl.k_next : kt_first;
    CHK(settle(p, B0, B1, cur, prev));
    if (info) {
      inf.fft_calls = p->stats.fft_calls;
      *info = inf;
    }
    return m.psd_noconv ? FCH_E_NOCONV : FCH_OK;
  }
  // nested factor-of-two steps (o->dyadic): the trial is kb 2^jt; the accepted
  // time is tu units of kb 2^kJmin (exact, so that alignment with the grid of
  // a doubled step is an integer test)
  constexpr int kJmin = -24, kJmax = 38;
  const double kb = kt;
  int jt = 0;
  long long tu = 0;
  auto ladder = [&](int j) { return std::ldexp(kb, j); };
  if (o->dyadic) {
    if (o->startup) tu = 1LL << (0 - kJmin);  // the startup step is kb
    while (jt > kJmin && ladder(jt) > ad->k_max) --jt;
  }
  while (t < t_end * (1.0 - 1e-14) && inf.accepted < max_acc) {
    if (o->dyadic) kt = ladder(jt);
    if (kt > t_end - t) kt = t_end - t;
    double r_new = 0.0;
    int64_t it = 0;
    StepCtl v = ctl_zero();
    set_bdf2(v, kt, k_n);
    set_am3(v, kt, k_n);
    set_adapt(v, ad);
    if (o->scheme == FCH_ETD) {
      // ETDRK2 attempt from the cached F(u^n) (Ft holds u~ until the AM3
      // epilogue overwrites it with F of the trial state)
      v.kappa0 = ka0;
      v.kappa2 = ka2;
      CHK(ctl_set(p, v));
      CHK(etd_first_cached(p, cur, Fn, Ft));
      CHK(etd_second(p, Ft, spare, true));
      CHK(row_mu(p, nullptr));
      ColArgs b = col_args(p);
      b.s0 = spare;
      b.s1 = cur;
      b.f_n = Fn;
      b.f_nm1 = Fm;
      b.out = Ft;
      b.partial = p->cpart;
      CHK(col(p, fch::EPI_AM3, fch::PRO_NONE, b));
      CHK(finalize(p, fch::FIN_AM3, false, true));
      CHK(readback(p));
      CHK(status_from_ctl(p));
      p->stats.fft_calls += 4;
      p->stats.steps += 1;
    } else if (o->scheme == FCH_IMEX) {
      // fused: the step's column pass also starts the F(u~) evaluation
      CHK(ctl_set(p, v));
      ColArgs a = col_args(p);
      a.s0 = cur;
      a.s1 = prev;
      CHK(col(p, fch::EPI_NONE, fch::PRO_EXTRAP, a));
      CHK(row_mu(p, nullptr));
      a.out = spare;
      CHK(col(p, fch::EPI_IMEX, fch::PRO_NEXT_FIELD, a));
      CHK(row_mu(p, nullptr));
      ColArgs b = col_args(p);
      b.s0 = spare;
      b.s1 = cur;
      b.f_n = Fn;
      b.f_nm1 = Fm;
      b.out = Ft;
      b.partial = p->cpart;
      CHK(col(p, fch::EPI_AM3, fch::PRO_NONE, b));
      CHK(finalize(p, fch::FIN_AM3, false, true));
      CHK(readback(p));
      CHK(status_from_ctl(p));
      p->stats.fft_calls += 8;
    } else {
      CHK(sav_or_psd_step(p, o, cur, prev, kt, k_n, spare, rs, &r_new, &it));
      inf.psd_iters += it;
      int32_t acc = 0;
      double kn = 0, e = 0;
      CHK(fch_adapt_dt(p, (const fch_c128*)spare, (const fch_c128*)cur, (const fch_c128*)Fn,
                       (const fch_c128*)Fm, kt, k_n, ad, (fch_c128*)Ft, &acc, &kn, &e));
    }
    const bool accept = p->hctl->accept != 0;
    double k_next = p->hctl->k_next;
    if (o->dyadic) {
      // the step law's proposal k_next (capped and clamped) picks the next
      // ladder size: halve (or lower) after a rejection; after an acceptance
      // double only on the doubled grid, keep, or lower
      const bool clamped = kt < ladder(jt);  // the final step to t_end
      int jn = jt;
      if (accept && !clamped) {
        tu += 1LL << (jt - kJmin);
        const long long coarse = 1LL << (jt + 1 - kJmin);
        if (k_next >= 2.0 * kt && jt < kJmax && tu % coarse == 0)
          jn = jt + 1;
        else if (k_next < kt)
          while (jn > kJmin && ladder(jn) > k_next) --jn;
      } else if (!accept) {
        jn = jt - 1;
        while (jn > kJmin && ladder(jn) > k_next) --jn;
      }
      while (jn > kJmin && ladder(jn) > ad->k_max) --jn;
      while (jn < jt && ladder(jn) < ad->k_min) ++jn;
      jt = jn;
      k_next = ladder(jt);
    }
    if (accept) {
      cd* old_prev = prev;
      prev = cur;
      cur = spare;
      spare = old_prev;
      cd* old_Fm = Fm;
      Fm = Fn;
      Fn = Ft;
      Ft = old_Fm;
      if (o->scheme == FCH_SAV) { rs[1] = rs[0]; rs[0] = r_new; }
      t += kt;
      k_n = kt;
      inf.accepted += 1;
      inf.k_last = kt;
    } else {
      inf.rejected += 1;
      p->stats.rejected += 1;
    }
    kt = k_next;
  }
  inf.t = t;
  inf.k_next = kt;
  CHK(settle(p, B0, B1, cur, prev));
  if (info) {
    inf.fft_calls = p->stats.fft_calls;
    *info = inf;
  }
  return FCH_OK;
}

}  // extern "C"
