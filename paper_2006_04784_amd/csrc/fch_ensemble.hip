// fch_ensemble.hip -- batched ensembles of adaptive runs (BDF2-IMEX, BDF2-SAV or ETDRK2): size
// classes, device-side step control and HIP-graph replay of one attempt.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fch.h"
#include "fch_coef.hpp"
#include "fch_kernels.hpp"
#include "fch_plan.hpp"

using fch::cd;
using fch::EnsMember;

namespace {

struct EnsClass {
  int N = 0, first = 0, count = 0;
  fch_plan_t plan = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t join = nullptr;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
size_t spec_bytes(int N) { return (size_t)(N / 2 + 1) * (size_t)N * sizeof(cd); }

#define HCHK(x)                              \
  do {                                       \
    if ((x) != hipSuccess) return FCH_E_HIP; \
  } while (0)
#define SCHK(x)                   \
  do {                            \
    fch_status s_ = (x);          \
    if (s_ != FCH_OK) return s_;  \
  } while (0)

}  // namespace

struct fch_ensemble_s {
  int count = 0;
  std::vector<fch_params> prm;  // by internal index
  std::vector<int> order;       // user index -> internal index
  fch_ensemble_opts opts;
  std::vector<EnsClass> classes;
  std::vector<EnsMember> hmem;
  std::vector<char> loaded;
  EnsMember* dmem = nullptr;
  EnsMember* pinned = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;       // internal stream: attempts run (and are captured) here
  hipStream_t user_stream = nullptr;  // caller's stream: loads, and the start of a run
  hipEvent_t fork = nullptr;
  hipEvent_t start = nullptr;
  hipEvent_t finish = nullptr;  // end of the attempts queued by fch_ensemble_step
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

// three states, three F spectra, the pair buffer, aux (SAV q / ETDRK2 w), the
// column partials, the umax slots, the E_1 row partials (SAV) and the step log
size_t member_bytes(const fch_ensemble_s* e, int N) {
  const size_t S = a256(spec_bytes(N));
  return 9 * S + a256(sizeof(double) * 2 * (N / 2 + 1)) + a256(sizeof(double) * (size_t)N) +
         a256(sizeof(double) * 2 * (size_t)N) + a256(sizeof(double) * (size_t)e->opts.max_steps);
}

size_t layout(fch_ensemble_s* e, bool assign) {
  size_t off = a256(sizeof(EnsMember) * (size_t)e->count);
  if (assign) e->dmem = (EnsMember*)e->ws;
  for (auto& c : e->classes) {
    const size_t pb = a256(fch_plan_workspace_bytes(c.plan));
    if (assign) fch_plan_set_workspace(c.plan, e->ws + off, pb);
    off += pb;
  }
  for (int i = 0; i < e->count; ++i) {
    const int N = e->prm[i].N;
    const size_t S = a256(spec_bytes(N));
    if (assign) {
      char* b = e->ws + off;
      EnsMember& m = e->hmem[i];
      for (int k = 0; k < 3; ++k) m.ring[k] = (cd*)(b + k * S);
      for (int k = 0; k < 3; ++k) m.fring[k] = (cd*)(b + (3 + k) * S);
      m.P0 = (cd*)(b + 6 * S);
      m.P1 = (cd*)(b + 7 * S);
      m.aux = (cd*)(b + 8 * S);
      char* q = b + 9 * S;
      m.cpart = (double*)q;
      q += a256(sizeof(double) * 2 * (N / 2 + 1));
      m.umaxpart = (double*)q;
      q += a256(sizeof(double) * (size_t)N);
      m.rpart = (double*)q;
      q += a256(sizeof(double) * 2 * (size_t)N);
      m.klog = (double*)q;
      m.klog_cap = e->opts.max_steps;
    }
    off += member_bytes(e, N);
  }
  return off;
}

EnsClass* class_of(fch_ensemble_s* e, int idx) {
  for (auto& c : e->classes)
    if (idx >= c.first && idx < c.first + c.count) return &c;
  return nullptr;
}

// every class: PRO, row, IMEX(+u~ prologue), row, AM3, controller (SAV: PRO,
// row with E_1 partials, SAV, SAV_FIELD, row, AM3; ETDRK2: ETD_PRO, row, ETD2,
// row, AM3); classes on their own streams between a fork and a join on the
// ensemble stream
fch_status enqueue_class(fch_ensemble_s* e, const EnsClass& c, hipStream_t s) {
  const fch::RowVT* rv = c.plan->rv;
  const fch::ColVT* cv = c.plan->cv;
  const int sch = e->opts.scheme;
  HCHK(cv->col_ens(sch == FCH_ETD ? fch::ENS_ETD_PRO : fch::ENS_PRO, e->dmem, c.first, c.count, s));
  HCHK(rv->row_ens(e->dmem, c.first, c.count, fch::ENS_ROW, s));
  if (sch == FCH_SAV) {
    HCHK(cv->col_ens(fch::ENS_SAV, e->dmem, c.first, c.count, s));
    HCHK(cv->col_ens(fch::ENS_SAV_FIELD, e->dmem, c.first, c.count, s));
  } else {
    HCHK(cv->col_ens(sch == FCH_ETD ? fch::ENS_ETD2 : fch::ENS_IMEX, e->dmem, c.first, c.count, s));
  }
  HCHK(rv->row_ens(e->dmem, c.first, c.count, fch::ENS_ROW_TRACK, s));
  HCHK(cv->col_ens(fch::ENS_AM3, e->dmem, c.first, c.count, s));
  HCHK(fch::launch_ens_control(e->dmem, c.first, c.count, s));
  return FCH_OK;
}

fch_status enqueue_attempt(fch_ensemble_s* e) {
  HCHK(hipEventRecord(e->fork, e->stream));
  for (auto& c : e->classes) {
    HCHK(hipStreamWaitEvent(c.stream, e->fork, 0));
    SCHK(enqueue_class(e, c, c.stream));
    HCHK(hipEventRecord(c.join, c.stream));
    HCHK(hipStreamWaitEvent(e->stream, c.join, 0));
  }
  return FCH_OK;
}

// Batched tuning of one size class: every pair of compiled row and column
// variants runs `reps` whole attempts of all the class's members (after one
// untimed attempt), each pair from the same saved member memory, which is
// restored at the end; the fastest pair stays.  Timing the batched launches
// (not a single field's step) matters: with many members per launch the
// best tile and radix choice trades latency for occupancy differently.
fch_status tune_class(fch_ensemble_s* e, EnsClass& c, int reps) {
  const int N = c.N;
  const int nr = fch::row_variant_count(N), nc = fch::col_variant_count(N);
  const size_t region = member_bytes(e, N) * (size_t)c.count;
  char* base = (char*)e->hmem[c.first].ring[0];
  std::vector<EnsMember> saved((size_t)c.count);
  // everything below runs on the ensemble stream, which does not synchronize
  // with the legacy null stream: the snapshot is ordered there too
  HCHK(hipStreamSynchronize(e->user_stream));
  HCHK(hipMemcpyAsync(saved.data(), e->dmem + c.first, sizeof(EnsMember) * c.count,
                      hipMemcpyDeviceToHost, e->stream));
  HCHK(hipStreamSynchronize(e->stream));
  bool any = false;
  for (const auto& m : saved) any |= !m.ctl.done;
  if (!any) return FCH_OK;  // nothing would run
  char* keep = nullptr;
  if (hipMalloc((void**)&keep, region) != hipSuccess) return FCH_E_NOMEM;
  hipEvent_t ev[2] = {nullptr, nullptr};
  fch_status st = FCH_OK;
  // without a snapshot nothing may run, and nothing is restored
  const bool snap =
      hipMemcpyAsync(keep, base, region, hipMemcpyDeviceToDevice, e->stream) == hipSuccess;
  if (!snap || hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
    st = FCH_E_HIP;
  std::vector<EnsMember> trial = saved;
  auto restore = [&](const fch::RowVT* rv) -> fch_status {
    for (auto& m : trial) m.nrow = N / rv->R;
    HCHK(hipMemcpyAsync(base, keep, region, hipMemcpyDeviceToDevice, e->stream));
    HCHK(hipMemcpyAsync(e->dmem + c.first, trial.data(), sizeof(EnsMember) * c.count,
                        hipMemcpyHostToDevice, e->stream));
    return FCH_OK;
  };
  const fch::RowVT* keep_r = c.plan->rv;
  const fch::ColVT* keep_c = c.plan->cv;
  // every pair runs from the same snapshot in three sweeps; its time is the
  // best of the three
  std::vector<float> tbest((size_t)nr * nc, 3.0e38f);
  for (int sweep = 0; sweep < 3 && st == FCH_OK; ++sweep) {
    for (int ri = 0; ri < nr && st == FCH_OK; ++ri) {
      for (int ci = 0; ci < nc && st == FCH_OK; ++ci) {
        c.plan->rv = fch::row_variant(N, ri);
        c.plan->cv = fch::col_variant(N, ci);
        st = restore(c.plan->rv);
        if (st == FCH_OK) st = enqueue_class(e, c, e->stream);  // untimed
        if (st == FCH_OK && hipEventRecord(ev[0], e->stream) != hipSuccess) st = FCH_E_HIP;
        for (int r = 0; r < reps && st == FCH_OK; ++r) st = enqueue_class(e, c, e->stream);
        if (st == FCH_OK && (hipEventRecord(ev[1], e->stream) != hipSuccess ||
                             hipEventSynchronize(ev[1]) != hipSuccess))
          st = FCH_E_HIP;
        float ms = 0.f;
        if (st == FCH_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) st = FCH_E_HIP;
        float& tb = tbest[(size_t)ri * nc + ci];
        if (st == FCH_OK && ms < tb) tb = ms;
      }
    }
  }
  // the fastest pair; pairs within 3% of it are ties, and among ties the first
  // in list order whose row variant takes at most 4 rows per workgroup wins
  // (the 8-row batched variants fetch 1.2-1.8x their algorithmic bytes), so
  // that timing noise does not switch between near-equal variants
  const fch::RowVT* best_r = keep_r;
  const fch::ColVT* best_c = keep_c;
  if (st == FCH_OK) {
    size_t bi = 0;
    for (size_t i = 1; i < tbest.size(); ++i)
      if (tbest[i] < tbest[bi]) bi = i;
    const float tmin = tbest[bi];
    for (size_t i = 0; i < tbest.size(); ++i) {
      if (tbest[i] <= 1.03f * tmin && fch::row_variant(N, (int)(i / nc))->R <= 4) {
        bi = i;
        break;
      }
    }
    best_r = fch::row_variant(N, (int)(bi / nc));
    best_c = fch::col_variant(N, (int)(bi % nc));
  }
  c.plan->rv = (st == FCH_OK) ? best_r : keep_r;
  c.plan->cv = (st == FCH_OK) ? best_c : keep_c;
  if (snap) {
    const fch_status rs = restore(c.plan->rv);
    if (st == FCH_OK) st = rs;
  }
  if (hipStreamSynchronize(e->stream) != hipSuccess && st == FCH_OK) st = FCH_E_HIP;
  for (int k = c.first; k < c.first + c.count; ++k) e->hmem[k].nrow = N / c.plan->rv->R;
  for (auto* x : ev)
    if (x) (void)hipEventDestroy(x);
  (void)hipFree(keep);
  return st;
}

fch_status check_runnable(fch_ensemble_s* e) {
  if (!e->ws) return FCH_E_NOMEM;
  for (int k = 0; k < e->count; ++k)
    if (!e->loaded[k]) return FCH_E_INVALID;
  return FCH_OK;
}

void drop_graph(fch_ensemble_s* e) {
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  e->gexec = nullptr;
  e->graph = nullptr;
}

}  // namespace

extern "C" {

fch_status fch_ensemble_create(const fch_params* members, int32_t count,
                               const fch_ensemble_opts* opts, fch_ensemble_t* out) {
  if (!members || count < 1 || !opts || !out) return FCH_E_INVALID;
  const fch_adapt_opts& ad = opts->adapt;
  if (!(ad.sigma_tol > 0.0) || !(ad.k_min > 0.0) || !(ad.k_max >= ad.k_min) ||
      !(ad.rho_s > 0.0) || std::isnan(ad.cap) || !(opts->t_end > 0.0) || opts->max_steps < 2 ||
      std::isnan(opts->umax_t0) ||
      (opts->scheme != FCH_IMEX && opts->scheme != FCH_SAV && opts->scheme != FCH_ETD) ||
      !(opts->etd.kappa0 >= 0.0) || !(opts->etd.kappa2 >= 0.0) ||
      !std::isfinite(opts->etd.kappa0) || !std::isfinite(opts->etd.kappa2))
    return FCH_E_INVALID;
  for (int i = 0; i < count; ++i) SCHK(fch::validate_params_internal(&members[i]));
  fch_ensemble_s* e = new (std::nothrow) fch_ensemble_s;
  if (!e) return FCH_E_NOMEM;
  e->count = count;
  e->opts = *opts;
  // internal order: by N descending (largest class first), stable
  std::vector<int> idx(count);
  for (int i = 0; i < count; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int a, int b) { return members[a].N > members[b].N; });
  e->order.assign(count, 0);
  e->prm.resize(count);
  for (int k = 0; k < count; ++k) {
    e->order[idx[k]] = k;
    e->prm[k] = members[idx[k]];
  }
  e->hmem.assign(count, EnsMember());
  std::memset(e->hmem.data(), 0, sizeof(EnsMember) * count);
  e->loaded.assign(count, 0);
  fch_status st = FCH_OK;
  for (int k = 0; k < count && st == FCH_OK;) {
    EnsClass c;
    c.N = e->prm[k].N;
    c.first = k;
    while (k < count && e->prm[k].N == c.N) ++k;
    c.count = k - c.first;
    st = fch_plan_create(&e->prm[c.first], &c.plan);
    if (st == FCH_OK &&
        (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&c.join, hipEventDisableTiming) != hipSuccess))
      st = FCH_E_HIP;
    e->classes.push_back(c);
  }
  if (st == FCH_OK && (hipEventCreateWithFlags(&e->fork, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&e->start, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&e->finish, hipEventDisableTiming) != hipSuccess ||
                       hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess ||
                       hipHostMalloc((void**)&e->pinned, sizeof(EnsMember) * count,
                                     hipHostMallocDefault) != hipSuccess))
    st = FCH_E_HIP;
  if (st != FCH_OK) {
    fch_ensemble_destroy(e);
    return st;
  }
  for (int k = 0; k < count; ++k) {
    EnsMember& m = e->hmem[k];
    m.c = fch::consts_from_params(e->prm[k]);
    m.tw = class_of(e, k)->plan->tw;
    m.H = e->prm[k].N / 2 + 1;
    m.ctl.done = 1;  // until loaded
  }
  *out = e;
  return FCH_OK;
}

fch_status fch_ensemble_destroy(fch_ensemble_t e) {
  if (!e) return FCH_E_INVALID;
  drop_graph(e);
  for (auto& c : e->classes) {
    if (c.plan) fch_plan_destroy(c.plan);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    if (c.join) (void)hipEventDestroy(c.join);
  }
  if (e->fork) (void)hipEventDestroy(e->fork);
  if (e->start) (void)hipEventDestroy(e->start);
  if (e->finish) (void)hipEventDestroy(e->finish);
  if (e->stream) (void)hipStreamDestroy(e->stream);
  if (e->pinned) (void)hipHostFree(e->pinned);
  delete e;
  return FCH_OK;
}

fch_status fch_ensemble_set_stream(fch_ensemble_t e, void* stream) {
  if (!e) return FCH_E_INVALID;
  e->user_stream = (hipStream_t)stream;
  for (auto& c : e->classes) fch_plan_set_stream(c.plan, stream);
  return FCH_OK;
}

size_t fch_ensemble_workspace_bytes(fch_ensemble_t e) { return e ? layout(e, false) : 0; }

fch_status fch_ensemble_set_workspace(fch_ensemble_t e, void* dptr, size_t bytes) {
  if (!e || !dptr || ((uintptr_t)dptr & 255)) return FCH_E_INVALID;
  if (bytes < layout(e, false)) return FCH_E_NOMEM;
  drop_graph(e);
  if (e->stream) HCHK(hipStreamSynchronize(e->stream));  // attempts on the old workspace
  e->ws = (char*)dptr;
  e->ws_bytes = bytes;
  layout(e, true);
  // members live in the workspace: a new one holds none of them yet
  for (int k = 0; k < e->count; ++k) {
    e->loaded[k] = 0;
    e->hmem[k].ctl.done = 1;
  }
  HCHK(hipMemcpy(e->dmem, e->hmem.data(), sizeof(EnsMember) * e->count, hipMemcpyHostToDevice));
  return FCH_OK;
}

fch_status fch_ensemble_load(fch_ensemble_t e, int32_t member, const double* u0) {
  if (!e || !u0 || member < 0 || member >= e->count) return FCH_E_INVALID;
  if (!e->ws) return FCH_E_NOMEM;
  const int k = e->order[member];
  EnsClass* c = class_of(e, k);
  fch_plan_t p = c->plan;
  EnsMember& m = e->hmem[k];
  HCHK(hipStreamSynchronize(e->stream));  // attempts still queued on the member
  const fch::Consts keep = p->c;
  p->c = m.c;  // the member's parameters for the setup calls
  // the startup step is clamped to the run like the last step (t_end > 0)
  const double k1 =
      std::min(e->opts.k_first > 0.0 ? e->opts.k_first : e->opts.adapt.k_min, e->opts.t_end);
  const int sch = e->opts.scheme;
  double r0 = 0.0, r1 = 0.0;
  fch_status st = fch_forward(p, u0, (fch_c128*)m.ring[0]);
  if (st == FCH_OK) st = fch_rhs(p, (const fch_c128*)m.ring[0], (fch_c128*)m.fring[0]);
  const fch_c128* u0h = (const fch_c128*)m.ring[0];
  fch_c128* u1h = (fch_c128*)m.ring[1];
  if (st == FCH_OK) {
    if (sch == FCH_SAV) {
      st = fch_sav_r(p, u0h, &r0);
      if (st == FCH_OK) st = fch_step_sav(p, u0h, nullptr, r0, r0, k1, -1.0, u1h, &r1);
    } else if (sch == FCH_ETD) {
      st = fch_step_etd(p, u0h, (const fch_c128*)m.fring[0], k1, &e->opts.etd, u1h);
    } else {
      st = fch_step_imex(p, u0h, nullptr, k1, -1.0, u1h);
    }
  }
  if (st == FCH_OK) st = fch_rhs(p, (const fch_c128*)m.ring[1], (fch_c128*)m.fring[1]);
  p->c = keep;
  SCHK(st);
  m.sav = (sch == FCH_SAV) ? 1 : 0;
  m.rslot = 0;
  m.nrow = m.c.N / p->rv->R;
  m.cur = 1;
  m.prev = 0;
  m.trial = 2;
  m.fn = 1;
  m.fm = 0;
  m.ft = 2;
  m.t = k1;
  m.t_end = e->opts.t_end;
  m.accepted = 1;
  m.rejected = 0;
  m.max_accepted = e->opts.max_steps;
  m.umax = -INFINITY;
  m.umax_t0 = e->opts.umax_t0;
  fch::StepCtl& v = m.ctl;
  std::memset(&v, 0, sizeof(v));
  v.sigma_tol = e->opts.adapt.sigma_tol;
  v.k_min = e->opts.adapt.k_min;
  v.k_max = e->opts.adapt.k_max;
  v.rho_s = e->opts.adapt.rho_s;
  v.cap = e->opts.adapt.cap;
  v.kappa0 = e->opts.etd.kappa0;
  v.kappa2 = e->opts.etd.kappa2;
  v.rring[0] = r1;  // SAV: r^n (slot rslot = 0) and r^{n-1}
  v.rring[2] = r0;
  // Step 0: the first trial step equals the last step
  double kt = k1;
  if (kt > m.t_end - m.t) kt = m.t_end - m.t;
  fch::set_bdf2(v, kt, k1);
  fch::set_am3(v, kt, k1);
  v.done = (m.t >= m.t_end * (1.0 - 1e-14) || m.accepted >= m.max_accepted) ? 1 : 0;
  HCHK(hipStreamSynchronize(p->stream));
  HCHK(hipMemcpy(m.klog, &k1, sizeof(double), hipMemcpyHostToDevice));
  const std::vector<double> ninf((size_t)m.c.N, -INFINITY);
  HCHK(hipMemcpy(m.umaxpart, ninf.data(), sizeof(double) * ninf.size(), hipMemcpyHostToDevice));
  HCHK(hipMemcpy(e->dmem + k, &m, sizeof(EnsMember), hipMemcpyHostToDevice));
  e->loaded[k] = 1;
  return FCH_OK;
}

fch_status fch_ensemble_autotune(fch_ensemble_t e, int32_t reps) {
  if (!e || reps < 1) return FCH_E_INVALID;
  SCHK(check_runnable(e));
  drop_graph(e);  // launch variants change
  for (auto& c : e->classes) SCHK(tune_class(e, c, reps));
  return FCH_OK;
}

namespace {
// captures one attempt of all members into a graph on first use
fch_status ensure_graph(fch_ensemble_s* e) {
  if (e->gexec) return FCH_OK;
  HCHK(hipStreamBeginCapture(e->stream, hipStreamCaptureModeGlobal));
  fch_status st = enqueue_attempt(e);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(e->stream, &g);
  if (st != FCH_OK || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != FCH_OK ? st : FCH_E_HIP;
  }
  e->graph = g;
  if (hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(e);
    return FCH_E_HIP;
  }
  return FCH_OK;
}
}  // namespace

fch_status fch_ensemble_step(fch_ensemble_t e, int32_t attempts, int32_t use_graph) {
  if (!e || attempts < 1) return FCH_E_INVALID;
  SCHK(check_runnable(e));
  if (use_graph) SCHK(ensure_graph(e));
  HCHK(hipEventRecord(e->start, e->user_stream));
  HCHK(hipStreamWaitEvent(e->stream, e->start, 0));
  for (int32_t i = 0; i < attempts; ++i) {
    if (use_graph) {
      HCHK(hipGraphLaunch(e->gexec, e->stream));
    } else {
      SCHK(enqueue_attempt(e));
    }
  }
  HCHK(hipEventRecord(e->finish, e->stream));
  HCHK(hipStreamWaitEvent(e->user_stream, e->finish, 0));
  return FCH_OK;
}

fch_status fch_ensemble_run(fch_ensemble_t e, int64_t max_attempts, int32_t sync_every,
                            int32_t use_graph, fch_ensemble_info* info) {
  if (!e || max_attempts < 1 || sync_every < 1) return FCH_E_INVALID;
  SCHK(check_runnable(e));
  if (use_graph) SCHK(ensure_graph(e));
  // order after the caller's stream
  HCHK(hipEventRecord(e->start, e->user_stream));
  HCHK(hipStreamWaitEvent(e->stream, e->start, 0));
  int64_t attempts = 0;
  int active = e->count;
  while (attempts < max_attempts && active > 0) {
    const int64_t n = std::min<int64_t>(sync_every, max_attempts - attempts);
    for (int64_t i = 0; i < n; ++i) {
      if (use_graph) {
        HCHK(hipGraphLaunch(e->gexec, e->stream));
      } else {
        SCHK(enqueue_attempt(e));
      }
    }
    attempts += n;
    HCHK(hipMemcpyAsync(e->pinned, e->dmem, sizeof(EnsMember) * e->count, hipMemcpyDeviceToHost,
                        e->stream));
    HCHK(hipStreamSynchronize(e->stream));
    active = 0;
    for (int k = 0; k < e->count; ++k) active += e->pinned[k].ctl.done ? 0 : 1;
  }
  bool bad = false;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->attempts = attempts;
    info->active = active;
  }
  for (int k = 0; k < e->count; ++k) {
    if (info) {
      info->accepted += e->pinned[k].accepted;
      info->rejected += e->pinned[k].rejected;
    }
    bad |= e->pinned[k].ctl.nonfinite != 0;
  }
  return bad ? FCH_E_NONFINITE : FCH_OK;
}

fch_status fch_ensemble_member(fch_ensemble_t e, int32_t member, fch_c128* uh, double* klog,
                               fch_member_info* info) {
  if (!e || member < 0 || member >= e->count) return FCH_E_INVALID;
  if (!e->ws) return FCH_E_NOMEM;
  const int k = e->order[member];
  EnsMember m;
  HCHK(hipStreamSynchronize(e->stream));
  HCHK(hipStreamSynchronize(e->user_stream));
  HCHK(hipMemcpy(&m, e->dmem + k, sizeof(EnsMember), hipMemcpyDeviceToHost));
  if (uh)
    HCHK(hipMemcpyAsync(uh, m.ring[m.cur], spec_bytes(e->prm[k].N), hipMemcpyDeviceToDevice,
                        e->user_stream));
  const long long nlog = std::min<long long>(m.accepted, m.klog_cap);
  if (klog && nlog > 0) HCHK(hipMemcpy(klog, m.klog, sizeof(double) * nlog, hipMemcpyDeviceToHost));
  if (info) {
    info->N = e->prm[k].N;
    info->done = m.ctl.done;
    info->nonfinite = m.ctl.nonfinite;
    info->accepted = m.accepted;
    info->rejected = m.rejected;
    info->t = m.t;
    info->k_last = m.ctl.k_n;
    info->k_next = m.ctl.k_next;
    info->err = m.ctl.err;
    info->umax = m.umax;
    info->invalid = m.ctl.invalid;
    info->r_n = m.sav ? m.ctl.rring[m.rslot] : 0.0;
    info->r_nm1 = m.sav ? m.ctl.rring[(m.rslot + 2) % 3] : 0.0;
  }
  return FCH_OK;
}

}  // extern "C"
