// fch_plan.hpp -- the plan object shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "fch.h"
#include "fch_kernels.hpp"

struct fch_plan_s {
  fch_params prm;
  fch::Consts c;
  int N, H;
  const fch::RowVT* rv;
  const fch::ColVT* cv;
  hipStream_t stream;
  fch::SideLane lane;  // the split column passes' side stream (N >= 4096; else null)
  int device;
  fch::cd* tw;
  fch::StepCtl* ctl;
  fch::StepCtl* hctl;  // pinned mirror for read-back
  char* ws;
  size_t ws_bytes;
  fch::cd *P0, *P1, *aux, *st, *Fc[3];
  double *rpart, *cpart;
  fch_stats stats;
  int psd_hint;
  // one-launch PSD solve (k_psd_solve): the compiled pair for N (nullptr if
  // none), its grid (every workgroup resident at once) and whether the
  // fch_step_psd calls use it
  const fch::PsdSolveVT* psd1;
  int psd1_grid, psd1_def_grid, psd1_max_grid;
  int psd1_on;
  // launches read the control block's done code (PSD solves, and the
  // device-scalar calls, whose invalid scalars stop every kernel)
  int check_done;
  // device-controlled adaptive IMEX (fch_run): the run described as one
  // ensemble member, in device memory, with a pinned mirror
  fch::EnsMember* dmem;
  fch::EnsMember* hmem;
  // kernel timing (fch_plan_profile)
  int prof_on;
  int prof_n;
  int* prof_prev;   // index of the timed launch just before on the stream, or -1
  int prof_last;    // last timed launch, -1 after any other stream work
  unsigned long long* prof_ts;  // mode 2: earliest workgroup start per launch (device)
  hipEvent_t* prof_ev;    // 2 per record
  int* prof_kind;
  // HIP-graph replay of the fixed-step fused IMEX chain (fch_plan_set_graph)
  int graph_steps;
  hipStream_t gstream;
  hipEvent_t gfork, gjoin;
  hipGraphExec_t chain_exec;
  const void* chain_key[6];
};


namespace fch {
// model constants of a parameter set (effective eta, alpha_m, wavenumber scale)
Consts consts_from_params(const fch_params& prm);
fch_status validate_params_internal(const fch_params* p);
}  // namespace fch
