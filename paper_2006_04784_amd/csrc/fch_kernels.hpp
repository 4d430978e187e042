// fch_kernels.hpp -- shared declarations between the HIP kernels and the
// host orchestration: argument blocks, the device control block and the
// per-grid-size launch table.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fch_device.hpp"

namespace fch {

// Per-call scalars live in device memory so that a captured launch sequence
// can be replayed with new values (written by ctl_set or by a finalize kernel).
struct StepCtl {
  double k_np1, k_n, a, b, c, gamma;  // BDF2 coefficients (eq. BDF2Coef), u* ratio
  double w1, w2, w3;                  // AM3 weights (eq. Predictor)
  double lambda, tol;                 // PSD search step and stopping tolerance
  double r_n, r_nm1, s_star, r_np1;   // SAV scalars
  double sigma_tol, k_min, k_max, rho_s, cap;
  double err, k_next, ratio, energy, E1;
  double kappa0, kappa2;              // ETDRK2 split constants (eq. ETD-L); step k_np1
  double rring[3];                    // SAV r history of the fused chain, slot n mod 3 = r^n
  int accept, iters, max_iter, fixed_iters;
  int done;       // PSD: 0 running, 1 converged / fixed count reached, 2 max_iter, 3 non-finite;
                  // 4 invalid device scalars (every kernel stops); 5 the one-launch
                  // solve's grid barrier gave up (not every workgroup ran)
  int nonfinite;  // set by any kernel that sees NaN/Inf
  int invalid;    // SAV: E1 + D0 <= 0
  unsigned bar;   // arrivals at the one-launch PSD solve's grid barrier (zeroed with the block)
};

enum RowMode { ROW_MU = 0, ROW_FWD = 1, ROW_INV = 2 };
enum Epi { EPI_NONE = 0, EPI_MU, EPI_F, EPI_IMEX, EPI_SAV, EPI_PSD, EPI_AM3, EPI_ETD1, EPI_ETD2 };
enum Pro {
  PRO_NONE = 0,
  PRO_FIELD,
  PRO_EXTRAP,
  PRO_PSD_INIT,
  PRO_NEXT_EXTRAP,
  PRO_NEXT_FIELD,
  PRO_ETD1,
  PRO_SAV_NEXT,
  PRO_SAV_FIELD
};
enum FinMode { FIN_SAV_S = 0, FIN_PSD, FIN_AM3, FIN_ENERGY };

struct RowArgs {
  Consts c;
  cd* P0;              // pair buffer channel 0 (kx-major), in place (ROW_MU)
  cd* P1;              // pair buffer channel 1
  const double* u_in;  // ROW_FWD physical input
  double* u_out;       // ROW_INV physical output
  const cd* X_in;      // ROW_INV column-inverted input (kx-major)
  cd* X_out;           // ROW_FWD row-transformed output (kx-major)
  double* partial;     // ROW_MU: 2 per workgroup (E_1 density, energy density), nullable
  StepCtl* ctl;
  const cd* tw;        // exp(-2 pi i m / N), m < N
  // ROW_MU inside a PSD solve (nullable): the column partial sums of the
  // previous iteration (psd_ncol pairs), whose stopping test every workgroup
  // evaluates first; psd_iter = the number of iterations that test completes
  const double* psd_part;
  int psd_ncol;
  int psd_iter;
  // device-controlled PSD rounds (nullable): workgroup 0 sets *psd_init_skip
  // (the initial iterate is consumed) and, when the test stops the solve,
  // clears *psd_eval_skip
  int* psd_init_skip;
  int* psd_eval_skip;
  // ROW_MU launches of a PSD solve: the pass returns at once when the
  // control block's done code is set (other launches never read it)
  int check_done;
  // kernel timing (nullable): the earliest workgroup start, in ticks of the
  // device's constant wall clock, is folded in with an atomic minimum
  unsigned long long* tstart;
};

struct ColArgs {
  Consts c;
  cd* P0;
  cd* P1;
  const cd* s0;     // state / field input (u^n, u, u~)
  const cd* s1;     // second input (u^{n-1}, u^n for EPI_AM3, w for EPI_ETD2)
  cd* out;          // output (u^{n+1}, mu, F, PSD iterate, ETD stage u~); may alias s1
  cd* aux;          // SAV q, PSD b u^n + c u^{n-1}, ETD w = u~ - k phi2 N(u^n)
  const cd* guess;  // PSD initial guess (nullable)
  const cd* f_n;    // AM3 F^n; PRO_ETD1 F(u^n)
  const cd* f_nm1;  // AM3 F^{n-1}
  const cd* X_in;   // single-field column transform input
  cd* X_out;        // single-field column transform output
  double* partial;  // 2 per column
  StepCtl* ctl;
  const cd* tw;
  // EPI_SAV (nullable): the row partial sums (E_1 densities, sav_nrow pairs)
  // from which every workgroup forms s*; otherwise ctl->s_star is used
  const double* sav_rpart;
  int sav_nrow;
  // PRO_SAV_NEXT / PRO_SAV_FIELD: the column partial sums (g_p, g_q; sav_ncol pairs) of the
  // SAV step, from which every workgroup solves for r^{n+1}; r^n and r^{n-1}
  // are ctl->rring[rslot] and ctl->rring[(rslot + 2) % 3], r^{n+1} goes to
  // ctl->rring[(rslot + 1) % 3]
  const double* sav_cpart;
  int sav_ncol;
  int rslot;
  unsigned long long* tstart;  // kernel timing (nullable), as in RowArgs
  int check_done;              // as in RowArgs (the launches of a PSD solve)
};

struct FinArgs {
  Consts c;
  const double* rpart;  // row partials (2 per row workgroup)
  int nrow;
  const double* cpart;  // column partials (2 per column)
  int ncol;
  StepCtl* ctl;
  int mode;
};

// One member of a batched ensemble (device memory).  The batched kernels
// read their buffers through the ring slots; the per-member controller
// rotates the slots on accepted steps and writes the next attempt's scalars
// into ctl, so an attempt is a fixed launch sequence that can be captured.
struct EnsMember {
  Consts c;
  StepCtl ctl;  // ctl.done = 1 once the member finished
  const cd* tw;
  cd* ring[3];   // states: slots cur, prev, trial
  cd* fring[3];  // F = Lap mu of the states: slots fn, fm, ft
  cd* P0;
  cd* P1;
  cd* aux;        // ETDRK2 attempts: w = u~ - k phi2 N(u^n) (u~ sits in fring[ft]); SAV: q
  double* rpart;  // SAV attempts: E_1 partial sums of the first row pass (2 per row workgroup)
  double* cpart;  // 2 per column
  double* umaxpart;  // N slots: largest u per row workgroup of the trial evaluation (-inf unused)
  double umax;       // running max of u over the accepted states after the startup step
  double umax_t0;    // ... at t >= umax_t0
  double* klog;   // accepted step sizes
  long long klog_cap;
  int cur, prev, trial, fn, fm, ft;
  int sav;    // SAV attempts: r^n = ctl.rring[rslot], r^{n-1} = ctl.rring[(rslot + 2) % 3]
  int rslot;  // (the controller advances rslot on acceptance)
  int nrow;   // row-pass workgroups (SAV: the E_1 partial pairs)
  double t, t_end;
  long long accepted, rejected, max_accepted;
  int H;
  // adaptive BDF2-PSD under device control (psd = 1): sctl is the solve's
  // control block (BDF2 coefficients, lambda, tolerance, completed iterations,
  // stop code in sctl.done); the attempt's stages run while their flag is 0:
  // psd_init_skip (the initial iterate, cleared by the controller for a new
  // attempt), sctl.done (the iterations) and psd_eval_skip (the F(u~)
  // evaluation and the controller, cleared when the solve stops)
  int psd;
  StepCtl sctl;
  int psd_init_skip, psd_eval_skip;
  int psd_noconv;      // a solve reached max_iter: the run stops
  int psd_last_iters;  // iterations of the latest attempt
  double psd_lambda;   // > 0: fixed search step, else Table SearchSize at the trial step
  long long psd_iters; // iterations of all attempts
};
// IMEX attempt: PRO, row, IMEX, row, AM3; ETDRK2 attempt: ETD_PRO, row, ETD2, row, AM3;
// SAV attempt: PRO, row (E_1 partials), SAV, SAV_FIELD, row, AM3; PSD round:
// PSD_INIT, c x (row with the stopping test, PSD), row, AM3 (the row pass
// that stops the solve leaves the final iterate's column-inverted (u, Lap u)
// in the pair buffer for the evaluation of F(u~))
enum EnsStage {
  ENS_PRO = 0,
  ENS_IMEX = 1,
  ENS_AM3 = 2,
  ENS_ETD_PRO = 3,
  ENS_ETD2 = 4,
  ENS_SAV = 5,
  ENS_SAV_FIELD = 6,
  ENS_PSD_INIT = 7,
  ENS_PSD = 8
};
// row_ens modes: the first evaluation of an attempt, the trial's evaluation
// (tracking the largest u), a PSD iteration (stopping test of the previous one)
enum EnsRow { ENS_ROW = 0, ENS_ROW_TRACK = 1, ENS_ROW_PSD = 2 };

// Launch tables of the compiled variants of one grid size.  Row-pass and
// column-pass variants are chosen independently.
struct RowVT {
  int N, R, E, twl, threads;
  // e0/e1 (nullable): events attached to the dispatch (kernel execution time)
  hipError_t (*row)(int mode, const RowArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  // batched row pass (chemical-potential pieces) over members [first, first+count);
  // mode (EnsRow): ENS_ROW_TRACK also records the largest u per workgroup
  // (into each member's umaxpart); ENS_ROW_PSD is a PSD iteration
  hipError_t (*row_ens)(EnsMember* m, int first, int count, int mode, hipStream_t s);
  // ROW_FWD / ROW_INV over `batch` fields stored back to back
  hipError_t (*row_batch)(int mode, const RowArgs& a, int batch, size_t pstride, size_t sstride,
                          hipStream_t s);
};
// A plan's second stream and two events.  A fused column pass split into its
// columns kx >= 1 and the self-conjugate pair launches the pair on this stream,
// beside the other launch: forked after the work before it, joined before the
// work after it (both are captured into a graph when the plan's stream is).
struct SideLane {
  hipStream_t stream;
  hipEvent_t fork, join;
};

struct ColVT {
  int N, E, twl, threads;
  // side (nullable): the plan's side lane for the split passes (without it
  // their two launches run one after the other)
  hipError_t (*col)(int epi, int pro, const ColArgs& a, hipStream_t s, hipEvent_t e0,
                    hipEvent_t e1, const SideLane* side);
  hipError_t (*col_fwd1)(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  hipError_t (*col_inv1)(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  hipError_t (*col_ens)(int stage, EnsMember* m, int first, int count, hipStream_t s);
  // single-field column transforms (dir -1 forward, +1 inverse) over `batch` fields
  hipError_t (*col1_batch)(int dir, const ColArgs& a, int batch, size_t sstride, hipStream_t s);
};

// One-launch PSD solve of a grid size (k_psd_solve with one fixed pair of
// row and column variants of equal workgroup size): func is the kernel for
// occupancy queries; launch runs it on `grid` persistent workgroups.
struct PsdSolveVT {
  int N, R, ER, rtwl, EC, ctwl, threads;
  const void* func;
  hipError_t (*launch)(const RowArgs& ra, const ColArgs& ca, int limit, int grid, hipStream_t s);
};
const PsdSolveVT* psd_solve_variant(int N);  // nullptr: none compiled for N

// registry: the first entry of each list is the default for N
int row_variant_count(int N);
const RowVT* row_variant(int N, int i);
int col_variant_count(int N);
const ColVT* col_variant(int N, int i);

hipError_t launch_ctl_set(StepCtl* ctl, const StepCtl& v, hipStream_t s);
// device-scalar steps: flags of k_ctl_dev, result kinds of k_ctl_out
enum CtlFlags { CTL_AM3 = 1, CTL_SAV = 2, CTL_LAMBDA = 4, CTL_K1_ONLY = 8 };
enum CtlOut { OUT_STATUS = 0, OUT_SAV = 1, OUT_PSD = 2, OUT_ADAPT = 3, OUT_ENERGY = 4 };
hipError_t launch_ctl_dev(StepCtl* ctl, const StepCtl& v, const double* k_dev,
                          const double* r_dev, double q, int flags, hipStream_t s);
hipError_t launch_ctl_out(const StepCtl* ctl, int what, double* d_out, int* i_out, int* status,
                          hipStream_t s);
hipError_t launch_finalize(const FinArgs& a, hipStream_t s);
// SAV combine u^{n+1} = p + r^{n+1} q, the r-solve done in every workgroup
hipError_t launch_sav_combine(cd* out, const cd* q, StepCtl* ctl, size_t n, const double* cpart,
                              int ncol, double pars, hipStream_t s);
// per-member AM3 decision, slot rotation and next-attempt scalars
hipError_t launch_ens_control(EnsMember* m, int first, int count, hipStream_t s);

}  // namespace fch
