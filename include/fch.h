/*
 * fch.h -- C ABI of the MI355X (gfx950) engine for the functionalized
 * Cahn-Hilliard (FCH) gradient flow with Fourier pseudo-spectral space
 * discretization and variable-step BDF2 time stepping.
 *
 * Model (paper Sec. 2): energy eq. Functional with the regularized well W_q
 * of eq. e:Wq-def; H^{-1} gradient flow u_t = Lap mu, mu = dE/du (eqs. sFCH,
 * FCH) on the periodic square [0, L)^2, N x N collocation points.
 *
 * Conventions shared by every call
 *  - Precision: IEEE FP64 throughout.
 *  - Memory: every array argument is a DEVICE pointer (HIP global memory)
 *    owned by the caller; scalars marked "host" are host memory.  The plan
 *    owns its twiddle table and a small control block, nothing else.
 *  - Physical field: double u[y*N + x], y = row index (coordinate y*h),
 *    x = column index, h = L/N.
 *  - Spectral field ("half spectrum", kx-major): fch_c128 uh[kx*N + ky],
 *    kx = 0..N/2 (N/2+1 columns), ky = 0..N-1; wavenumbers 2*pi*kx/L and
 *    2*pi*(ky <= N/2 ? ky : ky-N)/L.  This is the transpose of the
 *    numpy.fft.rfft2 layout.  Forward transforms are unnormalized; the inverse
 *    carries 1/N^2 and returns the real part of the inverse DFT of the
 *    Hermitian extension (imaginary parts at kx = 0 and kx = N/2 are ignored).
 *  - The state of every time stepper is the half spectrum; physical fields
 *    appear only through fch_forward / fch_inverse.
 *  - Streams: all work is enqueued on the plan's stream (fch_plan_set_stream)
 *    and calls return without synchronizing, except where an output is a host
 *    scalar (then the call waits for that value).
 *  - Aliasing: outputs must not alias inputs, except uh_np1 == uh_nm1 where
 *    stated (every column is read before it is written).
 *  - Errors: status codes only; nothing aborts.  Invalid arguments leave all
 *    outputs untouched.  A plan is bound to one device and is not
 *    thread-safe; calls on one plan must not overlap.
 */
#ifndef FCH_H
#define FCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fch_plan_s* fch_plan_t;
typedef struct { double re, im; } fch_c128;

typedef enum {
    FCH_OK = 0,
    FCH_E_INVALID = -1,     /* bad argument (size, null pointer, E1 + D0 <= 0, ...) */
    FCH_E_UNSUPPORTED = -2, /* N outside the supported powers of two 16..4096       */
    FCH_E_HIP = -3,         /* a HIP runtime call failed                            */
    FCH_E_NOMEM = -4,       /* workspace missing or too small                        */
    FCH_E_NOCONV = -5,      /* PSD reached max_iter; last iterate and stats written  */
    FCH_E_NONFINITE = -6    /* a reduction saw a NaN or Inf                          */
} fch_status;

/* Model parameters (paper Table t:Benchmark notation). */
typedef struct {
    int32_t N;                 /* grid points per side: power of two, 16..4096      */
    double  L;                 /* side of the periodic square, > 0                  */
    double  eps;               /* interface width epsilon, > 0                      */
    double  eta1, eta2;        /* functionalization parameters as given             */
    int32_t p;                 /* effective eta_i = eps^p * eta_i (p = 1 gives the
                                  paper's eta_1 = 1.45 eps, eta_2 = 3 eps form)     */
    double  q;                 /* well regularization q >= 0 (eq. e:Wq-def)         */
    double  gamma_w;           /* well asymmetry gamma (0.3)                        */
    double  b_minus, b_plus;   /* well minima (-1, +1)                              */
    double  beta1, beta2;      /* stabilization of L_0 (eq. e:SAV-L0) in SAV and IMEX,
                                  (2, 1) = L_IMEX                                    */
    double  zeta, D0;          /* SAV splitting constant (eq. 4.1) and energy shift
                                  D_0 > -min E_1 (Sec. 3.5); see fch_sav_constants */
} fch_params;

/* Default SAV constants: zeta = ceil(10 max(0, -min_u W_q''))/10 and
 * D0 = |Omega| (max(0, -min_u [W_q'^2/2 - eta2 W_q]) + 1), minima over a fine
 * sample of u in [-3, 3].  Host-only; writes *zeta and *D0. */
fch_status fch_sav_constants(const fch_params* prm, double* zeta, double* D0);

/* alpha_m = W_q''(b_-) (Sec. 3.3), host-only. */
double fch_alpha_m(const fch_params* prm);

/* ---- plan ---------------------------------------------------------------- */
/* Creates a plan on the current HIP device.  Allocates the twiddle table and a
 * control block (device) and a small pinned host block.  *out is set on
 * success only. */
fch_status fch_plan_create(const fch_params* prm, fch_plan_t* out);
fch_status fch_plan_destroy(fch_plan_t plan);
/* stream: a hipStream_t (NULL = the null stream). */
fch_status fch_plan_set_stream(fch_plan_t plan, void* stream);
/* Device workspace the caller must provide before any compute call
 * (intermediate half spectra, reduction partials).  No compute call allocates. */
size_t     fch_plan_workspace_bytes(fch_plan_t plan);
fch_status fch_plan_set_workspace(fch_plan_t plan, void* dptr, size_t bytes);
/* Launch configuration of the two kernel families: the row pass (R rows per
 * workgroup, row_E FFT elements per thread, twiddle table in LDS when
 * row_twl = 1, else read through the vector caches) and the column pass
 * (col_E FFT elements per thread, one column per workgroup, twiddles in LDS
 * when col_twl = 1).  NULL selects
 * the built-in default for N.  FCH_E_UNSUPPORTED for a configuration that was
 * not compiled. */
typedef struct { int32_t row_R, row_E, row_twl, col_E, col_twl; } fch_launch_cfg;
fch_status fch_plan_set_config(fch_plan_t plan, const fch_launch_cfg* cfg);
/* One-launch PSD solve (Sec. 3.3): the iterations of fch_step_psd and
 * fch_step_psd_dev run in a single persistent kernel whose workgroups, all
 * resident at once, alternate the row pass and the column pass with device-
 * wide barriers and stop on the stopping test evaluated on the device, so a
 * captured solve is two launches whatever its iteration count or max_iter.
 * Each barrier costs an agent-scope cache release and acquire per
 * workgroup, so an iteration takes 1.4-2.2x as long as with separate
 * launches (256^2: 24 against 16 us; 1024^2: 91 against 42 us): it pays
 * where a captured solve's max_iter far exceeds its iterations (the separate
 * launches of a converged solve still cost about 2.4 us each).  Off by
 * default.  Compiled for N = 256, 512, 1024 and 2048 with one fixed pair of
 * row and column variants (launch cfg 2,8,0 | 4,0 up to 1024; 2,16,0 | 8,0 at
 * 2048), independent of fch_plan_set_config; the default grid is one
 * workgroup per CU (fewer when a phase has fewer tasks).  A barrier that
 * waits half a second gives up; the solve then returns FCH_E_HIP (status -3
 * from the _dev call).
 * set: on = 1 or 0; grid > 0 sets the number of persistent workgroups (at
 * most what the device holds at once, else FCH_E_INVALID), grid <= 0 the
 * default; FCH_E_UNSUPPORTED for on = 1 without the solve for N.
 * get (host out): on, and its grid size (nullable; 0 without it). */
fch_status fch_plan_set_psd_solve(fch_plan_t plan, int32_t on, int32_t grid);
fch_status fch_plan_get_psd_solve(fch_plan_t plan, int32_t* on, int32_t* grid);
fch_status fch_plan_get_config(fch_plan_t plan, fch_launch_cfg* cfg);
/* Compiled variants for a grid size: row-pass variants (row fields of cfg)
 * and column-pass variants (col fields of cfg). */
int32_t    fch_row_config_count(int32_t N);
int32_t    fch_col_config_count(int32_t N);
fch_status fch_config_get(int32_t N, int32_t row_i, int32_t col_i, fch_launch_cfg* cfg);
/* Autotuner: runs the fused BDF2-IMEX chain (row pass, then column pass with
 * the next step's prologue, back to back) for every pair of compiled row-pass
 * and column-pass variants on scratch copies of the given state, reps steps
 * per chain (at least 2, at most N-1), in three timed sweeps after a warm-up
 * sweep, and keeps the pair with the shortest chain time per step (HIP events
 * around the chain; best of the sweeps).  Pairs within 1% of the fastest are
 * ties, resolved by list order, so the choice does not follow timing noise.
 * uh_n, uh_nm1 are read only (copied into the workspace); k is the step used.
 * best (host out, nullable) receives the choice; us (host out, nullable, 2
 * doubles) the chosen row and column passes' average shares of the chain in
 * microseconds (device clock, launch start to launch start).  Synchronizes
 * the plan's stream. */
fch_status fch_autotune(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1, double k,
                        int32_t reps, fch_launch_cfg* best, double* us);

typedef struct {
    int64_t fft_calls;     /* 2D real transforms (forward or inverse) of one N^2 field */
    int64_t launches;      /* kernels enqueued                                        */
    int64_t psd_iters;     /* PSD iterations performed                                */
    int64_t steps, rejected;
} fch_stats;
fch_status fch_plan_stats(fch_plan_t plan, fch_stats* out);   /* host out */
fch_status fch_plan_reset_stats(fch_plan_t plan);

/* Kernel timing.  While enabled, every row-pass and column-pass launch of the
 * steppers is timed (up to 16384 launches; later launches are not timed).
 * enable = 1: HIP events are recorded on the plan's stream before and after
 * each launch, so an interval also holds the dispatch of its kernel.
 * enable = 2: nothing enters the stream; each launch writes its start (the
 * earliest of its first eight workgroups on the device's constant wall
 * clock) to a device slot, and
 * a launch's time is the interval to the next launch's start, counted only
 * when that launch follows it directly on the stream (no other kernel, copy
 * or host wait in between): the kernel's share of a back-to-back chain.
 * Enabling mode 2 the first time allocates its slots (128 KiB of device
 * memory).  fch_plan_profile_read waits for the stream, sums
 * the elapsed times per kernel class and clears the records.  Classes:
 * 0 row pass (pointwise chemical potential), 1 column pass (forward FFT +
 * epilogue + inverse FFT), 2 column pass (one direction only),
 * 3 single-field transforms (fch_forward / fch_inverse passes; mode 1 only). */
typedef struct { int64_t count[4]; double ms[4]; } fch_profile;
fch_status fch_plan_profile(fch_plan_t plan, int32_t enable);
fch_status fch_plan_profile_read(fch_plan_t plan, fch_profile* out);
/* Replay of the fixed-step fused BDF2-IMEX chain of fch_run (Sec. 3.4) as a
 * HIP graph of `steps` steps (even, 2..256; 0 disables, the default).  The
 * graph runs on an internal stream ordered after the plan's stream, and the
 * plan's stream is ordered after it, so callers see the same stream
 * semantics.  Enabling creates that stream and two events; fch_run
 * instantiates one graph per (uh_n, uh_nm1) buffer pair, workspace and launch
 * configuration on first use (the HIP runtime's graph objects are the only
 * allocations).  Results are bit-identical to the unreplayed path: the same
 * kernels run in the same order.  Ignored while kernel timing is on.
 * FCH_E_INVALID for an odd or out-of-range count. */
fch_status fch_plan_set_graph(fch_plan_t plan, int32_t steps);

/* ---- transforms (pseudo-spectral discretization, Sec. 2.3 / Sec. 3) ------ */
/* uh = DFT(u), unnormalized.  u: N*N doubles; uh: (N/2+1)*N complex. */
fch_status fch_forward(fch_plan_t plan, const double* u, fch_c128* uh);
/* u = real part of IDFT(Hermitian extension of uh) / N^2. */
fch_status fch_inverse(fch_plan_t plan, const fch_c128* uh, double* u);
/* The same transforms over `batch` fields (1..65535) stored back to back:
 * u holds batch*N*N doubles, uh batch*(N/2+1)*N complex values, field b at
 * offset b*N*N and b*(N/2+1)*N.  Field b of the result equals fch_forward /
 * fch_inverse of field b bit for bit.  fch_forward_batch needs no workspace:
 * the row pass writes uh and the column pass transforms it in place.
 * fch_inverse_batch leaves uh unchanged and stages the column-inverted
 * spectra in ws, caller-owned device memory of at least
 * fch_inverse_batch_ws_bytes(plan, batch) = batch*16*N*(N/2+1) bytes
 * (FCH_E_INVALID if smaller).  Neither needs fch_plan_set_workspace.
 * u and uh must not overlap, nor ws either of them. */
fch_status fch_forward_batch(fch_plan_t plan, int32_t batch, const double* u, fch_c128* uh);
size_t     fch_inverse_batch_ws_bytes(fch_plan_t plan, int32_t batch);
fch_status fch_inverse_batch(fch_plan_t plan, int32_t batch, const fch_c128* uh, double* u,
                             void* ws, size_t ws_bytes);

/* ---- chemical potential (eq. FCH) ---------------------------------------- */
/* muh = half spectrum of mu(u) = (eps^2 Lap - W''(u)) omega + eps^2 eta1 Lap u
 * - eta2 W'(u), omega = eps^2 Lap u - W'(u); Laplacians as -|k|^2, products at
 * collocation points (no dealiasing).  energy (nullable, host out): the
 * discrete energy of eq. Functional, h^2 sum [omega^2/2 - eta2 W]
 * - (eps^2 eta1/2) ||grad u||^2 with the gradient term by Parseval. */
fch_status fch_chem_potential(fch_plan_t plan, const fch_c128* uh, fch_c128* muh,
                              double* energy);
/* The same evaluation with every output in device memory and nothing read
 * back (graph-capturable): muh as above; mu_phys (nullable, device, N x N
 * doubles, row-major, overlapping neither uh nor muh): mu on the grid, the
 * inverse transform of muh; energy_dev (nullable, device double): the energy
 * above; status_dev (nullable, device int32): 0, or -6 when a non-finite
 * value appeared.  FCH_E_INVALID for null or overlapping arrays. */
fch_status fch_chem_potential_dev(fch_plan_t plan, const fch_c128* uh, fch_c128* muh,
                                  double* mu_phys, double* energy_dev, int32_t* status_dev);

/* ---- BDF2 steps (eqs. BDF2Coef, BDF2-general) ---------------------------- */
/* Every step solves a u^{n+1} + b u^n + c u^{n-1} = (scheme's Lap mu) with
 * a, b, c from (k_np1, k_n).  k_n <= 0 selects the first-order startup step
 * (a = 1/k, b = -1/k, c = 0, u* = u^n); uh_nm1 is then not read and may be
 * NULL.  uh_np1 may alias uh_nm1. */

/* BDF2-IMEX (eqs. e:IMEX-op, IMEX, Richardson, IMEX-eq):
 * (a + |k|^2 L) u^{n+1} = -b u^n - c u^{n-1} - |k|^2 (mu(u*) - L u*),
 * u* = u^n + (k_np1/k_n)(u^n - u^{n-1}), with the stabilized
 * L = L_0 = eps^4 |k|^4 + beta1 alpha_m eps^2 |k|^2 + beta2 alpha_m^2 of eq. e:SAV-L0
 * (the plan's beta1, beta2), which is L_IMEX = (eps^2 |k|^2 + alpha_m)^2 at the
 * default beta = (2, 1); other values give the IMEX family of Figure Find-Beta. */
fch_status fch_step_imex(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                         double k_np1, double k_n, fch_c128* uh_np1);

/* The same BDF2-IMEX step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It needs no fch_plan_set_workspace: its two intermediate half
 * spectra live in a library-owned device array of 2 * 16 * N_max * (N_max/2+1)
 * bytes (4.02 MiB at N_max = FCH_STATIC_MAX_N = 512), which each GPU the
 * library runs on holds until the process ends.  It calls no hipMalloc,
 * hipFree or allocating library routine; the plan (created beforehand, on
 * this device) supplies twiddles and the control block.  Results equal
 * fch_step_imex's bit for bit under the same launch configuration.
 * FCH_E_UNSUPPORTED if the plan's N exceeds FCH_STATIC_MAX_N; other argument
 * rules as fch_step_imex.  Every call on one GPU shares that GPU's array and
 * leaves its contents behind (nothing in it has to start at zero): calls
 * that overlap on one GPU, from any plan, stream or thread, race and must be
 * serialized by the caller. */
#define FCH_STATIC_MAX_N 512
fch_status fch_step_imex_static(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                                double k_np1, double k_n, fch_c128* uh_np1);

/* BDF2-SAV (eqs. 4.7, 4.8) with L_0, L_1 of eqs. e:SAV-L0, e:SAV-L1:
 * u^{n+1} = p + r^{n+1} q, (a + |k|^2 L_0) p = -b u^n - c u^{n-1} - |k|^2 L_1 u*,
 * (a + |k|^2 L_0) q = -|k|^2 X, X = V(u*)/sqrt(E_1(u*) + D_0), V = mu - L_SAV u,
 * r^{n+1} = (-b r^n - c r^{n-1} + (X, a p + b u^n + c u^{n-1})/2) / (a - a (X, q)/2).
 * r_n, r_nm1 host scalars; *r_np1 host out.  FCH_E_INVALID if E_1(u*) + D_0 <= 0. */
fch_status fch_step_sav(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                        double r_n, double r_nm1, double k_np1, double k_n,
                        fch_c128* uh_np1, double* r_np1);
/* SAV scalar r = sqrt(E_1(u) + D_0) of a state (host out). */
fch_status fch_sav_r(fch_plan_t plan, const fch_c128* uh, double* r);

/* BDF2-PSD (eq. residual, Sec. 3.3): iterate d = -L_PSD^{-1} R(u_s),
 * u_{s+1} = u_s + lambda d with R = Pi_0 mu(u) - Lap^{-1}(a u + b u^n + c u^{n-1}),
 * L_PSD = eps^4 Lap^2 - 2 alpha eps^2 Lap + alpha^2 - a Lap^{-1}; stop once
 * ||d_s|| / ||u_{s+1}|| < tol.  guess (nullable): initial iterate, projected to
 * the mean of u^n; NULL selects the extrapolation of eq. recurrence.
 * lambda <= 0 selects Table SearchSize (linear in k; q in {0, 0.2, 0.5}).
 * fixed_iters > 0 runs exactly that many iterations (tol ignored).
 * Returns FCH_E_NOCONV after max_iter iterations (uh_np1 holds the last
 * iterate).  stats (nullable, host out). */
typedef struct { double tol; int32_t max_iter; double lambda; int32_t fixed_iters; } fch_psd_opts;
typedef struct { int32_t iters; int64_t fft_calls; double last_ratio; } fch_psd_stats;
fch_status fch_step_psd(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                        double k_np1, double k_n, const fch_c128* guess,
                        const fch_psd_opts* opts, fch_c128* uh_np1, fch_psd_stats* stats);

/* ---- ETDRK2 (Sec. 3.6, eqs. ODE, ETDRK1, ETDRK2, ETD-L) ------------------- */
/* u_t = L u + N(u) with the split of eq. ETD-L,
 *   L = Lap (eps^4 Lap^2 - 2 alpha eps^2 Lap + alpha^2) - kappa0 + kappa2 eps^2 Lap,
 *   N(u) = Lap N_IMEX(u) + kappa0 u - kappa2 eps^2 Lap u   (so L u + N(u) = Lap mu),
 * and one step of size k:
 *   u~      = e^{Lk} u^n + L^{-1}(e^{Lk} - I) N(u^n)                (eq. ETDRK1)
 *   u^{n+1} = u~ + L^{-1}[L^{-1}(e^{Lk} - I) - k I](N(u~) - N(u^n))/k (eq. ETDRK2).
 * L is diagonal in Fourier space and never positive; the multipliers are
 * formed per wavenumber at z = L k as e^z, k (e^z - 1)/z, k (e^z - 1 - z)/z^2
 * (a Taylor polynomial for |z| <= 1/2).  opts: kappa0, kappa2 >= 0; NULL
 * selects the paper's 1e-2 and 15.  F_n (nullable): F(u^n) = Lap mu(u^n) as
 * written by fch_rhs or fch_adapt_dt; with it the step evaluates the chemical
 * potential once (4 FFT calls), without it twice (8).  uh_np1 may alias uh_n
 * or F_n.  Device pointers; no synchronization. */
typedef struct { double kappa0, kappa2; } fch_etd_opts;
fch_status fch_step_etd(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* F_n, double k,
                        const fch_etd_opts* opts, fch_c128* uh_np1);

/* ---- adaptive time step (Sec. 3.2, Steps 2-4) ---------------------------- */
/* F_trial = F(u~) = Lap mu(u~) (device out, the next step's cache);
 * u_p = u^n + (k~/6)[(3+2g)/(1+g) F(u~) + (3+g) F^n - g^2/(1+g) F^{n-1}], g = k~/k_n;
 * e = ||u~ - u_p|| / ||u_p|| (Parseval); accept = (e <= sigma_tol or k~ <= k_min);
 * k_next = max(k_min, min(rho_s (sigma_tol/e)^{1/3} k~, k_max, cap k~)), cap <= 0
 * disables the zero-stability cap.  accept, k_next, err: host outs (nullable). */
typedef struct { double sigma_tol, k_min, k_max, rho_s, cap; } fch_adapt_opts;
fch_status fch_adapt_dt(fch_plan_t plan, const fch_c128* uh_trial, const fch_c128* uh_n,
                        const fch_c128* F_n, const fch_c128* F_nm1, double k_trial, double k_n,
                        const fch_adapt_opts* opts, fch_c128* F_trial,
                        int32_t* accept, double* k_next, double* err);
/* F(u) = Lap mu(u) as a half spectrum (device out). */
fch_status fch_rhs(fch_plan_t plan, const fch_c128* uh, fch_c128* Fh);

/* ---- the steps with device-resident scalars (graph-capturable) ------------
 * Same operations as fch_step_imex / fch_step_sav / fch_step_psd /
 * fch_step_etd / fch_adapt_dt (same kernels; results bit-identical for the
 * same values),
 * but every per-step scalar is read from device memory when the launched
 * kernels run, every scalar result is written to device memory, and nothing
 * allocates, synchronizes or copies to the host.  A sequence of these calls
 * can therefore be captured into a HIP graph on the plan's stream and replayed
 * after writing new values into the scalar buffers.
 *   k_dev[2]      = (k_{n+1}, k_n), doubles; k_n <= 0 selects the first-order
 *                   startup step (eq. BDF2Coef with u^{n-1} unused, but uh_nm1
 *                   must still point at a finite field, e.g. uh_n).
 *   r_dev[2]      = (r^n, r^{n-1}) (SAV, eq. 4.8); r_np1_dev: r^{n+1} out.
 *   iters_dev     = PSD iterations taken (int32, out).
 *   out_dev[3]    = (accept as 1.0 / 0.0, k_next, err) (adaptivity, out).
 *   status_dev    = int32 out (nullable): 0 ok, FCH_E_INVALID (k not positive
 *                   and finite, k_n <= 0 for fch_adapt_dt_dev, untabulated q
 *                   for the lambda table), FCH_E_NOCONV (PSD limit reached),
 *                   FCH_E_NONFINITE.
 * All pointers are device pointers.  The host return value covers only the
 * host-side checks (null pointers, aliasing, options).  fch_step_psd_dev
 * launches opts->max_iter (or fixed_iters) iterations, a number fixed when
 * the calls are captured (the graph API of this HIP has no conditional
 * nodes); once converged the remaining launches return at once, so a caller
 * capturing it sets max_iter near the expected count.  fch_run's adaptive
 * PSD needs no such bound: it queues rounds sized from the latest attempt. */
fch_status fch_step_imex_dev(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                             const double* k_dev, fch_c128* uh_np1, int32_t* status_dev);
fch_status fch_step_sav_dev(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                            const double* r_dev, const double* k_dev, fch_c128* uh_np1,
                            double* r_np1_dev, int32_t* status_dev);
fch_status fch_step_psd_dev(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* uh_nm1,
                            const double* k_dev, const fch_c128* guess,
                            const fch_psd_opts* opts, fch_c128* uh_np1, int32_t* iters_dev,
                            int32_t* status_dev);
/* ETDRK2 step of fch_step_etd with k = k_dev[0] read on the device (k_dev[1]
 * is not read); status_dev as above. */
fch_status fch_step_etd_dev(fch_plan_t plan, const fch_c128* uh_n, const fch_c128* F_n,
                            const double* k_dev, const fch_etd_opts* opts, fch_c128* uh_np1,
                            int32_t* status_dev);
fch_status fch_adapt_dt_dev(fch_plan_t plan, const fch_c128* uh_trial, const fch_c128* uh_n,
                            const fch_c128* F_n, const fch_c128* F_nm1, const double* k_dev,
                            const fch_adapt_opts* opts, fch_c128* F_trial, double* out_dev,
                            int32_t* status_dev);

/* ---- trajectories -------------------------------------------------------- */
/* Runs a scheme on the device state.  On entry uh_n holds u^n and uh_nm1
 * u^{n-1} (ignored when opts->startup = 1: a first-order step of size
 * k_first is taken from uh_n).  On return uh_n holds the last accepted state
 * and uh_nm1 the one before it.  Fixed-step runs (adaptive = 0) take nsteps
 * steps of size k (the startup step counts as one); adaptive runs follow
 * Sec. 3.2 until t_end or nsteps accepted steps, their startup step being
 * min(k_first, t_end) (k_first <= 0 selects adapt.k_min).  *rs (SAV only, host in/out):
 * r^n, r^{n-1}.  info (nullable, host out).
 * FCH_ETD (ETDRK2 with opts->etd, taken as given: zeros mean kappa0 = kappa2 = 0,
 * not the paper's values) is a one-step method: fixed runs take
 * nsteps ETDRK2 steps and ignore startup and the entering uh_nm1.  Adaptive
 * ETD runs take the startup step as one ETDRK2 step of k_first without error
 * control (the estimate needs F^{n-1}), then follow Sec. 3.2 with the ETDRK2
 * result as the primary approximation of Step 1; each attempt starts from
 * the cached F(u^n) (8 FFT calls, as for IMEX).
 * Adaptive attempts run under device control: a controller kernel accepts or
 * rejects, rotates the buffers and sets the next trial step, and the host
 * waits only between chunks of queued attempts.  Adaptive PSD attempts are
 * queued as rounds (the initial iterate; a number of iterations, each row pass
 * first evaluating the previous iteration's stopping test; the F(u~)
 * evaluation with the error estimate, starting from the final iterate's
 * column transform that the last iteration left; the controller), each stage running
 * only in its phase of the attempt, so an attempt that outruns its round
 * continues in the next; the iterations per round follow the latest
 * attempt's count.  A solve that reaches max_iter stops the run with
 * FCH_E_NOCONV, the last accepted state in uh_n.  With kernel timing on
 * (fch_plan_profile) the attempts run from a host loop instead, with the same
 * results. */
typedef enum { FCH_IMEX = 0, FCH_SAV = 1, FCH_PSD = 2, FCH_ETD = 3 } fch_scheme;
typedef struct {
    int32_t scheme, adaptive, startup;
    int64_t nsteps;
    double  k, k_prev, k_first, t_end;
    fch_adapt_opts adapt;
    fch_psd_opts psd;
    fch_etd_opts etd;
    /* dyadic = 1 (adaptive runs): nested factor-of-two step sizes, the
     * adaptive strategy the paper pairs with SAV's fixed-step energy law
     * (Sec. 1, Sec. 5.2): every step is k_first 2^j (the first trial when
     * startup = 0, k); a rejected step is halved (or cut to the largest such
     * size not above the step law's proposal); after an accepted step the
     * size doubles only when the proposal allows it and the new time lies on
     * the grid of the doubled size (so coarse steps nest over fine ones),
     * stays when the proposal allows it, and otherwise drops to the largest
     * ladder size not above the proposal; always within [k_min, k_max] on the
     * ladder, the last step clamped to t_end.  Attempts then run from the host
     * loop.  0: the step law of Sec. 3.2. */
    int32_t dyadic;
} fch_run_opts;
typedef struct {
    int64_t accepted, rejected, psd_iters, fft_calls;
    double  t, k_last, k_next;
} fch_run_info;
fch_status fch_run(fch_plan_t plan, const fch_run_opts* opts, fch_c128* uh_n, fch_c128* uh_nm1,
                   double* rs, fch_run_info* info);

/* ---- batched ensembles ---------------------------------------------------- */
/* Many independent adaptive runs (Sec. 3.2 step control, each member with its
 * own parameters, state and step size) advanced together, all with one scheme:
 * BDF2-IMEX (the default), BDF2-SAV (each member's r history on the device) or
 * ETDRK2.  The description below is for IMEX; SAV attempts add a column pass
 * (the r-solve and the trial) after the SAV step, and ETDRK2 attempts start
 * from the cached F(u^n).
 * Members are grouped by N into size classes; an attempt runs, for every
 * class, the batched column pass (u*, Lap u*), row pass, column pass (the
 * IMEX step, then u~, Lap u~), row pass, column pass (F(u~), AM3 sums) and a
 * per-member controller that accepts or rejects, picks the next step and
 * rotates the state and F buffers on the device.  Classes run on their own
 * streams; with use_graph the whole attempt is captured once into a HIP
 * graph and replayed.  The host reads member status every sync_every
 * attempts.  Members finish at t_end or after max_steps accepted steps. */
typedef struct fch_ensemble_s* fch_ensemble_t;
typedef struct {
    fch_adapt_opts adapt;
    double  t_end;       /* end time of every member                              */
    int64_t max_steps;   /* cap on accepted steps per member (startup included)   */
    double  k_first;     /* startup step (<= 0: adapt.k_min), at most t_end       */
    double  umax_t0;     /* umax counts the accepted states at t >= umax_t0        */
    int32_t scheme;      /* FCH_IMEX (0), FCH_SAV or FCH_ETD for every member      */
    fch_etd_opts etd;    /* FCH_ETD: kappa0, kappa2, taken as given                */
} fch_ensemble_opts;
typedef struct { int64_t attempts, accepted, rejected; int32_t active; } fch_ensemble_info;
typedef struct {
    int32_t N, done, nonfinite;
    int32_t invalid;  /* SAV: E_1 + D_0 <= 0 at a stage state; the member stopped */
    int64_t accepted, rejected;
    double  t, k_last, k_next, err;
    double  umax;   /* running max of u over the accepted states after the startup
                       step at t >= opts.umax_t0 (-inf before the first); the
                       defect-onset indicator of Sec. 5.1 and Table f:defect-onsetR */
    double  r_n, r_nm1;  /* SAV: the auxiliary scalar r of the last two accepted
                            states (eq. 4.8); 0 for the other schemes */
} fch_member_info;
/* Host-side setup: one plan (twiddles, launch variants) per size class on the
 * current device.  members: count parameter sets (N in 16..4096). */
fch_status fch_ensemble_create(const fch_params* members, int32_t count,
                               const fch_ensemble_opts* opts, fch_ensemble_t* out);
fch_status fch_ensemble_destroy(fch_ensemble_t ens);
fch_status fch_ensemble_set_stream(fch_ensemble_t ens, void* stream);
/* Device workspace for every member (three states, three F spectra, the
 * pair buffer, partial sums, the step log) and each class plan.  Setting a
 * workspace (again) leaves every member unloaded: load them before a run. */
size_t     fch_ensemble_workspace_bytes(fch_ensemble_t ens);
fch_status fch_ensemble_set_workspace(fch_ensemble_t ens, void* dptr, size_t bytes);
/* Loads member i from a physical N*N state (device): forward transform,
 * F(u^0), a startup step of size k_first (first-order BDF for IMEX and SAV,
 * with r^0 = sqrt(E_1(u^0) + D_0); an ETDRK2 step), F(u^1).  Synchronizes. */
fch_status fch_ensemble_load(fch_ensemble_t ens, int32_t member, const double* u0);
/* Autotunes each size class's launch variants on the batched work itself:
 * every compiled (row, column) variant pair runs 1 + reps whole attempts of
 * all the class's members, each pair from the same member memory, in three
 * sweeps (best time of the three).  Pairs within 3% of the fastest are ties;
 * among them the first in list order whose row variant takes at most 4 rows
 * per workgroup is kept.  Member states, times and counters are restored
 * afterwards, so tuning changes no result beyond rounding.  Needs every
 * member loaded (FCH_E_INVALID) and the workspace (FCH_E_NOMEM); holds a
 * temporary device copy of one class's member memory (hipMalloc) while it
 * runs.  Synchronizes. */
fch_status fch_ensemble_autotune(fch_ensemble_t ens, int32_t reps);
/* Runs attempts until every member finished or max_attempts attempts ran.
 * FCH_E_NONFINITE if a member reached a non-finite state (that member stopped,
 * the others ran on).  A SAV member that meets E_1 + D_0 <= 0 stops with
 * fch_member_info.invalid set; the call still returns FCH_OK. */
fch_status fch_ensemble_run(fch_ensemble_t ens, int64_t max_attempts, int32_t sync_every,
                            int32_t use_graph, fch_ensemble_info* info);
/* Queues `attempts` attempts of all members (captured graph replays when
 * use_graph) after the work already on the ensemble's stream, and orders that
 * stream after them; no synchronization, no host read-back.  Members that
 * finished skip their work on the device.  Status: fch_ensemble_member or a
 * later fch_ensemble_run. */
fch_status fch_ensemble_step(fch_ensemble_t ens, int32_t attempts, int32_t use_graph);
/* Status of member i (host out); uh (device out, nullable) receives its last
 * accepted state, copied in order on the ensemble's caller stream
 * (fch_ensemble_set_stream); klog (host out, nullable, max_steps doubles) its
 * accepted step sizes.  Waits for the work queued so far. */
fch_status fch_ensemble_member(fch_ensemble_t ens, int32_t member, fch_c128* uh, double* klog,
                               fch_member_info* info);

/* ---- learned PSD warm start (network kernels) ----------------------------- */
/* A 3x3 periodic convolutional network maps (u^n, u^{n-1}, k) to a correction
 * of the extrapolated initial iterate of eq. recurrence; PSD then iterates
 * from the corrected guess to the same stopping tolerance.  Tensors are
 * device memory owned by the caller:
 *   activations bf16 [B][H][W][32] (NHWC, unused channels zero),
 *   weights     bf16 [9][cout][32] (tap = (dy+1)*3 + (dx+1), out, in channel),
 *   bias        f32  [cout], net output f32 [B][H][W];
 * cout = 32 for hidden layers (SiLU), 16 for the output layer (channel 0 is
 * the output, no activation).  H % 16 == 0, W % 32 == 0.  Products run on the
 * BF16 matrix cores with FP32 accumulation; stored activations are rounded
 * to bfloat16 (nearest, ties to even).  stream: a hipStream_t. */
/* z = bias + conv(x, w); hidden: y = SiLU(z) and, unless z is null (inference:
 * only training's backward pass reads z), z (bf16); output: o (f32). */
fch_status fch_nn_conv_fwd(int32_t B, int32_t H, int32_t W, int32_t cout, const void* x,
                           const void* w, const float* bias, void* z, void* y, float* o,
                           void* stream);
/* dz_prev = SiLU'(z_prev) * (gradient of the layer input), bf16; wt: scratch
 * of 9*32*32 bf16 (the flipped, transposed weights). */
fch_status fch_nn_conv_bwd_data(int32_t B, int32_t H, int32_t W, int32_t cout, const void* dz,
                                const void* w, const void* z_prev, void* dz_prev, void* wt,
                                void* stream);
/* dw_db (f32): [9][cout][32] weight gradient then [cout] bias gradient, summed
 * over all pixels in a fixed order; scratch: fch_nn_bwd_w_scratch_floats f32. */
size_t     fch_nn_bwd_w_scratch_floats(int32_t B, int32_t H, int32_t W);
fch_status fch_nn_conv_bwd_w(int32_t B, int32_t H, int32_t W, int32_t cout, const void* dz,
                             const void* x, float* dw_db, float* scratch, void* stream);
/* partial sums of (o - t)^2 / n per block (part[nblocks]; their sum is the
 * mean squared error) and the output-layer
 * gradient dz (bf16, 32 channels, channel 0 = 2 (o - t) / n). */
fch_status fch_nn_mse(int32_t n, const float* o, const float* target, void* dz, float* part,
                      int32_t nblocks, void* stream);
/* Adam step on FP32 parameters (bias-corrected, step >= 1); p_bf16 (nullable)
 * receives the rounded copy used by the convolutions. */
fch_status fch_nn_adam(int32_t n, float* p, const float* g, float* m, float* v, void* p_bf16,
                       double lr, double beta1, double beta2, double eps, int32_t step,
                       void* stream);
fch_status fch_nn_to_bf16(int32_t n, const float* p, void* p_bf16, void* stream);
/* Features of B samples of physical fields (f64 [B][H][W]); k: [B][2] = (k_{n+1},
 * k_n).  d = (u^n - u^{n-1}) k_{n+1}/k_n, scale s = RMS(d) (f64 [B] out),
 * x = [u^n, d/s, (log10 k_{n+1} + 3)/2, 0, ...] (bf16), and the target
 * (u^{n+1} - u^n - d)/s (f32, only when u_np1 and target are non-NULL).
 * work: device scratch of fch_nn_features_work_doubles(B) doubles (partial
 * sums of the scale). */
int32_t    fch_nn_features_work_doubles(int32_t B);
fch_status fch_nn_features(int32_t B, int32_t H, int32_t W, const double* u_n, const double* u_nm1,
                           const double* u_np1, const double* k, void* x, float* target,
                           double* scale, double* work, void* stream);
/* g = u^n + d + s * o (physical f64 [B][H][W]). */
fch_status fch_nn_guess(int32_t B, int32_t H, int32_t W, const double* u_n, const double* u_nm1,
                        const double* k, const double* scale, const float* o, double* g,
                        void* stream);
/* sums of fixed-size partials: out[i] = sum_k part[k*len + i] (f32) */
fch_status fch_nn_reduce(int32_t nparts, int32_t len, const float* part, float* out, void* stream);

const char* fch_status_string(fch_status s);

#ifdef __cplusplus
}
#endif
#endif
