// fch_kernels_impl.hpp -- HIP kernel templates of the FCH pseudo-spectral BDF2 path for
// gfx950, FP64.
//
// A 2D real transform is split into a row pass (length-N FFTs along x, one
// workgroup per R rows) and a column pass (length-N FFTs along y, one
// workgroup per column kx).  Spectra are stored kx-major, so the column pass
// reads and writes contiguous columns and the row pass gathers R-row
// segments per kx (R*16 bytes).  Everything between two HBM round trips is
// fused:
//   row pass   : gather -> inverse FFT -> pointwise well / chemical-potential
//                pieces (omega, p, E_1 and energy densities) -> forward FFT ->
//                untangle -> scatter.  Physical rows never leave the CU.
//   column pass: forward FFT -> spectral epilogue (mu assembly and the IMEX /
//                SAV / PSD / AM3 diagonal algebra, Parseval partial sums) ->
//                spectral prologue of the next evaluation (u*, Lap u*) ->
//                inverse FFT.
// Two real rows are transformed as one complex sequence z = a + i b (the
// row pass always handles pairs: (u, Lap u) in, (omega, p) out).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fch_coef.hpp"
#include "fch_kernels.hpp"

namespace fch {


__device__ __forceinline__ double wavek2(const Consts& c, int kx, int ky) {
  const int N = c.N;
  const int kyi = (ky <= N / 2) ? ky : ky - N;
  return c.kscale * (double)(kx * kx + kyi * kyi);
}

// ---- ETDRK2 (Sec. 3.6) --------------------------------------------------------
// e^z, phi1 = (e^z - 1)/z and phi2 = (e^z - 1 - z)/z^2 at z = L k are the
// multipliers of eqs. ETDRK1 and ETDRK2: L^{-1}(e^{Lk} - I) = k phi1 and
// L^{-1}[L^{-1}(e^{Lk} - I) - k I]/k = k phi2.  Both quotients cancel near
// z = 0, so for |z| <= 1/2 phi2 is its degree-15 Taylor polynomial
// sum_m z^m/(m+2)! (truncation error below 3e-21), phi1 = 1 + z phi2 and
// e^z = 1 + z phi1; elsewhere all three come from expm1.
constexpr double inv_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;  // exact up to 18!
  return 1.0 / f;
}
__device__ __forceinline__ void etd_phi(double z, double& e, double& p1, double& p2) {
  if (fabs(z) <= 0.5) {
    double s = inv_factorial(17);
#pragma unroll
    for (int n = 16; n >= 2; --n) s = fma(s, z, inv_factorial(n));
    p2 = s;
    p1 = fma(z, p2, 1.0);
    e = fma(z, p1, 1.0);
  } else {
    const double m1 = expm1(z);
    const double iz = 1.0 / z;
    e = m1 + 1.0;
    p1 = m1 * iz;
    p2 = (m1 - z) * iz * iz;
  }
}

// the linear operator of eq. ETD-L at |k|^2 = k2 (Laplacian -> -k2):
// -k2 (eps^2 k2 + alpha)^2 - kappa0 - kappa2 eps^2 k2, never positive
__device__ __forceinline__ double etd_L(const Consts& c, const StepCtl* ctl, double k2) {
  const double e2k2 = c.eps2 * k2;
  const double li = e2k2 + c.alpha;
  return -k2 * li * li - ctl->kappa0 - ctl->kappa2 * e2k2;
}

// First stage at one wavenumber from u^n and F = Lap mu(u^n): the split's
// nonlinearity N(u^n) = F - L u^n (eq. ETD-L), the ETDRK1 stage
// u~ = e^{Lk} u^n + k phi1 N(u^n), and w = u~ - k phi2 N(u^n), so that the
// second stage is u^{n+1} = w + k phi2 N(u~) (eq. ETDRK2).  k = k_np1.
__device__ __forceinline__ void etd_stage1(const Consts& c, const StepCtl* ctl, double k2, cd un,
                                           cd F, cd& ut, cd& w) {
  const double L = etd_L(c, ctl, k2);
  const double k = ctl->k_np1;
  double e, p1, p2;
  etd_phi(L * k, e, p1, p2);
  const cd Nn = {F.x - L * un.x, F.y - L * un.y};
  const double kp1 = k * p1, kp2 = k * p2;
  ut = cd{e * un.x + kp1 * Nn.x, e * un.y + kp1 * Nn.y};
  w = cd{ut.x - kp2 * Nn.x, ut.y - kp2 * Nn.y};
}

// Second stage from u~, F = Lap mu(u~) and w: u^{n+1} = w + k phi2 (F - L u~).
__device__ __forceinline__ cd etd_stage2(const Consts& c, const StepCtl* ctl, double k2, cd ut,
                                         cd F, cd w) {
  const double L = etd_L(c, ctl, k2);
  const double k = ctl->k_np1;
  double e, p1, p2;
  etd_phi(L * k, e, p1, p2);
  const double kp2 = k * p2;
  return cd{w.x + kp2 * (F.x - L * ut.x), w.y + kp2 * (F.y - L * ut.y)};
}

// deterministic reduction of K values over NT threads (a fixed butterfly
// inside each wavefront, then the wavefront sums in order); thread 0 writes
template <int NT, int K>
__device__ __forceinline__ void block_reduce(const double (&v)[K], double* red, double* out) {
  constexpr int NW = (NT + 63) / 64;
  const int tid = threadIdx.x;
  double w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k] = v[k];
#pragma unroll
    for (int off = (NT < 64 ? NT : 64) / 2; off >= 1; off >>= 1) w[k] += __shfl_xor(w[k], off, 64);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * NW + (tid >> 6)] = w[k];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) s += red[k * NW + i];
      out[k] = s;
    }
  }
}

// Sums of the two interleaved partial-sum columns p[2i], p[2i+1], i < n, in
// one fixed order whatever the caller's workgroup size: 64 lanes take
// i = l, l+64, ... each, then a fixed XOR butterfly.  Called by the threads
// 0..NT-1 of a workgroup; with NT >= 64 the first wavefront computes it,
// with fewer threads thread 0 reproduces the same additions.  Valid in
// thread 0.  NMAX > 0 (a bound on n known at compile time): each lane
// issues up to CHMAX of its loads before the first addition, so the sum
// costs one memory latency per 64 CHMAX partials instead of one per 64; the
// additions and their order are unchanged.
template <int NT, int NMAX = 0, int CHMAX = 16>
__device__ __forceinline__ void fixed_sum2(const double* p, int n, double& s0, double& s1) {
  if constexpr (NT >= 64 && NMAX > 0) {
    constexpr int PER = (NMAX + 63) / 64;
    constexpr int CH = PER < CHMAX ? PER : CHMAX;
    if (threadIdx.x < 64) {
      const int l = threadIdx.x;
      double a = 0.0, b = 0.0;
      for (int i0 = 0; i0 < n; i0 += 64 * CH) {
        double xa[CH], xb[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = min(i0 + l + 64 * k, n - 1);  // in bounds; unused past n
          xa[k] = p[2 * i];
          xb[k] = p[2 * i + 1];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          if (i0 + l + 64 * k < n) {
            a += xa[k];
            b += xb[k];
          }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
      }
      s0 = a;
      s1 = b;
    }
  } else if constexpr (NT >= 64) {
    if (threadIdx.x < 64) {
      const int l = threadIdx.x;
      double a = 0.0, b = 0.0;
      for (int i = l; i < n; i += 64) {
        a += p[2 * i];
        b += p[2 * i + 1];
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
      }
      s0 = a;
      s1 = b;
    }
  } else {
    if (threadIdx.x == 0) {
      double a[64], b[64];
      for (int l = 0; l < 64; ++l) {
        a[l] = 0.0;
        b[l] = 0.0;
        for (int i = l; i < n; i += 64) {
          a[l] += p[2 * i];
          b[l] += p[2 * i + 1];
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        double na[64], nb[64];
        for (int l = 0; l < 64; ++l) {
          na[l] = a[l] + a[l ^ off];
          nb[l] = b[l] + b[l ^ off];
        }
        for (int l = 0; l < 64; ++l) {
          a[l] = na[l];
          b[l] = nb[l];
        }
      }
      s0 = a[0];
      s1 = b[0];
    }
  }
}

// The stopping test of a PSD solve (Sec. 3.3) after `iter` iterations, from
// the column partial sums (sum |d|^2, sum |u_{s+1}|^2 per column): every
// workgroup of the next pass forms the same sums in the same order and gets
// the same done code (returned in all threads); the recording workgroup
// (rec) writes the ratio, the count and the code into the control block.
// NMAX bounds ncol at compile time (0: none).  done (nullable): the solve's
// stop flag; when it is already set the test is not taken, nothing is
// recorded and its code is returned.  iter == 0: there is no previous
// iteration to test.
template <int NT, int NMAX = 0>
__device__ __forceinline__ int psd_verdict(const double* part, int ncol, StepCtl* ctl, int iter,
                                           bool rec, int* eval_skip, const int* done = nullptr) {
  __shared__ int verdict;
  double c0 = 0.0, c1 = 0.0;
  // the stop flag and the control fields are requested before the partial
  // sums, so all of these loads are in flight together (thread 0 alone
  // consumes the flag, so no uniform branch waits for it first)
  int stopped = 0, fixed = 0, maxit = 0;
  double tol = 0.0;
  if (threadIdx.x == 0) {
    stopped = done ? *done : 0;
    fixed = ctl->fixed_iters;
    tol = ctl->tol;
    maxit = ctl->max_iter;
  }
  // (up to 32 loads per lane in flight: the 2049 column partials of 4096^2
  // in two rounds, those of 2048^2 in one; this sits at the head of the row
  // pass, where few other values are live)
  fixed_sum2<NT, NMAX, 32>(part, ncol, c0, c1);
  if (threadIdx.x == 0) {
    const double ratio = sqrt(c0 / c1);
    const int code =
        stopped ? stopped : (iter > 0 ? psd_done_code(fixed, tol, maxit, ratio, iter) : 0);
    verdict = code;
    if (rec && !stopped && iter > 0) {
      ctl->ratio = ratio;
      ctl->iters = iter;
      if (code) ctl->done = code;
      if (code == 3) ctl->nonfinite = 1;
      if (code && eval_skip) *eval_skip = 0;
    }
  }
  __syncthreads();
  const int v = verdict;
  __syncthreads();  // verdict is read before any later test writes it
  return v;
}

template <int NT, int NMAX>
__device__ __forceinline__ int psd_check(const RowArgs& a, const int* done) {
  return psd_verdict<NT, NMAX>(a.psd_part, a.psd_ncol, a.ctl, a.psd_iter, blockIdx.x == 0,
                               a.psd_eval_skip, done);
}

// ===========================================================================
// Row pass
// ===========================================================================
// TWL: twiddle table copied to LDS (1) or read from global memory through
// the vector caches (0, frees N*16 bytes of LDS per workgroup)
// UMAX (ROW_MU, ensembles): the workgroup's largest u goes to umax_part[tile]
// vblk >= 0: the tile of a persistent workgroup (vblk of vgrid tiles) instead
// of the launch's own block index
template <int N, int R, int E, int MODE, int TWL, bool UMAX = false>
__device__ __forceinline__ void row_body(const RowArgs& a, const int* done,
                                         double* umax_part = nullptr, int vblk = -1,
                                         int vgrid = 0) {
  constexpr int T = N / E;
  constexpr int NT = R * T;
  constexpr int M = N / 2;
  constexpr int H = M + 1;
  // row r of the scratch starts at r*ZS; ZS = 8/R (mod 8) places the R rows
  // of one kx in distinct bank groups
  constexpr int ZS0 = lp_size(N);
  constexpr int ZS = ZS0 + (((8 / R) - ZS0 % 8) % 8 + 8) % 8;
  __shared__ cd Zs[R * ZS];
  __shared__ cd twl[TWL ? N : 1];
  __shared__ double red[2 * ((NT + 63) / 64)];
  if constexpr (MODE == ROW_MU) {
    if (a.psd_part) {
      // the stop flag is read with the stopping test's inputs (its loads all
      // in flight together), not behind a branch of its own
      if (a.psd_init_skip && blockIdx.x == 0 && threadIdx.x == 0 && !(done && *done))
        *a.psd_init_skip = 1;
      if (psd_check<NT, N / 2 + 1>(a, done)) return;
    } else {
      if (done && *done) return;
      if (a.psd_init_skip && blockIdx.x == 0 && threadIdx.x == 0) *a.psd_init_skip = 1;
    }
  } else {
    if (done && *done) return;
  }

  const int tid = threadIdx.x;
  const int seq = tid / T;
  const int t = tid - seq * T;
  const int tile = (vblk < 0) ? xcd_remap(blockIdx.x, gridDim.x) : xcd_remap(vblk, vgrid);
  // ROW_MU: rows y0 .. y0+R-1, one (u, Lap u) pair per row.
  // ROW_FWD/ROW_INV: rows y0 .. y0+2R-1, sequence s pairs rows y0+s, y0+R+s.
  const int y0 = (MODE == ROW_MU) ? tile * R : tile * 2 * R;

  const cd* tw = a.tw;
  if constexpr (TWL) {
    for (int i = tid; i < N; i += NT) twl[i] = a.tw[i];
    tw = twl;
    __syncthreads();  // the FFT exchanges below may be wave-local
  }

  cd v[1][E];
  cd* const base[1] = {Zs + seq * ZS};

  if constexpr (MODE == ROW_MU || MODE == ROW_INV) {
    // gather the column-inverted half spectra of R rows (all loads issued
    // before any use), then build the full length-N spectrum of z = a + i b
    // from the two Hermitian halves
    constexpr int NIT = (R * H + NT - 1) / NT;
    cd ga[NIT], gb[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + it * NT;
      if (idx < R * H) {
        const int kx = idx / R, rr = idx - kx * R;
        const size_t g = (size_t)kx * N + y0 + rr;
        if constexpr (MODE == ROW_MU) {
          ga[it] = a.P0[g];
          gb[it] = a.P1[g];
        } else {
          ga[it] = a.X_in[g];
          gb[it] = a.X_in[g + R];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + it * NT;
      if (idx < R * H) {
        const int kx = idx / R, rr = idx - kx * R;
        const cd xa = ga[it], xb = gb[it];
        if (kx == 0 || kx == M) {
          Zs[rr * ZS + lp(kx)] = cd{xa.x, xb.x};  // real parts only: C2R of the Hermitian extension
        } else {
          Zs[rr * ZS + lp(kx)] = cd{xa.x - xb.y, xa.y + xb.x};
          Zs[rr * ZS + lp(N - kx)] = cd{xa.x + xb.y, xb.x - xa.y};
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) v[0][s] = Zs[seq * ZS + lp(t + s * T)];
    fft<N, E, 1, +1, (T == 64)>(v, base, tw, t);
  }

  if constexpr (MODE == ROW_INV) {
    double* ua = a.u_out + (size_t)(y0 + seq) * N;
    double* ub = a.u_out + (size_t)(y0 + R + seq) * N;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      ua[t + s * T] = v[0][s].x * a.c.invN2;
      ub[t + s * T] = v[0][s].y * a.c.invN2;
    }
    return;
  }

  double acc[2] = {0.0, 0.0};
  double umax = -INFINITY;
  if constexpr (MODE == ROW_MU) {
    const Consts& c = a.c;
    bool bad = false;
    // the q test is hoisted out of the point loop: one branch-free body per
    // case, so the E points' well evaluations interleave
    auto points = [&](auto qc) {
      constexpr bool Q = decltype(qc)::value;
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const double u = v[0][s].x * c.invN2;
        const double lap = v[0][s].y * c.invN2;
        double W, W1, W2;
        well_t<Q>(c, u, W, W1, W2);
        const double om = c.eps2 * lap - W1;
        const double p = -W2 * om - c.eta2 * W1;
        acc[0] += -c.eps2 * lap * (W1 + c.zeta * u) + 0.5 * W1 * W1 - c.eta2 * W;  // G (eq. e:G-def)
        acc[1] += 0.5 * om * om - c.eta2 * W;                                       // energy density
        bad |= !(isfinite(u) && isfinite(lap));
        if constexpr (UMAX) umax = fmax(umax, u);
        v[0][s] = cd{om, p};
      }
    };
    if (c.q != 0.0)
      points(std::integral_constant<bool, true>{});
    else
      points(std::integral_constant<bool, false>{});
    if (bad) a.ctl->nonfinite = 1;
  } else {  // ROW_FWD: two physical rows as one complex sequence
    const double* ua = a.u_in + (size_t)(y0 + seq) * N;
    const double* ub = a.u_in + (size_t)(y0 + R + seq) * N;
#pragma unroll
    for (int s = 0; s < E; ++s) v[0][s] = cd{ua[t + s * T], ub[t + s * T]};
  }

  fft<N, E, 1, -1, (T == 64)>(v, base, tw, t);
  pass_sync<(T == 64)>();
#pragma unroll
  for (int s = 0; s < E; ++s) Zs[seq * ZS + lp(t + s * T)] = v[0][s];
  __syncthreads();

  // untangle: A[k] = (Z[k] + conj Z[N-k])/2, B[k] = (Z[k] - conj Z[N-k])/(2i)
  constexpr int NIT2 = (R * H + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < NIT2; ++it) {
    const int idx = tid + it * NT;
    if (idx >= R * H) break;
    const int kx = idx / R, rr = idx - kx * R;
    const cd zk = Zs[rr * ZS + lp(kx)];
    const cd zn = Zs[rr * ZS + lp((N - kx) & (N - 1))];
    const cd xa = {0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y)};
    const cd xb = {0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x)};
    const size_t g = (size_t)kx * N + y0 + rr;
    if constexpr (MODE == ROW_MU) {
      a.P0[g] = xa;
      a.P1[g] = xb;
    } else {
      a.X_out[g] = xa;
      a.X_out[g + R] = xb;
    }
  }

  if constexpr (MODE == ROW_MU) {
    if (a.partial) block_reduce<NT, 2>(acc, red, a.partial + 2 * tile);
  }
  if constexpr (UMAX) {
    constexpr int NW = (NT + 63) / 64;
#pragma unroll
    for (int off = (NT < 64 ? NT : 64) / 2; off >= 1; off >>= 1)
      umax = fmax(umax, __shfl_xor(umax, off, 64));
    __syncthreads();  // red may still be read by the partial sums above
    if ((tid & 63) == 0) red[tid >> 6] = umax;
    __syncthreads();
    if (tid == 0) {
      double m = red[0];
      for (int i = 1; i < NW; ++i) m = fmax(m, red[i]);
      umax_part[tile] = m;
    }
  }
}

// ===========================================================================
// Column pass
// ===========================================================================

// Columns kx = 0 and kx = N/2 of the half spectrum of a real field obey
// U(ky) = conj U(N - ky).  Rounding breaks this slightly; the explicit linear
// terms of the schemes act on that non-real component while the pointwise
// terms (computed from real fields) never see it, so it would grow from step
// to step.  The single-field column transforms project their output:
// U(ky) <- (U(ky) + conj U(N - ky)) / 2, exchanging partners through LDS.
// Call only where kx is 0 or N/2 (uniform per group).  (The first NF of the
// NV register fields are projected.)  The column pass of the schemes keeps
// these columns exactly Hermitian by construction instead (col_body).
template <int N, int E, int NF, int NV>
__device__ __forceinline__ void hermitian_fix(cd (&f)[NV][E], cd* const (&lds)[2], int t) {
  constexpr int T = N / E;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NF; ++q)
#pragma unroll
    for (int s = 0; s < E; ++s) lds[q][lp(t + s * T)] = f[q][s];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NF; ++q)
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const cd p = lds[q][lp((N - (t + s * T)) & (N - 1))];
      f[q][s] = cd{0.5 * (f[q][s].x + p.x), 0.5 * (f[q][s].y - p.y)};
    }
  __syncthreads();
}

// ---- per-wavenumber algebra of the column pass --------------------------------
// State values read at one wavenumber before the forward FFT: u^n, u^{n-1}
// (IMEX, SAV), the PSD iterate and b u^n + c u^{n-1} (PSD), u~ and w (ETD2),
// or the field U whose (U, Lap U) fed the evaluation (MU, F, AM3, ETD1).
template <int EPI>
__device__ __forceinline__ void load_pre(const ColArgs& a, size_t g, cd& p0, cd& p1) {
  if constexpr (EPI == EPI_IMEX || EPI == EPI_SAV || EPI == EPI_ETD2) {
    p0 = a.s0[g];
    p1 = a.s1[g];
  } else if constexpr (EPI == EPI_PSD) {
    p0 = a.out[g];
    p1 = a.aux[g];
  } else {
    p0 = a.s0[g];
    p1 = cd{0.0, 0.0};
  }
}

// Epilogue at one wavenumber from the forward-transformed omega^, p^:
// mu^ = -eps^2 |k|^2 omega^ + p^ - eps^2 eta1 |k|^2 U^ (eq. FCH with Lap ->
// -|k|^2), then the scheme's diagonal algebra.  o0: the output (u^{n+1},
// mu^, F^, the next PSD iterate, F(u~), the ETD stage u~); o1: SAV q^, PSD d^
// or ETD w; Ua: the field the partial sums need (U, or X for SAV); un, um:
// u^n, u^{n-1}.
template <int EPI>
__device__ __forceinline__ void epi_point(const Consts& c, const StepCtl* ctl, double sstar,
                                          double k2, double wgt, cd om, cd pp, cd p0, cd p1,
                                          cd& o0, cd& o1, cd& Ua, cd& un, cd& um,
                                          double (&acc)[2]) {
  const double e2k2 = c.eps2 * k2;
  cd U;
  un = cd{0.0, 0.0};
  um = cd{0.0, 0.0};
  if constexpr (EPI == EPI_IMEX || EPI == EPI_SAV) {
    un = p0;
    um = p1;
    U = cadd(un, cscale(csub(un, um), ctl->gamma));
  } else {
    U = p0;
  }
  Ua = U;
  o1 = cd{0.0, 0.0};
  const cd mu = {-e2k2 * om.x + pp.x - e2k2 * c.eta1 * U.x,
                 -e2k2 * om.y + pp.y - e2k2 * c.eta1 * U.y};
  if constexpr (EPI == EPI_MU) {
    o0 = mu;
    acc[0] += wgt * k2 * cnorm2(U);
  } else if constexpr (EPI == EPI_F) {
    o0 = cscale(mu, -k2);
  } else if constexpr (EPI == EPI_IMEX) {
    // L_0(beta) of eq. e:SAV-L0; L_IMEX = (eps^2 |k|^2 + alpha)^2 at beta = (2, 1)
    const double Lk = e2k2 * e2k2 + c.beta1 * c.alpha * e2k2 + c.beta2 * c.alpha * c.alpha;
    const cd Nh = csub(mu, cscale(U, Lk));
    const double inv = 1.0 / (ctl->a + k2 * Lk);
    o0 = cd{(-ctl->b * un.x - ctl->c * um.x - k2 * Nh.x) * inv,
            (-ctl->b * un.y - ctl->c * um.y - k2 * Nh.y) * inv};
  } else if constexpr (EPI == EPI_SAV) {
    const double lsav = e2k2 * e2k2 - e2k2 * (c.eta1 + 2.0 * c.zeta);
    const double inv_s = 1.0 / sstar;
    const cd X = cscale(csub(mu, cscale(U, lsav)), inv_s);
    const double L0 = e2k2 * e2k2 + c.beta1 * c.alpha * e2k2 + c.beta2 * c.alpha * c.alpha;
    const double L1 = -e2k2 * (c.eta1 + 2.0 * c.zeta) - c.beta1 * c.alpha * e2k2 -
                      c.beta2 * c.alpha * c.alpha;
    const double inv = 1.0 / (ctl->a + k2 * L0);
    o0 = cd{(-ctl->b * un.x - ctl->c * um.x - k2 * L1 * U.x) * inv,
            (-ctl->b * un.y - ctl->c * um.y - k2 * L1 * U.y) * inv};
    o1 = cscale(X, -k2 * inv);
    Ua = X;  // the SAV sums need X
  } else if constexpr (EPI == EPI_PSD) {
    const cd G = p1;
    cd d = {0.0, 0.0};
    if (k2 != 0.0) {
      const double Lk = (e2k2 + c.alpha) * (e2k2 + c.alpha);
      const double inv = -1.0 / (k2 * Lk + ctl->a);
      d = cd{(k2 * mu.x + ctl->a * U.x + G.x) * inv, (k2 * mu.y + ctl->a * U.y + G.y) * inv};
    }
    o0 = cadd(U, cscale(d, ctl->lambda));
    o1 = d;
  } else if constexpr (EPI == EPI_AM3) {
    o0 = cscale(mu, -k2);
  } else if constexpr (EPI == EPI_ETD1) {
    etd_stage1(c, ctl, k2, U, cscale(mu, -k2), o0, o1);
  } else if constexpr (EPI == EPI_ETD2) {
    o0 = etd_stage2(c, ctl, k2, U, cscale(mu, -k2), p1);
  }
}

// After the epilogue: the stores, the Parseval partial sums and the field
// handed to the next prologue (unext).
template <int EPI, int PRO>
__device__ __forceinline__ void post_point(const ColArgs& a, const StepCtl* ctl, size_t g,
                                           double wgt, cd o0, cd o1, cd Ua, cd un, cd um,
                                           cd& unext, double (&acc)[2]) {
  a.out[g] = o0;
  if constexpr (EPI == EPI_MU || EPI == EPI_F) {
    unext = Ua;
  } else if constexpr (EPI == EPI_IMEX) {
    if constexpr (PRO == PRO_NEXT_EXTRAP)
      unext = cadd(o0, cscale(csub(o0, un), ctl->gamma));
    else
      unext = o0;
  } else if constexpr (EPI == EPI_SAV) {
    a.aux[g] = o1;
    const cd rp = {ctl->a * o0.x + ctl->b * un.x + ctl->c * um.x,
                   ctl->a * o0.y + ctl->b * un.y + ctl->c * um.y};
    acc[0] += wgt * cdotr(Ua, rp);
    acc[1] += wgt * cdotr(Ua, o1);
  } else if constexpr (EPI == EPI_PSD) {
    acc[0] += wgt * cnorm2(o1);
    acc[1] += wgt * cnorm2(o0);
    unext = o0;
  } else if constexpr (EPI == EPI_ETD1) {
    a.aux[g] = o1;
    unext = o0;
  } else if constexpr (EPI == EPI_ETD2) {
    unext = o0;
  } else if constexpr (EPI == EPI_AM3) {
    const cd u_n = a.s1[g], fn = a.f_n[g], fm = a.f_nm1[g];
    const cd up = {u_n.x + ctl->w1 * o0.x + ctl->w2 * fn.x + ctl->w3 * fm.x,
                   u_n.y + ctl->w1 * o0.y + ctl->w2 * fn.y + ctl->w3 * fm.y};
    acc[0] += wgt * cnorm2(csub(Ua, up));
    acc[1] += wgt * cnorm2(up);
  }
}

// State values the prologue reads at one wavenumber (PRO_FIELD: U; EXTRAP and
// PSD_INIT: u^n, u^{n-1} and, for PSD_INIT, the guess; ETD1: u^n, F(u^n)).
template <int PRO>
__device__ __forceinline__ void load_pro(const ColArgs& a, size_t g, cd& s0v, cd& s1v, cd& gv) {
  s0v = a.s0[g];
  s1v = cd{0.0, 0.0};
  gv = cd{0.0, 0.0};
  if constexpr (PRO == PRO_EXTRAP || PRO == PRO_PSD_INIT) s1v = a.s1[g];
  if constexpr (PRO == PRO_ETD1) s1v = a.f_n[g];
  if constexpr (PRO == PRO_SAV_NEXT || PRO == PRO_SAV_FIELD) {
    s1v = a.out[g];
    gv = a.aux[g];
  }
  if constexpr (PRO == PRO_PSD_INIT) {
    if (a.guess) gv = a.guess[g];
  }
}

// Prologue at one wavenumber: U whose (U, Lap U) the next evaluation needs:
// the field, the extrapolation u^n + gamma (u^n - u^{n-1}) (eq. Richardson),
// the PSD initial iterate (guess, keeping the mean of u^n; PSD_INIT also
// writes b u^n + c u^{n-1} and the iterate), the ETDRK1 stage u~ from the
// cached F(u^n) (ETD1 also writes u~ and w), or, after a SAV step, the
// extrapolation of u^{n+1} = p + r^{n+1} q (eq. 4.8; SAV_NEXT writes u^{n+1}
// over p; rr = r^{n+1}), or u^{n+1} itself (SAV_FIELD, for F of a trial
// state).  PRO_NEXT_*: unext.
template <int PRO>
__device__ __forceinline__ cd pro_point(const ColArgs& a, const StepCtl* ctl, size_t g,
                                        double k2, bool mean_mode, cd s0v, cd s1v, cd gv,
                                        cd unext, double rr) {
  if constexpr (PRO == PRO_SAV_NEXT || PRO == PRO_SAV_FIELD) {
    const cd u1 = {fma(rr, gv.x, s1v.x), fma(rr, gv.y, s1v.y)};
    a.out[g] = u1;
    if constexpr (PRO == PRO_SAV_FIELD) return u1;
    return cadd(u1, cscale(csub(u1, s0v), ctl->gamma));
  } else if constexpr (PRO == PRO_ETD1) {
    cd ut, w;
    etd_stage1(a.c, ctl, k2, s0v, s1v, ut, w);
    a.out[g] = ut;
    a.aux[g] = w;
    return ut;
  } else if constexpr (PRO == PRO_FIELD) {
    return s0v;
  } else if constexpr (PRO == PRO_EXTRAP) {
    return cadd(s0v, cscale(csub(s0v, s1v), ctl->gamma));
  } else if constexpr (PRO == PRO_PSD_INIT) {
    a.aux[g] = cd{ctl->b * s0v.x + ctl->c * s1v.x, ctl->b * s0v.y + ctl->c * s1v.y};
    cd U;
    if (a.guess)
      U = mean_mode ? s0v : gv;  // keep the mass of u^n
    else
      U = cadd(s0v, cscale(csub(s0v, s1v), ctl->gamma));
    a.out[g] = U;
    return U;
  } else {
    return unext;
  }
}

// Member fields that no kernel changes while it runs (the model constants, the
// buffer pointers, the slot indices and flags, which only the controller
// kernel rotates) are read through the constant address space: scalar loads,
// issued together at the start of every workgroup.  Control blocks and the
// stage flags, which workgroup 0 of some stages writes, are read directly,
// except by the column passes, which never write them: there a flag's
// scalar load joins the others instead of a vector load and a wait of its
// own.
template <class T>
__device__ __forceinline__ T ldc(const T& x) {
  if constexpr (std::is_scalar<T>::value) {
    return *(const __attribute__((address_space(4))) T*)(&x);
  } else {  // a struct of 8-byte words (the model constants)
    static_assert(sizeof(T) % 8 == 0 && alignof(T) >= 8, "struct of 8-byte words");
    using W = unsigned long long;
    const __attribute__((address_space(4))) W* p = (const __attribute__((address_space(4))) W*)(&x);
    T r;
    W* q = reinterpret_cast<W*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i) q[i] = p[i];
    return r;
  }
}

// Hermitian part of a column of a real field's half spectrum at ky, from its
// values at ky and N - ky (exactly conjugate at the two points)
__device__ __forceinline__ cd herm(cd x, cd xr) {
  return cd{0.5 * (x.x + xr.x), 0.5 * (x.y - xr.y)};
}

// N/2 workgroups.  Workgroup kx > 0 transforms column kx.  Workgroup 0
// transforms the two self-conjugate columns kx = 0 and N/2 together: the
// row-transformed fields are real there, so each field's two columns pack
// into one complex sequence z = X_0 + i X_{N/2}, and after the FFT
// X^_0(k) = (Z(k) + conj Z(-k))/2, X^_{N/2}(k) = (Z(k) - conj Z(-k))/(2i).
// The state values its epilogue reads are replaced by their Hermitian parts,
// so every state it writes is exactly the spectrum of a real field (a
// non-Hermitian component of these columns would be amplified by the
// explicit terms of the schemes); the inverse transforms pack the same way.
// vcol >= 0: the column task of a persistent workgroup instead of the
// launch's own block index (task 0 is the self-conjugate pair).
// PART: 0 every column (N/2 workgroups); 1 the columns kx = 1 .. N/2-1 only
// (N/2 - 1 workgroups, kx = block index + 1), 2 the self-conjugate pair only
// (one workgroup).  A launch split into parts 1 and 2 compiles each path
// alone, so neither holds the other's registers (the pair's path carries both
// of its columns' state values).
template <int N, int E, int EPI, int PRO, int TWL, int PART = 0>
__device__ __forceinline__ void col_body(const ColArgs& a, const int* done, int vcol = -1) {
  constexpr int T = N / E;
  constexpr int M = N / 2;
  __shared__ cd buf[2][lp_size(N)];
  __shared__ cd twl[TWL ? N : 1];
  __shared__ double red[2 * ((T + 63) / 64)];
  // The stop flag (set only by earlier launches) is read as a scalar load.
  // A pass that writes nothing before its main loads tests it after issuing
  // them, so the flag's latency and theirs overlap; the others test it first.
  // Measured: the late test speeds up the E = 4 variants (two or three
  // workgroups per CU; the fused IMEX pass at 1024^2 by 3%) and slows the
  // E = 8 ones (one workgroup per CU) by about 2%, and it costs the AM3 pass
  // a third of its occupancy, so those test first.
  constexpr bool LATE_STOP = (E <= 4 && EPI != EPI_NONE && EPI != EPI_SAV && EPI != EPI_AM3 &&
                              PRO != PRO_SAV_NEXT && PRO != PRO_SAV_FIELD);
  int stopped = 0;
  if constexpr (LATE_STOP) {
    stopped = done ? ldc(*done) : 0;
  } else {
    if (done && ldc(*done)) return;
  }

  const Consts& c = a.c;
  const int t = threadIdx.x;
  const int kx = (vcol >= 0) ? vcol : (PART == 1) ? (int)blockIdx.x + 1 : (PART == 2) ? 0
                                                                                : (int)blockIdx.x;
  const bool sc = (PART == 2) || (PART == 0 && kx == 0);  // the self-conjugate pair kx = 0, N/2
  const size_t col = (size_t)kx * N;
  constexpr size_t colM = (size_t)M * N;
  const double wgt = sc ? 1.0 : 2.0;  // Parseval weight of the half spectrum

  const cd* tw = a.tw;
  if constexpr (TWL) {
    for (int i = t; i < N; i += T) twl[i] = a.tw[i];
    __syncthreads();
    tw = twl;
  }

  // SAV: s* = sqrt(E_1(u*) + D0) from the row pass's partial sums, formed
  // by every workgroup in the same order (workgroup 0 records it)
  double sstar = 0.0;
  if constexpr (EPI == EPI_SAV) {
    __shared__ double sh_s;
    if (a.sav_rpart) {
      double r0 = 0.0, r1 = 0.0;
      fixed_sum2<T, N, 32>(a.sav_rpart, a.sav_nrow, r0, r1);  // N / R rows
      if (t == 0) {
        const double E1 = c.h2 * r0;
        double sst;
        const int st = sav_sstar(E1, c.D0, sst);
        sh_s = sst;
        if (kx == 0) {
          a.ctl->E1 = E1;
          a.ctl->s_star = sst;
          if (st == 1) a.ctl->nonfinite = 1;
          if (st == 2) a.ctl->invalid = 1;
        }
      }
      __syncthreads();
      sstar = sh_s;
    } else {
      sstar = a.ctl->s_star;
    }
  }

  // SAV_NEXT / SAV_FIELD: r^{n+1} from the SAV step's partial sums (g_p, g_q),
  // solved by every workgroup in the same order (eq. 4.8); workgroup 0 records it
  double rnew = 0.0;
  if constexpr (PRO == PRO_SAV_NEXT || PRO == PRO_SAV_FIELD) {
    __shared__ double sh_r;
    double c0 = 0.0, c1 = 0.0;
    fixed_sum2<T, N / 2 + 1, 32>(a.sav_cpart, a.sav_ncol, c0, c1);
    if (t == 0) {
      const int sl = a.rslot;
      const double r = sav_r_solve(*a.ctl, a.ctl->rring[sl], a.ctl->rring[(sl + 2) % 3],
                                   c.pars * c0, c.pars * c1);
      sh_r = r;
      if (kx == 0) {
        a.ctl->rring[(sl + 1) % 3] = r;
        if (!isfinite(r)) a.ctl->nonfinite = 1;
      }
    }
    __syncthreads();
    rnew = sh_r;
  }

  cd v[2][E];
  cd* const base[2] = {buf[0], buf[1]};
  // PRO_NEXT_*: the epilogue hands the next evaluation's field to the
  // prologue by writing (U, -|k|^2 U) (packed for the self-conjugate pair)
  // straight into v[.][s], whose FFT output it has just consumed
  constexpr bool NEXT = (PRO == PRO_NEXT_EXTRAP || PRO == PRO_NEXT_FIELD);
  double acc[2] = {0.0, 0.0};
  const StepCtl* ctl = a.ctl;

  if constexpr (EPI != EPI_NONE) {
    // the FFT inputs are requested first; the state values after them,
    // before the FFT, so that they arrive while it runs.  Workgroup 0 reads
    // both of its columns here: every state value it uses is read before it
    // writes any output (outputs may alias u^{n-1} or, for PSD, the iterate).
    cd pre0[E], pre1[E], preM0[E], preM1[E];
    if (sc) {
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const int ky = t + s * T;
        const cd a0 = a.P0[ky], aM = a.P0[colM + ky];
        const cd b0 = a.P1[ky], bM = a.P1[colM + ky];
        v[0][s] = cd{a0.x - aM.y, a0.y + aM.x};
        v[1][s] = cd{b0.x - bM.y, b0.y + bM.x};
      }
#pragma unroll
      for (int s = 0; s < E; ++s) load_pre<EPI>(a, colM + t + s * T, preM0[s], preM1[s]);
    } else {
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const size_t g = col + t + s * T;
        v[0][s] = a.P0[g];
        v[1][s] = a.P1[g];
      }
    }
#pragma unroll
    for (int s = 0; s < E; ++s) load_pre<EPI>(a, col + t + s * T, pre0[s], pre1[s]);
    if constexpr (LATE_STOP) {
      if (stopped) {
        // an empty asm reading the column values: without a use on this
        // path the compiler would sink their loads behind the test
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int s = 0; s < E; ++s) asm volatile("" ::"v"(v[q][s].x), "v"(v[q][s].y));
        return;
      }
    }
    fft<N, E, 2, -1>(v, base, tw, t);

    if (!sc) {
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const int ky = t + s * T;
        const double k2 = wavek2(c, kx, ky);
        cd o0, o1, Ua, un, um, U;
        epi_point<EPI>(c, ctl, sstar, k2, wgt, v[0][s], v[1][s], pre0[s], pre1[s], o0, o1, Ua, un,
                       um, acc);
        post_point<EPI, PRO>(a, ctl, col + ky, wgt, o0, o1, Ua, un, um, U, acc);
        if constexpr (NEXT) {
          v[0][s] = U;
          v[1][s] = cscale(U, -k2);
        }
      }
    } else {
      // separate the two columns; Z(-k) comes from the thread holding N - ky:
      // omega^, p^ of column 0 are (Z + conj Z(-k))/2, of column N/2
      // (Z - conj Z(-k))/(2i)
      constexpr bool P1 = (EPI == EPI_IMEX || EPI == EPI_SAV || EPI == EPI_PSD || EPI == EPI_ETD2);
      cd sep[4][E];  // omega^_0, p^_0, omega^_{N/2}, p^_{N/2}
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < E; ++s) base[q][lp(t + s * T)] = v[q][s];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const cd z = v[q][s], zr = base[q][lp((N - (t + s * T)) & (N - 1))];
          sep[q][s] = herm(z, zr);
          sep[2 + q][s] = cd{0.5 * (z.y + zr.y), -0.5 * (z.x - zr.x)};
        }
      // the state values of each column are replaced by their Hermitian
      // parts through the same exchange; then that column's epilogue
      cd U0[E];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        cd(&p0)[E] = h ? preM0 : pre0;
        cd(&p1)[E] = h ? preM1 : pre1;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) {
          base[0][lp(t + s * T)] = p0[s];
          if constexpr (P1) base[1][lp(t + s * T)] = p1[s];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const int kr = (N - (t + s * T)) & (N - 1);
          p0[s] = herm(p0[s], base[0][lp(kr)]);
          if constexpr (P1) p1[s] = herm(p1[s], base[1][lp(kr)]);
        }
        const int kxh = h ? M : 0;
        const size_t colh = h ? colM : 0;
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const int ky = t + s * T;
          const double k2 = wavek2(c, kxh, ky);
          cd o0, o1, Ua, un, um, U;
          epi_point<EPI>(c, ctl, sstar, k2, 1.0, sep[2 * h][s], sep[2 * h + 1][s], p0[s], p1[s],
                         o0, o1, Ua, un, um, acc);
          post_point<EPI, PRO>(a, ctl, colh + ky, 1.0, o0, o1, Ua, un, um, U, acc);
          if constexpr (NEXT) {
            if (h == 0) {
              U0[s] = U;
            } else {
              const double k20 = wavek2(c, 0, ky);
              v[0][s] = cd{U0[s].x - U.y, U0[s].y + U.x};
              v[1][s] = cd{-k20 * U0[s].x + k2 * U.y, -k20 * U0[s].y - k2 * U.x};
            }
          }
        }
      }
    }
  }

  if constexpr (PRO != PRO_NONE) {
    if constexpr (!NEXT) {
      // each point is read and written by the same thread; workgroup 0 then
      // replaces U of columns 0 and N/2 by its Hermitian part (U is linear in
      // the state with real coefficients, so this equals projecting the
      // state) and packs their inverse transforms as the real and the
      // imaginary part of one sequence
      if (!sc) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const int ky = t + s * T;
          cd s0v, s1v, gv;
          load_pro<PRO>(a, col + ky, s0v, s1v, gv);
          const double k2 = wavek2(c, kx, ky);
          const cd U =
              pro_point<PRO>(a, ctl, col + ky, k2, false, s0v, s1v, gv, cd{0.0, 0.0}, rnew);
          v[0][s] = U;
          v[1][s] = cscale(U, -k2);
        }
      } else {
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const int ky = t + s * T;
          cd s0v, s1v, gv;
          load_pro<PRO>(a, ky, s0v, s1v, gv);
          v[0][s] = pro_point<PRO>(a, ctl, ky, wavek2(c, 0, ky), ky == 0, s0v, s1v, gv,
                                   cd{0.0, 0.0}, rnew);
          load_pro<PRO>(a, colM + ky, s0v, s1v, gv);
          v[1][s] = pro_point<PRO>(a, ctl, colM + ky, wavek2(c, M, ky), false, s0v, s1v, gv,
                                   cd{0.0, 0.0}, rnew);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int s = 0; s < E; ++s) base[q][lp(t + s * T)] = v[q][s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < E; ++s) {
          const int ky = t + s * T;
          const int kr = (N - ky) & (N - 1);
          const cd U = herm(v[0][s], base[0][lp(kr)]), UM = herm(v[1][s], base[1][lp(kr)]);
          const double k2 = wavek2(c, 0, ky), k2M = wavek2(c, M, ky);
          v[0][s] = cd{U.x - UM.y, U.y + UM.x};
          v[1][s] = cd{-k2 * U.x + k2M * UM.y, -k2 * U.y - k2M * UM.x};
        }
      }
    }
    fft<N, E, 2, +1>(v, base, tw, t);
    if (!sc) {
#pragma unroll
      for (int s = 0; s < E; ++s) {
        a.P0[col + t + s * T] = v[0][s];
        a.P1[col + t + s * T] = v[1][s];
      }
    } else {
      // the inverse transforms of the two real columns are the real and the
      // imaginary part (the row pass reads real parts at kx = 0, N/2)
#pragma unroll
      for (int s = 0; s < E; ++s) {
        const int ky = t + s * T;
        a.P0[ky] = cd{v[0][s].x, 0.0};
        a.P0[colM + ky] = cd{v[0][s].y, 0.0};
        a.P1[ky] = cd{v[1][s].x, 0.0};
        a.P1[colM + ky] = cd{v[1][s].y, 0.0};
      }
    }
  }

  if constexpr (EPI == EPI_MU || EPI == EPI_SAV || EPI == EPI_PSD || EPI == EPI_AM3) {
    if (a.partial) {
      block_reduce<T, 2>(acc, red, a.partial + 2 * kx);
      if (sc && t == 0) {  // the sums of column N/2 are in workgroup 0's
        a.partial[2 * M] = 0.0;
        a.partial[2 * M + 1] = 0.0;
      }
    }
  }
}

// kernel timing: the launch's start on the device's constant clock.  The
// dispatcher hands out workgroups in index order, one per XCD in turn, so the
// first eight hold the earliest start; only they fold theirs in (a minimum
// over every workgroup would queue hundreds of atomics on one address).
__device__ __forceinline__ void stamp_start(unsigned long long* t) {
  if (t && threadIdx.x == 0 && blockIdx.x < 8 && blockIdx.y == 0)
    atomicMin(t, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}

template <int N, int R, int E, int MODE, int TWL>
__global__ __launch_bounds__(R*(N / E)) void k_row(RowArgs a, const int* done) {
  stamp_start(a.tstart);
  row_body<N, R, E, MODE, TWL>(a, done);
}

template <int N, int E, int EPI, int PRO, int TWL, int PART = 0>
__global__ __launch_bounds__(N / E) void k_col(ColArgs a, const int* done) {
  if constexpr (PART != 2) stamp_start(a.tstart);
  col_body<N, E, EPI, PRO, TWL, PART>(a, done);
}

// ---- one-launch PSD solve (Sec. 3.3) ------------------------------------------
// Grid barrier of a persistent launch whose G workgroups are all resident at
// once: thread 0 of each workgroup releases its writes at agent scope, counts
// its arrival in *bar and polls until `target` arrivals (round r completes at
// (r + 1) G; *bar is zeroed with the control block).  The wait gives up after
// half a second of the device's constant clock, which only happens when not
// every workgroup could run at once; then false.
__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned target) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (__builtin_amdgcn_s_memrealtime() - t0 > 50000000ull) {  // 0.5 s at 100 MHz
        good = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  const bool r = ok;
  __syncthreads();  // ok is read before a later barrier writes it
  return r;
}

// A whole PSD solve in one launch: G persistent workgroups run the row pass
// (chemical-potential pieces of the iterate, N/R row tiles) and the column
// pass (EPI_PSD with the next iterate's prologue, N/2 column tasks) in turn,
// separated by grid barriers, and before each iteration but the first they
// all evaluate the stopping test of the iterations done so far from the
// column partial sums; the solve ends on the test's code (converged, the
// fixed count, max_iter or non-finite, as psd_done_code decides) or when a
// barrier gives up (done code 5).  A control block already stopped (invalid
// device scalars) stops it before any work.  The initial iterate and its column-inverted
// (u, Lap u) come from a PRO_PSD_INIT column pass launched before; ra and ca
// are the arguments of the separate passes with no stopping test and no done
// flag.  The row and column variants must use the same number of threads.
// The two passes are separate (not inlined) functions, so that each keeps its
// own register allocation and nothing is held live from one into the other.
template <int N, int R, int ER, int RTWL>
__device__ __attribute__((noinline)) void psd_row_task(const RowArgs& ra, int v) {
  row_body<N, R, ER, ROW_MU, RTWL>(ra, nullptr, nullptr, v, N / R);
}
template <int N, int EC, int CTWL>
__device__ __attribute__((noinline)) void psd_col_task(const ColArgs& ca, int v) {
  col_body<N, EC, EPI_PSD, PRO_NEXT_FIELD, CTWL>(ca, nullptr, v);
}
// WPE: waves per SIMD the launch bound asks for (1 when LDS allows one
// workgroup per CU anyway)
template <int N, int R, int ER, int RTWL, int EC, int CTWL, int WPE>
__global__ __launch_bounds__(N / EC, WPE) void k_psd_solve(RowArgs ra, ColArgs ca, int limit) {
  constexpr int NT = N / EC;
  static_assert(R * (N / ER) == NT, "row and column variants of unequal workgroup size");
  constexpr int NROW = N / R, NCOL = N / 2;
  const int G = gridDim.x, b = blockIdx.x;
  StepCtl* ctl = ca.ctl;
  if (ctl->done) return;
  unsigned target = 0;
  for (int it = 0;; ++it) {
    if (it > 0 && psd_verdict<NT, NCOL + 1>(ca.partial, NCOL + 1, ctl, it, b == 0, nullptr)) break;
    if (it >= limit) break;  // not reached: the test stops at the limit
    for (int v = b; v < NROW; v += G) {
      psd_row_task<N, R, ER, RTWL>(ra, v);
      __syncthreads();
    }
    target += (unsigned)G;
    if (!grid_sync(&ctl->bar, target)) {
      if (threadIdx.x == 0) ctl->done = 5;
      break;
    }
    for (int v = b; v < NCOL; v += G) {
      psd_col_task<N, EC, CTWL>(ca, v);
      __syncthreads();
    }
    target += (unsigned)G;
    if (!grid_sync(&ctl->bar, target)) {
      if (threadIdx.x == 0) ctl->done = 5;
      break;
    }
  }
}

// ---- batched ensemble entry points (member = blockIdx.y) --------------------

__device__ __forceinline__ void ens_col_args(const EnsMember* m, ColArgs& a) {
  a.c = ldc(m->c);
  a.P0 = ldc(m->P0);
  a.P1 = ldc(m->P1);
  a.s0 = nullptr;
  a.s1 = nullptr;
  a.out = nullptr;
  a.aux = nullptr;
  a.guess = nullptr;
  a.f_n = nullptr;
  a.f_nm1 = nullptr;
  a.X_in = nullptr;
  a.X_out = nullptr;
  a.partial = nullptr;
  a.ctl = const_cast<StepCtl*>(&m->ctl);
  a.tw = ldc(m->tw);
  a.sav_rpart = nullptr;
  a.sav_nrow = 0;
  a.sav_cpart = nullptr;
  a.sav_ncol = 0;
  a.rslot = 0;
  a.tstart = nullptr;
}

// the buffers of the member's state and F slots
__device__ __forceinline__ cd* ring_at(const EnsMember* m, int slot) { return ldc(m->ring[slot]); }
__device__ __forceinline__ cd* fring_at(const EnsMember* m, int slot) { return ldc(m->fring[slot]); }

template <int N, int R, int E, int TWL, int ROWMODE>
__global__ __launch_bounds__(R*(N / E)) void k_row_ens(EnsMember* mem, int first) {
  EnsMember* m = mem + first + blockIdx.y;
  constexpr bool UMAX = (ROWMODE == ENS_ROW_TRACK);
  const int psd = ldc(m->psd);
  RowArgs a;
  a.c = ldc(m->c);
  a.P0 = ldc(m->P0);
  a.P1 = ldc(m->P1);
  a.u_in = nullptr;
  a.u_out = nullptr;
  a.X_in = nullptr;
  a.X_out = nullptr;
  a.partial = (ROWMODE == ENS_ROW && ldc(m->sav)) ? ldc(m->rpart) : nullptr;  // SAV: E_1 of u*
  a.ctl = &m->ctl;
  a.tw = ldc(m->tw);
  a.psd_part = nullptr;
  a.psd_ncol = 0;
  a.psd_iter = 0;
  a.psd_init_skip = nullptr;
  a.psd_eval_skip = nullptr;
  a.tstart = nullptr;
  const int* done = &m->ctl.done;
  if constexpr (ROWMODE == ENS_ROW_PSD) {
    // a PSD iteration of the solve whose control block is sctl: first the
    // stopping test of the previous iteration (none before the first)
    a.ctl = &m->sctl;
    const int it = m->sctl.iters;
    a.psd_part = ldc(m->cpart);  // no test before the first iteration (it == 0)
    a.psd_ncol = ldc(m->H);
    a.psd_iter = it;
    a.psd_init_skip = &m->psd_init_skip;
    a.psd_eval_skip = &m->psd_eval_skip;
    done = &m->sctl.done;
  } else {
    if (psd) done = &m->psd_eval_skip;  // the F(u~) evaluation of a PSD attempt
  }
  row_body<N, R, E, ROW_MU, TWL, UMAX>(a, done, ldc(m->umaxpart));
}

// one attempt of adaptive BDF2-IMEX: PRO (u* and Lap u* of the step),
// IMEX (the step, then u~ and Lap u~ for F(u~)), AM3 (F(u~) and the error sums);
// of adaptive ETDRK2: ETD_PRO (first stage from the cached F(u^n)), ETD2 (the
// step, then the trial's (u, Lap u)), AM3; of adaptive SAV: PRO, SAV (p, q and
// the r-solve sums), SAV_FIELD (r^{n+1}, the trial and its (u, Lap u)), AM3;
// of adaptive PSD (rounds): PSD_INIT, PSD iterations, AM3
template <int N, int E, int TWL, int STAGE>
__global__ __launch_bounds__(N / E) void k_col_ens(EnsMember* mem, int first) {
  EnsMember* m = mem + first + blockIdx.y;
  ColArgs a;
  ens_col_args(m, a);
  const int cur = ldc(m->cur), prev = ldc(m->prev), trial = ldc(m->trial);
  if constexpr (STAGE == ENS_PRO) {
    a.s0 = ring_at(m, cur);
    a.s1 = ring_at(m, prev);
    col_body<N, E, EPI_NONE, PRO_EXTRAP, TWL>(a, &m->ctl.done);
  } else if constexpr (STAGE == ENS_IMEX) {
    a.s0 = ring_at(m, cur);
    a.s1 = ring_at(m, prev);
    a.out = ring_at(m, trial);
    col_body<N, E, EPI_IMEX, PRO_NEXT_FIELD, TWL>(a, &m->ctl.done);
  } else if constexpr (STAGE == ENS_ETD_PRO) {
    // u~ and w from u^n and the cached F(u^n); u~ goes to the F slot that the
    // attempt's AM3 stage overwrites last
    a.s0 = ring_at(m, cur);
    a.f_n = fring_at(m, ldc(m->fn));
    a.out = fring_at(m, ldc(m->ft));
    a.aux = ldc(m->aux);
    col_body<N, E, EPI_NONE, PRO_ETD1, TWL>(a, &m->ctl.done);
  } else if constexpr (STAGE == ENS_ETD2) {
    a.s0 = fring_at(m, ldc(m->ft));
    a.s1 = ldc(m->aux);
    a.out = ring_at(m, trial);
    col_body<N, E, EPI_ETD2, PRO_NEXT_FIELD, TWL>(a, &m->ctl.done);
  } else if constexpr (STAGE == ENS_SAV) {
    // p into the trial slot, q into aux, the (g_p, g_q) partials; s* from the
    // first row pass's E_1 partials
    a.s0 = ring_at(m, cur);
    a.s1 = ring_at(m, prev);
    a.out = ring_at(m, trial);
    a.aux = ldc(m->aux);
    a.partial = ldc(m->cpart);
    a.sav_rpart = ldc(m->rpart);
    a.sav_nrow = ldc(m->nrow);
    col_body<N, E, EPI_SAV, PRO_NONE, TWL>(a, &m->ctl.done);
  } else if constexpr (STAGE == ENS_PSD_INIT) {
    // a new attempt's initial iterate u^n + gamma (u^n - u^{n-1}) (eq.
    // recurrence) into the trial slot, b u^n + c u^{n-1} into aux, and the
    // iterate's (u, Lap u) for the first iteration
    a.ctl = &m->sctl;
    a.s0 = ring_at(m, cur);
    a.s1 = ring_at(m, prev);
    a.out = ring_at(m, trial);
    a.aux = ldc(m->aux);
    col_body<N, E, EPI_NONE, PRO_PSD_INIT, TWL>(a, &m->psd_init_skip);
  } else if constexpr (STAGE == ENS_PSD) {
    // one iteration (the direction, the update in place, the stopping sums)
    // and the next iterate's (u, Lap u); workgroup 0 counts the iteration
    if (m->sctl.done) return;
    a.ctl = &m->sctl;
    a.out = ring_at(m, trial);
    a.aux = ldc(m->aux);
    a.partial = ldc(m->cpart);
    col_body<N, E, EPI_PSD, PRO_NEXT_FIELD, TWL>(a, &m->sctl.done);
    if (blockIdx.x == 0 && threadIdx.x == 0) m->sctl.iters += 1;
  } else if constexpr (STAGE == ENS_SAV_FIELD) {
    // r^{n+1}, u^{n+1} = p + r^{n+1} q over p, and its (u, Lap u) for F
    a.s0 = ring_at(m, cur);
    a.out = ring_at(m, trial);
    a.aux = ldc(m->aux);
    a.sav_cpart = ldc(m->cpart);
    a.sav_ncol = ldc(m->H);
    a.rslot = ldc(m->rslot);
    col_body<N, E, EPI_NONE, PRO_SAV_FIELD, TWL>(a, &m->ctl.done);
  } else {
    a.s0 = ring_at(m, trial);
    a.s1 = ring_at(m, cur);
    a.f_n = fring_at(m, ldc(m->fn));
    a.f_nm1 = fring_at(m, ldc(m->fm));
    a.out = fring_at(m, ldc(m->ft));
    a.partial = ldc(m->cpart);
    col_body<N, E, EPI_AM3, PRO_NONE, TWL>(a, ldc(m->psd) ? &m->psd_eval_skip : &m->ctl.done);
  }
}

// single-field column transforms (boundary fch_forward / fch_inverse):
// two columns per workgroup, one sequence each
template <int N, int E, int DIR, int TWL>
__device__ __forceinline__ void col1_body(const ColArgs& a) {
  constexpr int T = N / E;
  constexpr int H = N / 2 + 1;
  __shared__ cd buf[2][lp_size(N)];
  __shared__ cd twl[TWL ? N : 1];
  const int t = threadIdx.x;
  const int kx0 = 2 * blockIdx.x;
  const cd* tw = a.tw;
  if constexpr (TWL) {
    for (int i = t; i < N; i += T) twl[i] = a.tw[i];
    __syncthreads();
    tw = twl;
  }
  cd v[2][E];
  cd* const base[2] = {buf[0], buf[1]};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int kx = kx0 + q;
#pragma unroll
    for (int s = 0; s < E; ++s)
      v[q][s] = (kx < H) ? a.X_in[(size_t)kx * N + t + s * T] : cd{0.0, 0.0};
  }
  fft<N, E, 2, DIR>(v, base, tw, t);
  if (DIR < 0 && (kx0 == 0 || kx0 == N / 2)) hermitian_fix<N, E, 1, 2>(v, base, t);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int kx = kx0 + q;
    if (kx < H) {
#pragma unroll
      for (int s = 0; s < E; ++s) a.X_out[(size_t)kx * N + t + s * T] = v[q][s];
    }
  }
}

template <int N, int E, int DIR, int TWL>
__global__ __launch_bounds__(N / E) void k_col1(ColArgs a) {
  col1_body<N, E, DIR, TWL>(a);
}

// ---- batched single-field transforms (field = blockIdx.y) --------------------
// Fields are stored back to back: physical fields pstride doubles apart, half
// spectra sstride complex values apart.  Each field runs the single-field body.
template <int N, int R, int E, int MODE, int TWL>
__global__ __launch_bounds__(R*(N / E)) void k_row_b(RowArgs a, size_t pstride, size_t sstride) {
  const size_t b = blockIdx.y;
  if constexpr (MODE == ROW_FWD) {
    a.u_in += b * pstride;
    a.X_out += b * sstride;
  } else {
    a.X_in += b * sstride;
    a.u_out += b * pstride;
  }
  row_body<N, R, E, MODE, TWL>(a, nullptr);
}

template <int N, int E, int DIR, int TWL>
__global__ __launch_bounds__(N / E) void k_col1_b(ColArgs a, size_t sstride) {
  const size_t b = blockIdx.y;
  a.X_in += b * sstride;
  a.X_out += b * sstride;
  col1_body<N, E, DIR, TWL>(a);
}

}  // namespace fch
