// fch_device.hpp -- device building blocks for gfx950 (wave64, FP64):
// complex arithmetic, in-register radix-2^k DFTs, a workgroup Stockham FFT
// staged through LDS, and the regularized FCH well W_q (eq. e:Wq-def).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fch {

struct cd {
  double x, y;
};

__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
// Re(a * conj(b))
__device__ __forceinline__ double cdotr(cd a, cd b) { return fma(a.x, b.x, a.y * b.y); }
__device__ __forceinline__ double cnorm2(cd a) { return fma(a.x, a.x, a.y * a.y); }

// ---------------------------------------------------------------------------
// In-register DFT of R = 2, 4, 8 or 16 points:  v[k] <- sum_n v[n] w^{nk},
// w = exp(DIR * 2 pi i / R).  Radix-2 decimation in time over a bit-reversed
// copy; every index is a compile-time constant after unrolling, so the array
// lives in VGPRs.  The internal twiddles are powers of exp(DIR 2 pi i / 16).
// ---------------------------------------------------------------------------
constexpr double kC1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kS1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kC2 = 0.70710678118654752440;  // cos(pi/4)

constexpr int bitrev(int i, int R) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// multiply by exp(DIR * 2 pi i k / 16), k = 0..7
template <int K, int DIR>
__device__ __forceinline__ cd rot16(cd a) {
  constexpr double d = (double)DIR;
  if constexpr (K == 0) {
    return a;
  } else if constexpr (K == 4) {
    return {-d * a.y, d * a.x};
  } else if constexpr (K == 2) {
    return {kC2 * (a.x - d * a.y), kC2 * (a.y + d * a.x)};
  } else if constexpr (K == 6) {
    return {kC2 * (-a.x - d * a.y), kC2 * (-a.y + d * a.x)};
  } else {
    constexpr double c = (K == 1) ? kC1 : (K == 3) ? kS1 : (K == 5) ? -kS1 : -kC1;
    constexpr double s = (K == 1) ? kS1 : (K == 3) ? kC1 : (K == 5) ? kC1 : kS1;
    return cmul(a, cd{c, d * s});
  }
}

template <int LEN, int J, int DIR>
__device__ __forceinline__ cd rot_len(cd a) {
  return rot16<(J * (16 / LEN)), DIR>(a);
}

template <int R, int DIR, int LEN, int I, int J>
__device__ __forceinline__ void dft_bfly(cd* a) {
  if constexpr (I < R) {
    if constexpr (J < LEN / 2) {
      cd u = a[I + J];
      cd t = rot_len<LEN, J, DIR>(a[I + J + LEN / 2]);
      a[I + J] = cadd(u, t);
      a[I + J + LEN / 2] = csub(u, t);
      dft_bfly<R, DIR, LEN, I, J + 1>(a);
    } else {
      dft_bfly<R, DIR, LEN, I + LEN, 0>(a);
    }
  }
}

template <int R, int DIR, int LEN>
__device__ __forceinline__ void dft_stage(cd* a) {
  if constexpr (LEN <= R) {
    dft_bfly<R, DIR, LEN, 0, 0>(a);
    dft_stage<R, DIR, LEN * 2>(a);
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(cd* v) {
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
  cd a[R];
#pragma unroll
  for (int i = 0; i < R; ++i) a[bitrev(i, R)] = v[i];
  dft_stage<R, DIR, 2>(a);
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = a[i];
}

// ---------------------------------------------------------------------------
// LDS layout of FFT scratch: one padding slot after every 8 complex
// elements (128 bytes, one row of the 32 four-byte banks).  Stockham stores
// at lane strides of 2..16 elements then spread over distinct bank groups.
__host__ __device__ constexpr int lp(int i) { return i + (i >> 3); }
// elements of a padded length-n sequence
__host__ __device__ constexpr int lp_size(int n) { return n + (n >> 3) + 1; }

// Radix schedule of a length-L transform with E elements per thread: the
// first and the last pass have radix E (so a thread's registers hold
// positions t + s*T both before the first and after the last pass, T = L/E),
// the middle factor L/E^2 is split into radices <= E.
// ---------------------------------------------------------------------------
template <int L, int E>
struct Sched {
  static_assert(L == E || L >= E * E, "schedule needs L == E or L >= E^2");
  static constexpr int T = L / E;
  static constexpr int MID = (L == E) ? 1 : L / (E * E);
  static constexpr int nmid() {
    int m = MID, n = 0;
    while (m > 1) {
      int r = m < E ? m : E;
      m /= r;
      ++n;
    }
    return n;
  }
  static constexpr int NPASS = (L == E) ? 1 : 2 + nmid();
  static constexpr int radix(int p) {
    if (p == 0 || p == NPASS - 1) return E;
    int m = MID;
    for (int i = 1; i < p; ++i) {
      int r = m < E ? m : E;
      m /= r;
    }
    return m < E ? m : E;
  }
  static constexpr int span(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= radix(i);
    return s;
  }
};

// Exchange point between Stockham passes.  When one wavefront owns the
// whole sequence (WAVE), its own LDS writes are ordered before its reads by
// the LDS pipeline; only compiler reordering has to be prevented.
template <bool WAVE>
__device__ __forceinline__ void pass_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Twiddles of pass P held by thread t: w[b (R-1) + r - 1] is
// w^{(j mod Ns) r L/(Ns R)} for butterfly j = t + b T.  Issued one pass ahead
// so that their latency overlaps the current pass and its exchange.
template <int L, int E, int P>
__device__ __forceinline__ void load_tw(cd (&w)[E], const cd* tw, int t) {
  using S = Sched<L, E>;
  if constexpr (P < S::NPASS) {
    constexpr int R = S::radix(P);
    constexpr int Ns = S::span(P);
    constexpr int B = E / R;
    if constexpr (Ns > 1) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int jm = (t + b * S::T) & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[b * (R - 1) + r - 1] = tw[jm * r * (L / (Ns * R))];
      }
    }
  }
}

// One Stockham autosort pass (radix R, span Ns) over NSEQ independent
// length-L sequences held by the same T threads.  Butterfly j reads
// positions j + r L/R, twiddles by w^{(j mod Ns) r L/(Ns R)} and writes
// (j div Ns) Ns R + (j mod Ns) + r Ns.  tw holds exp(-2 pi i m / L); w holds
// this pass's twiddles (load_tw).
template <int L, int E, int NSEQ, int DIR, int P, bool WAVE = false>
__device__ __forceinline__ void fft_pass(cd (&v)[NSEQ][E], cd* const (&lds)[NSEQ], const cd* tw,
                                         const cd (&w)[E], int t) {
  using S = Sched<L, E>;
  constexpr int R = S::radix(P);
  constexpr int Ns = S::span(P);
  constexpr int B = E / R;
  constexpr int T = S::T;
  constexpr bool FIRST = (P == 0);
  constexpr bool LAST = (P == S::NPASS - 1);
  cd wn[E];
  load_tw<L, E, P + 1>(wn, tw, t);
  if constexpr (!FIRST) {
#pragma unroll
    for (int q = 0; q < NSEQ; ++q)
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][b * R + r] = lds[q][lp(t + b * T + r * (L / R))];
  }
  if constexpr (Ns > 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cd wr = w[b * (R - 1) + r - 1];
        if (DIR > 0) wr.y = -wr.y;
#pragma unroll
        for (int q = 0; q < NSEQ; ++q) v[q][b * R + r] = cmul(v[q][b * R + r], wr);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NSEQ; ++q)
#pragma unroll
    for (int b = 0; b < B; ++b) dft<R, DIR>(&v[q][b * R]);
  if constexpr (!LAST) {
    pass_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * T;
      const int base = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
      for (int q = 0; q < NSEQ; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) lds[q][lp(base + r * Ns)] = v[q][b * R + r];
    }
    pass_sync<WAVE>();
    fft_pass<L, E, NSEQ, DIR, P + 1, WAVE>(v, lds, tw, wn, t);
  }
}

// Length-L FFT of NSEQ sequences.  On entry and on exit v[q][s] is position
// t + s*T of sequence q.  lds[q] is an LDS scratch of lp_size(L) elements per
// sequence, indexed through lp().
// Unnormalized in both directions.
// WAVE: the T = L/E threads of each sequence form one wavefront (T == 64),
// so the exchanges need no workgroup barrier.
template <int L, int E, int NSEQ, int DIR, bool WAVE = false>
__device__ __forceinline__ void fft(cd (&v)[NSEQ][E], cd* const (&lds)[NSEQ], const cd* tw, int t) {
  static_assert(!WAVE || L / E == 64, "a wave-local FFT needs 64 threads per sequence");
  cd w0[E];  // the first pass (span 1) has no twiddles
  fft_pass<L, E, NSEQ, DIR, 0, WAVE>(v, lds, tw, w0, t);
}

// ---------------------------------------------------------------------------
// Model constants and the regularized well (eq. e:Wq-def):
//   W = A B,  A = (u-b_-)^2/2 + q eps (1 - sech z),  z = (u-b_-)/eps,
//             B = (u-b_+)^2/2 + (gamma/3)(u - (3 b_+ - b_-)/2),
// with sech, tanh from exp(-|z|) (no overflow).
// ---------------------------------------------------------------------------
struct Consts {
  int N;
  double L, eps, inv_eps, eps2;
  double eta1, eta2;  // effective (eps^p eta_i)
  double q, gw3, bm, bp, bshift;
  double alpha, beta1, beta2, zeta, D0;
  double kscale;  // (2 pi / L)^2
  double invN2;   // 1 / N^2
  double h2;      // (L/N)^2
  double pars;    // L^2 / N^4: h^2 sum_x f g = pars * sum_half w Re(f g*)
};

// W, W', W'' at u.  Q = (q != 0) is a template argument so that a caller
// evaluating many points tests the uniform q once, outside its point loop,
// and the points' chains interleave.
template <bool Q>
__device__ __forceinline__ void well_t(const Consts& c, double u, double& W, double& W1,
                                       double& W2) {
  const double dm = u - c.bm, dp = u - c.bp;
  double A = 0.5 * dm * dm, A1 = dm, A2 = 1.0;
  if constexpr (Q) {
    const double z = dm * c.inv_eps;
    const double e = exp(-fabs(z));
    const double den = 1.0 / (1.0 + e * e);
    const double sech = 2.0 * e * den;
    const double th = copysign((1.0 - e * e) * den, z);
    A += c.q * c.eps * (1.0 - sech);
    A1 += c.q * sech * th;
    A2 += c.q * c.inv_eps * sech * (sech * sech - th * th);
  }
  const double B = 0.5 * dp * dp + c.gw3 * (u - c.bshift);
  const double B1 = dp + c.gw3;
  W = A * B;
  W1 = A1 * B + A * B1;
  W2 = A2 * B + 2.0 * A1 * B1 + A;
}

// Workgroup index remap so that consecutive logical tiles land on the same
// XCD (the dispatcher deals workgroups to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int blk, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = blk & 7, i = blk >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace fch
