// fch_nn.hip -- the learned PSD warm start: a 3x3 periodic convolutional
// network with BF16 weights and activations and FP32 accumulation on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16), trained on the GPU.
//
// Tensors (all device memory, owned by the caller):
//   activations  bf16 [B][H][W][32]   (NHWC, 32 channels; unused channels 0)
//   weights      bf16 [9][Cout][32]   (tap = (dy+1)*3 + (dx+1), out channel,
//                                      in channel); Cout is 32, or 16 for the
//                                      output layer (channel 0 used)
//   bias         f32  [Cout]
//   net output   f32  [B][H][W]       (channel 0 of the output layer)
// A conv computes z[p][co] = bias[co] + sum_{tap,ci} x[p+tap][ci] w[tap][co][ci]
// with periodic neighbours.  Rounding to BF16 is round-to-nearest-even.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "fch.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ u16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

// 16-byte chunk of 8 bf16 values, reinterpreted as the MFMA operand type
union Chunk {
  uint4 u;
  bf16x8 v;
};

constexpr int C = 32;  // channels of every activation tensor
constexpr int TILE = 16;
constexpr int HALO = TILE + 2;

// orders one wave's LDS writes before its other lanes read them
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup of NW waves computes a 16 x 16 pixel tile for all COUT output
// channels.  Wave w handles tile rows w, w+NW, ... (16/NW 16-pixel M tiles);
// the 9 taps x COUT/16 N tiles of B operands stay in registers.  Small
// batches (inference) take NW = 16 so that each SIMD holds four waves.  MODE 0: forward
// hidden layer (store SiLU(z) and, when z is not null, z as bf16; each M tile
// is regrouped through LDS so that a lane stores 8 channels of one pixel,
// 16 bytes, and a wave 16 whole pixels); MODE 1: forward output layer (store
// channel 0 of z as f32); MODE 2: backward data (the input is dz of the next
// layer, the weights are flipped/transposed, and the output is
// dz_prev = dy * SiLU'(z_prev) as bf16).
template <int COUT, int MODE, int NW = 4>
__global__ __launch_bounds__(NW * 64) void k_conv(int H, int W, const u16* __restrict__ x,
                                              const u16* __restrict__ w,
                                              const float* __restrict__ bias,
                                              const u16* __restrict__ zprev, u16* __restrict__ z,
                                              u16* __restrict__ y, float* __restrict__ o) {
  constexpr int NT = COUT / 16;
  __shared__ uint4 xs[HALO * HALO * (C / 8)];
  __shared__ uint4 ws[9 * COUT * (C / 8)];
  // MODE 0: per wave, one M tile of z and of y (16 pixels x 32 channels bf16,
  // pixel stride PS = 40 values: the four lane groups' writes fall in distinct
  // banks and every pixel starts on 16 bytes)
  constexpr int PS = C + 8;
  __shared__ uint4 ost[MODE == 0 ? NW : 1][2][MODE == 0 ? TILE * PS / 8 : 1];
  static_assert(TILE % NW == 0, "each wave takes TILE / NW tile rows");
  constexpr int NTHR = NW * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_w = W / TILE;
  const int b = blockIdx.y;
  const int r0 = (blockIdx.x / tiles_w) * TILE, c0 = (blockIdx.x % tiles_w) * TILE;
  const uint4* xg = (const uint4*)(x + (size_t)b * H * W * C);
  for (int i = tid; i < HALO * HALO * (C / 8); i += NTHR) {
    const int q = i & 3, pix = i >> 2;
    const int hr = pix / HALO, hc = pix - hr * HALO;
    const int gr = (r0 + hr - 1 + H) % H, gc = (c0 + hc - 1 + W) % W;
    xs[i] = xg[((size_t)gr * W + gc) * (C / 8) + q];
  }
  const uint4* wg = (const uint4*)w;
  for (int i = tid; i < 9 * COUT * (C / 8); i += NTHR) ws[i] = wg[i];
  __syncthreads();

  const int li = lane & 15, kb = lane >> 4;
  Chunk bop[9][NT];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int n = 0; n < NT; ++n) bop[t][n].u = ws[(t * COUT + n * 16 + li) * (C / 8) + kb];

#pragma unroll
  for (int m = 0; m < TILE / NW; ++m) {
    const int tr = wave + NW * m;  // tile row
    f32x4 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      Chunk a;
      a.u = xs[((tr + dy + 1) * HALO + (li + dx + 1)) * (C / 8) + kb];
#pragma unroll
      for (int n = 0; n < NT; ++n)
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, bop[t][n].v, acc[n], 0, 0, 0);
    }
    // D layout: lane holds column j = lane & 15, rows 4*(lane>>4) + e
    const int gr = r0 + tr;
    if constexpr (MODE == 0) {
      u16* zt = (u16*)ost[wave][0];
      u16* yt = (u16*)ost[wave][1];
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + li;
        const float bco = bias[co];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = (4 * kb + e) * PS + co;  // pixel c0 + 4 kb + e of the tile row
          const u16 zb = f2bf(acc[n][e] + bco);
          const float zf = bf2f(zb);
          zt[q] = zb;
          yt[q] = f2bf(zf * sigm(zf));
        }
      }
      wave_sync();
      // lane -> pixel lane / 4, channels 8 (lane % 4) .. + 7
      const int sidx = (lane >> 2) * (PS / 8) + (lane & 3);
      const size_t p = ((size_t)b * H + gr) * W + c0 + (lane >> 2);
      if (z) *(uint4*)(z + p * C + (lane & 3) * 8) = ost[wave][0][sidx];
      *(uint4*)(y + p * C + (lane & 3) * 8) = ost[wave][1][sidx];
      wave_sync();  // the next M tile rewrites the staging tile
      continue;
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int co = n * 16 + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gc = c0 + 4 * kb + e;
        const size_t p = ((size_t)b * H + gr) * W + gc;
        const float acc_v = acc[n][e];
        if constexpr (MODE == 1) {
          if (co == 0) o[p] = acc_v + bias[0];
        } else {
          const float zf = bf2f(zprev[p * C + co]);
          const float s = sigm(zf);
          y[p * C + co] = f2bf(acc_v * (s * (1.0f + zf * (1.0f - s))));
        }
      }
    }
  }
}

// flip taps and swap channel roles: wt[t'][ci][co] = w[8 - t][co][ci] (zero for
// co >= Cout), the weights of the backward-data convolution
__global__ void k_flip_weights(int cout, const u16* __restrict__ w, u16* __restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * C * C) return;
  const int co = i % C, ci = (i / C) % C, t = i / (C * C);
  wt[i] = (co < cout) ? w[((8 - t) * cout + co) * C + ci] : (u16)0;
}

// Weight and bias gradients dW[t][co][ci] = sum_p dz[p][co] x[p + t][ci],
// db[co] = sum_p dz[p][co]: a reduction over pixels, which the MFMA takes as
// its K dimension.  A workgroup owns WROWS output rows of one sample and
// walks them in 32-pixel chunks.  Per chunk it stages, channel-major in LDS,
// the WROWS + 2 input rows it needs (34 pixels with the periodic halo) and
// the WROWS dz rows, each from 16-byte global loads written as pixel pairs.
// The three horizontal tap shifts read the same input lines at offsets 0, 1,
// 2 pixels: two aligned 16-byte reads and a byte-align for the odd shift.
// Wave w owns taps w, w+4, w+8 over all rows, so its accumulators need no
// cross-wave sum.  Per-workgroup partials are reduced in a fixed order.
constexpr int WROWS = 8;
constexpr int LP = 40;  // u16 per staged line: 34 pixels + pad (80 B, 16-B aligned)
template <int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(int H, int W, const u16* __restrict__ dz,
                                                    const u16* __restrict__ x,
                                                    float* __restrict__ part) {
  constexpr int MT = COUT / 16;
  constexpr int XR = WROWS + 2;
  __shared__ __attribute__((aligned(16))) u16 xT[XR][C][LP];
  __shared__ __attribute__((aligned(16))) u16 dzT[WROWS][COUT][LP];
  __shared__ float dbs[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kb = lane >> 4;
  const int bands = H / WROWS;
  const int b = blockIdx.x / bands, r0 = (blockIdx.x % bands) * WROWS;
  const uint4* dzb = (const uint4*)(dz + (size_t)b * H * W * C);
  const uint4* xb = (const uint4*)(x + (size_t)b * H * W * C);
  f32x4 acc[3][MT][2];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[s][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // bias: thread (co, row) sums its row's 32 pixels per chunk
  constexpr int DBT = COUT * WROWS;  // threads that take part (<= 256)
  float dbacc = 0.f;
  for (int c0 = 0; c0 < W; c0 += 32) {
    __syncthreads();
    // input lines: rows r0-1 .. r0+WROWS, pixels c0-1 .. c0+32 as pairs
    for (int i = tid; i < XR * 17 * (C / 8); i += 256) {
      const int q = i % (C / 8), pr = (i / (C / 8)) % 17, rr = i / ((C / 8) * 17);
      const int gr = (r0 + rr - 1 + H) % H;
      const int g0 = (c0 + 2 * pr - 1 + W) % W, g1 = (c0 + 2 * pr + W) % W;
      const uint4 v0 = xb[((size_t)gr * W + g0) * (C / 8) + q];
      const uint4 v1 = xb[((size_t)gr * W + g1) * (C / 8) + q];
      const uint32_t a0[4] = {v0.x, v0.y, v0.z, v0.w}, a1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // channels q*8 + 2j (low halves) and q*8 + 2j + 1 (high halves)
        *(uint32_t*)&xT[rr][q * 8 + 2 * j][2 * pr] = (a0[j] & 0xffffu) | (a1[j] << 16);
        *(uint32_t*)&xT[rr][q * 8 + 2 * j + 1][2 * pr] = (a0[j] >> 16) | (a1[j] & 0xffff0000u);
      }
    }
    // dz lines: rows r0 .. r0+WROWS-1, pixels c0 .. c0+31 as pairs
    for (int i = tid; i < WROWS * 16 * (COUT / 8); i += 256) {
      const int q = i % (COUT / 8), pr = (i / (COUT / 8)) % 16, rr = i / ((COUT / 8) * 16);
      const size_t p0 = (size_t)(r0 + rr) * W + c0 + 2 * pr;
      const uint4 v0 = dzb[p0 * (C / 8) + q];
      const uint4 v1 = dzb[(p0 + 1) * (C / 8) + q];
      const uint32_t a0[4] = {v0.x, v0.y, v0.z, v0.w}, a1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        *(uint32_t*)&dzT[rr][q * 8 + 2 * j][2 * pr] = (a0[j] & 0xffffu) | (a1[j] << 16);
        *(uint32_t*)&dzT[rr][q * 8 + 2 * j + 1][2 * pr] = (a0[j] >> 16) | (a1[j] & 0xffff0000u);
      }
    }
    __syncthreads();
    if (tid < DBT) {
      const int co = tid % COUT, rr = tid / COUT;
      float sacc = 0.f;
      for (int px = 0; px < 32; ++px) sacc += bf2f(dzT[rr][co][px]);
      dbacc += sacc;
    }
#pragma unroll 1
    for (int rr = 0; rr < WROWS; ++rr) {
      Chunk a[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) a[m].u = *(const uint4*)&dzT[rr][m * 16 + li][kb * 8];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int t = wave + 4 * s;
        if (t < 9) {
          const int dy = t / 3 - 1, sh = t % 3;  // line offset (pixels) = dx + 1
#pragma unroll
          for (int n = 0; n < 2; ++n) {
            const u16* line = &xT[rr + dy + 1][n * 16 + li][kb * 8];
            const uint4 lo = *(const uint4*)line;
            Chunk bb;
            if (sh == 0) {
              bb.u = lo;
            } else {
              const uint4 hi = *(const uint4*)(line + 8);
              if (sh == 2) {
                bb.u = uint4{lo.y, lo.z, lo.w, hi.x};
              } else {
                bb.u = uint4{__builtin_amdgcn_alignbyte(lo.y, lo.x, 2),
                             __builtin_amdgcn_alignbyte(lo.z, lo.y, 2),
                             __builtin_amdgcn_alignbyte(lo.w, lo.z, 2),
                             __builtin_amdgcn_alignbyte(hi.x, lo.w, 2)};
              }
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
              acc[s][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m].v, bb.v, acc[s][m][n], 0,
                                                                    0, 0);
          }
        }
      }
    }
  }
  // partial layout per workgroup: [9][COUT][32] weights, then [COUT] bias
  float* pw = part + (size_t)blockIdx.x * (9 * COUT * C + COUT);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int t = wave + 4 * s;
    if (t < 9) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int co = m * 16 + 4 * kb + e, ci = n * 16 + li;
            pw[(t * COUT + co) * C + ci] = acc[s][m][n][e];
          }
    }
  }
  dbs[tid] = (tid < DBT) ? dbacc : 0.f;
  __syncthreads();
  if (tid < COUT) {
    float sdb = 0.f;
    for (int rr = 0; rr < WROWS; ++rr) sdb += dbs[rr * COUT + tid];
    pw[9 * COUT * C + tid] = sdb;
  }
}

// fixed-order sum of nparts partial vectors (one thread per element)
__global__ void k_reduce_parts(int nparts, int len, const float* __restrict__ part,
                               float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int k = 0; k < nparts; ++k) s += part[(size_t)k * len + i];
  out[i] = s;
}

// fixed-order sum of the per-workgroup partials, in two stages: RG groups of
// consecutive partials, then the groups in order
constexpr int RG = 16;
__global__ void k_reduce_stage1(int nparts, int len, const float* __restrict__ part,
                                float* __restrict__ tmp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (i >= len) return;
  const int per = (nparts + RG - 1) / RG;
  const int k0 = g * per, k1 = min(nparts, k0 + per);
  float s = 0.f;
  for (int k = k0; k < k1; ++k) s += part[(size_t)k * len + i];
  tmp[(size_t)g * len + i] = s;
}
__global__ void k_reduce_stage2(int len, const float* __restrict__ tmp, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int g = 0; g < RG; ++g) s += tmp[(size_t)g * len + i];
  out[i] = s;
}

// loss = mean (o - t)^2 over B*H*W; dz (bf16, 32 channels) = 2 (o - t) / n in
// channel 0 and 0 elsewhere; per-block partial sums of the squared error / n
__global__ __launch_bounds__(256) void k_mse(int n, const float* __restrict__ o,
                                             const float* __restrict__ t, u16* __restrict__ dz,
                                             float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0.f;
  const float sc = 2.0f / (float)n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float d = o[i] - t[i];
    s += d * d;
    uint4* row = (uint4*)(dz + (size_t)i * C);
    uint4 zero = {0, 0, 0, 0};
    uint4 first = zero;
    first.x = f2bf(sc * d);
    row[0] = first;
    row[1] = zero;
    row[2] = zero;
    row[3] = zero;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] / (float)n;
}

// Adam on FP32 master parameters, with the bf16 copy used by the convs
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, u16* __restrict__ pb,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void k_to_bf16(int n, const float* __restrict__ p, u16* __restrict__ pb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

// Features of B samples, over the whole grid: d = (u^n - u^{n-1}) k_{n+1}/k_n,
// s = RMS(d), x = [u^n, d/s, (log10 k_{n+1} + 3)/2, 0...] as bf16, and the
// target (u^{n+1} - u^n - d)/s when u^{n+1} is given.  First kernel: partial
// sums of d^2 over FEAT_BLK chunks of each sample; second: every block forms
// s from its sample's partials in the same order (block 0 records it) and
// writes its chunk.
constexpr int FEAT_BLK = 64;
__global__ __launch_bounds__(256) void k_feat_part(int HW, const double* __restrict__ un,
                                                   const double* __restrict__ um,
                                                   const double* __restrict__ kk,
                                                   double* __restrict__ work) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const double r = kk[2 * b] / kk[2 * b + 1];
  const double* a = un + (size_t)b * HW;
  const double* p = um + (size_t)b * HW;
  const int chunk = (HW + FEAT_BLK - 1) / FEAT_BLK;
  const int lo = blockIdx.x * chunk, hi = min(HW, lo + chunk);
  double s2 = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += 256) {
    const double d = (a[i] - p[i]) * r;
    s2 += d * d;
  }
  red[threadIdx.x] = s2;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) work[b * FEAT_BLK + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_feat_write(int HW, const double* __restrict__ un,
                                                    const double* __restrict__ um,
                                                    const double* __restrict__ unp1,
                                                    const double* __restrict__ kk,
                                                    const double* __restrict__ work,
                                                    u16* __restrict__ x, float* __restrict__ tgt,
                                                    double* __restrict__ scale) {
  __shared__ double sh;
  const int b = blockIdx.y;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < FEAT_BLK; ++i) t += work[b * FEAT_BLK + i];
    double s = sqrt(t / HW);
    if (!(s > 1e-300)) s = 1e-300;
    sh = s;
    if (blockIdx.x == 0) scale[b] = s;
  }
  __syncthreads();
  const double s = sh;
  const double r = kk[2 * b] / kk[2 * b + 1];
  const float lk = (float)((log10(kk[2 * b]) + 3.0) * 0.5);
  const u16 lkb = f2bf(lk);
  const size_t base = (size_t)b * HW;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < HW; i += gridDim.x * 256) {
    const double a = un[base + i];
    const double d = (a - um[base + i]) * r;
    uint4* row = (uint4*)(x + (base + i) * C);
    uint4 first = {0, 0, 0, 0};
    first.x = (uint32_t)f2bf((float)a) | ((uint32_t)f2bf((float)(d / s)) << 16);
    first.y = lkb;
    const uint4 zero = {0, 0, 0, 0};
    row[0] = first;
    row[1] = zero;
    row[2] = zero;
    row[3] = zero;
    if (unp1 && tgt) tgt[base + i] = (float)((unp1[base + i] - a - d) / s);
  }
}

// guess g = u^n + d + s * o (the extrapolation of eq. recurrence plus the
// learned correction)
__global__ void k_guess(int HW, int B, const double* __restrict__ un, const double* __restrict__ um,
                        const double* __restrict__ kk, const double* __restrict__ scale,
                        const float* __restrict__ o, double* __restrict__ g) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)HW * B) return;
  const int b = (int)(i / HW);
  const double d = (un[i] - um[i]) * (kk[2 * b] / kk[2 * b + 1]);
  g[i] = un[i] + d + scale[b] * (double)o[i];
}

bool ok_dims(int B, int H, int W) { return B > 0 && H >= 16 && W >= 32 && H % 16 == 0 && W % 32 == 0; }

}  // namespace

extern "C" {

fch_status fch_nn_conv_fwd(int32_t B, int32_t H, int32_t W, int32_t cout, const void* x,
                           const void* w, const float* bias, void* z, void* y, float* o,
                           void* stream) {
  if (!ok_dims(B, H, W) || !x || !w || !bias) return FCH_E_INVALID;
  const dim3 grid((H / 16) * (W / 16), B);
  hipStream_t s = (hipStream_t)stream;
  // fewer tiles than two per CU: 16-wave workgroups, one tile row per wave
  const bool small = (size_t)grid.x * grid.y < 512;
  if (cout == 32) {
    if (!y) return FCH_E_INVALID;  // z may be null (inference)
    if (small)
      hipLaunchKernelGGL((k_conv<32, 0, 16>), grid, dim3(1024), 0, s, H, W, (const u16*)x,
                         (const u16*)w, bias, nullptr, (u16*)z, (u16*)y, nullptr);
    else
      hipLaunchKernelGGL((k_conv<32, 0>), grid, dim3(256), 0, s, H, W, (const u16*)x,
                         (const u16*)w, bias, nullptr, (u16*)z, (u16*)y, nullptr);
  } else if (cout == 16) {
    if (!o) return FCH_E_INVALID;
    if (small)
      hipLaunchKernelGGL((k_conv<16, 1, 16>), grid, dim3(1024), 0, s, H, W, (const u16*)x,
                         (const u16*)w, bias, nullptr, nullptr, nullptr, o);
    else
      hipLaunchKernelGGL((k_conv<16, 1>), grid, dim3(256), 0, s, H, W, (const u16*)x,
                         (const u16*)w, bias, nullptr, nullptr, nullptr, o);
  } else {
    return FCH_E_INVALID;
  }
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_conv_bwd_data(int32_t B, int32_t H, int32_t W, int32_t cout, const void* dz,
                                const void* w, const void* z_prev, void* dz_prev, void* wt,
                                void* stream) {
  if (!ok_dims(B, H, W) || !dz || !w || !z_prev || !dz_prev || !wt) return FCH_E_INVALID;
  if (cout != 32 && cout != 16) return FCH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_flip_weights, dim3((9 * C * C + 255) / 256), dim3(256), 0, s, cout,
                     (const u16*)w, (u16*)wt);
  const dim3 grid((H / 16) * (W / 16), B);
  hipLaunchKernelGGL((k_conv<32, 2>), grid, dim3(256), 0, s, H, W, (const u16*)dz,
                     (const u16*)wt, nullptr, (const u16*)z_prev, nullptr, (u16*)dz_prev,
                     nullptr);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

size_t fch_nn_bwd_w_scratch_floats(int32_t B, int32_t H, int32_t W) {
  // per-workgroup partials, then the RG group sums of the reduction
  return (size_t)(B * (H / WROWS) + RG) * (9 * C * C + C);
}

fch_status fch_nn_conv_bwd_w(int32_t B, int32_t H, int32_t W, int32_t cout, const void* dz,
                             const void* x, float* dw_db, float* scratch, void* stream) {
  if (!ok_dims(B, H, W) || H % WROWS || !dz || !x || !dw_db || !scratch) return FCH_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const int nwg = B * (H / WROWS);
  const int len = 9 * cout * C + cout;
  if (cout == 32) {
    hipLaunchKernelGGL((k_conv_bwd_w<32>), dim3(nwg), dim3(256), 0, s, H, W, (const u16*)dz,
                       (const u16*)x, scratch);
  } else if (cout == 16) {
    hipLaunchKernelGGL((k_conv_bwd_w<16>), dim3(nwg), dim3(256), 0, s, H, W, (const u16*)dz,
                       (const u16*)x, scratch);
  } else {
    return FCH_E_INVALID;
  }
  float* tmp = scratch + (size_t)nwg * len;
  hipLaunchKernelGGL(k_reduce_stage1, dim3((len + 255) / 256, RG), dim3(256), 0, s, nwg, len,
                     scratch, tmp);
  hipLaunchKernelGGL(k_reduce_stage2, dim3((len + 255) / 256), dim3(256), 0, s, len, tmp, dw_db);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_reduce(int32_t nparts, int32_t len, const float* part, float* out,
                         void* stream) {
  if (nparts < 1 || len < 1 || !part || !out) return FCH_E_INVALID;
  hipLaunchKernelGGL(k_reduce_parts, dim3((len + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     nparts, len, part, out);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_mse(int32_t n, const float* o, const float* target, void* dz, float* part,
                      int32_t nblocks, void* stream) {
  if (n < 1 || !o || !target || !dz || !part || nblocks < 1) return FCH_E_INVALID;
  hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, n, o, target,
                     (u16*)dz, part);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_adam(int32_t n, float* p, const float* g, float* m, float* v, void* p_bf16,
                       double lr, double b1, double b2, double eps, int32_t step, void* stream) {
  if (n < 1 || !p || !g || !m || !v || step < 1) return FCH_E_INVALID;
  const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, p, g, m,
                     v, (u16*)p_bf16, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_to_bf16(int32_t n, const float* p, void* p_bf16, void* stream) {
  if (n < 1 || !p || !p_bf16) return FCH_E_INVALID;
  hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, p,
                     (u16*)p_bf16);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

int32_t fch_nn_features_work_doubles(int32_t B) { return B > 0 ? B * FEAT_BLK : 0; }

fch_status fch_nn_features(int32_t B, int32_t H, int32_t W, const double* u_n, const double* u_nm1,
                           const double* u_np1, const double* k, void* x, float* target,
                           double* scale, double* work, void* stream) {
  if (!ok_dims(B, H, W) || !u_n || !u_nm1 || !k || !x || !scale || !work) return FCH_E_INVALID;
  const hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_feat_part, dim3(FEAT_BLK, B), dim3(256), 0, st, H * W, u_n, u_nm1, k, work);
  const int nblk = (H * W + 255) / 256 < 128 ? (H * W + 255) / 256 : 128;
  hipLaunchKernelGGL(k_feat_write, dim3(nblk, B), dim3(256), 0, st, H * W, u_n, u_nm1, u_np1, k,
                     work, (u16*)x, target, scale);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

fch_status fch_nn_guess(int32_t B, int32_t H, int32_t W, const double* u_n, const double* u_nm1,
                        const double* k, const double* scale, const float* o, double* g,
                        void* stream) {
  if (!ok_dims(B, H, W) || !u_n || !u_nm1 || !k || !scale || !o || !g) return FCH_E_INVALID;
  const size_t n = (size_t)B * H * W;
  hipLaunchKernelGGL(k_guess, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     H * W, B, u_n, u_nm1, k, scale, o, g);
  return hipGetLastError() == hipSuccess ? FCH_OK : FCH_E_HIP;
}

}  // extern "C"
