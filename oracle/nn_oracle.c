/*
 * nn_oracle.c -- FP64 reference of the learned PSD warm start network.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the product
 * library never links it.
 *
 * A 3x3 periodic convolution over NHWC tensors with 32 channels:
 *   z[p][co] = bias[co] + sum_{tap, ci} x[p + off(tap)][ci] w[tap][co][ci],
 *   off(tap) = (tap/3 - 1, tap%3 - 1) in (row, column), periodic.
 * Hidden layers apply SiLU(z) = z / (1 + exp(-z)); the output layer keeps
 * channel 0 of z.  Gradients follow the chain rule written out per layer.
 * With round_bf16 = 1 the quantities the GPU stores in bfloat16 (inputs,
 * weights, z, SiLU(z), dz operands) are rounded to the nearest bfloat16
 * (ties to even) at the same points; with 0 everything stays FP64 (used for
 * the finite-difference check of the gradients).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NC 32

double nn_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double rnd(double v, int r) { return r ? nn_bf16(v) : v; }
static double sig(double z) { return 1.0 / (1.0 + exp(-z)); }

static long pix(int H, int W, int b, int r, int c) {
    r = (r % H + H) % H;
    c = (c % W + W) % W;
    return ((long)b * H + r) * W + c;
}

/* forward of one layer: x [B][H][W][32] (values), w [9][cout][32], bias[cout];
 * hidden (cout = 32): z, y [B][H][W][32]; output (cout = 16): o [B][H][W] */
void nn_conv_fwd(int B, int H, int W, int cout, const double* x, const double* w,
                 const double* bias, double* z, double* y, double* o, int round_bf16) {
    for (int b = 0; b < B; ++b)
        for (int r = 0; r < H; ++r)
            for (int c = 0; c < W; ++c) {
                long p = pix(H, W, b, r, c);
                for (int co = 0; co < cout; ++co) {
                    double s = 0.0;
                    for (int t = 0; t < 9; ++t) {
                        long q = pix(H, W, b, r + t / 3 - 1, c + t % 3 - 1);
                        const double* xp = x + q * NC;
                        const double* wp = w + ((long)t * cout + co) * NC;
                        for (int ci = 0; ci < NC; ++ci) s += xp[ci] * wp[ci];
                    }
                    s += bias[co];
                    if (cout == 32) {
                        double zb = rnd(s, round_bf16);
                        z[p * NC + co] = zb;
                        y[p * NC + co] = rnd(zb * sig(zb), round_bf16);
                    } else if (co == 0) {
                        o[p] = s;
                    }
                }
            }
}

/* dx[q][ci] = SiLU'(z_prev[q][ci]) * sum_{tap, co} dz[q - off(tap)][co] w[tap][co][ci] */
void nn_conv_bwd_data(int B, int H, int W, int cout, const double* dz, const double* w,
                      const double* z_prev, double* dz_prev, int round_bf16) {
    for (int b = 0; b < B; ++b)
        for (int r = 0; r < H; ++r)
            for (int c = 0; c < W; ++c) {
                long q = pix(H, W, b, r, c);
                for (int ci = 0; ci < NC; ++ci) {
                    double s = 0.0;
                    for (int t = 0; t < 9; ++t) {
                        long p = pix(H, W, b, r - (t / 3 - 1), c - (t % 3 - 1));
                        for (int co = 0; co < cout; ++co)
                            s += dz[p * NC + co] * w[((long)t * cout + co) * NC + ci];
                    }
                    double zp = z_prev[q * NC + ci];
                    double sg = sig(zp);
                    dz_prev[q * NC + ci] = rnd(s * sg * (1.0 + zp * (1.0 - sg)), round_bf16);
                }
            }
}

/* dw[tap][co][ci] = sum_p dz[p][co] x[p + off(tap)][ci], db[co] = sum_p dz[p][co] */
void nn_conv_bwd_w(int B, int H, int W, int cout, const double* dz, const double* x, double* dw,
                   double* db) {
    memset(dw, 0, sizeof(double) * 9 * cout * NC);
    memset(db, 0, sizeof(double) * cout);
    for (int b = 0; b < B; ++b)
        for (int r = 0; r < H; ++r)
            for (int c = 0; c < W; ++c) {
                long p = pix(H, W, b, r, c);
                for (int co = 0; co < cout; ++co) {
                    double g = dz[p * NC + co];
                    if (g == 0.0) continue;
                    db[co] += g;
                    for (int t = 0; t < 9; ++t) {
                        long q = pix(H, W, b, r + t / 3 - 1, c + t % 3 - 1);
                        for (int ci = 0; ci < NC; ++ci)
                            dw[((long)t * cout + co) * NC + ci] += g * x[q * NC + ci];
                    }
                }
            }
}

/* mean squared error over n values and dz of the output layer (32 channels,
 * channel 0 = 2 (o - t)/n) */
double nn_mse(long n, const double* o, const double* t, double* dz, int round_bf16) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = o[i] - t[i];
        s += d * d;
        for (int c = 0; c < NC; ++c) dz[i * NC + c] = 0.0;
        dz[i * NC] = rnd(2.0 * d / (double)n, round_bf16);
    }
    return s / (double)n;
}
