/*
 * fch_oracle.c -- plain FP64 CPU oracle for the FCH pseudo-spectral BDF2 path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  The product library never links it.
 *
 * Every routine is written for a reader with the paper beside them: the
 * transforms are the plain DFT definition (a naive O(n^2) line DFT, and a
 * textbook radix-2 FFT that reaches the same numbers faster), the model
 * pieces are the paper's formulas evaluated pointwise with pseudo-spectral
 * Laplacians, and the schemes take the paper's steps in its order.
 * Reductions are serial (deterministic); OpenMP only splits independent lines.
 */
#include "fch_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.28318530717958647692528676655900577;

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* exp(sign * 2 pi i m / n) for an integer m already reduced mod n */
static cplx unit_root(long m, long n, int sign) {
    double ang = TWO_PI * (double)m / (double)n;
    return cos(ang) + (double)sign * sin(ang) * I;
}

/* ------------------------------------------------------------------------ */
/* Transforms: the DFT definition  X[k] = sum_j x[j] exp(sign 2 pi i j k / n) */
/* ------------------------------------------------------------------------ */

void oracle_dft_1d(int n, const double* in, double* out, int sign) {
    const cplx* x = (const cplx*)in;
    cplx* X = (cplx*)out;
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    for (int k = 0; k < n; ++k) {
        cplx s = 0.0;
        for (int j = 0; j < n; ++j) {
            long m = ((long)j * (long)k) % n;   /* exact argument reduction */
            s += x[j] * unit_root(m, n, sign);
        }
        tmp[k] = s;
    }
    memcpy(X, tmp, sizeof(cplx) * (size_t)n);
    free(tmp);
}

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* iterative radix-2 decimation-in-time FFT (bit reversal, then butterflies);
 * each twiddle is evaluated directly from cos/sin, never by recurrence */
int oracle_fft_1d(int n, double* data, int sign) {
    if (!is_pow2(n)) return -1;
    cplx* a = (cplx*)data;
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1;
        for (int i = 0; i < n; i += len) {
            for (int j = 0; j < half; ++j) {
                cplx w = unit_root(j, len, sign);
                cplx u = a[i + j];
                cplx v = a[i + j + half] * w;
                a[i + j] = u + v;
                a[i + j + half] = u - v;
            }
        }
    }
    return 0;
}

static void line_transform(int n, cplx* line, cplx* scratch, int sign, int method) {
    if (method == 0) {
        oracle_dft_1d(n, (const double*)line, (double*)scratch, sign);
        memcpy(line, scratch, sizeof(cplx) * (size_t)n);
    } else {
        oracle_fft_1d(n, (double*)line, sign);
    }
}

void oracle_dft2_brute(int N, const double* u, double* uh_) {
    cplx* uh = (cplx*)uh_;
    int H = N / 2 + 1;
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            cplx s = 0.0;
            for (int y = 0; y < N; ++y)
                for (int x = 0; x < N; ++x) {
                    long m = ((long)ky * y + (long)kx * x) % N;
                    s += u[y * N + x] * unit_root(m, N, -1);
                }
            uh[ky * H + kx] = s;
        }
}

int oracle_r2c(int N, const double* u, double* uh_, int method) {
    if (N < 2 || (method == 1 && !is_pow2(N)) || (N % 2)) return -1;
    cplx* uh = (cplx*)uh_;
    int H = N / 2 + 1;
    /* rows: transform along x, keep kx = 0..N/2 */
#pragma omp parallel
    {
        cplx* line = (cplx*)malloc(sizeof(cplx) * (size_t)N);
        cplx* scr = (cplx*)malloc(sizeof(cplx) * (size_t)N);
#pragma omp for schedule(static)
        for (int y = 0; y < N; ++y) {
            for (int x = 0; x < N; ++x) line[x] = u[y * N + x];
            line_transform(N, line, scr, -1, method);
            for (int kx = 0; kx < H; ++kx) uh[y * H + kx] = line[kx];
        }
        /* columns: transform along y */
#pragma omp for schedule(static)
        for (int kx = 0; kx < H; ++kx) {
            for (int y = 0; y < N; ++y) line[y] = uh[y * H + kx];
            line_transform(N, line, scr, -1, method);
            for (int ky = 0; ky < N; ++ky) uh[ky * H + kx] = line[ky];
        }
        free(line);
        free(scr);
    }
    return 0;
}

int oracle_c2r(int N, const double* uh_, double* u, int method) {
    if (N < 2 || (method == 1 && !is_pow2(N)) || (N % 2)) return -1;
    const cplx* uh = (const cplx*)uh_;
    int H = N / 2 + 1;
    cplx* g = (cplx*)malloc(sizeof(cplx) * (size_t)N * H);
    double scale = 1.0 / ((double)N * (double)N);
#pragma omp parallel
    {
        cplx* line = (cplx*)malloc(sizeof(cplx) * (size_t)N);
        cplx* scr = (cplx*)malloc(sizeof(cplx) * (size_t)N);
        /* columns: inverse along ky */
#pragma omp for schedule(static)
        for (int kx = 0; kx < H; ++kx) {
            for (int ky = 0; ky < N; ++ky) line[ky] = uh[ky * H + kx];
            line_transform(N, line, scr, +1, method);
            for (int y = 0; y < N; ++y) g[y * H + kx] = line[y];
        }
        /* rows: Hermitian extension in kx, inverse, real part */
#pragma omp for schedule(static)
        for (int y = 0; y < N; ++y) {
            for (int kx = 0; kx < N; ++kx)
                line[kx] = (kx < H) ? g[y * H + kx] : conj(g[y * H + (N - kx)]);
            line_transform(N, line, scr, +1, method);
            for (int x = 0; x < N; ++x) u[y * N + x] = creal(line[x]) * scale;
        }
        free(line);
        free(scr);
    }
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Model pieces                                                              */
/* ------------------------------------------------------------------------ */

static int method_for(int N) { return is_pow2(N) ? 1 : 0; }

static double eff_eta(const oracle_params* P, double eta) { return eta * pow(P->eps, P->p); }

static double k2_at(const oracle_params* P, int ky, int kx) {
    int N = P->N;
    double kxv = TWO_PI * (double)kx / P->L;
    double kyv = TWO_PI * (double)(ky <= N / 2 ? ky : ky - N) / P->L;
    return kxv * kxv + kyv * kyv;
}

/* W_q of eq. e:Wq-def as the product A(u) B(u), with its first two
 * derivatives by the product rule.  sech and tanh of z = (u - b_-)/eps are
 * formed from exp(-|z|) so that nothing overflows. */
void oracle_well(const oracle_params* P, int n, const double* u,
                 double* W, double* W1, double* W2) {
    const double eps = P->eps, q = P->q, g = P->gamma_w;
    const double bm = P->b_minus, bp = P->b_plus;
    for (int i = 0; i < n; ++i) {
        double v = u[i];
        double z = (v - bm) / eps;
        double e = exp(-fabs(z));
        double sech = 2.0 * e / (1.0 + e * e);
        double tnh = (z >= 0 ? 1.0 : -1.0) * (1.0 - e * e) / (1.0 + e * e);
        double dm = v - bm, dp = v - bp;
        double A = 0.5 * dm * dm + q * eps * (1.0 - sech);
        double A1 = dm + q * sech * tnh;
        double A2 = 1.0 + (q / eps) * sech * (sech * sech - tnh * tnh);
        double B = 0.5 * dp * dp + (g / 3.0) * (v - 0.5 * (3.0 * bp - bm));
        double B1 = dp + g / 3.0;
        double B2 = 1.0;
        if (W) W[i] = A * B;
        if (W1) W1[i] = A1 * B + A * B1;
        if (W2) W2[i] = A2 * B + 2.0 * A1 * B1 + A * B2;
    }
}

double oracle_alpha_m(const oracle_params* P) {
    double u = P->b_minus, w2;
    oracle_well(P, 1, &u, NULL, NULL, &w2);
    return w2;
}

static size_t nphys(const oracle_params* P) { return (size_t)P->N * (size_t)P->N; }
static size_t nspec(const oracle_params* P) { return (size_t)P->N * (size_t)(P->N / 2 + 1); }

/* pseudo-spectral Laplacian of a physical field */
void oracle_laplacian(const oracle_params* P, const double* u, double* lap) {
    int N = P->N, H = N / 2 + 1;
    cplx* h = (cplx*)malloc(sizeof(cplx) * nspec(P));
    oracle_r2c(N, u, (double*)h, method_for(N));
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) h[ky * H + kx] *= -k2_at(P, ky, kx);
    oracle_c2r(N, (const double*)h, lap, method_for(N));
    free(h);
}

/* physical u, Laplacian of u, W', W'' and omega = eps^2 Lap u - W'(u) */
typedef struct {
    double *u, *lap, *W, *W1, *W2, *omega;
} fields_t;

static void fields_alloc(const oracle_params* P, fields_t* f) {
    size_t n = nphys(P);
    f->u = malloc(n * sizeof(double));
    f->lap = malloc(n * sizeof(double));
    f->W = malloc(n * sizeof(double));
    f->W1 = malloc(n * sizeof(double));
    f->W2 = malloc(n * sizeof(double));
    f->omega = malloc(n * sizeof(double));
}
static void fields_free(fields_t* f) {
    free(f->u); free(f->lap); free(f->W); free(f->W1); free(f->W2); free(f->omega);
}
static void fields_eval(const oracle_params* P, const double* uh, fields_t* f) {
    int N = P->N;
    size_t n = nphys(P);
    oracle_c2r(N, uh, f->u, method_for(N));
    oracle_laplacian(P, f->u, f->lap);
    oracle_well(P, (int)n, f->u, f->W, f->W1, f->W2);
    double e2 = P->eps * P->eps;
    for (size_t i = 0; i < n; ++i) f->omega[i] = e2 * f->lap[i] - f->W1[i];
}

/* mu = (eps^2 Lap - W''(u)) omega + eps^2 eta1 Lap u - eta2 W'(u),
 * the bracket of eq. FCH, with omega = eps^2 Lap u - W'(u). */
int oracle_mu(const oracle_params* P, const double* uh, double* muh) {
    int N = P->N;
    size_t n = nphys(P);
    fields_t f;
    fields_alloc(P, &f);
    fields_eval(P, uh, &f);
    double* lap_om = malloc(n * sizeof(double));
    double* mu = malloc(n * sizeof(double));
    oracle_laplacian(P, f.omega, lap_om);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1), eta2 = eff_eta(P, P->eta2);
    for (size_t i = 0; i < n; ++i)
        mu[i] = e2 * lap_om[i] - f.W2[i] * f.omega[i] + e2 * eta1 * f.lap[i] - eta2 * f.W1[i];
    int rc = oracle_r2c(N, mu, muh, method_for(N));
    free(lap_om);
    free(mu);
    fields_free(&f);
    return rc;
}

/* F(u) = Lap mu (eq. sFCH) */
int oracle_F(const oracle_params* P, const double* uh, double* Fh_) {
    int N = P->N, H = N / 2 + 1;
    int rc = oracle_mu(P, uh, Fh_);
    cplx* Fh = (cplx*)Fh_;
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) Fh[ky * H + kx] *= -k2_at(P, ky, kx);
    return rc;
}

/* h^2 sum f g over the grid, both given as half spectra */
double oracle_inner(const oracle_params* P, const double* fh, const double* gh) {
    int N = P->N;
    size_t n = nphys(P);
    double* f = malloc(n * sizeof(double));
    double* g = malloc(n * sizeof(double));
    oracle_c2r(N, fh, f, method_for(N));
    oracle_c2r(N, gh, g, method_for(N));
    double h = P->L / N, s = 0.0;
    for (size_t i = 0; i < n; ++i) s += f[i] * g[i];
    free(f);
    free(g);
    return h * h * s;
}

/* E_h = h^2 sum [ omega^2/2 - eta2 W ] - (eps^2 eta1 / 2) ||grad u||^2 with
 * ||grad u||^2 = -h^2 sum u Lap u (eq. Functional) */
double oracle_energy(const oracle_params* P, const double* uh) {
    size_t n = nphys(P);
    fields_t f;
    fields_alloc(P, &f);
    fields_eval(P, uh, &f);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1), eta2 = eff_eta(P, P->eta2);
    double s = 0.0, grad2 = 0.0;
    for (size_t i = 0; i < n; ++i) {
        s += 0.5 * f.omega[i] * f.omega[i] - eta2 * f.W[i];
        grad2 += -f.u[i] * f.lap[i];
    }
    double h = P->L / P->N;
    fields_free(&f);
    return h * h * (s - 0.5 * e2 * eta1 * grad2);
}

double oracle_mass(const oracle_params* P, const double* uh) {
    size_t n = nphys(P);
    double* u = malloc(n * sizeof(double));
    oracle_c2r(P->N, uh, u, method_for(P->N));
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += u[i] + 1.0;
    free(u);
    double h = P->L / P->N;
    return 0.5 * h * h * s;
}

/* E_1(u) = int G(u), G = -eps^2 Lap u (W' + zeta u) + W'^2/2 - eta2 W (eq. e:G-def) */
double oracle_E1(const oracle_params* P, const double* uh) {
    size_t n = nphys(P);
    fields_t f;
    fields_alloc(P, &f);
    fields_eval(P, uh, &f);
    double e2 = P->eps * P->eps, eta2 = eff_eta(P, P->eta2);
    double s = 0.0;
    for (size_t i = 0; i < n; ++i)
        s += -e2 * f.lap[i] * (f.W1[i] + P->zeta * f.u[i]) + 0.5 * f.W1[i] * f.W1[i] - eta2 * f.W[i];
    double h = P->L / P->N;
    fields_free(&f);
    return h * h * s;
}

/* V = dE_1/du written out by the chain rule:
 * V = -eps^2 Lap(W') - eps^2 W'' Lap u - 2 zeta eps^2 Lap u + W' W'' - eta2 W' */
int oracle_V(const oracle_params* P, const double* uh, double* Vh) {
    size_t n = nphys(P);
    fields_t f;
    fields_alloc(P, &f);
    fields_eval(P, uh, &f);
    double* lapW1 = malloc(n * sizeof(double));
    double* V = malloc(n * sizeof(double));
    oracle_laplacian(P, f.W1, lapW1);
    double e2 = P->eps * P->eps, eta2 = eff_eta(P, P->eta2);
    for (size_t i = 0; i < n; ++i)
        V[i] = -e2 * lapW1[i] - e2 * f.W2[i] * f.lap[i] - 2.0 * P->zeta * e2 * f.lap[i]
             + f.W1[i] * f.W2[i] - eta2 * f.W1[i];
    int rc = oracle_r2c(P->N, V, Vh, method_for(P->N));
    free(lapW1);
    free(V);
    fields_free(&f);
    return rc;
}

/* physical-space operators of the SAV split (eqs. e:def-LSAV, e:SAV-L1) */
static void apply_LSAV(const oracle_params* P, const double* f, double* out) {
    size_t n = nphys(P);
    double* l1 = malloc(n * sizeof(double));
    double* l2 = malloc(n * sizeof(double));
    oracle_laplacian(P, f, l1);
    oracle_laplacian(P, l1, l2);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1);
    for (size_t i = 0; i < n; ++i) out[i] = e2 * e2 * l2[i] + e2 * (eta1 + 2.0 * P->zeta) * l1[i];
    free(l1);
    free(l2);
}
static void apply_L1(const oracle_params* P, const double* f, double* out) {
    size_t n = nphys(P);
    double* l1 = malloc(n * sizeof(double));
    oracle_laplacian(P, f, l1);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1), al = oracle_alpha_m(P);
    for (size_t i = 0; i < n; ++i)
        out[i] = e2 * (eta1 + 2.0 * P->zeta) * l1[i] + P->beta1 * al * e2 * l1[i]
               - P->beta2 * al * al * f[i];
    free(l1);
}
static double phys_inner(const oracle_params* P, const double* f, const double* g) {
    size_t n = nphys(P);
    double s = 0.0, h = P->L / P->N;
    for (size_t i = 0; i < n; ++i) s += f[i] * g[i];
    return h * h * s;
}

/* modified energy of Theorem t:SAV */
double oracle_E_aux(const oracle_params* P, const double* uh_n, const double* uh_nm1,
                    double r_n, double r_nm1) {
    size_t n = nphys(P);
    int N = P->N;
    double* un = malloc(n * sizeof(double));
    double* um = malloc(n * sizeof(double));
    double* d = malloc(n * sizeof(double));
    double* e = malloc(n * sizeof(double));
    double* t = malloc(n * sizeof(double));
    oracle_c2r(N, uh_n, un, method_for(N));
    oracle_c2r(N, uh_nm1, um, method_for(N));
    for (size_t i = 0; i < n; ++i) { d[i] = un[i] - um[i]; e[i] = 2.0 * un[i] - um[i]; }
    double E = 0.0;
    apply_LSAV(P, un, t);
    E += 0.5 * phys_inner(P, un, t);
    apply_L1(P, d, t);
    E -= phys_inner(P, d, t);
    apply_LSAV(P, e, t);
    E += 0.5 * phys_inner(P, e, t);
    E += r_n * r_n + (2.0 * r_n - r_nm1) * (2.0 * r_n - r_nm1);
    free(un); free(um); free(d); free(e); free(t);
    return E;
}

/* ------------------------------------------------------------------------ */
/* Time stepping                                                             */
/* ------------------------------------------------------------------------ */

/* eq. BDF2Coef; k_n <= 0 selects the first-order startup step */
void oracle_bdf2_coef(double k_np1, double k_n, double* a, double* b, double* c) {
    if (k_n <= 0.0) {
        *a = 1.0 / k_np1;
        *b = -1.0 / k_np1;
        *c = 0.0;
        return;
    }
    *a = 1.0 / k_np1 + 1.0 / (k_np1 + k_n);
    *b = -1.0 / k_np1 - 1.0 / k_n;
    *c = 1.0 / k_n - 1.0 / (k_np1 + k_n);
}

/* eq. Predictor: weights of F(u~), F(u^n), F(u^{n-1}) */
void oracle_am3_weights(double k_np1, double k_n, double* w1, double* w2, double* w3) {
    double g = k_np1 / k_n;
    *w1 = k_np1 / 6.0 * (3.0 + 2.0 * g) / (1.0 + g);
    *w2 = k_np1 / 6.0 * (3.0 + g);
    *w3 = -k_np1 / 6.0 * g * g / (1.0 + g);
}

/* u* = u^n + (k_{n+1}/k_n)(u^n - u^{n-1}) (eq. Richardson); startup: u* = u^n */
static void extrapolate(const oracle_params* P, const cplx* un, const cplx* um,
                        double k_np1, double k_n, cplx* ustar) {
    size_t m = nspec(P);
    double g = (k_n <= 0.0) ? 0.0 : k_np1 / k_n;
    for (size_t i = 0; i < m; ++i) ustar[i] = (g == 0.0) ? un[i] : un[i] + g * (un[i] - um[i]);
}

/* The IMEX nonlinearity N = mu - L u (eqs. e:IMEX-op, IMEX) as a half spectrum,
 * for the linear part L = eps^4 Lap^2 - beta1 alpha eps^2 Lap + beta2 alpha^2 of
 * eq. e:SAV-L0, which is (eps^2 Lap - alpha)^2 at beta = (2, 1).  Written out
 * term by term:
 *   N = eps^2 (alpha - W'') Lap u + eps^2 Lap(alpha u - W') + W'' W'
 *       - alpha^2 u + eps^2 eta1 Lap u - eta2 W'
 *       + (beta1 - 2) alpha eps^2 Lap u + (1 - beta2) alpha^2 u
 * (the last line vanishes at beta = (2, 1)). */
static void imex_nonlin(const oracle_params* P, const cplx* uh, double beta1, double beta2,
                        cplx* Nh) {
    int N = P->N, H = N / 2 + 1;
    size_t n = nphys(P), m = nspec(P);
    double al = oracle_alpha_m(P);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1), eta2 = eff_eta(P, P->eta2);
    fields_t f;
    fields_alloc(P, &f);
    fields_eval(P, (const double*)uh, &f);
    double* t1 = malloc(n * sizeof(double));
    double* t2 = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        t1[i] = e2 * (al - f.W2[i] + eta1) * f.lap[i] + f.W2[i] * f.W1[i] - al * al * f.u[i]
              - eta2 * f.W1[i];
        if (beta1 != 2.0 || beta2 != 1.0)
            t1[i] += (beta1 - 2.0) * al * e2 * f.lap[i] + (1.0 - beta2) * al * al * f.u[i];
        t2[i] = al * f.u[i] - f.W1[i];
    }
    cplx* T1 = malloc(m * sizeof(cplx));
    cplx* T2 = malloc(m * sizeof(cplx));
    oracle_r2c(N, t1, (double*)T1, method_for(N));
    oracle_r2c(N, t2, (double*)T2, method_for(N));
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            Nh[i] = T1[i] - k2_at(P, ky, kx) * e2 * T2[i];
        }
    free(T1); free(T2); free(t1); free(t2);
    fields_free(&f);
}

/* BDF2-IMEX (eqs. IMEX, IMEX-eq):
 * (a - Lap L) u^{n+1} = -b u^n - c u^{n-1} + Lap N(u*), with L = L_IMEX at the
 * default beta = (2, 1) and the stabilized L_0 of eq. e:SAV-L0 otherwise (the
 * paper's IMEX family of Figure Find-Beta). */
int oracle_imex_step(const oracle_params* P, const double* uh_n_, const double* uh_nm1_,
                     double k_np1, double k_n, const double* fh_, double* uh_np1_) {
    int N = P->N, H = N / 2 + 1;
    size_t m = nspec(P);
    const cplx* un = (const cplx*)uh_n_;
    const cplx* um = (const cplx*)uh_nm1_;
    const cplx* fh = (const cplx*)fh_;
    cplx* out = (cplx*)uh_np1_;
    double a, b, c;
    oracle_bdf2_coef(k_np1, k_n, &a, &b, &c);
    double al = oracle_alpha_m(P);
    double e2 = P->eps * P->eps;

    cplx* us = malloc(m * sizeof(cplx));
    extrapolate(P, un, um, k_np1, k_n, us);
    cplx* Nh = malloc(m * sizeof(cplx));
    imex_nonlin(P, us, P->beta1, P->beta2, Nh);
    cplx* tmp = malloc(m * sizeof(cplx));
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            double k2 = k2_at(P, ky, kx);
            double Lh = e2 * e2 * k2 * k2 + P->beta1 * al * e2 * k2 + P->beta2 * al * al;
            cplx rhs = -b * un[i] - (c != 0.0 ? c * um[i] : 0.0) - k2 * Nh[i];
            if (fh) rhs += fh[i];
            tmp[i] = rhs / (a + k2 * Lh);
        }
    memcpy(out, tmp, m * sizeof(cplx));
    free(tmp); free(Nh); free(us);
    return 0;
}

/* BDF2-SAV (eqs. 4.7, 4.8).  The paper defers the linear algebra to its
 * references; here u^{n+1} = p + r^{n+1} q where p and q solve
 * (a - Lap L_0) p = -b u^n - c u^{n-1} + Lap L_1 u* (+ f) and
 * (a - Lap L_0) q = Lap X with X = V[u*]/sqrt(E_1(u*) + D_0); substituting
 * into eq. 4.8 gives a scalar linear equation for r^{n+1}. */
int oracle_sav_step(const oracle_params* P, const double* uh_n_, const double* uh_nm1_,
                    double r_n, double r_nm1, double k_np1, double k_n,
                    const double* fh_, double* uh_np1_, double* r_np1,
                    double* s_star_out, double* qh_out) {
    int N = P->N, H = N / 2 + 1;
    size_t m = nspec(P);
    const cplx* un = (const cplx*)uh_n_;
    const cplx* um = (const cplx*)uh_nm1_;
    const cplx* fh = (const cplx*)fh_;
    double a, b, c;
    oracle_bdf2_coef(k_np1, k_n, &a, &b, &c);
    double al = oracle_alpha_m(P);
    double e2 = P->eps * P->eps, eta1 = eff_eta(P, P->eta1);

    cplx* us = malloc(m * sizeof(cplx));
    extrapolate(P, un, um, k_np1, k_n, us);
    double E1 = oracle_E1(P, (const double*)us);
    double s2 = E1 + P->D0;
    if (!(s2 > 0.0)) { free(us); return -2; }
    double s = sqrt(s2);
    cplx* X = malloc(m * sizeof(cplx));
    oracle_V(P, (const double*)us, (double*)X);
    for (size_t i = 0; i < m; ++i) X[i] /= s;

    cplx* ph = malloc(m * sizeof(cplx));
    cplx* qh = malloc(m * sizeof(cplx));
    cplx* rp = malloc(m * sizeof(cplx));   /* a p + b u^n + c u^{n-1} */
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            double k2 = k2_at(P, ky, kx);
            double L0 = e2 * e2 * k2 * k2 + P->beta1 * al * e2 * k2 + P->beta2 * al * al;
            double L1 = -e2 * (eta1 + 2.0 * P->zeta) * k2 - P->beta1 * al * e2 * k2
                      - P->beta2 * al * al;
            double A = a + k2 * L0;
            cplx rhs = -b * un[i] - (c != 0.0 ? c * um[i] : 0.0) - k2 * L1 * us[i];
            if (fh) rhs += fh[i];
            ph[i] = rhs / A;
            qh[i] = -k2 * X[i] / A;
            rp[i] = a * ph[i] + b * un[i] + (c != 0.0 ? c * um[i] : 0.0);
        }
    double gp = oracle_inner(P, (const double*)X, (const double*)rp);
    double gq = oracle_inner(P, (const double*)X, (const double*)qh);
    double r = (-b * r_n - c * r_nm1 + 0.5 * gp) / (a - 0.5 * a * gq);
    cplx* out = (cplx*)uh_np1_;
    for (size_t i = 0; i < m; ++i) out[i] = ph[i] + r * qh[i];
    *r_np1 = r;
    if (s_star_out) *s_star_out = s;
    if (qh_out) memcpy(qh_out, qh, m * sizeof(cplx));
    free(us); free(X); free(ph); free(qh); free(rp);
    return 0;
}

/* Table SearchSize: optimal search step lambda(q, k), linear in k between
 * the printed columns and constant outside them. */
double oracle_lambda_table(double q, double k) {
    static const double ks[10] = {1e-6, 1e-5, 5e-5, 1e-4, 5e-4, 1e-3, 5e-3, 0.01, 0.02, 0.03};
    static const double qs[3] = {0.0, 0.2, 0.5};
    static const double lam[3][10] = {
        {1.0, 1.07, 1.11, 1.14, 1.24, 1.34, 1.60, 1.738, 1.804, 1.855},
        {1.0, 1.04, 1.15, 1.28, 1.50, 1.70, 1.87, 1.92, 1.95, 1.97},
        {1.0, 1.20, 1.32, 1.45, 1.72, 1.83, 1.965, 1.97, 1.985, 1.99}};
    int row = -1;
    for (int i = 0; i < 3; ++i)
        if (fabs(q - qs[i]) < 1e-12) row = i;
    if (row < 0) return -1.0;
    if (k <= ks[0]) return lam[row][0];
    if (k >= ks[9]) return lam[row][9];
    for (int j = 0; j < 9; ++j)
        if (k <= ks[j + 1]) {
            double t = (k - ks[j]) / (ks[j + 1] - ks[j]);
            return lam[row][j] + t * (lam[row][j + 1] - lam[row][j]);
        }
    return lam[row][9];
}

/* BDF2-PSD (eq. residual, Sec. 3.3): preconditioned steepest descent with
 * the residual R = Pi_0 mu(u) - Lap^{-1}(a u + b u^n + c u^{n-1}), the
 * preconditioner L_PSD = eps^4 Lap^2 - 2 alpha eps^2 Lap + alpha^2 - a Lap^{-1},
 * direction d = -L_PSD^{-1} R and update u_{s+1} = u_s + lambda d; stop once
 * ||d_s|| / ||u_{s+1}|| < tol. */
int oracle_psd_step(const oracle_params* P, const double* uh_n_, const double* uh_nm1_,
                    double k_np1, double k_n, const double* guess_, const double* fh_,
                    double tol, int max_iter, double lambda, int fixed_iters,
                    double* uh_np1_, int* iters_out, double* last_ratio) {
    int N = P->N, H = N / 2 + 1;
    size_t m = nspec(P);
    const cplx* un = (const cplx*)uh_n_;
    const cplx* um = (const cplx*)uh_nm1_;
    const cplx* fh = (const cplx*)fh_;
    double a, b, c;
    oracle_bdf2_coef(k_np1, k_n, &a, &b, &c);
    double al = oracle_alpha_m(P);
    double e2 = P->eps * P->eps;
    double lam = lambda > 0.0 ? lambda : oracle_lambda_table(P->q, k_np1);
    if (!(lam > 0.0)) return -1;

    cplx* u = malloc(m * sizeof(cplx));
    if (guess_) {
        memcpy(u, guess_, m * sizeof(cplx));
        u[0] = un[0];   /* project the guess to the mass of u^n */
    } else {
        extrapolate(P, un, um, k_np1, k_n, u);
    }
    cplx* mu = malloc(m * sizeof(cplx));
    cplx* d = malloc(m * sizeof(cplx));
    int it = 0, rc = 1;
    double ratio = 0.0;
    for (;;) {
        oracle_mu(P, (const double*)u, (double*)mu);
        for (int ky = 0; ky < N; ++ky)
            for (int kx = 0; kx < H; ++kx) {
                size_t i = (size_t)ky * H + kx;
                if (ky == 0 && kx == 0) { d[i] = 0.0; continue; }  /* Pi_0 */
                double k2 = k2_at(P, ky, kx);
                cplx g = a * u[i] + b * un[i] + (c != 0.0 ? c * um[i] : 0.0);
                if (fh) g -= fh[i];
                cplx R = mu[i] + g / k2;                          /* Lap^{-1} -> -1/k2 */
                double Lpsd = e2 * e2 * k2 * k2 + 2.0 * al * e2 * k2 + al * al + a / k2;
                d[i] = -R / Lpsd;
            }
        for (size_t i = 0; i < m; ++i) u[i] += lam * d[i];
        ++it;
        double dn = sqrt(oracle_inner(P, (const double*)d, (const double*)d));
        double unrm = sqrt(oracle_inner(P, (const double*)u, (const double*)u));
        ratio = dn / unrm;
        if (fixed_iters > 0) {
            if (it >= fixed_iters) { rc = 0; break; }
        } else if (ratio < tol) {
            rc = 0;
            break;
        } else if (it >= max_iter) {
            rc = 1;
            break;
        }
    }
    memcpy(uh_np1_, u, m * sizeof(cplx));
    if (iters_out) *iters_out = it;
    if (last_ratio) *last_ratio = ratio;
    free(u); free(mu); free(d);
    return rc;
}

/* Steps 2-3 of the adaptive algorithm: AM3 predictor and relative error */
double oracle_am3_error(const oracle_params* P, const double* uh_trial_, const double* uh_n_,
                        const double* F_trial_, const double* F_n_, const double* F_nm1_,
                        double k_trial, double k_n) {
    size_t m = nspec(P);
    const cplx* ut = (const cplx*)uh_trial_;
    const cplx* un = (const cplx*)uh_n_;
    const cplx *Ft = (const cplx*)F_trial_, *Fn = (const cplx*)F_n_, *Fm = (const cplx*)F_nm1_;
    double w1, w2, w3;
    oracle_am3_weights(k_trial, k_n, &w1, &w2, &w3);
    cplx* up = malloc(m * sizeof(cplx));
    cplx* df = malloc(m * sizeof(cplx));
    for (size_t i = 0; i < m; ++i) {
        up[i] = un[i] + w1 * Ft[i] + w2 * Fn[i] + w3 * Fm[i];
        df[i] = ut[i] - up[i];
    }
    double e = sqrt(oracle_inner(P, (const double*)df, (const double*)df))
             / sqrt(oracle_inner(P, (const double*)up, (const double*)up));
    free(up);
    free(df);
    return e;
}

/* Step 4: accept if e <= sigma_tol or the trial step is already k_min; the
 * next trial step is rho_s (sigma_tol / e)^{1/3} k~, clamped to [k_min, k_max]
 * and (when cap > 0) to cap * k~ for zero-stability of variable-step BDF2. */
void oracle_adapt_decide(double e, double k_trial, double sigma_tol, double k_min,
                         double k_max, double rho_s, double cap, int* accept,
                         double* k_next) {
    double ee = e > 1e-300 ? e : 1e-300;
    double kn = rho_s * cbrt(sigma_tol / ee) * k_trial;
    if (cap > 0.0 && kn > cap * k_trial) kn = cap * k_trial;
    if (kn > k_max) kn = k_max;
    if (kn < k_min) kn = k_min;
    *accept = (e <= sigma_tol) || (k_trial <= k_min);
    *k_next = kn;
}

/* ------------------------------------------------------------------------ */
/* ETDRK2 (Sec. 3.6)                                                         */
/* ------------------------------------------------------------------------ */

/* phi0 = e^z, phi1 = (e^z - 1)/z, phi2 = (e^z - 1 - z)/z^2: the multipliers
 * of eqs. ETDRK1 and ETDRK2 at z = L k, since L^{-1}(e^{Lk} - I) = k phi1 and
 * L^{-1}[L^{-1}(e^{Lk} - I) - k I] / k = k phi2.  Both quotients cancel near
 * z = 0, so for |z| < 1 they are summed from their Taylor series
 * phi_j(z) = sum_m z^m / (m + j)!; elsewhere phi1 comes from exp and
 * phi2 = (phi1 - 1)/z. */
void oracle_etd_phi(double z, double* phi0, double* phi1, double* phi2) {
    *phi0 = exp(z);
    if (fabs(z) < 1.0) {
        double t1 = 1.0, t2 = 0.5, s1 = 0.0, s2 = 0.0;
        for (int m = 0; m < 40; ++m) {
            s1 += t1;
            s2 += t2;
            t1 *= z / (double)(m + 2);
            t2 *= z / (double)(m + 3);
        }
        *phi1 = s1;
        *phi2 = s2;
    } else {
        *phi1 = (exp(z) - 1.0) / z;
        *phi2 = (*phi1 - 1.0) / z;
    }
}

/* the linear operator of eq. ETD-L at |k|^2 = k2 (Lap -> -k2):
 * Lap (eps^4 Lap^2 - 2 alpha eps^2 Lap + alpha^2) - kappa0 + kappa2 eps^2 Lap */
static double etd_L(const oracle_params* P, double k2, double kappa0, double kappa2) {
    double e2 = P->eps * P->eps, al = oracle_alpha_m(P);
    return -k2 * (e2 * e2 * k2 * k2 + 2.0 * al * e2 * k2 + al * al) - kappa0 - kappa2 * e2 * k2;
}

/* the nonlinearity of eq. ETD-L, N(u) = Lap N_IMEX(u) + kappa0 u - kappa2 eps^2 Lap u,
 * plus the forcing fh (nullable) */
static void etd_N(const oracle_params* P, const cplx* uh, double kappa0, double kappa2,
                  const cplx* fh, cplx* out) {
    int N = P->N, H = N / 2 + 1;
    size_t m = nspec(P);
    double e2 = P->eps * P->eps;
    cplx* Ni = malloc(m * sizeof(cplx));
    imex_nonlin(P, uh, 2.0, 1.0, Ni);   /* eq. ETD-L takes L_IMEX itself */
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            double k2 = k2_at(P, ky, kx);
            out[i] = -k2 * Ni[i] + kappa0 * uh[i] + kappa2 * e2 * k2 * uh[i];
            if (fh) out[i] += fh[i];
        }
    free(Ni);
}

/* One ETDRK2 step of size k (eq. ETDRK2) with the split of eq. ETD-L:
 *   u~      = e^{Lk} u^n + L^{-1}(e^{Lk} - I) N(u^n)            (eq. ETDRK1)
 *   u^{n+1} = u~ + L^{-1}[L^{-1}(e^{Lk} - I) - k I] (N(u~) - N(u^n)) / k
 * fh_n, fh_np1 (nullable): a forcing at t^n and t^{n+1}, treated as part of
 * N (manufactured solutions only).  uh_stage (nullable out): u~. */
int oracle_etd_step(const oracle_params* P, const double* uh_n_, double k, double kappa0,
                    double kappa2, const double* fh_n, const double* fh_np1, double* uh_np1_,
                    double* uh_stage_) {
    if (!(k > 0.0)) return -1;
    int N = P->N, H = N / 2 + 1;
    size_t m = nspec(P);
    const cplx* un = (const cplx*)uh_n_;
    cplx* Nn = malloc(m * sizeof(cplx));
    cplx* Nt = malloc(m * sizeof(cplx));
    cplx* ut = malloc(m * sizeof(cplx));
    etd_N(P, un, kappa0, kappa2, (const cplx*)fh_n, Nn);
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            double p0, p1, p2;
            oracle_etd_phi(etd_L(P, k2_at(P, ky, kx), kappa0, kappa2) * k, &p0, &p1, &p2);
            ut[i] = p0 * un[i] + k * p1 * Nn[i];
        }
    etd_N(P, ut, kappa0, kappa2, (const cplx*)fh_np1, Nt);
    cplx* out = (cplx*)uh_np1_;
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < H; ++kx) {
            size_t i = (size_t)ky * H + kx;
            double p0, p1, p2;
            oracle_etd_phi(etd_L(P, k2_at(P, ky, kx), kappa0, kappa2) * k, &p0, &p1, &p2);
            out[i] = ut[i] + k * p2 * (Nt[i] - Nn[i]);
        }
    if (uh_stage_) memcpy(uh_stage_, ut, m * sizeof(cplx));
    free(Nn); free(Nt); free(ut);
    return 0;
}
