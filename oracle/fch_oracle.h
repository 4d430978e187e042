/*
 * fch_oracle.h -- plain FP64 CPU oracle for the functionalized Cahn-Hilliard
 * (FCH) pseudo-spectral BDF2 path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Layouts (all arrays owned by the caller, host memory):
 *   physical  u[i*N + j]            i = row (y = i*h), j = column (x = j*h), h = L/N
 *   spectrum  uh[i*(N/2+1) + j]     i = ky index 0..N-1, j = kx index 0..N/2
 *             (the layout of numpy.fft.rfft2)
 *   wavenumbers kx_j = 2*pi*j/L, ky_i = 2*pi*(i <= N/2 ? i : i-N)/L,
 *   |k|^2 = kx^2 + ky^2, and the Laplacian is the multiplier -|k|^2.
 *   Forward transforms are unnormalized; inverse transforms carry 1/N^2.
 *
 * Parameters follow the paper's statement of the model:
 *   regularized well W_q (eq. e:Wq-def), energy (eq. Functional),
 *   H^{-1} gradient flow (eqs. sFCH, FCH), BDF2 coefficients (eq. BDF2Coef),
 *   AM3 predictor (eq. Predictor), the PSD residual and preconditioner
 *   (eq. residual, Sec. 3.3), the IMEX split (eqs. e:IMEX-op, IMEX-eq) and the
 *   SAV scheme (eqs. 4.1-4.8), and the ETDRK2 scheme (Sec. 3.6, eqs.
 *   ETDRK1, ETDRK2, ETD-L).
 */
#ifndef FCH_ORACLE_H
#define FCH_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    N;          /* grid points per side (power of two for the FFT route) */
    double L;          /* periodic square [0, L)^2                               */
    double eps;        /* interface width epsilon                                */
    double eta1, eta2; /* functionalization parameters as given                  */
    int    p;          /* effective eta_i = eps^p * eta_i                         */
    double q;          /* well regularization q >= 0                              */
    double gamma_w;    /* well asymmetry gamma (0.3 in the paper)                 */
    double b_minus, b_plus; /* well minima (-1, +1)                               */
    double beta1, beta2;    /* SAV stabilization (2, 1)                           */
    double zeta, D0;        /* SAV splitting constant and energy shift            */
} oracle_params;

/* ---- transforms -------------------------------------------------------- */
/* naive O(n^2) DFT of one complex line (interleaved re,im); sign = -1 forward,
 * +1 inverse (unnormalized) */
void oracle_dft_1d(int n, const double* in, double* out, int sign);
/* iterative radix-2 FFT of one complex line in place (n a power of two) */
int  oracle_fft_1d(int n, double* data, int sign);
/* brute-force O(N^4) 2D DFT of a real field into the half spectrum */
void oracle_dft2_brute(int N, const double* u, double* uh);
/* 2D real-to-half-spectrum transform; method 0 = naive DFT lines, 1 = FFT */
int  oracle_r2c(int N, const double* u, double* uh, int method);
/* inverse: real part of the inverse DFT of the Hermitian extension, times 1/N^2 */
int  oracle_c2r(int N, const double* uh, double* u, int method);
void oracle_set_threads(int n);   /* OpenMP threads over lines (timing only) */

/* ---- model pieces ------------------------------------------------------ */
void   oracle_well(const oracle_params* P, int n, const double* u,
                   double* W, double* W1, double* W2);
double oracle_alpha_m(const oracle_params* P);      /* W_q''(b_-)           */
void   oracle_laplacian(const oracle_params* P, const double* u, double* lap);
/* chemical potential mu = dE/du (eq. FCH bracket), returned as a half spectrum */
int    oracle_mu(const oracle_params* P, const double* uh, double* muh);
/* F(u) = Laplacian(mu) as a half spectrum */
int    oracle_F(const oracle_params* P, const double* uh, double* Fh);
/* discrete energy, mass (1/2) int (u+1), and SAV pieces */
double oracle_energy(const oracle_params* P, const double* uh);
double oracle_mass(const oracle_params* P, const double* uh);
double oracle_E1(const oracle_params* P, const double* uh);        /* int G(u) */
int    oracle_V(const oracle_params* P, const double* uh, double* Vh);  /* dE1/du */
/* modified SAV energy E_aux(u^n, u^{n-1}, r^n, r^{n-1}) */
double oracle_E_aux(const oracle_params* P, const double* uh_n, const double* uh_nm1,
                    double r_n, double r_nm1);
/* L2 inner product h^2 sum f g computed in physical space */
double oracle_inner(const oracle_params* P, const double* fh, const double* gh);

/* ---- time stepping ----------------------------------------------------- */
/* BDF2 coefficients a, b, c for steps k_np1, k_n; k_n <= 0 gives the BDF1
 * startup step (a = 1/k, b = -1/k, c = 0) */
void oracle_bdf2_coef(double k_np1, double k_n, double* a, double* b, double* c);
/* AM3 weights w1, w2, w3 such that u_p = u^n + w1 F(u~) + w2 F^n + w3 F^{n-1} */
void oracle_am3_weights(double k_np1, double k_n, double* w1, double* w2, double* w3);

/* forcing fh (nullable) is added to the right-hand side u_t = Delta mu + f
 * (manufactured solutions only) */
int oracle_imex_step(const oracle_params* P, const double* uh_n, const double* uh_nm1,
                     double k_np1, double k_n, const double* fh, double* uh_np1);
int oracle_sav_step(const oracle_params* P, const double* uh_n, const double* uh_nm1,
                    double r_n, double r_nm1, double k_np1, double k_n,
                    const double* fh, double* uh_np1, double* r_np1,
                    double* s_star /* nullable out */, double* qh /* nullable out */);
/* PSD solve; guess nullable (extrapolation).  lambda <= 0 selects the table.
 * fixed_iters > 0 runs exactly that many iterations and ignores tol.
 * returns 0 on convergence, 1 if max_iter was reached, <0 on bad input. */
int oracle_psd_step(const oracle_params* P, const double* uh_n, const double* uh_nm1,
                    double k_np1, double k_n, const double* guess, const double* fh,
                    double tol, int max_iter, double lambda, int fixed_iters,
                    double* uh_np1, int* iters, double* last_ratio);
double oracle_lambda_table(double q, double k);     /* <0 if q not tabulated */

/* ETDRK2 (Sec. 3.6, eqs. ETDRK1, ETDRK2, ETD-L).  phi0 = e^z,
 * phi1 = (e^z - 1)/z, phi2 = (e^z - 1 - z)/z^2 (the limits 1, 1/2 at z = 0). */
void oracle_etd_phi(double z, double* phi0, double* phi1, double* phi2);
/* one step of size k; fh_n, fh_np1 nullable forcing at t^n, t^{n+1};
 * uh_stage nullable out (the ETDRK1 stage u~).  Returns -1 for k <= 0. */
int oracle_etd_step(const oracle_params* P, const double* uh_n, double k, double kappa0,
                    double kappa2, const double* fh_n, const double* fh_np1, double* uh_np1,
                    double* uh_stage);

/* AM3 local error estimate e = ||u~ - u_p|| / ||u_p|| (physical L2 norms) */
double oracle_am3_error(const oracle_params* P, const double* uh_trial, const double* uh_n,
                        const double* F_trial, const double* F_n, const double* F_nm1,
                        double k_trial, double k_n);
/* step-size controller: accept flag and next trial step */
void oracle_adapt_decide(double e, double k_trial, double sigma_tol, double k_min,
                         double k_max, double rho_s, double cap, int* accept,
                         double* k_next);

#ifdef __cplusplus
}
#endif
#endif
