/*
 * CPU FP64 oracle of the marginal likelihood of the power spectrum.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do. It shares no code, header or constant with the GPU
 * path.
 *
 * What it computes (Summary and Statement of need: joint EoR + foreground
 * fit with the instrument forward-modelled and the sky coefficients
 * marginalised out so that only the per-k-bin power is sampled; eq. 1: one
 * power value per spherical k-shell):
 *
 *   model    d = T a + e,  a ~ CN(0, Phi),  e ~ CN(0, N),  N = diag(sigma^2)
 *   marginal d ~ CN(0, C),  C = N + T Phi T^H
 *   logL     = -m ln(pi) - ln det C - d^H C^{-1} d                       (D1)
 *
 * The route taken is the Woodbury identity and the matrix-determinant lemma:
 *   A = T^H N^{-1} T,  dbar = T^H N^{-1} d,  c = d^H N^{-1} d,
 *   Sigma = A + Phi^{-1},
 *   logL = -m ln(pi) - sum ln sigma_i^2 - ln det Phi - ln det Sigma
 *          - (c - dbar^H Sigma^{-1} dbar)                                 (M1)
 * with Sigma = L L^H, ln det Sigma = 2 sum ln L_jj, and the quadratic form
 * taken as dbar^H x where L L^H x = dbar (forward then back substitution).
 *
 * Plain loops, std C99, no BLAS, built with -O2 -fno-fast-math
 * -ffp-contract=off. Complex numbers are explicit (re, im) pairs.
 * Parallelism: OpenMP over independent outputs only (rows of A, theta).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Mutation hooks: every MUT(k) is 0 in the normal build. The tests compile
 * mutants (-DORACLE_MUTANT=k) to show that each planted mistake fails a pin. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif
#define MUT(k) (ORACLE_MUTANT == (k))

#define RE(p, k) ((p)[2 * (k)])
#define IM(p, k) ((p)[2 * (k) + 1])

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/*
 * Precompute (once per dataset).
 *   T          [m x ldT] complex, row-major, interleaved (re, im)
 *   noise_var  [m] sigma_i^2 > 0
 *   d          [m] complex
 * Outputs:
 *   A          [n x n] complex, row-major, full Hermitian (both triangles)
 *   dbar       [n] complex
 *   c_out      d^H N^{-1} d
 *   K0_out     -m ln(pi) - sum_i ln sigma_i^2
 * Returns 0, or -1 on a bad argument.
 */
int oracle_precompute(int64_t m, int64_t n, const double *T, int64_t ldT,
                      const double *noise_var, const double *d, double *A,
                      double *dbar, double *c_out, double *K0_out, int nthreads) {
    if (m <= 0 || n <= 0 || ldT < n) return -1;
    for (int64_t i = 0; i < m; ++i)
        if (!(noise_var[i] > 0.0)) return -1;
    set_threads(nthreads);

    /* A_jk = sum_i conj(T_ij) T_ik / sigma_i^2, for k <= j, increasing i. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t k = 0; k <= j; ++k) {
            double sr = 0.0, si = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                const double *tj = T + 2 * (i * ldT + j);
                const double *tk = T + 2 * (i * ldT + k);
                const double w = 1.0 / noise_var[i];
                /* conj(tj) * tk = (ar - i ai)(br + i bi) */
                double pr = tj[0] * tk[0] + tj[1] * tk[1];
                double pi = tj[0] * tk[1] - tj[1] * tk[0];
                if (MUT(1)) pi = -pi;
                sr += pr * w;
                si += pi * w;
            }
            RE(A, j * n + k) = sr;
            IM(A, j * n + k) = si;
        }
    }
    /* Hermitian mirror; the diagonal is real by construction. */
    for (int64_t j = 0; j < n; ++j) {
        IM(A, j * n + j) = 0.0;
        for (int64_t k = 0; k < j; ++k) {
            RE(A, k * n + j) = RE(A, j * n + k);
            IM(A, k * n + j) = -IM(A, j * n + k);
        }
    }
    /* dbar_j = sum_i conj(T_ij) d_i / sigma_i^2 */
    for (int64_t j = 0; j < n; ++j) {
        double sr = 0.0, si = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double *tj = T + 2 * (i * ldT + j);
            const double w = MUT(2) ? 1.0 : 1.0 / noise_var[i];
            sr += (tj[0] * RE(d, i) + tj[1] * IM(d, i)) * w;
            si += (tj[0] * IM(d, i) - tj[1] * RE(d, i)) * w;
        }
        RE(dbar, j) = sr;
        IM(dbar, j) = si;
    }
    double c = 0.0, K0 = -(double)m * log(MUT(3) ? 2.0 * ORACLE_PI : ORACLE_PI);
    for (int64_t i = 0; i < m; ++i) {
        c += (RE(d, i) * RE(d, i) + IM(d, i) * IM(d, i)) / noise_var[i];
        K0 -= log(noise_var[i]);
    }
    *c_out = c;
    *K0_out = K0;
    return 0;
}

/*
 * Prior variance of coefficient j: s_b 10^theta_b for an EoR coefficient in
 * k-bin b (eq. 1: every voxel of a shell shares its bin's power), else the
 * fixed foreground variance v_j.
 */
static double prior_var(int64_t j, const double *theta, const int32_t *bin_of,
                        const double *fixed_var, const double *bin_scale) {
    int32_t b = bin_of[j];
    if (b < 0) return fixed_var[j];
    if (MUT(4) && b > 0) b -= 1;
    double s = bin_scale ? bin_scale[b] : 1.0;
    return s * pow(10.0, theta[b]);
}

/*
 * Per-theta likelihood.
 *   A [n x n] full Hermitian row-major (from oracle_precompute), dbar [n].
 *   theta [B x n_k] row-major.
 * Outputs logL[B]; info[B] (0 ok, -1 non-finite theta or prior variance,
 * k>0 the 1-based column whose pivot was not positive and finite);
 * terms[B x 4] if not NULL: ln det Sigma, dbar^H x, ln det Phi, ||L^{-1} dbar||^2.
 * Returns 0, or -1 on a bad argument.
 */
int oracle_loglike(int64_t n, const double *A, const double *dbar, double c,
                   double K0, int32_t n_k, const int32_t *bin_of,
                   const double *fixed_var, const double *bin_scale, int64_t B,
                   const double *theta, double *logL, int32_t *info,
                   double *terms, int nthreads) {
    if (n <= 0 || n_k < 0 || B < 0) return -1;
    for (int64_t j = 0; j < n; ++j) {
        if (bin_of[j] >= n_k || bin_of[j] < -1) return -1;
        if (bin_of[j] < 0 && !(fixed_var[j] > 0.0)) return -1;
    }
    set_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < B; ++t) {
        const double *th = theta + t * n_k;
        double *L = (double *)malloc(sizeof(double) * 2 * (size_t)n * (size_t)n);
        double *y = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        double *x = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        double *phi = (double *)malloc(sizeof(double) * (size_t)n);
        int32_t status = 0;
        double out = -INFINITY;
        double ldS = NAN, quad = NAN, ldP = NAN, yy = NAN;

        for (int32_t b = 0; b < n_k; ++b)
            if (!isfinite(th[b])) status = -1;
        for (int64_t j = 0; j < n && status == 0; ++j) {
            phi[j] = prior_var(j, th, bin_of, fixed_var, bin_scale);
            if (!(phi[j] > 0.0) || !isfinite(phi[j])) status = -1;
        }
        if (status == 0) {
            /* Sigma = A + Phi^{-1} (lower triangle is all that is read) */
            memcpy(L, A, sizeof(double) * 2 * (size_t)n * (size_t)n);
            for (int64_t j = 0; j < n; ++j) RE(L, j * n + j) += MUT(7) ? phi[j] : 1.0 / phi[j];

            /* Cholesky-Banachiewicz, row by row: L_ij for k<=j<=i. */
            for (int64_t i = 0; i < n && status == 0; ++i) {
                for (int64_t j = 0; j <= i; ++j) {
                    double sr = RE(L, i * n + j), si = IM(L, i * n + j);
                    for (int64_t k = 0; k < j; ++k) {
                        /* L_ik * conj(L_jk) */
                        double ar = RE(L, i * n + k), ai = IM(L, i * n + k);
                        double br = RE(L, j * n + k), bi = IM(L, j * n + k);
                        sr -= ar * br + ai * bi;
                        si -= MUT(8) ? ai * br + ar * bi : ai * br - ar * bi;
                    }
                    if (j == i) {
                        if (!(sr > 0.0) || !isfinite(sr)) {
                            status = (int32_t)(i + 1);
                            break;
                        }
                        RE(L, i * n + i) = sqrt(sr);
                        IM(L, i * n + i) = 0.0;
                    } else {
                        double djj = RE(L, j * n + j);
                        RE(L, i * n + j) = sr / djj;
                        IM(L, i * n + j) = si / djj;
                    }
                }
            }
        }
        if (status == 0) {
            /* forward substitution L y = dbar */
            for (int64_t i = 0; i < n; ++i) {
                double sr = RE(dbar, i), si = IM(dbar, i);
                for (int64_t k = 0; k < i; ++k) {
                    double ar = RE(L, i * n + k), ai = IM(L, i * n + k);
                    sr -= ar * RE(y, k) - ai * IM(y, k);
                    si -= ar * IM(y, k) + ai * RE(y, k);
                }
                double dii = RE(L, i * n + i);
                RE(y, i) = sr / dii;
                IM(y, i) = si / dii;
            }
            /* back substitution L^H x = y; (L^H)_ik = conj(L_ki) */
            for (int64_t i = n - 1; i >= 0; --i) {
                double sr = RE(y, i), si = IM(y, i);
                for (int64_t k = i + 1; k < n; ++k) {
                    double ar = RE(L, k * n + i), ai = -IM(L, k * n + i);
                    sr -= ar * RE(x, k) - ai * IM(x, k);
                    si -= ar * IM(x, k) + ai * RE(x, k);
                }
                double dii = RE(L, i * n + i);
                RE(x, i) = sr / dii;
                IM(x, i) = si / dii;
            }
            ldS = 0.0;
            for (int64_t j = 0; j < n; ++j) ldS += 2.0 * log(RE(L, j * n + j));
            /* ln det Phi summed per coefficient (not per bin) */
            ldP = 0.0;
            for (int64_t j = 0; j < n; ++j) ldP += MUT(5) ? 0.0 : log(phi[j]);
            /* quad = Re(dbar^H x) */
            quad = 0.0;
            yy = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                quad += RE(dbar, j) * RE(x, j) + IM(dbar, j) * IM(x, j);
                yy += RE(y, j) * RE(y, j) + IM(y, j) * IM(y, j);
            }
            out = K0 - ldP - ldS - (c - (MUT(6) ? -quad : quad));
        }
        logL[t] = out;
        if (info) info[t] = status;
        if (terms) {
            terms[4 * t + 0] = ldS;
            terms[4 * t + 1] = quad;
            terms[4 * t + 2] = ldP;
            terms[4 * t + 3] = yy;
        }
        free(L);
        free(y);
        free(x);
        free(phi);
    }
    return 0;
}

/* Identification string, so a caller can confirm which build it loaded. */
const char *oracle_build_id(void) {
    return ORACLE_MUTANT ? "oracle-mutant" : "oracle";
}
