/*
 * Test infrastructure only: the plain FP64 CPU oracle of the kernelised periodogram sums.
 *
 * Nothing in the product path may include, link or call this file.  It shares no code, header,
 * table or constant with the HIP library; it is written straight from the definitions:
 *
 *   Gaussian kernel          G_s(x)      = exp(-x^2 / (2 s^2)) / (sqrt(2 pi) s)        (Sec. 2, Gaussian kernel)
 *   periodic kernel          G^P_s(f,dt) = exp(-2 sin^2(pi f dt) / s^2) / (sqrt(2 pi) s)  (Sec. 2.1)
 *   information potential    IP_y = (1/N^2) sum_i sum_j G_sy(y_i - y_j)                  (Sec. 3)
 *   CKP                      (1/N^2) sum_i sum_j (G_sy(dy_ij) - IP_y) G^P_st(f, dt_ij)   (Sec. 3)
 *
 * From the same pair sums the oracle returns the three information potentials of the
 * Cauchy-Schwarz quadratic mutual information between the periodic time warp and the magnitude:
 *
 *   V_J(f)  = (1/N^2) sum_i sum_j G_sy(dy_ij) G^P_st(f, dt_ij)        (joint)
 *   IP_t(f) = (1/N^2) sum_i sum_j G^P_st(f, dt_ij)                    (so V_M = IP_y IP_t)
 *   V_C(f)  = (1/N^3) sum_i [sum_k G_sy(dy_ik)] [sum_j G^P_st(f, dt_ij)]   (cross)
 *
 * so that CKP = V_J - V_M exactly.  Every sum runs over all ordered pairs, diagonal included, as
 * the CKP and information-potential definitions of Sec. 3 are written.  The periodic kernel is
 * evaluated in the sin^2 form of Sec. 2.1
 * (not the chord form that a fast implementation would use), with the product f * dt folded to
 * [-1/2, 1/2] in FP64 before the sine.  Sums use Neumaier compensation.
 *
 * mode 0 ("plain"): the double loop over all (i, j) exactly as written above.
 * mode 1 ("fast") : the loop over i < j only, doubled, plus the diagonal added in closed form
 *                   (G^P(f, 0) = A, G_sy(0) = B).  Same quantities; validated against mode 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double s, c;
} nsum_t;

static inline void nsum_add(nsum_t *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nsum_val(const nsum_t *a) { return a->s + a->c; }

static const double kPi = 3.14159265358979323846264338327950288;

/* Gaussian kernel of Sec. 2 evaluated at difference x with width s. */
static double gauss_kernel(double x, double s) {
    return exp(-(x * x) / (2.0 * s * s)) / (sqrt(2.0 * kPi) * s);
}

/* Periodic kernel of Sec. 2.1 at frequency f and time difference dt, width s. */
static double periodic_kernel(double f, double dt, double s) {
    double x = f * dt;
    x -= nearbyint(x); /* the kernel has period 1 in f*dt; fold in FP64 */
    double sn = sin(kPi * x);
    return exp(-2.0 * sn * sn / (s * s)) / (sqrt(2.0 * kPi) * s);
}

/* Magnitude Gram matrix K[i][j] = G_sy(y_i - y_j) and its row sums r_i (diagonal included). */
static int magnitude_gram(int64_t n, const double *y, double sigma_y, double *K, double *r) {
    for (int64_t i = 0; i < n; ++i) {
        nsum_t acc = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            double k = gauss_kernel(y[i] - y[j], sigma_y);
            K[i * n + j] = k;
            nsum_add(&acc, k);
        }
        r[i] = nsum_val(&acc);
    }
    return 0;
}

/* Sums at one frequency. */
static void sums_at(int64_t n, const double *t, const double *K, const double *r, double sigma_t,
                    double f, int mode, double *vj, double *ipt, double *vc) {
    nsum_t J = {0, 0}, T = {0, 0}, C = {0, 0};
    double N = (double)n;
    if (mode == 0) {
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t j = 0; j < n; ++j) {
                double g = periodic_kernel(f, t[i] - t[j], sigma_t);
                nsum_add(&J, K[i * n + j] * g);
                nsum_add(&T, g);
                nsum_add(&C, r[i] * g);
            }
        }
    } else {
        double A = 1.0 / (sqrt(2.0 * kPi) * sigma_t);
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t j = i + 1; j < n; ++j) {
                double g = periodic_kernel(f, t[i] - t[j], sigma_t);
                nsum_add(&J, 2.0 * K[i * n + j] * g);
                nsum_add(&T, 2.0 * g);
                nsum_add(&C, (r[i] + r[j]) * g);
            }
        }
        /* diagonal: G^P(f, 0) = A and G_sy(0) = K[i][i] */
        for (int64_t i = 0; i < n; ++i) {
            nsum_add(&J, K[i * n + i] * A);
            nsum_add(&T, A);
            nsum_add(&C, r[i] * A);
        }
    }
    *vj = nsum_val(&J) / (N * N);
    *ipt = nsum_val(&T) / (N * N);
    *vc = nsum_val(&C) / (N * N * N);
}

/*
 * Information potentials of a batch of curves (CSR: curve c is samples [offsets[c], offsets[c+1]))
 * at per-curve frequency lists (CSR: curve c has freqs[foffsets[c] .. foffsets[c+1])).
 * sigma_t[c], sigma_y[c] are the kernel widths.  Outputs are indexed like freqs (vj, ipt, vc) and
 * per curve (ipy).  n_threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad input,
 * -2 on allocation failure.
 */
int oracle_batch_ips(int64_t n_curves, const int64_t *offsets, const double *t, const double *y,
                     const double *sigma_t, const double *sigma_y, const int64_t *foffsets,
                     const double *freqs, int mode, double *vj, double *ipt, double *vc,
                     double *ipy, int n_threads) {
    if (n_curves < 0 || !offsets || !foffsets || (mode != 0 && mode != 1)) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    for (int64_t c = 0; c < n_curves; ++c) {
        int64_t n = offsets[c + 1] - offsets[c];
        if (n < 1 || !(sigma_t[c] > 0.0) || !(sigma_y[c] > 0.0)) return -1;
        const double *tc = t + offsets[c];
        const double *yc = y + offsets[c];
        double *K = (double *)malloc(sizeof(double) * (size_t)(n * n));
        double *r = (double *)malloc(sizeof(double) * (size_t)n);
        if (!K || !r) {
            free(K);
            free(r);
            return -2;
        }
        magnitude_gram(n, yc, sigma_y[c], K, r);
        nsum_t R = {0, 0};
        for (int64_t i = 0; i < n; ++i) nsum_add(&R, r[i]);
        ipy[c] = nsum_val(&R) / ((double)n * (double)n);
        int64_t f0 = foffsets[c], f1 = foffsets[c + 1];
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t q = f0; q < f1; ++q)
            sums_at(n, tc, K, r, sigma_t[c], freqs[q], mode, &vj[q], &ipt[q], &vc[q]);
        free(K);
        free(r);
    }
    return 0;
}

/* Number of OpenMP threads a parallel region would use (for reporting the CPU baseline). */
int oracle_threads(int n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
    int m = 1;
#pragma omp parallel
    {
#pragma omp single
        m = omp_get_num_threads();
    }
    return m;
#else
    (void)n_threads;
    return 1;
#endif
}
