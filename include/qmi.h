/*
 * qmi.h - C ABI of libqmi, the MI355X (gfx950) kernelised-periodogram period search.
 *
 * The method is from Protopapas et al., "A novel, fully automated pipeline for period estimation
 * in the EROS 2 data set" (arXiv:1412.1840).  For every lightcurve {t_i, y_i}, i = 1..N, and every
 * trial frequency f, the library forms the pair sums of the Gaussian kernel on magnitude
 * differences (Sec. 2, Gaussian kernel) times the periodic kernel on time differences (Sec. 2.1):
 *
 *     K_y(i,j) = B exp(-(y_i - y_j)^2 / (2 sy^2)),        B = 1 / (sqrt(2 pi) sy)
 *     K_t(i,j) = A exp(-2 sin^2(pi f (t_i - t_j)) / st^2), A = 1 / (sqrt(2 pi) st)
 *
 * and reduces them, over all ordered pairs with the diagonal included, to the information
 * potentials
 *
 *     V_J(f)  = (1/N^2) sum_ij K_y(i,j) K_t(i,j)            joint
 *     IP_y    = (1/N^2) sum_ij K_y(i,j)                     magnitude marginal (Sec. 3)
 *     IP_t(f) = (1/N^2) sum_ij K_t(i,j)                     warped-time marginal
 *     V_M(f)  = IP_y IP_t(f)
 *     V_C(f)  = (1/N^3) sum_i [sum_k K_y(i,k)] [sum_j K_t(i,j)]   cross
 *
 * From these come two scores:
 *     QMI(f)  = ln V_J + ln V_M - 2 ln V_C       Cauchy-Schwarz quadratic mutual information (>= 0)
 *     nCKP(f) = sqrt(N st) / IP_y * (V_J - V_M)  the normalised CKP of Sec. 3 (V_J - V_M is the CKP)
 *
 * Units: t in days, f in 1/day, y and e in magnitudes.  All floating-point arguments and results
 * are IEEE double.  Inside, the phase fold frac(f t) and the final scores are FP64; in the default
 * mixed precision the kernel values and the pair sums run in FP32 with FP64 block accumulation.
 *
 * Error behaviour: every function returns QMI_OK (0) or a negative QMI_E* code.  A call-level error
 * leaves every output buffer untouched and records a message for qmi_last_error.  A problem with
 * one curve (N < 2, a non-finite sample, a degenerate width rule) does not fail the call: that
 * curve's status is set and its outputs are NaN.  No C++ exception crosses this interface.
 *
 * Threading: a context is used by one host thread at a time; several contexts may share a device.
 */
#ifndef QMI_H
#define QMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define QMI_OK 0
#define QMI_EINVAL (-1)      /* invalid argument (bad sizes, sigma_t <= 0, f_max <= f_min, ...) */
#define QMI_ENOMEM (-2)      /* device memory: a single curve does not fit the HBM budget */
#define QMI_EDEVICE (-3)     /* HIP runtime error; text in qmi_last_error */
#define QMI_EDEGENERATE (-4) /* width rule gives zero (per-curve status only) */
#define QMI_EAGAIN (-5)      /* serving: admission budget full, submit again later */
#define QMI_EINTERNAL (-6)   /* internal error */

/* Limits. */
#define QMI_MAX_N 8192  /* samples per curve */
#define QMI_MAX_TOPK 32 /* refined peaks per curve */
#define QMI_MAX_BANDS 32    /* magnitude bands of the bands method */
#define QMI_MAX_TRIALS 1024 /* trial frequencies per band of the bands method */
#define QMI_MAX_MASKS 32     /* spurious-period masks (qmi_set_masks) */

/* sigma_y rules (qmi_kernel_params.sigma_y <= 0 selects a rule). */
#define QMI_SIGMA_SILVERMAN (-1.0)  /* 0.9 min(s, IQR/1.34) N^(-1/5); s on N-1, linear quartiles */
#define QMI_SIGMA_MEDIAN_ERR (-2.0) /* median of the error bars (Sec. 3) */

/* Scores. */
#define QMI_SCORE_CS_QMI 0
#define QMI_SCORE_NCKP 1

/* Arithmetic of the pair sums. */
#define QMI_PREC_MIXED 0 /* FP64 fold + FP32 kernel values + FP32 short sums folded into FP64 */
#define QMI_PREC_FP64 1  /* every step in FP64 */
/* Negative control for precision studies, not for use: QMI_PREC_MIXED with the phase fold
 * f t - rint(f t) taken in FP32 instead of FP64.  Over long baselines at high frequencies f t
 * reaches 1e5 cycles, where an FP32 ulp is ~0.01 cycle, and the scores degrade accordingly. */
#define QMI_PREC_FOLD32 2

/* Discriminator output values. */
#define QMI_NOT_PERIODIC 0
#define QMI_PERIODIC 1
#define QMI_UNDECIDED 255 /* bad status, non-finite score, or pSNR outside every bin */

typedef struct qmi_ctx qmi_ctx;

/*
 * One batch of curves in CSR form: curve k is samples [offsets[k], offsets[k+1]).
 * offsets is always a host array of n_curves + 1 non-decreasing int64 values starting at 0.
 * t, y (and e, which may be NULL) are host arrays for qmi_periodogram / qmi_best_period and device
 * arrays for the *_dev variants.  Samples may be in any order.  The library only reads them during
 * the call (the *_dev variants: until the call returns, after it has synchronised its stream).
 */
typedef struct {
    int32_t n_curves;
    const int64_t *offsets;
    const double *t; /* days */
    const double *y; /* magnitudes */
    const double *e; /* error bars, nullable (needed by QMI_SIGMA_MEDIAN_ERR and for pSNR) */
} qmi_batch;

/* sigma_t rule (qmi_kernel_params.sigma_t == QMI_SIGMA_T_SKEWNESS): per curve,
 * sigma_t = skew_lambda + 0.5 exp(-skew_mu S^2), S = (Q3 + Q1 - 2 Q2) / (Q3 - Q1) the quartile
 * estimator of the skewness of the magnitudes (Sec. 3, the skewness rule; S = 0 when Q3 = Q1), with
 * Q2 the median and Q1, Q3 the medians of the lower and upper half of the sorted magnitudes (for
 * odd N the middle value belongs to neither half).  Symmetric distributions get about
 * skew_lambda + 0.5, very skewed ones (eclipses) about skew_lambda.  The paper reports
 * skew_lambda = 0.1 and skew_mu = 12 for its survey; both zero selects these. */
#define QMI_SIGMA_T_SKEWNESS (-1.0)
#define QMI_SKEW_LAMBDA 0.1
#define QMI_SKEW_MU 12.0

/* sigma_t > 0: periodic-kernel width (Sec. 3 finds 0.1 - 0.6 typical), or QMI_SIGMA_T_SKEWNESS.
 * sigma_y > 0: explicit magnitude-kernel width, or one of the QMI_SIGMA_* rules.  precision:
 * QMI_PREC_*.  skew_lambda > 0 and skew_mu >= 0: constants of the sigma_t rule (both 0: the
 * paper's), read only when the rule is selected. */
typedef struct {
    double sigma_t;
    double sigma_y;
    int32_t precision;
    int32_t reserved;
    double skew_lambda;
    double skew_mu;
} qmi_kernel_params;

/*
 * Coarse-to-fine search for the frequency that maximises the score (Sec. 3; the refined peaks are
 * the highest local maxima of the coarse periodogram, the selection the bands method of Sec. 3.1
 * applies to its spectral windows).  The coarse grid is
 * f_k = f_min + k * ((f_max - f_min) / (n_coarse - 1)),
 * k = 0 .. n_coarse-1.  Its local maxima (q_k > q_{k-1} and q_k >= q_{k+1}; q_0 >= q_1 at the first
 * point, q_{F-1} > q_{F-2} at the last) are ranked by score, ties to the lower k, and the best top_k
 * are each refined on n_fine evenly spaced points of [f_{k-1}, f_{k+1}] ([f_0, f_1], [f_{F-2},
 * f_{F-1}] at the ends).  The best is the highest refined score, ties to the lower frequency, then
 * to the lower peak rank.  top_k = 0 (or n_fine = 0) returns the coarse argmax (ties to lower k).
 * Masks set with qmi_set_masks leave their candidates out of each of these selections.
 * Requirements: 0 <= f_min < f_max, 1 <= n_coarse <= 2^26, 0 <= top_k <= QMI_MAX_TOPK,
 * n_fine == 0 or 2 <= n_fine <= 2^20, score one of QMI_SCORE_*.
 */
typedef struct {
    double f_min, f_max;
    int32_t n_coarse, top_k, n_fine;
    int32_t score;
} qmi_search;

/*
 * Trial frequencies by the bands method (Sec. 3.1), for qmi_bands_best_period.  Per curve, samples
 * are taken in time order (stable) and split by magnitude rank into n_bands equal-count bands
 * (rank r goes to band floor(n_bands r / N)).  Band j is ranked by D_j = sum of |d_i| over its
 * samples i, d_i = (y_{i+1} - y_i) / (t_{i+1} - t_i) (summed in time order; a pair of equal times
 * adds nothing); the n_keep bands with the largest D_j (ties to the lower band) are kept.  For
 * each kept band the spectral window S_j(f) = |sum_{i in band} exp(2 pi i f t_i)|^2 is evaluated on
 * the grid f_k = f_lo + k * ((f_hi - f_lo) / (n_grid - 1)) (FP64), and its n_trials highest local
 * maxima (the local-maximum and tie rules of qmi_search), leaving out any with |1/f_k - 1| < 1e-4
 * (the one-day sampling period), are the band's trial frequencies.  The paper uses n_bands 10,
 * n_keep 3, n_trials 150 and the grid [0.00125, 3] 1/d; its grid density is not stated.
 * Requirements: 0 < f_lo < f_hi, 2 <= n_grid <= 2^24, 1 <= n_keep <= n_bands <= QMI_MAX_BANDS,
 * 1 <= n_trials <= QMI_MAX_TRIALS, score one of QMI_SCORE_*.
 */
typedef struct {
    double f_lo, f_hi;
    int32_t n_grid;
    int32_t n_bands, n_keep, n_trials;
    int32_t score;
    int32_t reserved;
} qmi_bands;

/*
 * One spurious-period mask (Sec. 6.1): a Gaussian in period, amplitude * exp(-(P - period)^2 /
 * (2 sigma^2)), with the amplitude in units of the searched score.  A candidate frequency f with
 * score s lies inside it when s < amplitude * exp(-(1/f - period)^2 / (2 sigma^2)).  The paper
 * centres masks on the periods of its table of spurious periods (the solar day, the synodic month,
 * the tropical year, the survey's mean span and their aliases) and tunes widths and amplitudes
 * on the survey's period histogram; it does not publish them.
 */
typedef struct {
    double period;    /* days, > 0 */
    double sigma;     /* days, > 0 */
    double amplitude; /* score units, finite */
} qmi_mask;

/* Per-curve result of qmi_best_period (and of qmi_bands_best_period, which uses the integer
 * fields as noted in its description). */
typedef struct {
    double f_best;      /* 1/day */
    double period;      /* 1 / f_best, days */
    double score;       /* the searched score at f_best */
    double score_qmi;   /* QMI at f_best */
    double score_nckp;  /* nCKP at f_best */
    double sigma_y;     /* magnitude-kernel width used */
    double psnr;        /* 0.7413 iqr(y) / median(e) (Sec. 5.2, alpha = 1); NaN without e */
    double coarse_best; /* coarse score at coarse_argmax */
    int32_t coarse_index;  /* k of the refined peak holding f_best (coarse_argmax without refinement) */
    int32_t peak_rank;     /* its rank among the refined peaks (-1 without refinement) */
    int32_t fine_index;    /* index of f_best inside that peak's fine grid (-1 without refinement) */
    int32_t coarse_argmax; /* argmax of the coarse scores outside every mask (-1: none) */
    int32_t n_peaks;       /* number of refined peaks */
    int32_t n;             /* samples */
    int32_t status;        /* QMI_OK or the per-curve QMI_E* code */
    int32_t reserved;
    double sigma_t;        /* periodic-kernel width used */
} qmi_result;

/* SNR-binned thresholds (Sec. 4.1): bin b is [edges[b], edges[b+1]); periodic iff score > th[b]. */
typedef struct {
    int32_t n_bins;
    int32_t score; /* QMI_SCORE_* the thresholds apply to */
    const double *edges; /* [n_bins + 1], non-decreasing */
    const double *th;    /* [n_bins] */
} qmi_thresholds;

/* Timing of the last qmi_periodogram / qmi_best_period call on this context, from HIP events on the
 * context stream (pair kernels only, and the whole device section). */
typedef struct {
    double pair_kernel_ms;   /* summed duration of the pair-sum kernel launches */
    double device_ms;        /* first kernel start to last kernel end */
    double pair_items;       /* sum over curves of N(N-1)/2 x evaluated frequencies */
    int32_t pair_launches;   /* number of pair-sum kernel launches */
    int32_t used_graph;      /* 1 if the device section ran as a captured hipGraph */
    int32_t pair_variant;    /* pair-kernel variant used (autotuned unless QMI_OPT_TILE is set) */
    int32_t reserved;
} qmi_stats;

/*
 * Create a context on HIP device hip_device.  hbm_budget_bytes caps the device memory the context
 * allocates (0: 80% of the device's free memory at creation).  hip_stream is the hipStream_t to
 * work on (NULL: the context creates its own stream at default priority).  Returns QMI_EDEVICE
 * when no usable device is present.  *out is set only on success.
 */
int qmi_create(qmi_ctx **out, int hip_device, size_t hbm_budget_bytes, void *hip_stream);

/* Release the context and all device memory it owns.  NULL is allowed. */
void qmi_destroy(qmi_ctx *ctx);

/* Message of the last error on ctx (never NULL; "" when none).  With ctx == NULL: the last
 * qmi_create failure of this thread. */
const char *qmi_last_error(const qmi_ctx *ctx);

/* Options (qmi_set_option). */
#define QMI_OPT_USE_GRAPH 1 /* 1: capture the device section into a hipGraph and replay it (default 1) */
#define QMI_OPT_TILE 2      /* pair-kernel variant: 0 autotuned per length bucket, k > 0 variant k-1 */
/* Variants 0-3: 2 or 4 waves per SIMD with 64- or 32-column chunks.  They give the same bits; the
 * autotuner times them on the first large call of each length bucket and keeps the fastest. */
#define QMI_OPT_SYNC 3      /* reserved */
/* Serving: at most this many pair x frequency items (sum over a launch's requests of
 * N(N-1)/2 x (n_coarse + top_k n_fine)) per launch of a lane (0: no bound, the default; a single
 * larger request still runs alone).  Read by qmi_serve_start. */
#define QMI_OPT_SERVE_BATCH_ITEMS 4
int qmi_set_option(qmi_ctx *ctx, int32_t option, int64_t value);

/* Copy the timing of the last call into *out. */
int qmi_get_stats(const qmi_ctx *ctx, qmi_stats *out);

/*
 * Spurious-period filter (Sec. 6.1) for the searches that follow on this context: qmi_best_period
 * (and _dev), qmi_bands_best_period and serving started afterwards.  Candidates inside any mask
 * take no part in a selection: the coarse argmax, the local maxima kept for refinement (the
 * local-maximum test still compares raw neighbours), the best refined point, and the best trial of
 * the bands method are each taken over candidates outside every mask.  A curve with no candidate
 * left gets f_best = period = score = NaN and coarse_index = coarse_argmax = -1 (status stays
 * QMI_OK).  Periodograms are not masked.
 *   masks    host, [n_masks], copied; NULL with n_masks = 0 removes every mask (the default)
 * QMI_EINVAL when n_masks < 0 or > QMI_MAX_MASKS, masks is NULL with n_masks > 0, a period or sigma
 * is not finite and positive, an amplitude is not finite, or serving is running on ctx.
 */
int qmi_set_masks(qmi_ctx *ctx, const qmi_mask *masks, int32_t n_masks);

/*
 * Periodogram at a caller-supplied frequency list (the same list for every curve).
 *   freqs      host, [n_freq] frequencies (finite, >= 0)
 *   score      QMI_SCORE_* written to score_out
 *   score_out  host, [n_curves * n_freq] row-major (curve, frequency)
 *   ips_out    nullable host, [n_curves * n_freq * 3]: V_J, IP_t, V_C per (curve, frequency)
 *   ip_y_out   nullable host, [n_curves]: IP_y
 *   status_out nullable host, [n_curves]: per-curve status
 * The inputs of the paper's problem statement: a curve, its kernel widths and a list of trial
 * frequencies (Sec. 3 maximises the CKP over trial frequencies for fixed widths).
 */
int qmi_periodogram(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                    const double *freqs, int32_t n_freq, int32_t score, double *score_out,
                    double *ips_out, double *ip_y_out, int32_t *status_out);

/*
 * Best period of each curve by the coarse-to-fine search of qmi_search.  The period estimate is the
 * trial frequency that maximises the score for fixed kernel widths (Sec. 3, where the CKP is
 * maximised over trial frequencies); the trial frequencies are refinement windows around the
 * highest local maxima of a coarse periodogram, as the bands method of Sec. 3.1 takes the highest
 * local maxima of its spectral windows.
 *   out         host, [n_curves]; coarse_index, peak_rank, fine_index locate f_best in the search
 *   coarse_out  nullable host, [n_curves * n_coarse]: the coarse periodogram of the searched score
 * Per-curve problems set out[k].status (QMI_EINVAL for N < 2 or a non-finite sample,
 * QMI_EDEGENERATE for a zero width) with NaN scores; call-level errors leave out untouched.
 */
int qmi_best_period(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                    const qmi_search *search, qmi_result *out, double *coarse_out);

/* Device-pointer variants: batch->t, y, e, freqs, score_out, ips_out and coarse_out are device
 * pointers (e.g. PyTorch-owned); offsets, ip_y_out, status_out and out stay host arrays.  They run
 * on the context's stream and return after it has completed. */
int qmi_periodogram_dev(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                        const double *freqs, int32_t n_freq, int32_t score, double *score_out,
                        double *ips_out, double *ip_y_out, int32_t *status_out);
int qmi_best_period_dev(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                        const qmi_search *search, qmi_result *out, double *coarse_out);

/*
 * For callers that cannot allocate device memory during the call (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): qmi_periodogram_dev computed
 * in a fixed scratch area instead of the context's buffers.  Arguments, layouts and results are
 * those of qmi_periodogram_dev (device t, y, e, freqs, score_out, ips_out; host offsets, ip_y_out,
 * status_out), and the results are bit-identical to it.  The call allocates nothing: every
 * intermediate table (per-curve parameters, magnitude Gram tables, row and column sums, partial
 * sums) lives in one static device array of QMI_NOALLOC_SCRATCH_BYTES per GPU, whose address is
 * resolved when the first context on that GPU is created and which the GPU holds until the
 * process ends.  The whole batch must fit it at once (about N * ceil(N/256) * 256 * 4 bytes per
 * curve of N samples, so one curve of up to ~3800 samples, or ~15 curves of 1000); a batch that
 * does not fit returns QMI_ENOMEM before any device work, outputs untouched.  Nothing in the
 * array needs to start at zero.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (from several contexts or threads) race and must be serialised by the caller.  No
 * timing is recorded (qmi_get_stats reads zeros) and no hipGraph is captured.
 */
#define QMI_NOALLOC_SCRATCH_BYTES (64u << 20)
int qmi_periodogram_noalloc(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                            const double *freqs, int32_t n_freq, int32_t score, double *score_out,
                            double *ips_out, double *ip_y_out, int32_t *status_out);

/*
 * Best period over the trial frequencies of the bands method (Sec. 3.1 followed by the score of
 * Sec. 3): the score at each of the n_keep * n_trials trial frequencies of every curve, and the
 * best (highest score, ties to the lower frequency, then the earlier trial).  Trials are listed band
 * by band in rank order, each band's maxima by rank; a band with fewer local maxima leaves its
 * remaining entries empty (NaN).
 *   out          host, [n_curves]; f_best, period, score, score_qmi, score_nckp, sigma_y, psnr,
 *                n and status as for qmi_best_period; coarse_index = the best trial's position in
 *                the list, peak_rank = its band's rank, fine_index = its rank inside the band,
 *                coarse_argmax = its index on the spectral-window grid, n_peaks = the number of
 *                trials found, coarse_best = NaN
 *   trials_out   nullable host, [n_curves * n_keep * n_trials] trial frequencies (NaN: empty)
 *   scores_out   nullable host, same shape: the score at each trial (NaN: empty)
 * Needs per curve about n_keep * n_grid * 8 bytes of device memory for the spectral windows, in
 * addition to the pair sums' tables.
 */
int qmi_bands_best_period(qmi_ctx *ctx, const qmi_batch *batch, const qmi_kernel_params *kp,
                          const qmi_bands *bands, qmi_result *out, double *trials_out,
                          double *scores_out);

/*
 * Preprocessing of Sec. 5.2, per curve: with error_cut, samples with e_i >= mean(e) + 3 sd(e) are
 * removed (sd with N - 1; when all error bars are equal nothing is removed); a curve left with
 * fewer than min_samples samples is rejected (the paper: 50); with detrend, the chi^2 line
 * a0 + a1 t minimising sum (a0 + a1 t_i - y_i)^2 / e_i^2 is subtracted from y when the Pearson
 * correlation between the line and the magnitudes exceeds 0.5.  error_cut and detrend need error
 * bars (detrend needs e > 0; a curve with e <= 0 is rejected).
 */
typedef struct {
    int32_t error_cut;
    int32_t min_samples; /* 2 .. QMI_MAX_N */
    int32_t detrend;
    int32_t reserved;
} qmi_preprocess_params;

/*
 * Preprocess a host batch.  Outputs (host, caller-owned) form a new batch: offsets_out
 * [n_curves + 1], t_out / y_out / e_out with room for the input's total sample count (e_out may
 * be NULL only when the batch has no error bars).  A rejected curve (invalid input, too short
 * after the cut) keeps no samples and gets status QMI_EINVAL in status_out (nullable,
 * [n_curves]); detrended_out (nullable, [n_curves]) is 1 where the line was subtracted.  The kept
 * samples stay in input order.
 */
int qmi_preprocess(qmi_ctx *ctx, const qmi_batch *batch, const qmi_preprocess_params *params,
                   int64_t *offsets_out, double *t_out, double *y_out, double *e_out,
                   int32_t *status_out, uint8_t *detrended_out);

/*
 * Whitening for the search of further modes (Sec. 7.1): per curve, fold with periods[k] (phase
 * t/P - floor(t/P)), order the samples by phase (stable), take as template at folded position i
 * the mean of the w = min(window, N) samples at positions i - w/2 .. i - w/2 + w - 1 (cyclic),
 * and write y - template to y_out (host, [total samples], input order).  The paper uses window 30.
 * A curve with invalid input or a period that is not finite and > 0 gets status QMI_EINVAL
 * (status_out nullable) and NaN outputs.
 */
int qmi_whiten(qmi_ctx *ctx, const qmi_batch *batch, const double *periods, int32_t window,
               double *y_out, int32_t *status_out);

/*
 * Periodic / non-periodic decision (Sec. 4.1): for curve k with status QMI_OK, pSNR p (psnr[k] if
 * psnr is not NULL, else best[k].psnr) in bin b and score s = best[k].score_qmi or score_nckp as
 * th->score selects, is_periodic[k] = QMI_PERIODIC iff s > th->th[b] (strict).  Curves with a bad
 * status, a non-finite score or pSNR outside every bin get QMI_UNDECIDED.  Host-only; needs no
 * device.  Returns QMI_EINVAL for bad threshold tables.
 */
int qmi_discriminate(const qmi_result *best, int32_t n_curves, const double *psnr,
                     const qmi_thresholds *th, uint8_t *is_periodic);

/*
 * Threshold calibration (Sec. 4.1): for each SNR bin b = [edges[b], edges[b+1]), over the curves k
 * with psnr[k] in the bin and a finite score, sweep n_points thresholds evenly spaced on
 * [min score, max score] (th_j = min + j * ((max - min) / (n_points - 1))), label a curve periodic
 * iff score > th_j, and keep the threshold of the highest F1 = 2 p r / (p + r) against truth[k]
 * (1 periodic, 0 not); ties go to the lowest threshold.  A bin with no periodic member gets
 * th = max score and F1 = p = r = 0; an empty bin th = +inf.  Outputs are [n_bins] host arrays
 * (f1_out, precision_out, recall_out nullable).  Host-only; returns QMI_EINVAL on bad arguments.
 */
int qmi_calibrate(const double *scores, const double *psnr, const uint8_t *truth, int32_t n,
                  const double *edges, int32_t n_bins, int32_t n_points, double *th_out,
                  double *f1_out, double *precision_out, double *recall_out);

/*
 * Serving (continuous batching).  qmi_serve_start starts max_inflight (1..8) worker threads, each
 * with a private context and stream on ctx's device (ctx's HBM budget split between them), and
 * fixes the kernel parameters and search of every request.  qmi_submit copies one curve (host
 * arrays of n samples; e nullable) into a host-side queue with a caller tag and returns QMI_OK, or
 * QMI_EAGAIN when the queued requests' estimated device footprint would exceed admit_budget_bytes
 * (0: half of ctx's budget); the caller owns t / y / e and may reuse them at once.  A free worker
 * takes queued requests in arrival order while they fit its share of the admission budget, at
 * most max_batch of them, runs them as one qmi_best_period call on its stream, and posts the
 * results; the launches of different workers overlap on the device.  A request's result does not
 * depend on the other requests it was batched with (bitwise).  qmi_poll moves up to max completed
 * results (with their tags) into out / tags and returns their count, waiting up to timeout_us
 * microseconds for at least one.  qmi_serve_stop finishes the queued requests, joins the workers
 * and discards results not yet polled.  A context serves at most one stream of requests at a time;
 * its other entry points stay usable meanwhile.
 */
int qmi_serve_start(qmi_ctx *ctx, const qmi_kernel_params *kp, const qmi_search *search,
                    size_t admit_budget_bytes, int32_t max_batch, int32_t max_inflight);
int qmi_submit(qmi_ctx *ctx, const double *t, const double *y, const double *e, int32_t n,
               uint64_t tag);
int qmi_poll(qmi_ctx *ctx, qmi_result *out, uint64_t *tags, int32_t max, int32_t timeout_us);
int qmi_serve_stop(qmi_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* QMI_H */
