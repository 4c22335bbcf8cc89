// Internal declarations shared by the device code (qmi_kernels.hip) and the host runtime
// (qmi_api.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qmi.h"

namespace qmi {

// Pair-kernel geometry.  A work item is (curve, tile of kLanes frequency slots); one lane owns one
// frequency.  The pair triangle i < j is walked in passes of kPass rows; inside a pass wave w owns
// the interleaved rows base + w + kWaves*m (m < rows per wave), so every wave has nearly the same
// number of valid pairs in the diagonal region.  Columns j stream through LDS in chunks of kChunk.
constexpr int kLanes = 64;
constexpr int kWaves = 8;
constexpr int kThreads = kWaves * kLanes;
constexpr int kXcds = 8;    // accelerator complex dies of an MI355X, one L2 each
constexpr int kPass = 256;  // rows per pass; the K-table permutation is defined on it
constexpr int kChunk = 64;  // columns per LDS chunk

// Position of row i inside its pass in the K-table layout: rows of one wave are contiguous, so a
// wave reads its rows' kernel values for one column with scalar loads.
__host__ __device__ inline int64_t kperm(int64_t i) {
    int64_t b = i & ~int64_t(kPass - 1);
    int64_t r = i & (kPass - 1);
    return b + (r & (kWaves - 1)) * (kPass / kWaves) + (r >> 3);
}
__host__ __device__ inline int64_t kperm_inv(int64_t s) {
    int64_t b = s & ~int64_t(kPass - 1);
    int64_t r = s & (kPass - 1);
    return b + (r / (kPass / kWaves)) + kWaves * (r % (kPass / kWaves));
}

// Per-curve state, written by the host (off, koff, n, npad, status, sigma_t) and completed by the
// prologue and Gram kernels.
struct CurveParams {
    int64_t off;   // first sample in the packed t / y / e arrays
    int64_t koff;  // first element of this curve's K table
    int64_t poff;  // first element of this curve's permuted FP64 row-sum array (npad entries)
    int64_t ksoff; // first element of this curve's column K-sum table (passes * kWaves * n)
    int32_t n;     // samples
    int32_t npad;  // K-table row length (multiple of kPass)
    int32_t status;
    int32_t has_e;
    double sigma_t;       // > 0; QMI_SIGMA_T_SKEWNESS until the prologue sets it
    double sigma_y_rule;  // > 0 explicit, -1 Silverman, -2 median error bar
    double sigma_y;
    double A, B;   // 1 / (sqrt(2 pi) sigma)
    double ipy;    // IP_y
    double rsum;   // sum_i r_i
    double psnr;
    double bk;     // diagonal value of the stored K table (B rounded to the kernel type)
    double sjc;    // sum_{i<j} K(i,j)            (FP64, from the stored K table)
    int64_t pqoff; // first piece of this curve in a one-piece-per-workgroup launch's partial sums
};

// Interleaved partial sums of a column's terms over a wave's rows (row m goes to partial
// m mod kPartials), combined at the end of the column: the pair kernel and the column-sum tables
// it subtracts use the same order.  Two partials issue 1% faster than four (two adds fewer per
// column and sum) and as fast as one.
constexpr int kPartials = 2;
static_assert(kPartials == 1 || kPartials == 2 || kPartials == 4, "1, 2 or 4 partial sums");

template <typename R>
__host__ __device__ inline R combine_partials(const R* p) {
    if constexpr (kPartials == 1) return p[0];
    else if constexpr (kPartials == 2) return p[0] + p[1];
    else return (p[0] + p[1]) + (p[2] + p[3]);
}

// Rows per wave of the pair kernel for each arithmetic type (a pass is kWaves times this).
template <typename R>
constexpr int rows_per_wave() {
    return sizeof(R) == 4 ? 32 : 16;
}

// How frequency slot s of curve c maps to a frequency.
struct FreqPlan {
    int32_t kind;   // 0 linear grid, 1 explicit list, 2 refinement windows, 3 per-curve lists
    int32_t count;  // slots per curve
    int32_t n_fine;
    int32_t top_k;
    int32_t stride;  // kind 3: row length of the per-curve lists
    int32_t tile_cap;  // > 0: the pair kernel runs only the first tile_cap tiles of kLanes slots
    double f0, df;           // kind 0: f = f0 + s * df
    const double* list;      // kind 1: [count]; kind 3: [curve][stride], NaN = no frequency
    const double* win;       // kind 2: [curve][top_k][2] = (lo, step)
    const int32_t* npk;      // kind 2: [curve] refined peaks
};

struct PairOut {
    double* score;   // [curve][count] primary score
    double* score2;  // nullable: [curve][count] the other score
    double* ips;     // nullable: [curve][count][3] V_J, IP_t, V_C
    int32_t score_kind;
    int32_t pad;
    double* part;    // one piece per workgroup: [piece (pqoff + q)][count][3] FP64 piece sums
};

struct PeakOut {
    int32_t* peak_k;   // [curve][top_k]
    int32_t* npk;      // [curve]
    double* win;       // [curve][top_k][2]
    int32_t* argmax;   // [curve]
};

// Spurious-period masks (Sec. 6.1), passed to the selection kernels by value.  A candidate (f, s)
// is inside mask i when s < amp[i] exp(-(1/f - period[i])^2 / (2 sigma[i]^2)).
struct MaskDev {
    int32_t n;
    int32_t pad;
    double period[QMI_MAX_MASKS];
    double sigma[QMI_MAX_MASKS];
    double amp[QMI_MAX_MASKS];
};

__device__ __forceinline__ bool in_mask(const MaskDev& md, double f, double s) {
    if (md.n == 0) return false;
    const double P = 1.0 / f;
    for (int i = 0; i < md.n; ++i) {
        const double d = P - md.period[i];
        if (s < md.amp[i] * exp(-(d * d) / (2.0 * md.sigma[i] * md.sigma[i]))) return true;
    }
    return false;
}

// Result record written by the best-of kernel (mirrors qmi_result field order).
struct DevResult {
    double f_best, period, score, score_qmi, score_nckp, sigma_y, psnr, coarse_best;
    int32_t coarse_index, peak_rank, fine_index, coarse_argmax, n_peaks, n, status, reserved;
    double sigma_t;
};

// Bands method (qmi_bands.hip): per-group device buffers and parameters.
struct BandsDev {
    double f_lo, df;      // spectral-window grid f_k = f_lo + k df
    int32_t n_grid, n_bands, n_keep, n_trials;
    int32_t stride;       // band_t row length (at least the largest band)
    int32_t pad;
    double* ts;           // [samples] times in time order (at each curve's offset)
    double* ys;           // [samples] magnitudes in the same order
    double* band_t;       // [curve][n_keep][stride] sample times of the kept bands
    int32_t* band_cnt;    // [curve][n_keep]
    int32_t* band_id;     // [curve][n_keep] band index of each kept band
    double* S;            // [curve][n_keep][n_grid] spectral windows
    double* trials;       // [curve][n_keep * n_trials] trial frequencies, NaN = none
    int32_t* trial_k;     // [curve][n_keep * n_trials] their grid indices, -1 = none
};
size_t bands_prep_lds(int max_n);
hipError_t launch_bands(hipStream_t st, const CurveParams* cp, int n_curves, int max_n,
                        const double* t, const double* y, const BandsDev& bd);
hipError_t launch_bands_best(hipStream_t st, const CurveParams* cp, int n_curves,
                             const double* score, const double* score2, int score_kind,
                             const BandsDev& bd, const MaskDev& md, DevResult* res);

// Preprocessing and whitening (qmi_prep.hip).
struct PrepDev {
    int32_t error_cut, detrend, min_samples, pad;
    const int32_t* status_in;  // [curve] host validation (nonzero: skip the curve)
    int32_t* counts;           // [curve] samples kept
    int32_t* status;           // [curve] QMI_OK or QMI_EINVAL (too short)
    uint8_t* detrended;        // [curve] 1 if the chi^2 line was subtracted
    double* t_out;             // kept samples, compacted inside each curve's input span
    double* y_out;
    double* e_out;
};
size_t whiten_lds(int max_n);
hipError_t launch_prep(hipStream_t st, int n_curves, const int64_t* offsets, const double* t,
                       const double* y, const double* e, const PrepDev& pd);
hipError_t launch_whiten(hipStream_t st, int n_curves, int max_n, const int64_t* offsets,
                         const double* t, const double* y, const double* periods, int window,
                         const int32_t* status, double* y_out);

// Launchers (qmi_kernels.hip).  All launch on `st` and return hipGetLastError().
// skew_lambda, skew_mu: constants of the sigma_t rule, applied to curves whose sigma_t is
// QMI_SIGMA_T_SKEWNESS.
hipError_t launch_prologue(hipStream_t st, CurveParams* cp, int n_curves, int max_n,
                           const double* t, const double* y, const double* e, double skew_lambda,
                           double skew_mu);
template <typename R>
hipError_t launch_gram(hipStream_t st, CurveParams* cp, int n_curves, int64_t total_rows,
                       const int64_t* row_curve_start, const double* y, R* K, double* rp,
                       double* rd);
template <typename R>
hipError_t launch_gram_finalize(hipStream_t st, CurveParams* cp, int n_curves, const double* rd,
                                double* rp);
template <typename R>
hipError_t launch_ksum(hipStream_t st, const CurveParams* cp, int n_curves, int max_n, const R* K,
                       R* ks);
// Pair-kernel variants: ids 0 .. pair_variants<R>() - 1 (0 is the default), and for R = float
// kVariantFold32, the shape of variant 0 with the phase fold in FP32 (a precision control).
// split_pmax > 0 (with out.part): one (pass, column segment) piece per workgroup, at most
// split_pmax pieces per curve, then the epilogue kernel; 0: every piece of a (curve, tile) in one
// workgroup.  Both give the same bits.
constexpr int kVariantFold32 = -1;
template <typename R>
int pair_variants();
template <typename R>
hipError_t launch_pairs(hipStream_t st, const CurveParams* cp, const int32_t* order,
                        int n_work_curves, const FreqPlan& fp, const double* t, const R* K,
                        const double* rd, const double* rp, const R* ks, const PairOut& out,
                        int variant, int split_pmax);
// The last kRemSlots slots of per-curve frequency lists (fp.kind 3) from slot0 on, one row per
// lane (FP32 path; pairs with fp.tile_cap = slot0 / kLanes on the main launch).
constexpr int kRemSlots = kLanes / 32;
hipError_t launch_pairs_rows(hipStream_t st, const CurveParams* cp, const int32_t* order,
                             int n_work_curves, const FreqPlan& fp, int slot0, const double* t,
                             const float* K, const double* rd, const PairOut& out);
hipError_t launch_peaks(hipStream_t st, const CurveParams* cp, int n_curves, const double* coarse,
                        int n_coarse, double f0, double df, int top_k, int n_fine,
                        const MaskDev& md, const PeakOut& po);
hipError_t launch_best(hipStream_t st, const CurveParams* cp, int n_curves, const double* coarse,
                       const double* coarse2, int n_coarse, const double* fine,
                       const double* fine2, int top_k, int n_fine, int score_kind, double f0,
                       double df, const MaskDev& md, const PeakOut& po, DevResult* res);

}  // namespace qmi
