// HIP kernels for gfx950 (MI355X): the per-curve preprocessing of Protopapas et al.,
// arXiv:1412.1840, Sec. 5.2 (error-bar cut, minimum length, chi^2 linear detrending) and the
// whitening of Sec. 7.1 (fold at a period, subtract a moving-average template) that turns a
// searched curve into the input of a search for a second mode.  One block per curve.
#include <math.h>

#include "qmi_internal.h"

namespace qmi {

namespace {

constexpr int kPrepBlock = 256;

// Deterministic block sum (wave shuffles, then the waves in order).
__device__ double prep_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kPrepBlock / 64; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__device__ double prep_min(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int i = 1; i < kPrepBlock / 64; ++i) s = fmin(s, sh[i]);
    __syncthreads();
    return s;
}

__device__ double prep_max(double v, double* sh) {
    return -prep_min(-v, sh);
}

// Error-bar cut, in-order compaction into the curve's own span of the output arrays, minimum
// length, chi^2 line and detrending.  counts[c] receives the kept length, status[c] QMI_OK or
// QMI_EINVAL (too short), detrended[c] 1 if the line was subtracted.
__global__ void __launch_bounds__(kPrepBlock)
prep_kernel(const int64_t* __restrict__ offsets, const double* __restrict__ t,
            const double* __restrict__ y, const double* __restrict__ e, PrepDev pd) {
    __shared__ double sh[kPrepBlock / 64];
    __shared__ int32_t scan[kPrepBlock];
    __shared__ int32_t s_base;
    const int c = blockIdx.x;
    const int64_t off = offsets[c], n = offsets[c + 1] - off;
    if (pd.status_in[c] != 0) {
        if (threadIdx.x == 0) {
            pd.counts[c] = 0;
            pd.status[c] = pd.status_in[c];
            pd.detrended[c] = 0;
        }
        return;
    }
    const double* tc = t + off;
    const double* yc = y + off;
    const double* ec = e + off;
    // Threshold of the error-bar cut: mean + 3 sd (sd with N - 1); no cut when all are equal.
    const bool has_e = e != nullptr;
    double thr = INFINITY;
    if (pd.error_cut) {
        double lo = INFINITY, hi = -INFINITY, s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += kPrepBlock) {
            lo = fmin(lo, ec[i]);
            hi = fmax(hi, ec[i]);
            s += ec[i];
        }
        lo = prep_min(lo, sh);
        hi = prep_max(hi, sh);
        const double mean = prep_sum(s, sh) / (double)n;
        double ss = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += kPrepBlock) ss += (ec[i] - mean) * (ec[i] - mean);
        ss = prep_sum(ss, sh);
        if (lo != hi) thr = mean + 3.0 * sqrt(n > 1 ? ss / (double)(n - 1) : 0.0);
    }
    // In-order compaction, 256 samples at a time (block-wide exclusive scan of the keep flags).
    double* to = pd.t_out + off;
    double* yo = pd.y_out + off;
    double* eo = pd.e_out + off;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (int64_t i0 = 0; i0 < n; i0 += kPrepBlock) {
        const int64_t i = i0 + threadIdx.x;
        const int keep = (i < n) && (!pd.error_cut || ec[i] < thr);
        scan[threadIdx.x] = keep;
        __syncthreads();
        for (int d = 1; d < kPrepBlock; d <<= 1) {
            const int v = threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        const int base = s_base;
        if (keep) {
            const int p = base + scan[threadIdx.x] - 1;
            to[p] = tc[i];
            yo[p] = yc[i];
            eo[p] = has_e ? ec[i] : 0.0;
        }
        __syncthreads();
        if (threadIdx.x == kPrepBlock - 1) s_base = base + scan[threadIdx.x];
        __syncthreads();
    }
    const int64_t m = s_base;
    if (m < pd.min_samples) {
        if (threadIdx.x == 0) {
            pd.counts[c] = (int32_t)m;
            pd.status[c] = -1;  // QMI_EINVAL: too short after the cut
            pd.detrended[c] = 0;
        }
        return;
    }
    int applied = 0;
    if (pd.detrend) {
        double S = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0;
        for (int64_t i = threadIdx.x; i < m; i += kPrepBlock) {
            const double w = 1.0 / (eo[i] * eo[i]);
            S += w;
            Sx += w * to[i];
            Sy += w * yo[i];
            Sxx += w * to[i] * to[i];
            Sxy += w * to[i] * yo[i];
        }
        S = prep_sum(S, sh);
        Sx = prep_sum(Sx, sh);
        Sy = prep_sum(Sy, sh);
        Sxx = prep_sum(Sxx, sh);
        Sxy = prep_sum(Sxy, sh);
        const double den = S * Sxx - Sx * Sx;
        const double a1 = den != 0.0 ? (S * Sxy - Sx * Sy) / den : 0.0;
        const double a0 = (Sy - a1 * Sx) / S;
        // Pearson correlation of the fitted line with the magnitudes.
        double mf = 0, my = 0;
        for (int64_t i = threadIdx.x; i < m; i += kPrepBlock) {
            mf += a0 + a1 * to[i];
            my += yo[i];
        }
        mf = prep_sum(mf, sh) / (double)m;
        my = prep_sum(my, sh) / (double)m;
        double sfy = 0, sff = 0, syy = 0;
        for (int64_t i = threadIdx.x; i < m; i += kPrepBlock) {
            const double df = a0 + a1 * to[i] - mf, dy = yo[i] - my;
            sfy += df * dy;
            sff += df * df;
            syy += dy * dy;
        }
        sfy = prep_sum(sfy, sh);
        sff = prep_sum(sff, sh);
        syy = prep_sum(syy, sh);
        const double r = (sff > 0.0 && syy > 0.0) ? sfy / sqrt(sff * syy) : 0.0;
        if (r > 0.5) {
            applied = 1;
            __syncthreads();
            for (int64_t i = threadIdx.x; i < m; i += kPrepBlock) yo[i] = yo[i] - (a0 + a1 * to[i]);
        }
    }
    if (threadIdx.x == 0) {
        pd.counts[c] = (int32_t)m;
        pd.status[c] = 0;
        pd.detrended[c] = (uint8_t)applied;
    }
}

// Bitonic sort of (key, idx) in LDS by key then idx (the stable order of the keys).
__device__ void prep_sort_pairs(double* key, int32_t* idx, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += kPrepBlock) {
                const int l = i ^ j;
                if (l > i) {
                    const double a = key[i], b = key[l];
                    const int32_t ia = idx[i], ib = idx[l];
                    const bool gt = (a > b) || (a == b && ia > ib);
                    const bool up = (i & k) == 0;
                    if (gt == up) {
                        key[i] = b;
                        key[l] = a;
                        idx[i] = ib;
                        idx[l] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Whitening: phase order at period P, template = mean of the w cyclic neighbours in phase order
// (positions i - w/2 .. i - w/2 + w - 1), y - template written at the sample's input position.
// Dynamic LDS: pow2(max_n) x 12 bytes.
__global__ void __launch_bounds__(kPrepBlock)
whiten_kernel(const int64_t* __restrict__ offsets, const double* __restrict__ t,
              const double* __restrict__ y, const double* __restrict__ periods, int window,
              const int32_t* __restrict__ status, double* __restrict__ y_out) {
    extern __shared__ double wsh[];
    const int c = blockIdx.x;
    const int64_t off = offsets[c];
    const int n = (int)(offsets[c + 1] - off);
    if (status[c] != 0) return;
    int m = 1;
    while (m < n) m <<= 1;
    double* key = wsh;
    int32_t* idx = reinterpret_cast<int32_t*>(wsh + m);
    const double P = periods[c];
    for (int i = threadIdx.x; i < m; i += kPrepBlock) {
        if (i < n) {
            const double x = t[off + i] / P;
            key[i] = x - floor(x);
            idx[i] = i;
        } else {
            key[i] = INFINITY;
            idx[i] = 0x7fffffff;
        }
    }
    __syncthreads();
    prep_sort_pairs(key, idx, m);
    const int w = window < n ? window : n;
    for (int i = threadIdx.x; i < n; i += kPrepBlock) {
        double s = 0.0;
        for (int q = 0; q < w; ++q) {
            int p = (i - w / 2 + q) % n;
            if (p < 0) p += n;
            s += y[off + idx[p]];
        }
        y_out[off + idx[i]] = y[off + idx[i]] - s / (double)w;
    }
}

}  // namespace

size_t whiten_lds(int max_n) {
    int m = 1;
    while (m < max_n) m <<= 1;
    return (size_t)m * 12;
}

hipError_t launch_prep(hipStream_t st, int n_curves, const int64_t* offsets, const double* t,
                       const double* y, const double* e, const PrepDev& pd) {
    if (n_curves <= 0) return hipSuccess;
    prep_kernel<<<n_curves, kPrepBlock, 0, st>>>(offsets, t, y, e, pd);
    return hipGetLastError();
}

hipError_t launch_whiten(hipStream_t st, int n_curves, int max_n, const int64_t* offsets,
                         const double* t, const double* y, const double* periods, int window,
                         const int32_t* status, double* y_out) {
    if (n_curves <= 0) return hipSuccess;
    whiten_kernel<<<n_curves, kPrepBlock, whiten_lds(max_n), st>>>(offsets, t, y, periods, window,
                                                                   status, y_out);
    return hipGetLastError();
}

}  // namespace qmi
