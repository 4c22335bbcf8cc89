// HIP kernels for gfx950 (MI355X): trial frequencies by the bands method of Protopapas et al.,
// arXiv:1412.1840, Sec. 3.1, and the best trial after the pair sums have scored them.
//
// Per curve: samples in time order, equal-count magnitude bands, the bands ranked by the summed
// absolute first derivative of their samples, the spectral window of each kept band's sample times
// on a linear grid (FP64), and the band's highest local maxima of the window as trial frequencies.
// The pair kernel then scores the per-curve trial lists (frequency plan kind 3).
#include <math.h>

#include "qmi_internal.h"

namespace qmi {

namespace {

constexpr int kBandsBlock = 256;
constexpr int kWindowBlock = 256;
constexpr int kTrialsBlock = 256;
constexpr int kTieCap = 2048;  // equal-valued maxima gathered in LDS when selecting by value

__device__ __forceinline__ double band_grid_f(double f0, double df, int k) {
    return __dadd_rn(f0, __dmul_rn((double)k, df));
}

// Bitonic sort of (key, idx) pairs in LDS by key, then idx (a total order, so the result is the
// stable order of the keys).  m is a power of two; entries n..m-1 must hold (+inf, large idx).
template <int BLOCK>
__device__ void sort_pairs(double* key, int32_t* idx, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += BLOCK) {
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

// One block per curve: time order, magnitude bands, D_j, the kept bands and their sample times.
// Dynamic LDS: pow2(max_n) x (8 + 4 + 4) bytes.
__global__ void __launch_bounds__(kBandsBlock)
bands_prep_kernel(const CurveParams* __restrict__ cp, const double* __restrict__ t_all,
                  const double* __restrict__ y_all, BandsDev bd) {
    extern __shared__ double sh[];
    __shared__ double D[QMI_MAX_BANDS];
    __shared__ int32_t keep[QMI_MAX_BANDS];
    const int c = blockIdx.x;
    const CurveParams P = cp[c];
    const int nk = bd.n_keep, nb = bd.n_bands;
    if (P.status != 0) {
        if (threadIdx.x < nk) {
            bd.band_cnt[(int64_t)c * nk + threadIdx.x] = 0;
            bd.band_id[(int64_t)c * nk + threadIdx.x] = -1;
        }
        return;
    }
    const int n = P.n;
    int m = 1;
    while (m < n) m <<= 1;
    double* key = sh;
    int32_t* idx = reinterpret_cast<int32_t*>(sh + m);
    int32_t* band = idx + m;
    const double* t = t_all + P.off;
    const double* y = y_all + P.off;
    double* ts = bd.ts + P.off;
    double* ys = bd.ys + P.off;

    // Time order (stable).
    for (int i = threadIdx.x; i < m; i += kBandsBlock) {
        key[i] = i < n ? t[i] : INFINITY;
        idx[i] = i < n ? i : 0x7fffffff;
    }
    __syncthreads();
    sort_pairs<kBandsBlock>(key, idx, m);
    for (int i = threadIdx.x; i < n; i += kBandsBlock) {
        ts[i] = key[i];
        ys[i] = y[idx[i]];
    }
    __syncthreads();
    // Magnitude ranks in time order (stable), then the equal-count bands.
    for (int i = threadIdx.x; i < m; i += kBandsBlock) {
        key[i] = i < n ? ys[i] : INFINITY;
        idx[i] = i < n ? i : 0x7fffffff;
    }
    __syncthreads();
    sort_pairs<kBandsBlock>(key, idx, m);
    for (int r = threadIdx.x; r < n; r += kBandsBlock)
        band[idx[r]] = (int32_t)(((int64_t)r * nb) / n);
    __syncthreads();
    // D_j: |first derivative| summed over the band's samples in time order (one thread per band,
    // so the order of the additions is fixed).
    if (threadIdx.x < nb) {
        double d = 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            if (band[i] != (int)threadIdx.x) continue;
            const double dt = ts[i + 1] - ts[i];
            if (dt != 0.0) d += fabs((ys[i + 1] - ys[i]) / dt);
        }
        D[threadIdx.x] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned used = 0;
        for (int b = 0; b < nk; ++b) {
            int best = -1;
            for (int j = 0; j < nb; ++j) {
                if (used & (1u << j)) continue;
                if (best < 0 || D[j] > D[best]) best = j;  // ties keep the lower band
            }
            used |= 1u << best;
            keep[b] = best;
        }
    }
    __syncthreads();
    // The kept bands' sample times, in time order.
    if (threadIdx.x < nk) {
        const int b = threadIdx.x, j = keep[b];
        double* out = bd.band_t + ((int64_t)c * nk + b) * bd.stride;
        int cnt = 0;
        for (int i = 0; i < n; ++i)
            if (band[i] == j) out[cnt++] = ts[i];
        bd.band_cnt[(int64_t)c * nk + b] = cnt;
        bd.band_id[(int64_t)c * nk + b] = j;
    }
}

// Spectral window S(f_k) = |sum_i exp(2 pi i f_k t_i)|^2 over a kept band's times (FP64).  A
// thread owns kWinRun consecutive grid points: per sample it forms exp(2 pi i f t) at its first
// point from the folded phase x - rint(x), x = f t, and steps to the next points by multiplying
// with exp(2 pi i df t) (one complex product per point instead of a sine and a cosine; the
// rounding error grows by a few ulp per step).  Blocks walk (curve, band, grid tile).
constexpr int kWinRun = 16;

__device__ __forceinline__ void cis2pi(double x, double& c, double& s) {
    const double p = x - rint(x);
    sincospi(2.0 * p, &s, &c);
}

__global__ void __launch_bounds__(kWindowBlock)
window_kernel(const CurveParams* __restrict__ cp, int tiles, BandsDev bd) {
    extern __shared__ double2 step[];  // [cnt] (cos, sin) of 2 pi df t_i
    const int64_t blk = blockIdx.x;
    const int tile = (int)(blk % tiles);
    const int64_t cb = blk / tiles;  // curve * n_keep + band
    const int c = (int)(cb / bd.n_keep);
    const int cnt = (cp[c].status == 0) ? bd.band_cnt[cb] : 0;
    const double* bt = bd.band_t + cb * bd.stride;
    for (int i = threadIdx.x; i < cnt; i += kWindowBlock) {
        double sc, ss;
        cis2pi(bd.df * bt[i], sc, ss);
        step[i] = make_double2(sc, ss);
    }
    __syncthreads();
    const int k0 = (tile * kWindowBlock + threadIdx.x) * kWinRun;
    if (k0 >= bd.n_grid) return;
    const double f0 = band_grid_f(bd.f_lo, bd.df, k0);
    double re[kWinRun], im[kWinRun];
#pragma unroll
    for (int g = 0; g < kWinRun; ++g) re[g] = im[g] = 0.0;
    for (int i = 0; i < cnt; ++i) {
        double zr, zi;
        cis2pi(f0 * bt[i], zr, zi);
        const double2 w = step[i];
#pragma unroll
        for (int g = 0; g < kWinRun; ++g) {
            re[g] += zr;
            im[g] += zi;
            const double nr = zr * w.x - zi * w.y;
            zi = zr * w.y + zi * w.x;
            zr = nr;
        }
    }
    double* out = bd.S + cb * bd.n_grid;
#pragma unroll
    for (int g = 0; g < kWinRun; ++g)
        if (k0 + g < bd.n_grid) out[k0 + g] = re[g] * re[g] + im[g] * im[g];
}

// Candidate key of grid point k: 1 + the bits of S(k) (S >= 0, so the order of the keys is the
// order of the values) for a local maximum outside the one-day window, else 0.
__device__ __forceinline__ uint64_t cand_key(const double* S, int F, int k, double f0, double df) {
    const double v = S[k];
    bool peak;
    if (F == 1) peak = (v == v);
    else if (k == 0) peak = v >= S[1];
    else if (k == F - 1) peak = v > S[k - 1];
    else peak = v > S[k - 1] && v >= S[k + 1];
    if (!peak) return 0;
    const double f = band_grid_f(f0, df, k);
    if (fabs(1.0 / f - 1.0) < 1e-4) return 0;
    return (uint64_t)__double_as_longlong(v) + 1;
}

// The n_trials highest local maxima of one band's window (ties to the lower grid index), by a
// radix select of the n_trials-th largest key over 8-bit digits, then a sort of the selection.
__global__ void __launch_bounds__(kTrialsBlock)
trials_kernel(const CurveParams* __restrict__ cp, BandsDev bd) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t s_prefix;
    __shared__ int32_t s_need, s_total, s_ngt, s_neq;
    __shared__ double sel_key[QMI_MAX_TRIALS];
    __shared__ int32_t sel_k[QMI_MAX_TRIALS];
    __shared__ int32_t tie_k[kTieCap];
    const int64_t cb = blockIdx.x;
    const int c = (int)(cb / bd.n_keep);
    const int b = (int)(cb % bd.n_keep);
    const int F = bd.n_grid, nt = bd.n_trials;
    double* out_f = bd.trials + (int64_t)c * bd.n_keep * nt + (int64_t)b * nt;
    int32_t* out_k = bd.trial_k + (int64_t)c * bd.n_keep * nt + (int64_t)b * nt;
    if (cp[c].status != 0) {
        for (int r = threadIdx.x; r < nt; r += kTrialsBlock) {
            out_f[r] = NAN;
            out_k[r] = -1;
        }
        return;
    }
    const double* S = bd.S + cb * F;
    if (threadIdx.x == 0) {
        s_total = 0;
        s_ngt = 0;
        s_neq = 0;
    }
    __syncthreads();
    int local = 0;
    for (int k = threadIdx.x; k < F; k += kTrialsBlock)
        local += cand_key(S, F, k, bd.f_lo, bd.df) != 0;
    atomicAdd(&s_total, local);
    __syncthreads();
    const int total = s_total;
    const int take = total < nt ? total : nt;
    uint64_t T = 1;  // with total <= nt every candidate (key >= 1) is taken
    int need_eq = 0;
    if (total > nt) {
        uint64_t prefix = 0;
        int need = nt;
        for (int shift = 56; shift >= 0; shift -= 8) {
            for (int i = threadIdx.x; i < 256; i += kTrialsBlock) hist[i] = 0;
            __syncthreads();
            const uint64_t hi = (shift == 56) ? 0ull : (~0ull << (shift + 8));
            for (int k = threadIdx.x; k < F; k += kTrialsBlock) {
                const uint64_t key = cand_key(S, F, k, bd.f_lo, bd.df);
                if (key != 0 && (key & hi) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int d = 255;
                for (; d > 0; --d) {
                    if ((int)hist[d] >= need) break;
                    need -= (int)hist[d];
                }
                s_prefix = prefix | ((uint64_t)d << shift);
                s_need = need;
            }
            __syncthreads();
            prefix = s_prefix;
            need = s_need;
            __syncthreads();
        }
        T = prefix;
        need_eq = need;
    }
    // Gather: every key above T, and the need_eq lowest grid indices with key == T (all keys >= T
    // when every candidate is taken).
    for (int k = threadIdx.x; k < F; k += kTrialsBlock) {
        const uint64_t key = cand_key(S, F, k, bd.f_lo, bd.df);
        if (key == 0) continue;
        if (total <= nt || key > T) {
            const int p = atomicAdd(&s_ngt, 1);
            if (p < nt) {  // at most nt keys lie above T (radix-select invariant)
                sel_key[p] = __longlong_as_double((long long)(key - 1));
                sel_k[p] = k;
            }
        } else if (key == T) {
            const int p = atomicAdd(&s_neq, 1);
            if (p < kTieCap) tie_k[p] = k;
        }
    }
    __syncthreads();
    if (total > nt) {
        const int neq = s_neq, ngt = s_ngt < nt ? s_ngt : nt;
        if (need_eq > nt - ngt) need_eq = nt - ngt;
        if (threadIdx.x == 0) {
            // The need_eq lowest indices among the ties (a selection over at most kTieCap entries;
            // beyond that, a scan of the grid in index order).
            const double tv = __longlong_as_double((long long)(T - 1));
            if (neq <= kTieCap) {
                for (int q = 0; q < need_eq; ++q) {
                    int bi = q;
                    for (int r = q + 1; r < neq; ++r)
                        if (tie_k[r] < tie_k[bi]) bi = r;
                    const int tmp = tie_k[q];
                    tie_k[q] = tie_k[bi];
                    tie_k[bi] = tmp;
                    sel_key[ngt + q] = tv;
                    sel_k[ngt + q] = tie_k[q];
                }
            } else {
                int q = 0;
                for (int k = 0; k < F && q < need_eq; ++k)
                    if (cand_key(S, F, k, bd.f_lo, bd.df) == T) {
                        sel_key[ngt + q] = tv;
                        sel_k[ngt + q] = k;
                        ++q;
                    }
            }
        }
        __syncthreads();
    }
    // Order the selection by value (descending), then grid index, and write it out.
    int m = 1;
    while (m < take) m <<= 1;
    for (int i = take + threadIdx.x; i < m; i += kTrialsBlock) {
        sel_key[i] = -INFINITY;
        sel_k[i] = 0x7fffffff;
    }
    __syncthreads();
    for (int kk = 2; kk <= m; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += kTrialsBlock) {
                const int l = i ^ j;
                if (l > i) {
                    const double a = sel_key[i], bv = sel_key[l];
                    const int32_t ka = sel_k[i], kb = sel_k[l];
                    // "a after b" in the output order: smaller value, or equal value and larger k.
                    const bool after = (a < bv) || (a == bv && ka > kb);
                    const bool up = (i & kk) == 0;
                    if (after == up) {
                        sel_key[i] = bv;
                        sel_key[l] = a;
                        sel_k[i] = kb;
                        sel_k[l] = ka;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < nt; r += kTrialsBlock) {
        if (r < take) {
            out_f[r] = band_grid_f(bd.f_lo, bd.df, sel_k[r]);
            out_k[r] = sel_k[r];
        } else {
            out_f[r] = NAN;
            out_k[r] = -1;
        }
    }
}

// Best trial per curve: highest score outside every spurious-period mask (Sec. 6.1), ties to the
// lower frequency, then the earlier trial.
constexpr int kBandsBestBlock = 256;

__device__ __forceinline__ bool trial_before(double qa, double fa, int sa, double qb, double fb,
                                             int sb) {
    if (!(qa == qa)) return false;
    if (!(qb == qb)) return true;
    if (qa != qb) return qa > qb;
    if (fa != fb) return fa < fb;
    return sa < sb;
}

__global__ void __launch_bounds__(kBandsBestBlock)
bands_best_kernel(const CurveParams* __restrict__ cp, const double* __restrict__ score,
                  const double* __restrict__ score2, int score_kind, BandsDev bd, MaskDev md,
                  DevResult* __restrict__ res) {
    __shared__ double sq[kBandsBestBlock], sf[kBandsBestBlock];
    __shared__ int ss[kBandsBestBlock], sfound[kBandsBestBlock];
    const int c = blockIdx.x;
    const CurveParams P = cp[c];
    const int F = bd.n_keep * bd.n_trials;
    const double* q = score + (int64_t)c * F;
    const double* fr = bd.trials + (int64_t)c * F;
    double bq = NAN, bf = INFINITY;
    int bs = 0x7fffffff, found = 0;
    if (P.status == 0) {
        for (int s = threadIdx.x; s < F; s += kBandsBestBlock) {
            const double f = fr[s];
            if (!(f == f)) continue;
            ++found;
            if (trial_before(q[s], f, s, bq, bf, bs) && !in_mask(md, f, q[s])) {
                bq = q[s];
                bf = f;
                bs = s;
            }
        }
    }
    sq[threadIdx.x] = bq;
    sf[threadIdx.x] = bf;
    ss[threadIdx.x] = bs;
    sfound[threadIdx.x] = found;
    __syncthreads();
    for (int h = kBandsBestBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = threadIdx.x + h;
            if (trial_before(sq[o], sf[o], ss[o], sq[threadIdx.x], sf[threadIdx.x],
                             ss[threadIdx.x])) {
                sq[threadIdx.x] = sq[o];
                sf[threadIdx.x] = sf[o];
                ss[threadIdx.x] = ss[o];
            }
            sfound[threadIdx.x] += sfound[o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    DevResult r;
    r.sigma_y = P.sigma_y;
    r.sigma_t = P.sigma_t > 0.0 ? P.sigma_t : NAN;  // the rule flag until the prologue ran
    r.psnr = P.psnr;
    r.coarse_best = NAN;
    r.n = P.n;
    r.status = P.status;
    r.reserved = 0;
    r.n_peaks = sfound[0];
    const int s = ss[0];
    if (P.status != 0 || s == 0x7fffffff) {
        r.f_best = r.period = r.score = r.score_qmi = r.score_nckp = NAN;
        r.coarse_index = r.peak_rank = r.fine_index = r.coarse_argmax = -1;
    } else {
        r.f_best = sf[0];
        r.period = 1.0 / sf[0];
        r.score = sq[0];
        const double other = score2 ? score2[(int64_t)c * F + s] : NAN;
        r.score_qmi = score_kind == 0 ? sq[0] : other;
        r.score_nckp = score_kind == 0 ? other : sq[0];
        r.coarse_index = s;
        r.peak_rank = s / bd.n_trials;
        r.fine_index = s % bd.n_trials;
        r.coarse_argmax = bd.trial_k[(int64_t)c * F + s];
    }
    res[c] = r;
}

}  // namespace

size_t bands_prep_lds(int max_n) {
    int m = 1;
    while (m < max_n) m <<= 1;
    return (size_t)m * (8 + 4 + 4);
}

hipError_t launch_bands(hipStream_t st, const CurveParams* cp, int n_curves, int max_n,
                        const double* t, const double* y, const BandsDev& bd) {
    if (n_curves <= 0) return hipSuccess;
    bands_prep_kernel<<<n_curves, kBandsBlock, bands_prep_lds(max_n), st>>>(cp, t, y, bd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per_block = kWindowBlock * kWinRun;
    const int tiles = (bd.n_grid + per_block - 1) / per_block;
    const int64_t blocks = (int64_t)n_curves * bd.n_keep * tiles;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    window_kernel<<<(unsigned)blocks, kWindowBlock, (size_t)bd.stride * 16, st>>>(cp, tiles, bd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    trials_kernel<<<(unsigned)((int64_t)n_curves * bd.n_keep), kTrialsBlock, 0, st>>>(cp, bd);
    return hipGetLastError();
}

hipError_t launch_bands_best(hipStream_t st, const CurveParams* cp, int n_curves,
                             const double* score, const double* score2, int score_kind,
                             const BandsDev& bd, const MaskDev& md, DevResult* res) {
    if (n_curves <= 0) return hipSuccess;
    bands_best_kernel<<<n_curves, kBandsBestBlock, 0, st>>>(cp, score, score2, score_kind, bd,
                                                             md, res);
    return hipGetLastError();
}

}  // namespace qmi
