// HIP kernels for gfx950 (MI355X): prologue (kernel widths, pSNR), magnitude Gram matrix, column
// K sums and the pair x frequency sums (the hot path).  The peak search and best-of kernels are in
// qmi_search.hip.
//
// Method: Protopapas et al., arXiv:1412.1840.  Gaussian kernel (Sec. 2), periodic kernel and the
// warp identity ||u_f(z) - u_f(y)||^2 = 4 sin^2(pi f (z - y)) (Sec. 2.1), CKP and information
// potential (Sec. 3), normalised CKP (Sec. 3), pSNR (Sec. 5.2).
#include <float.h>
#include <math.h>

#include "qmi_internal.h"

namespace qmi {

namespace {

constexpr double kLog2e = 1.4426950408889634073599246810018921;
constexpr double kInvSqrt2Pi = 0.39894228040143267793994605993438187;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// --------------------------------------------------------------------------------------------
// Block-wide helpers
// --------------------------------------------------------------------------------------------

template <int BLOCK>
__device__ double block_sum(double v, double* sh) {
    // Deterministic tree: wave shuffles, then one value per wave combined in wave order.
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < BLOCK / 64; ++k) s += sh[k];
        sh[0] = s;
    }
    __syncthreads();
    double r = sh[0];
    __syncthreads();
    return r;
}

// In-LDS bitonic sort of n values (padded to a power of two with +inf) by one block.
template <int BLOCK>
__device__ void block_sort(double* a, int n) {
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = n + threadIdx.x; i < m; i += BLOCK) a[i] = INFINITY;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += BLOCK) {
                int l = i ^ j;
                if (l > i) {
                    double x = a[i], y = a[l];
                    bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Quantile by linear interpolation at position (n-1) p of sorted a[0..n).
__device__ double sorted_quantile(const double* a, int n, double p) {
    double h = (n - 1) * p;
    int lo = (int)floor(h);
    int hi = lo + 1 < n ? lo + 1 : n - 1;
    return a[lo] + (h - lo) * (a[hi] - a[lo]);
}

__device__ double sorted_median(const double* a, int n) {
    return (n & 1) ? a[n / 2] : 0.5 * (a[n / 2 - 1] + a[n / 2]);
}

// --------------------------------------------------------------------------------------------
// Prologue: validity, sigma_y (Silverman or median error bar), sigma_t (given, or the skewness
// rule of Sec. 3), pSNR, A, B.  One block per curve.
// --------------------------------------------------------------------------------------------

constexpr int kPrologueBlock = 256;

__global__ void __launch_bounds__(kPrologueBlock)
prologue_kernel(CurveParams* __restrict__ cp, const double* __restrict__ t,
                const double* __restrict__ y, const double* __restrict__ e, double skew_lambda,
                double skew_mu) {
    extern __shared__ double sbuf[];  // [QMI_MAX_N rounded to pow2] + 64 scratch
    __shared__ double red[kPrologueBlock / 64 + 1];
    __shared__ int bad;
    const int c = blockIdx.x;
    CurveParams P = cp[c];
    const int n = P.n;
    if (P.status != 0) return;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const double* tc = t + P.off;
    const double* yc = y + P.off;
    const double* ec = P.has_e ? e + P.off : nullptr;
    for (int i = threadIdx.x; i < n; i += kPrologueBlock) {
        bool ok = isfinite(tc[i]) && isfinite(yc[i]);
        if (ec) ok = ok && isfinite(ec[i]);
        if (!ok) bad = 1;
    }
    __syncthreads();
    if (bad || n < 2) {
        if (threadIdx.x == 0) cp[c].status = -1;  // QMI_EINVAL
        return;
    }
    // Mean and sample deviation of y.
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kPrologueBlock) s += yc[i];
    const double mean = block_sum<kPrologueBlock>(s, red) / n;
    s = 0.0;
    for (int i = threadIdx.x; i < n; i += kPrologueBlock) {
        double d = yc[i] - mean;
        s += d * d;
    }
    const double sdev = sqrt(block_sum<kPrologueBlock>(s, red) / (n - 1));
    // Quartiles of y.
    for (int i = threadIdx.x; i < n; i += kPrologueBlock) sbuf[i] = yc[i];
    block_sort<kPrologueBlock>(sbuf, n);
    const double iqr = sorted_quantile(sbuf, n, 0.75) - sorted_quantile(sbuf, n, 0.25);
    // sigma_t rule (Sec. 3): S = (Q3 + Q1 - 2 Q2) / (Q3 - Q1) with Q2 the median and Q1, Q3 the
    // medians of the lower and upper n / 2 sorted magnitudes; S = 0 when Q3 = Q1.
    double sigma_t = P.sigma_t;
    if (!(sigma_t > 0.0)) {
        const int h = n / 2;
        const double q1 = sorted_median(sbuf, h), q2 = sorted_median(sbuf, n);
        const double q3 = sorted_median(sbuf + (n - h), h);
        const double S = (q3 == q1) ? 0.0 : (q3 + q1 - 2.0 * q2) / (q3 - q1);
        sigma_t = skew_lambda + 0.5 * exp(-skew_mu * S * S);
    }
    __syncthreads();
    double med_e = NAN;
    if (ec) {
        for (int i = threadIdx.x; i < n; i += kPrologueBlock) sbuf[i] = ec[i];
        block_sort<kPrologueBlock>(sbuf, n);
        med_e = sorted_median(sbuf, n);
    }
    if (threadIdx.x != 0) return;
    double sy = 0.0;
    int status = 0;
    if (P.sigma_y_rule > 0.0) {
        sy = P.sigma_y_rule;
    } else if (P.sigma_y_rule == -1.0) {
        if (sdev == 0.0) {
            status = -4;  // QMI_EDEGENERATE
        } else {
            double spread = (iqr == 0.0) ? sdev : fmin(sdev, iqr / 1.34);
            sy = 0.9 * spread * pow((double)n, -0.2);
        }
    } else {
        if (!(med_e > 0.0)) status = ec ? -4 : -1;
        sy = med_e;
    }
    cp[c].status = status;
    cp[c].sigma_y = status ? NAN : sy;
    cp[c].sigma_t = sigma_t;
    cp[c].A = kInvSqrt2Pi / sigma_t;
    cp[c].B = status ? NAN : kInvSqrt2Pi / sy;
    cp[c].psnr = (ec && med_e > 0.0) ? 0.7413 * iqr / med_e : NAN;
}

// --------------------------------------------------------------------------------------------
// Magnitude Gram matrix K(j, i) = B exp(-(y_j - y_i)^2 / (2 sy^2)) in the permuted row layout, and
// r_j = sum_i K(j, i) (diagonal B included).  One block per row j of one curve.
// --------------------------------------------------------------------------------------------

constexpr int kGramBlock = 256;

template <typename R>
__global__ void __launch_bounds__(kGramBlock)
gram_kernel(const CurveParams* __restrict__ cp, const int64_t* __restrict__ row_curve_start,
            int n_curves, const double* __restrict__ y, R* __restrict__ K,
            double* __restrict__ rp, double* __restrict__ rd) {
    __shared__ double red[kGramBlock / 64 + 1];
    const int64_t row = blockIdx.x;
    // Curve of this row: binary search over the prefix of row counts.
    int lo = 0, hi = n_curves - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (row_curve_start[mid] <= row) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const CurveParams P = cp[c];
    const int j = (int)(row - row_curve_start[c]);
    if (P.status != 0) return;
    const double* yc = y + P.off;
    const double yj = yc[j];
    const double inv2s2 = 1.0 / (2.0 * P.sigma_y * P.sigma_y);
    R* Krow = K + P.koff + (int64_t)j * P.npad;
    double acc = 0.0;
    for (int s = threadIdx.x; s < P.npad; s += kGramBlock) {
        int64_t i = kperm_inv(s);
        R v = R(0);
        if (i < P.n) {
            double d = yj - yc[i];
            v = (R)(P.B * exp(-d * d * inv2s2));
        }
        Krow[s] = v;
        acc += (double)v;
    }
    acc = block_sum<kGramBlock>(acc, red);
    if (threadIdx.x == 0) {
        rp[P.poff + kperm(j)] = acc;
        rd[P.off + j] = acc;
    }
}

constexpr int kFinBlock = 256;

// IP_y = sum_i r_i / N^2, and zero the padding rows of the permuted row-sum array.
template <typename R>
__global__ void __launch_bounds__(kFinBlock)
gram_finalize_kernel(CurveParams* __restrict__ cp, const double* __restrict__ rd,
                     double* __restrict__ rp) {
    __shared__ double red[kFinBlock / 64 + 1];
    const int c = blockIdx.x;
    const CurveParams P = cp[c];
    if (P.status != 0 || P.npad == 0) return;
    for (int s = threadIdx.x; s < P.npad; s += kFinBlock)
        if (kperm_inv(s) >= P.n) rp[P.poff + s] = 0.0;
    double acc = 0.0;
    for (int i = threadIdx.x; i < P.n; i += kFinBlock) acc += rd[P.off + i];
    acc = block_sum<kFinBlock>(acc, red);
    if (threadIdx.x == 0) {
        const double N = (double)P.n;
        const double bk = (double)(R)P.B;  // K(i,i) as stored
        cp[c].rsum = acc;
        cp[c].ipy = acc / (N * N);
        cp[c].bk = bk;
        cp[c].sjc = 0.5 * (acc - N * bk);  // the table is symmetric: sum_{i<j} K = (sum - diag)/2
    }
}

// Column K-sums in the pair kernel's own rounding order: for pass p, wave w and column j, the
// sum over the wave's rows i < j of K(i, j), accumulated in the kernel type exactly as the pair
// kernel accumulates K(i, j) g_ij: kPartials interleaved partials (rows m mod kPartials, each row
// by row with an fma), combined as the kernel combines them.  Where every g_ij of a column is
// exactly 1 (coincident phases, f = 0) the kernel's column sum equals this value bit for bit, so
// their difference is exactly zero.  blockIdx.x is the curve; the curve's (pass, wave, column)
// entries are dealt over the gridDim.y blocks of its row (each entry is computed alone, so the
// split does not change a value).
constexpr int kKsBlock = 256;

template <typename R>
__global__ void __launch_bounds__(kKsBlock)
ksum_kernel(const CurveParams* __restrict__ cp, const R* __restrict__ K, R* __restrict__ ks) {
    constexpr int ROWS = rows_per_wave<R>();
    constexpr int PASS = kWaves * ROWS;
    const int c = blockIdx.x;
    const CurveParams P = cp[c];
    if (P.status != 0 || P.npad == 0) return;
    const int n = P.n;
    const int passes = (n + PASS - 1) / PASS;
    const int64_t total = (int64_t)passes * kWaves * n;
    for (int64_t e = (int64_t)blockIdx.y * kKsBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.y * kKsBlock) {
        const int j = (int)(e % n);
        const int pw = (int)(e / n);
        const int w = pw % kWaves, base = (pw / kWaves) * PASS;
        const int nrows = min(ROWS, max(0, (n - base - w + kWaves - 1) / kWaves));
        int cnt = (j - base - w + kWaves - 1) / kWaves;
        cnt = cnt < 0 ? 0 : (cnt > nrows ? nrows : cnt);
        // The wave's ROWS values of column j are one aligned 128-byte run of row j of the
        // permuted table (always inside the row: kperm(base + w) + ROWS <= base + PASS <= npad);
        // read it whole with 16-byte loads, then add its first cnt values in row order.
        const R* kr = K + P.koff + (int64_t)j * P.npad + kperm(base + w);
        R kv[ROWS];
        const float4* kr4 = reinterpret_cast<const float4*>(kr);
#pragma unroll
        for (int q = 0; q < (int)(ROWS * sizeof(R) / 16); ++q)
            *reinterpret_cast<float4*>(&kv[q * 16 / sizeof(R)]) = kr4[q];
        R acc[kPartials];
#pragma unroll
        for (int q = 0; q < kPartials; ++q) acc[q] = R(0);
#pragma unroll
        for (int m = 0; m < ROWS; ++m)
            if (m < cnt) acc[m % kPartials] = fma(kv[m], R(1), acc[m % kPartials]);
        ks[P.ksoff + e] = combine_partials(acc);
    }
}

// --------------------------------------------------------------------------------------------
// Pair x frequency sums.
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ double slot_freq(const FreqPlan& fp, int c, int s, bool& active) {
    active = s < fp.count;
    if (!active) return 0.0;
    if (fp.kind == 0) return __dadd_rn(fp.f0, __dmul_rn((double)s, fp.df));
    if (fp.kind == 1) return fp.list[s];
    if (fp.kind == 3) {
        const double v = fp.list[(int64_t)c * fp.stride + s];
        active = v == v;
        return active ? v : 0.0;
    }
    const int p = s / fp.n_fine, m = s - p * fp.n_fine;
    if (p >= fp.npk[c]) {
        active = false;
        return 0.0;
    }
    const double* w = fp.win + ((int64_t)c * fp.top_k + p) * 2;
    return __dadd_rn(w[0], __dmul_rn((double)m, w[1]));
}

// sin(2 pi p) and cos(2 pi p) for p in [-1/2, 1/2] (an FP64-folded phase), accurate to about 1e-9:
// 2 pi p = (pi/2)(q + r) with q = rint(4p) and |r| <= 1/2, then the Taylor series of sin and cos of
// theta = (pi/2) r (|theta| <= pi/4; the first omitted terms are below 7e-10) and the quadrant
// identities sin(q pi/2 + theta), cos(q pi/2 + theta).
__device__ __forceinline__ void sincos_2pi_reduced(double p, double& sn, double& cs) {
    const double x = 4.0 * p;
    const double q = rint(x);
    const double th = (x - q) * 1.5707963267948966192313216916397514;
    const double t2 = th * th;
    const double s = th * fma(t2, fma(t2, fma(t2, fma(t2, 1.0 / 362880.0, -1.0 / 5040.0),
                                                  1.0 / 120.0), -1.0 / 6.0), 1.0);
    const double c = fma(t2, fma(t2, fma(t2, fma(t2, fma(t2, -1.0 / 3628800.0, 1.0 / 40320.0),
                                                     -1.0 / 720.0), 1.0 / 24.0), -0.5), 1.0);
    const int iq = ((int)q) & 3;
    sn = (iq == 0) ? s : (iq == 1) ? c : (iq == 2) ? -s : -c;
    cs = (iq == 0) ? c : (iq == 1) ? -s : (iq == 2) ? -c : s;
}

// Half-angle warp of a sample: h(t) = (2 log2(e) / sigma_t^2)^(1/4) (cos pi p, sin pi p) with p the
// phase f t folded to [-1/2, 1/2] in FP64 (fma gives f t - rint(f t) with one rounding).  For two
// samples d = h_s(i) h_c(j) - h_c(i) h_s(j) = sqrt(2 log2 e) / sigma_t * sin(pi f (t_i - t_j)), so
// exp2(-d^2) = exp(-2 sin^2(pi f (t_i - t_j)) / sigma_t^2), the periodic kernel of Sec. 2.1 without
// its constant (sin^2 of half the angle between the warp points u_f(t_i), u_f(t_j), whose chord is
// 2 |sin|).  d is formed from a difference of products, so it is exact to rounding when the two
// phases coincide and the kernel value is then exactly 1.
template <typename R, bool FOLD32 = false>
struct Warp;

template <bool FOLD32>
struct Warp<float, FOLD32> {
    using V = float2;
    __device__ __forceinline__ static V at(double f, double t, double scale) {
        double p;
        if constexpr (FOLD32) {
            // Precision control only: the fold in FP32 (one rounding of f t to FP32).
            const float x = (float)f * (float)t;
            p = (double)(x - rintf(x));
        } else {
            const double n = rint(f * t);
            p = fma(f, t, -n);
        }
        double sn, cs;
        sincos_2pi_reduced(0.5 * p, sn, cs);  // sin(pi p), cos(pi p)
        return make_float2((float)(cs * scale), (float)(sn * scale));
    }
    __device__ __forceinline__ static float kexp(float a) { return __builtin_amdgcn_exp2f(a); }
};

template <>
struct Warp<double, false> {
    using V = double2;
    __device__ __forceinline__ static V at(double f, double t, double scale) {
        const double n = rint(f * t);
        const double p = fma(f, t, -n);
        double sn, cs;
        sincospi(p, &sn, &cs);
        return make_double2(cs * scale, sn * scale);
    }
    __device__ __forceinline__ static double kexp(double a) { return exp2(a); }
};


// The lane index, formed afresh from the lane count.  The empty asm keeps the compiler from
// reusing an earlier copy, so that no register holds the lane index (or an address derived from
// it) across the pair kernel's loops only to be spilled.
__device__ __forceinline__ int fresh_lane() {
    int l = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    asm volatile("" : "+v"(l));
    return l;
}

// Exponent offset of a row in the diagonal region: 0, or +inf for a masked row (g = 0).  The
// choice is wave-uniform and made on the scalar unit (an integer select of the bit pattern), so
// that the offset is a scalar operand of the kernel-argument FMA and costs no VALU instruction.
template <typename R>
__device__ __forceinline__ R mask_offset(bool masked) {
    if constexpr (sizeof(R) == 4) {
        return __int_as_float(__builtin_amdgcn_readfirstlane(masked ? 0x7f800000 : 0));
    } else {
        const int hi = __builtin_amdgcn_readfirstlane(masked ? 0x7ff00000 : 0);
        return __longlong_as_double((long long)hi << 32);
    }
}

// Adds v to a lane-private LDS accumulator without returning the old value (ds_add_f64).
__device__ __forceinline__ void ladd(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// One term of the pair sums for row i of this wave and the current column j: the kernel value
// g = exp2(-(d^2 + moff)) with d = h_s(i) h_c(j) - h_c(i) h_s(j) and moff = 0 (or +inf for a row
// that is masked out, giving g = 0), added to a column partial T, the row sum G and a K-weighted
// column partial J.  With FIRST the term starts the column partials instead (T = g, J = k g): the
// same values as adding to partials of zero, since g and k are never negative, without the
// additions of zero.
template <typename R, bool FIRST = false>
__device__ __forceinline__ void pair_term(R hc, R hs, R ux, R uy, R moff, R k, R& T, R& G, R& J) {
    const R pr = hc * uy;
    const R d = fma(hs, ux, -pr);
    const R a = fma(d, d, moff);
    const R g = Warp<R>::kexp(-a);
    G += g;
    if constexpr (FIRST) {
        T = g;
        J = k * g;
    } else {
        T += g;
        J = fma(k, g, J);
    }
}

// Scheduling request for a straight-line column body of ROWS rows: the exp of each row placed
// between VALU work (three VALU instructions, the exp, three more), so that the exps of a wave
// spread over the column instead of each row's chain (multiply-adds, exp, accumulations) issuing
// back to back.
template <typename R, int ROWS>
__device__ __forceinline__ void interleave_exps() {
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int m = 0; m < ROWS; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
            __builtin_amdgcn_sched_group_barrier(0x400, 1, 0);  // transcendental
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
        }
    }
}

// The epilogue of a (curve, slot): V_J, IP_t, V_C from the FP64 pair sums and the Gram-stage
// constants, then QMI and nCKP (Sec. 3).
__device__ __forceinline__ void pair_scores(const CurveParams& P, double SJ, double ST, double SC,
                                            int64_t obase, const PairOut& out) {
    const double N = (double)P.n;
    const double VJ = P.A * (N * P.bk + 2.0 * (P.sjc + SJ)) / (N * N);
    const double IPt = P.A * (N + 2.0 * ST) / (N * N);
    const double VC = P.A * (P.rsum + SC) / (N * N * N);
    const double VM = P.ipy * IPt;
    const double q = log(VJ) + log(VM) - 2.0 * log(VC);
    const double nckp = sqrt(N * P.sigma_t) / P.ipy * (VJ - VM);
    out.score[obase] = out.score_kind == 0 ? q : nckp;
    if (out.score2) out.score2[obase] = out.score_kind == 0 ? nckp : q;
    if (out.ips) {
        out.ips[obase * 3 + 0] = VJ;
        out.ips[obase * 3 + 1] = IPt;
        out.ips[obase * 3 + 2] = VC;
    }
}

// One work item = (curve, kLanes frequency slots).  Accumulators per lane (one frequency), FP64:
//   ST  = sum_{i<j} g_ij                 SJ  = sum_{i<j} K(i,j) g_ij - sum_{i<j} K(i,j)
//   SC  = sum_{i<j} (r_i + r_j) g_ij
// with g_ij = exp(-2 sin^2(pi f (t_i - t_j)) / sigma_t^2) and r_i = sum_k K(i,k).  A column's
// terms over the wave's rows are summed in R in kPartials interleaved partials and folded
// into FP64 per column; the r-weighted sums multiply R sums by FP64 row sums.  Where all kernel
// values are 1 (coincident phases, f = 0) every R sum is exact: the column sums of g and the row
// sums are integers, and the K-weighted column sum equals, bit for bit, the precomputed sum of K
// over the same rows in the same order, so that SJ is 0 and the scores come out exactly.
// Summation order.  The work of a (curve, tile) is cut into pieces (pass p, column segment s >= p),
// a segment being the PASS columns [s PASS, (s + 1) PASS): a piece's sums are its waves' sums added
// in wave order, and the totals are the pieces' sums added in the order (0,0), (0,1), ..., (1,1),
// ....  A workgroup either runs every piece of its (curve, tile) and adds each into the totals
// (SPLIT false), or - in a launch with too few (curve, tile) items to fill the chip - runs a
// single piece and stores its sums in out.part, for pair_epilogue_kernel to add in the same order
// (SPLIT true): both give the same bits.
// Variants: WPE is the occupancy target in waves per SIMD (2: the registers of 2 waves; 4: at most
// 128 VGPRs, so two workgroups share a CU), CH the columns per LDS chunk; all four give the same
// bits (the row sums are folded every 64 columns whatever the chunk), and the host autotuner
// chooses among them per length bucket.  PULLK (per-curve frequency lists) reads each column's K
// block while staging it.
template <typename R, int WPE, int CH, bool FOLD32 = false, bool PULLK = false, bool SPLIT = false>
__global__ void __launch_bounds__(kThreads, WPE)
pairs_kernel(const CurveParams* __restrict__ cp, const int32_t* __restrict__ order,
             FreqPlan fp, const double* __restrict__ t_all, const R* __restrict__ K_all,
             const double* __restrict__ rd_all, const double* __restrict__ rp_all,
             const R* __restrict__ ks_all, int n_work, int xcd_grouped, int split_pmax,
             PairOut out) {
    using W = Warp<R, FOLD32>;
    using V = typename W::V;
    constexpr int ROWS = rows_per_wave<R>();
    constexpr int PASS = kWaves * ROWS;
    constexpr int GRP = 4;  // rows skipped together in the diagonal region
    __shared__ V ph[2][CH][kLanes];
    __shared__ double fq[kLanes];  // the lane's frequency, re-read where the warp is formed
    __shared__ double acc[3][kWaves][kLanes];  // this piece's SJ, ST, SC per wave (added to in place)
    __shared__ double tot[3][kLanes];          // totals over the pieces done so far (wave x: x)

    const int lane = threadIdx.x & 63;
    const int w = uniform((int)(threadIdx.x >> 6));
    const int tiles = fp.tile_cap > 0 ? fp.tile_cap : (fp.count + kLanes - 1) / kLanes;
    // The dispatcher deals blocks to the XCDs round robin (block b runs on XCD b mod kXcds), and
    // each XCD has its own L2.  With enough curves (xcd_grouped), every XCD gets whole curves
    // (work ranks x, x + kXcds, ...) with their frequency tiles in consecutive blocks, so that a
    // curve's K table is fetched into one L2 only; the grid is then padded to a multiple of kXcds
    // curves.  Otherwise consecutive blocks are the tiles of one curve, spread over all XCDs.
    int rank, tile, piece = -1;
    if (SPLIT) {
        // One piece per workgroup: blocks are (rank, piece, tile), pieces of a curve in order.
        const int per_rank = split_pmax * tiles;
        rank = (int)(blockIdx.x / (unsigned)per_rank);
        const int rem = (int)(blockIdx.x - (unsigned)rank * per_rank);
        piece = rem / tiles;
        tile = rem - piece * tiles;
    } else if (xcd_grouped) {
        const int xcd = (int)(blockIdx.x % kXcds);
        const int seq = (int)(blockIdx.x / kXcds);
        rank = (seq / tiles) * kXcds + xcd;
        tile = seq - (seq / tiles) * tiles;
    } else {
        rank = (int)(blockIdx.x / tiles);
        tile = (int)(blockIdx.x - (unsigned)rank * tiles);
    }
    if (rank >= n_work) return;
    const int c = order[rank];
    const CurveParams P = cp[c];
    const int slot = tile * kLanes + lane;
    bool active;
    const double f = slot_freq(fp, c, slot, active);

    const int nb = (P.n + PASS - 1) / PASS;  // passes (and column segments)
    int p_lo = 0, p_hi = nb, s_only = -1;
    if (SPLIT) {
        // A curve with a bad status has its outputs written by the epilogue kernel.
        if (P.status != 0 || piece >= nb * (nb + 1) / 2) return;
        int pp = 0, q = piece;
        while (q >= nb - pp) {
            q -= nb - pp;
            ++pp;
        }
        p_lo = pp;
        p_hi = pp + 1;
        s_only = pp + q;
    }

    if (P.status != 0) {
        const int64_t obase = (int64_t)c * fp.count + slot;
        if (active && w == 0) {
            out.score[obase] = NAN;
            if (out.score2) out.score2[obase] = NAN;
            if (out.ips) {
                out.ips[obase * 3 + 0] = NAN;
                out.ips[obase * 3 + 1] = NAN;
                out.ips[obase * 3 + 2] = NAN;
            }
        }
        return;
    }

    const int n = P.n;
    const double* t = t_all + P.off;
    const double* rr = rd_all + P.off;
    const double scale = uniform(sqrt(sqrt(2.0 * kLog2e) / P.sigma_t));
    const R zero = R(0);

    // The FP64 sums SJ, ST and SC = SCa + SCb of this lane live in LDS and are added to in place,
    // so that no registers are held for them across the column loops.
    double* aSJ = &acc[0][w][lane];
    double* aST = &acc[1][w][lane];
    double* aSC = &acc[2][w][lane];
    *aSJ = 0.0;
    *aST = 0.0;
    *aSC = 0.0;
    if (w < 3) tot[w][lane] = 0.0;
    // Kept in LDS rather than in two registers across the column loops.
    if (w == 0) fq[lane] = f;
    __syncthreads();

    const int base_end = SPLIT ? p_hi * PASS : n;
    for (int base = SPLIT ? p_lo * PASS : 0; base < base_end; base += PASS) {
        // This wave's rows: base + w + kWaves * m, m < nrows.
        const int nrows = uniform(min(ROWS, max(0, (n - base - w + kWaves - 1) / kWaves)));
        // Columns [cbeg, cend): the whole pass, or the piece's segment.
        const int cbeg = SPLIT ? s_only * PASS : base;
        const int cend = SPLIT ? min(n, cbeg + PASS) : n;
        const int nch = (cend - cbeg + CH - 1) / CH;
        // Where the columns start at the pass's own rows (every launch but the off-diagonal
        // pieces of a split one), the rows' warp vectors are the staged vectors of the diagonal
        // block's columns, read from LDS as each chunk arrives (rows_from_chunk below); they
        // start at zero, as do rows past the end of the curve.  Otherwise they are formed here.
        const bool rows_staged = (cbeg == base);
        R ci[ROWS], si[ROWS], G[ROWS];
#pragma unroll
        for (int m = 0; m < ROWS; ++m) {
            const int i = base + w + kWaves * m;
            V u = (!rows_staged && m < nrows) ? W::at(fq[lane], t[i], scale) : V{R(0), R(0)};
            ci[m] = u.x;
            si[m] = u.y;
            G[m] = R(0);
        }
        const int64_t kofs = kperm(base + w);
        const R* Kbase = K_all + P.koff + kofs;
        const double* rpb = rp_all + P.poff + kofs;
        const R* ksb = ks_all + P.ksoff + (int64_t)((base / PASS) * kWaves + w) * n;

        // With per-curve frequency lists (a few tiles per curve, as in the bands method) the
        // workgroups of a curve run side by side and every column's scalar K loads would miss the
        // L2; staging a column then also reads its 1 KB K block of this pass (16 bytes per lane,
        // padding rows included), a chunk before the column is used.  The value only feeds an
        // empty asm statement, which keeps the load and changes nothing.
        constexpr bool pull_k = PULLK && sizeof(R) == 4;
        auto stage = [&](int j0, int buf) {
            for (int q = w; q < CH; q += kWaves) {
                const int j = j0 + q;
                const int ls = fresh_lane();
                if (pull_k && j < n) {
                    const float4 kb = reinterpret_cast<const float4*>(
                        K_all + P.koff + (int64_t)j * P.npad + base)[ls];
                    asm volatile("" ::"v"(kb.x));
                }
                ph[buf][q][ls] = (j < n) ? W::at(fq[ls], t[j], scale) : V{R(0), R(0)};
            }
        };
        stage(cbeg, 0);
        __syncthreads();
        // Chunks in segment order: the inner loop runs the chunks of one column segment, the
        // segment's piece is folded into the totals after it.
        constexpr int kSegChunks = PASS / CH;
        // Chunk k of the diagonal block holds the columns base + k CH ... + CH - 1, among them
        // this wave's rows m in [k RPC, (k + 1) RPC), at the chunk's columns w + kWaves r,
        // r = m - k RPC: they are read from it before its columns are used.  A column j pairs
        // only with rows i < j, so that every row a column of chunk k pairs with has been read
        // by then (and the masked groups of GRP rows stay inside the rows read, RPC being a
        // multiple of GRP).  k is wave-uniform; a row takes the value read for it by a select on
        // k, so that every register index stays static.
        constexpr int RPC = CH / kWaves;
        static_assert(CH % kWaves == 0 && PASS % CH == 0, "chunks tile the diagonal block");
        static_assert(RPC % GRP == 0, "masked groups stay inside the rows read");
        auto rows_from_chunk = [&](int k, int buf) {
            V u[RPC];
#pragma unroll
            for (int r = 0; r < RPC; ++r) u[r] = ph[buf][w + kWaves * r][lane];
#pragma unroll
            for (int m = 0; m < ROWS; ++m) {
                const bool mine = (m / RPC == k);
                ci[m] = mine ? u[m % RPC].x : ci[m];
                si[m] = mine ? u[m % RPC].y : si[m];
            }
        };
        constexpr int kRowFold = 64;  // columns per FP32 run of the row sums
        for (int k = 0; k < nch;) {
          const int kend = min(nch, (k / kSegChunks + 1) * kSegChunks);
          for (; k < kend; ++k) {
            const int j0 = cbeg + k * CH;
            if (k + 1 < nch) stage(j0 + CH, (k + 1) & 1);
            const int buf = k & 1;
            if (rows_staged && k < kSegChunks) rows_from_chunk(k, buf);
            const int jend = min(CH, n - j0);
            // Columns of this chunk.  Past the diagonal block of the pass every row of a full wave
            // pairs with every column (straight-line body); in the diagonal block, or for a wave
            // with fewer than ROWS rows, rows with i >= j are masked.
            const bool straight = (nrows == ROWS) && (j0 >= base + PASS);
            if (straight) {
                for (int q = 0; q < jend; ++q) {
                    const int j = j0 + q;
                    const V u = ph[buf][q][lane];
                    const R* kr = Kbase + (int64_t)j * P.npad;
                    R kk[ROWS];
#pragma unroll
                    for (int m = 0; m < ROWS; ++m) kk[m] = kr[m];
                    const R ksj = ksb[j];
                    const double rj = rr[j];
                    R Tp[kPartials], Jp[kPartials];
#pragma unroll
                    for (int m = 0; m < kPartials; ++m)
                        pair_term<R, true>(ci[m], si[m], u.x, u.y, zero, kk[m], Tp[m], G[m],
                                           Jp[m]);
#pragma unroll
                    for (int m = kPartials; m < ROWS; ++m)
                        pair_term<R>(ci[m], si[m], u.x, u.y, zero, kk[m], Tp[m % kPartials], G[m],
                                     Jp[m % kPartials]);
                    interleave_exps<R, ROWS>();
                    const R Tq = combine_partials(Tp);
                    const R Jq = combine_partials(Jp);
                    const double Td = (double)Tq;
                    ladd(aST, Td);
                    ladd(aSJ, (double)(Jq - ksj));
                    ladd(aSC, Td * rj);
                }
            } else if (nrows == ROWS && j0 >= base + PASS / 2) {
                // The upper half of the diagonal block: every column pairs with all of the
                // wave's rows below base + PASS / 2 (the first half, a straight-line body) and
                // with the first cnt - ROWS / 2 of the others (masked in groups as below).  The
                // same terms in the same order as the general masked loop, so the same bits.
                constexpr int HALF = ROWS / 2;
                for (int q = 0; q < jend; ++q) {
                    const int j = j0 + q;
                    const int cnt = uniform(min(ROWS, (j - base - w + kWaves - 1) / kWaves));
                    const V u = ph[buf][q][lane];
                    const R* kr = Kbase + (int64_t)j * P.npad;
                    R kk[ROWS];
#pragma unroll
                    for (int m = 0; m < ROWS; ++m) kk[m] = kr[m];
#pragma unroll
                    for (int m = 0; m < ROWS; ++m) asm volatile("" : "+s"(kk[m]));
                    R Tp[kPartials], Jp[kPartials];
#pragma unroll
                    for (int m = 0; m < kPartials; ++m)
                        pair_term<R, true>(ci[m], si[m], u.x, u.y, zero, kk[m], Tp[m], G[m],
                                           Jp[m]);
#pragma unroll
                    for (int m = kPartials; m < HALF; ++m)
                        pair_term<R>(ci[m], si[m], u.x, u.y, zero, kk[m], Tp[m % kPartials],
                                     G[m], Jp[m % kPartials]);
                    interleave_exps<R, HALF>();
#pragma unroll
                    for (int g0 = HALF; g0 < ROWS; g0 += GRP) {
                        if (g0 < cnt) {
#pragma unroll
                            for (int m = g0; m < g0 + GRP; ++m)
                                pair_term<R>(ci[m], si[m], u.x, u.y, mask_offset<R>(m >= cnt),
                                             kk[m], Tp[m % kPartials], G[m], Jp[m % kPartials]);
                        }
                    }
                    const R Tq = combine_partials(Tp);
                    const R Jq = combine_partials(Jp);
                    const double Td = (double)Tq;
                    ladd(aST, Td);
                    ladd(aSJ, (double)(Jq - ksb[j]));
                    ladd(aSC, Td * rr[j]);
                }
            } else {
                for (int q = 0; q < jend; ++q) {
                    const int j = j0 + q;
                    int cnt = (j - base - w + kWaves - 1) / kWaves;
                    cnt = uniform(cnt < 0 ? 0 : (cnt > nrows ? nrows : cnt));
                    if (cnt == 0) continue;
                    const V u = ph[buf][q][lane];
                    const R* kr = Kbase + (int64_t)j * P.npad;
                    R kk[ROWS];
#pragma unroll
                    for (int m = 0; m < ROWS; ++m) kk[m] = kr[m];
                    // The column's kernel values are loaded together here, before the groups'
                    // branches, so that the column waits once for its scalar loads rather than
                    // once in each group that needs more of them.
#pragma unroll
                    for (int m = 0; m < ROWS; ++m) asm volatile("" : "+s"(kk[m]));
                    R Tp[kPartials], Jp[kPartials];
                    // Masked rows get an exponent offset of +inf (g = 0, adding exactly nothing);
                    // groups of GRP rows that are entirely masked are skipped.  cnt and the
                    // branches are wave-uniform.  The first kPartials rows start the partials (a
                    // skipped group's partials start at zero; cnt > 0, so the first group runs).
                    static_assert(kPartials % GRP == 0 || kPartials < GRP, "group layout");
#pragma unroll
                    for (int g0 = 0; g0 < ROWS; g0 += GRP) {
                        if (g0 < cnt) {
#pragma unroll
                            for (int m = g0; m < g0 + GRP; ++m) {
                                const R off = mask_offset<R>(m >= cnt);
                                if (m < kPartials)
                                    pair_term<R, true>(ci[m], si[m], u.x, u.y, off, kk[m], Tp[m],
                                                       G[m], Jp[m]);
                                else
                                    pair_term<R>(ci[m], si[m], u.x, u.y, off, kk[m],
                                                 Tp[m % kPartials], G[m], Jp[m % kPartials]);
                            }
                        } else if (g0 < kPartials) {
#pragma unroll
                            for (int m = g0; m < g0 + GRP && m < kPartials; ++m) {
                                Tp[m] = zero;
                                Jp[m] = zero;
                            }
                        }
                    }
                    const R Tq = combine_partials(Tp);
                    const R Jq = combine_partials(Jp);
                    const double Td = (double)Tq;
                    ladd(aST, Td);
                    ladd(aSJ, (double)(Jq - ksb[j]));
                    ladd(aSC, Td * rr[j]);
                }
            }
            // Row sums of the last kRowFold columns (or of the segment's or pass's last,
            // shorter run), weighted by the FP64 row sums r_i.  The fold points do not depend on
            // CH, so that the variants' results are the same bits.
            static_assert(kRowFold % CH == 0, "chunks tile the row-sum runs");
            if ((k + 1) % (kRowFold / CH) == 0 || k + 1 == kend) {
                double rk[ROWS];
#pragma unroll
                for (int m = 0; m < ROWS; ++m) rk[m] = rpb[m];
                double sca = 0.0;
#pragma unroll
                for (int m = 0; m < ROWS; ++m) {
                    sca = fma((double)G[m], rk[m], sca);
                    G[m] = R(0);
                }
                ladd(aSC, sca);
            }
            __syncthreads();
          }
          // The segment's piece is complete: its sums, the waves' sums in wave order, are added
          // to the totals (wave x owns total x), and the waves start the next piece from zero.
          if (w < 3) {
              const int lf = fresh_lane();
              double sp = 0.0;
              for (int v = 0; v < kWaves; ++v) sp += acc[w][v][lf];
              tot[w][lf] += sp;
          }
          __syncthreads();
          *aSJ = 0.0;
          *aST = 0.0;
          *aSC = 0.0;
        }
    }

    if (w != 0 || !active) return;
    // The lane and slot are formed again here so that they need not stay in registers across
    // the loops.
    const int ln = fresh_lane();
    const int slot_e = tile * kLanes + ln;
    if (SPLIT) {
        double* pp = out.part + (((int64_t)P.pqoff + piece) * fp.count + slot_e) * 3;
        pp[0] = tot[0][ln];
        pp[1] = tot[1][ln];
        pp[2] = tot[2][ln];
        return;
    }
    pair_scores(P, tot[0][ln], tot[1][ln], tot[2][ln], (int64_t)c * fp.count + slot_e, out);
}

// Totals and scores of the launches that ran one piece per workgroup: one thread per (curve,
// slot) adds the pieces' sums in piece order, as the workgroups of the other launches do.
constexpr int kEpiBlock = 256;

__global__ void __launch_bounds__(kEpiBlock)
pair_epilogue_kernel(const CurveParams* __restrict__ cp, const int32_t* __restrict__ order,
                     FreqPlan fp, int n_work, int pass, PairOut out) {
    const int64_t idx = (int64_t)blockIdx.x * kEpiBlock + threadIdx.x;
    const int64_t rank = idx / fp.count;
    if (rank >= n_work) return;
    const int slot = (int)(idx - rank * fp.count);
    if (fp.tile_cap > 0 && slot >= fp.tile_cap * kLanes) return;  // another launch's slots
    const int c = order[rank];
    const CurveParams P = cp[c];
    bool active;
    (void)slot_freq(fp, c, slot, active);
    if (!active) return;
    const int64_t obase = (int64_t)c * fp.count + slot;
    if (P.status != 0) {
        out.score[obase] = NAN;
        if (out.score2) out.score2[obase] = NAN;
        if (out.ips) {
            out.ips[obase * 3 + 0] = NAN;
            out.ips[obase * 3 + 1] = NAN;
            out.ips[obase * 3 + 2] = NAN;
        }
        return;
    }
    const int nb = (P.n + pass - 1) / pass;
    const int pieces = nb * (nb + 1) / 2;
    double SJ = 0.0, ST = 0.0, SC = 0.0;
    for (int q = 0; q < pieces; ++q) {
        const double* pp = out.part + (((int64_t)P.pqoff + q) * fp.count + slot) * 3;
        SJ += pp[0];
        ST += pp[1];
        SC += pp[2];
    }
    pair_scores(P, SJ, ST, SC, obase, out);
}

// The last, nearly empty tile of per-curve frequency lists (the bands method's 3 x 150 trials
// leave 2 slots in a curve's eighth tile of 64): in pairs_kernel its 2 active lanes would cost a
// whole tile.  Here a workgroup takes the curve's last kRemSlots slots with lanes = (slot,
// row): lane l holds slot slot0 + l / 32 and row base + w + kWaves (l mod 32) of each pass, the
// interleaved rows of pairs_kernel, and every lane walks the pass's columns j >= base through LDS.
// Per pair (i, j), i < j: g_ij from the same warp vectors and exp as pairs_kernel; the lane adds g
// (its row's part of S_T and, times the FP64 r_i, of S_C), r_j g (the column part of S_C) and
// K(i, j) (g - 1) (S_J, exactly zero where g = 1), in FP32 runs of 64 columns folded into FP64.  The 32 row lanes of a slot and the waves are then added in a fixed order.  FP32 path only
// (the FP64 and FP32-fold instances keep the plain tiles).
__global__ void __launch_bounds__(kThreads, 2)
pairs_rows_kernel(const CurveParams* __restrict__ cp, const int32_t* __restrict__ order,
                  FreqPlan fp, int slot0, const double* __restrict__ t_all,
                  const float* __restrict__ K_all, const double* __restrict__ rd_all, int n_work,
                  PairOut out) {
    using W = Warp<float, false>;
    using V = W::V;
    constexpr int ROWS = rows_per_wave<float>();
    constexpr int PASS = kWaves * ROWS;
    constexpr int CH = kChunk;
    constexpr int kFold = 64;  // columns per FP32 run
    static_assert(ROWS * kRemSlots == kLanes, "one row per lane and slot");
    __shared__ V ph[CH][kLanes];
    __shared__ double fq[kLanes];
    __shared__ double red[3][kWaves][kRemSlots];

    const int lane = threadIdx.x & 63;
    const int w = uniform((int)(threadIdx.x >> 6));
    const int rank = (int)blockIdx.x;
    if (rank >= n_work) return;
    const int c = order[rank];
    const CurveParams P = cp[c];
    const int half = lane / ROWS, r = lane % ROWS;
    bool active;
    const double f = slot_freq(fp, c, slot0 + half, active);
    const int64_t obase = (int64_t)c * fp.count + slot0 + half;
    if (P.status != 0) {
        if (active && w == 0 && r == 0) {
            out.score[obase] = NAN;
            if (out.score2) out.score2[obase] = NAN;
            if (out.ips) {
                out.ips[obase * 3 + 0] = NAN;
                out.ips[obase * 3 + 1] = NAN;
                out.ips[obase * 3 + 2] = NAN;
            }
        }
        return;
    }
    const int n = P.n;
    const double* t = t_all + P.off;
    const double* rr = rd_all + P.off;
    const double scale = uniform(sqrt(sqrt(2.0 * kLog2e) / P.sigma_t));
    if (w == 0) fq[lane] = f;
    __syncthreads();

    double SJ = 0.0, ST = 0.0, SC = 0.0;
    for (int base = 0; base < n; base += PASS) {
        const int i = base + w + kWaves * r;  // this lane's row
        const bool has_row = i < n;
        const V ui = has_row ? W::at(fq[lane], t[i], scale) : V{0.f, 0.f};
        const double ri = has_row ? rr[i] : 0.0;
        // K(i, j) for this lane's row: column j's run of the wave's rows, element r.
        const float* kc = K_all + P.koff + kperm(base + w) + r;
        float gs = 0.f, cs = 0.f, js = 0.f;
        int run = 0;
        for (int j0 = base; j0 < n; j0 += CH) {
            __syncthreads();  // the previous chunk's columns have been read
            for (int q = w; q < CH; q += kWaves) {
                const int j = j0 + q;
                const int ls = fresh_lane();
                ph[q][ls] = (j < n) ? W::at(fq[ls], t[j], scale) : V{0.f, 0.f};
            }
            __syncthreads();
            const int jend = min(CH, n - j0);
            for (int q = 0; q < jend; ++q) {
                const int j = j0 + q;
                const V u = ph[q][lane];
                const bool pair = has_row && i < j;
                const float k = pair ? kc[(int64_t)j * P.npad] : 0.f;
                const float rj = (float)rr[j];
                const float pr = ui.x * u.y;
                const float d = fmaf(ui.y, u.x, -pr);
                const float a = fmaf(d, d, pair ? 0.f : INFINITY);
                const float g = W::kexp(-a);
                gs += g;
                cs = fmaf(rj, g, cs);
                js = fmaf(k, g - 1.f, js);
                if (++run == kFold) {
                    ST += (double)gs;
                    SC = fma((double)gs, ri, SC + (double)cs);
                    SJ += (double)js;
                    gs = cs = js = 0.f;
                    run = 0;
                }
            }
        }
        ST += (double)gs;
        SC = fma((double)gs, ri, SC + (double)cs);
        SJ += (double)js;
    }
    // The 32 row lanes of each slot (butterfly within the half-wave), then the waves in order.
    for (int o = ROWS / 2; o > 0; o >>= 1) {
        SJ += __shfl_xor(SJ, o, 64);
        ST += __shfl_xor(ST, o, 64);
        SC += __shfl_xor(SC, o, 64);
    }
    if (r == 0) {
        red[0][w][half] = SJ;
        red[1][w][half] = ST;
        red[2][w][half] = SC;
    }
    __syncthreads();
    if (w != 0 || r != 0 || !active) return;
    double sj = 0.0, st = 0.0, sc = 0.0;
    for (int v = 0; v < kWaves; ++v) {
        sj += red[0][v][half];
        st += red[1][v][half];
        sc += red[2][v][half];
    }
    pair_scores(P, sj, st, sc, obase, out);
}

}  // namespace

// --------------------------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------------------------

hipError_t launch_prologue(hipStream_t st, CurveParams* cp, int n_curves, int max_n,
                           const double* t, const double* y, const double* e, double skew_lambda,
                           double skew_mu) {
    if (n_curves <= 0) return hipSuccess;
    int m = 1;
    while (m < max_n) m <<= 1;
    size_t shm = sizeof(double) * (size_t)m;
    prologue_kernel<<<n_curves, kPrologueBlock, shm, st>>>(cp, t, y, e, skew_lambda, skew_mu);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gram(hipStream_t st, CurveParams* cp, int n_curves, int64_t total_rows,
                       const int64_t* row_curve_start, const double* y, R* K, double* rp,
                       double* rd) {
    if (total_rows <= 0) return hipSuccess;
    gram_kernel<R><<<(unsigned)total_rows, kGramBlock, 0, st>>>(cp, row_curve_start, n_curves, y,
                                                                 K, rp, rd);
    return hipGetLastError();
}
template hipError_t launch_gram<float>(hipStream_t, CurveParams*, int, int64_t, const int64_t*,
                                       const double*, float*, double*, double*);
template hipError_t launch_gram<double>(hipStream_t, CurveParams*, int, int64_t, const int64_t*,
                                        const double*, double*, double*, double*);

template <typename R>
hipError_t launch_gram_finalize(hipStream_t st, CurveParams* cp, int n_curves, const double* rd,
                                double* rp) {
    if (n_curves <= 0) return hipSuccess;
    gram_finalize_kernel<R><<<n_curves, kFinBlock, 0, st>>>(cp, rd, rp);
    return hipGetLastError();
}
template hipError_t launch_gram_finalize<float>(hipStream_t, CurveParams*, int, const double*,
                                                double*);
template hipError_t launch_gram_finalize<double>(hipStream_t, CurveParams*, int, const double*,
                                                 double*);

template <typename R>
hipError_t launch_ksum(hipStream_t st, const CurveParams* cp, int n_curves, int max_n, const R* K,
                       R* ks) {
    if (n_curves <= 0) return hipSuccess;
    // Enough blocks per curve for its longest member's entries to take a few steps per thread,
    // and no more than the chip needs when there are many curves.
    constexpr int PASS = kWaves * rows_per_wave<R>();
    const int64_t entries = (int64_t)((max_n + PASS - 1) / PASS) * kWaves * max_n;
    int per_curve = (int)std::min<int64_t>(64, (entries + 4 * kKsBlock - 1) / (4 * kKsBlock));
    per_curve = std::max(1, std::min(per_curve, (2048 + n_curves - 1) / n_curves));
    ksum_kernel<R><<<dim3(n_curves, per_curve), kKsBlock, 0, st>>>(cp, K, ks);
    return hipGetLastError();
}
template hipError_t launch_ksum<float>(hipStream_t, const CurveParams*, int, int, const float*,
                                       float*);
template hipError_t launch_ksum<double>(hipStream_t, const CurveParams*, int, int, const double*,
                                        double*);

template <typename R>
int pair_variants() {
    return sizeof(R) == 4 ? 4 : 1;
}
template int pair_variants<float>();
template int pair_variants<double>();

struct PairGrid {
    unsigned blocks;
    int n_work;
    int xcd_grouped;
    int split_pmax;
};

template <typename R, int WPE, int CH, bool FOLD32 = false, bool PULLK = false>
static hipError_t launch_pairs_v(hipStream_t st, const CurveParams* cp, const int32_t* order,
                                 const PairGrid& g, const FreqPlan& fp, const double* t,
                                 const R* K, const double* r, const double* rp, const R* ks,
                                 const PairOut& out) {
    if (g.split_pmax > 0)
        pairs_kernel<R, WPE, CH, FOLD32, PULLK, true><<<g.blocks, kThreads, 0, st>>>(
            cp, order, fp, t, K, r, rp, ks, g.n_work, g.xcd_grouped, g.split_pmax, out);
    else
        pairs_kernel<R, WPE, CH, FOLD32, PULLK, false><<<g.blocks, kThreads, 0, st>>>(
            cp, order, fp, t, K, r, rp, ks, g.n_work, g.xcd_grouped, g.split_pmax, out);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_pairs_grid(hipStream_t st, const CurveParams* cp, const int32_t* order,
                                    const PairGrid& g, const FreqPlan& fp, const double* t,
                                    const R* K, const double* r, const double* rp, const R* ks,
                                    const PairOut& out, int variant) {
    if constexpr (sizeof(R) == 4) {
        // Per-curve lists have few tiles per curve: their launches use the K-pulling instances.
        if (fp.kind == 3 && variant != kVariantFold32) {
            switch (variant) {
                case 1:
                    return launch_pairs_v<R, 4, 64, false, true>(st, cp, order, g, fp, t, K, r,
                                                                 rp, ks, out);
                case 2:
                    return launch_pairs_v<R, 2, 32, false, true>(st, cp, order, g, fp, t, K, r,
                                                                 rp, ks, out);
                case 3:
                    return launch_pairs_v<R, 4, 32, false, true>(st, cp, order, g, fp, t, K, r,
                                                                 rp, ks, out);
                default:
                    return launch_pairs_v<R, 2, 64, false, true>(st, cp, order, g, fp, t, K, r,
                                                                 rp, ks, out);
            }
        }
        switch (variant) {
            case kVariantFold32:
                return launch_pairs_v<R, 2, 64, true>(st, cp, order, g, fp, t, K, r, rp, ks, out);
            case 1: return launch_pairs_v<R, 4, 64>(st, cp, order, g, fp, t, K, r, rp, ks, out);
            case 2: return launch_pairs_v<R, 2, 32>(st, cp, order, g, fp, t, K, r, rp, ks, out);
            case 3: return launch_pairs_v<R, 4, 32>(st, cp, order, g, fp, t, K, r, rp, ks, out);
            default: return launch_pairs_v<R, 2, 64>(st, cp, order, g, fp, t, K, r, rp, ks, out);
        }
    } else {
        (void)variant;
        return launch_pairs_v<R, 2, 32>(st, cp, order, g, fp, t, K, r, rp, ks, out);
    }
}

template <typename R>
hipError_t launch_pairs(hipStream_t st, const CurveParams* cp, const int32_t* order,
                        int n_work_curves, const FreqPlan& fp, const double* t, const R* K,
                        const double* r, const double* rp, const R* ks, const PairOut& out,
                        int variant, int split_pmax) {
    if (n_work_curves <= 0 || fp.count <= 0) return hipSuccess;
    const int64_t tiles = fp.tile_cap > 0 ? fp.tile_cap : (fp.count + kLanes - 1) / kLanes;
    PairGrid g;
    g.n_work = n_work_curves;
    if (split_pmax > 0 && out.part) {
        // One piece per workgroup, then the epilogue kernel.
        g.xcd_grouped = 0;
        g.split_pmax = split_pmax;
        g.blocks = (unsigned)((int64_t)n_work_curves * split_pmax * tiles);
        hipError_t e = launch_pairs_grid<R>(st, cp, order, g, fp, t, K, r, rp, ks, out, variant);
        if (e != hipSuccess) return e;
        const int64_t threads = (int64_t)n_work_curves * fp.count;
        pair_epilogue_kernel<<<(unsigned)((threads + kEpiBlock - 1) / kEpiBlock), kEpiBlock, 0,
                               st>>>(cp, order, fp, n_work_curves,
                                     kWaves * rows_per_wave<R>(), out);
        return hipGetLastError();
    }
    // Whole curves per XCD once every XCD gets at least 8 of them (enough to balance the XCDs'
    // loads in the work order); below that, a curve's tiles spread over the whole chip.
    g.split_pmax = 0;
    g.xcd_grouped = n_work_curves >= 8 * kXcds;
    const int64_t rows = g.xcd_grouped ? (int64_t)(n_work_curves + kXcds - 1) / kXcds * kXcds
                                       : (int64_t)n_work_curves;
    g.blocks = (unsigned)(rows * tiles);
    return launch_pairs_grid<R>(st, cp, order, g, fp, t, K, r, rp, ks, out, variant);
}
hipError_t launch_pairs_rows(hipStream_t st, const CurveParams* cp, const int32_t* order,
                             int n_work_curves, const FreqPlan& fp, int slot0, const double* t,
                             const float* K, const double* rd, const PairOut& out) {
    if (n_work_curves <= 0 || slot0 >= fp.count) return hipSuccess;
    pairs_rows_kernel<<<(unsigned)n_work_curves, kThreads, 0, st>>>(cp, order, fp, slot0, t, K,
                                                                     rd, n_work_curves, out);
    return hipGetLastError();
}

template hipError_t launch_pairs<float>(hipStream_t, const CurveParams*, const int32_t*, int,
                                        const FreqPlan&, const double*, const float*,
                                        const double*, const double*, const float*,
                                        const PairOut&, int, int);
template hipError_t launch_pairs<double>(hipStream_t, const CurveParams*, const int32_t*, int,
                                         const FreqPlan&, const double*, const double*,
                                         const double*, const double*, const double*,
                                         const PairOut&, int, int);

}  // namespace qmi
