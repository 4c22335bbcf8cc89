// HIP kernels for gfx950 (MI355X): the search around the pair sums of Protopapas et al.,
// arXiv:1412.1840 - the top local maxima of the coarse periodogram and their refinement windows
// (the trial periods are kept at the highest maxima of a spectrum, Sec. 3.1), and the best
// frequency of a curve (the score is maximised over trial frequencies, Sec. 3).
#include <math.h>

#include "qmi_internal.h"

namespace qmi {

namespace {

// --------------------------------------------------------------------------------------------
// Peaks: local maxima of the coarse scores, best top_k by (score desc, k asc), and their
// refinement windows.  Candidates inside a spurious-period mask (Sec. 6.1) are left out of the
// argmax and of the maxima kept.  One block per curve.
// --------------------------------------------------------------------------------------------

constexpr int kPeakBlock = 256;
constexpr int kPeakBlockWide = 512;

__device__ __forceinline__ bool better(double qa, int ka, double qb, int kb) {
    // a ranks before b: higher score, ties to lower index.  NaN never ranks.
    if (!(qa == qa)) return false;
    if (!(qb == qb)) return true;
    return qa > qb || (qa == qb && ka < kb);
}

__device__ __forceinline__ double grid_f(double f0, double df, int k) {
    return __dadd_rn(f0, __dmul_rn((double)k, df));
}

// The wave's best (score, index) by the rank order of better(), in every lane (butterfly).
__device__ __forceinline__ void wave_best(double& q, int& k) {
    for (int o = 32; o > 0; o >>= 1) {
        const double q2 = __shfl_xor(q, o, 64);
        const int k2 = __shfl_xor(k, o, 64);
        if (better(q2, k2, q, k)) {
            q = q2;
            k = k2;
        }
    }
}

// The block's best of the waves' bests, in every thread; slot (0 or 1) alternates between
// consecutive calls so that one barrier per call suffices.
template <int NW>
__device__ __forceinline__ int block_best(double q, int k, double (*wq)[NW], int (*wk)[NW],
                                          int slot) {
    wave_best(q, k);
    if ((threadIdx.x & 63) == 0) {
        wq[slot][threadIdx.x >> 6] = q;
        wk[slot][threadIdx.x >> 6] = k;
    }
    __syncthreads();
    double bq = wq[slot][0];
    int bk = wk[slot][0];
    for (int v = 1; v < NW; ++v)
        if (better(wq[slot][v], wk[slot][v], bq, bk)) {
            bq = wq[slot][v];
            bk = wk[slot][v];
        }
    return bk;
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK)
peaks_kernel(const CurveParams* __restrict__ cp, const double* __restrict__ coarse, int F,
             double f0, double df, int top_k, int n_fine, MaskDev md, PeakOut po) {
    constexpr int NW = BLOCK / 64;
    __shared__ double wq[2][NW];
    __shared__ int wk[2][NW];
    __shared__ int chosen[64];
    extern __shared__ double peak_dyn[];  // [max(top_k, 1)][BLOCK] scores, then indices
    const int c = blockIdx.x;
    const double* q = coarse + (int64_t)c * F;
    const bool ok = cp[c].status == 0;
    // One scan of the coarse scores gives both this thread's candidate for the coarse argmax (ties
    // to lower k, candidates outside every mask) and its best top_k local maxima, kept sorted in
    // rank order (score descending, ties to the lower k) in its own LDS slots.  The scan takes
    // kUnroll grid points per step with their loads issued together.
    constexpr int kUnroll = 4;
    const int TK = top_k > 0 ? top_k : 1;
    // Entry i of a thread's list sits at i * BLOCK + thread (consecutive threads in
    // consecutive slots, so that the list operations of a wave do not conflict on LDS banks).
    double* mv0 = reinterpret_cast<double*>(peak_dyn) + threadIdx.x;
    int* mk0 = reinterpret_cast<int*>(reinterpret_cast<double*>(peak_dyn) + BLOCK * TK) +
               threadIdx.x;
    auto mv = [&](int i) -> double& { return mv0[i * BLOCK]; };
    auto mk = [&](int i) -> int& { return mk0[i * BLOCK]; };
    int n_loc = 0;
    double bq = NAN;
    int bk = 0x7fffffff;
    if (ok) {
        for (int k0 = threadIdx.x; k0 < F; k0 += kUnroll * BLOCK) {
            double v[kUnroll], lft[kUnroll], rgt[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int k = k0 + u * BLOCK;
                v[u] = k < F ? q[k] : NAN;
                lft[u] = (k < F && k > 0) ? q[k - 1] : NAN;
                rgt[u] = (k + 1 < F) ? q[k + 1] : NAN;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int k = k0 + u * BLOCK;
                if (k >= F) break;
                if (better(v[u], k, bq, bk) && !in_mask(md, grid_f(f0, df, k), v[u])) {
                    bq = v[u];
                    bk = k;
                }
                if (top_k <= 0) continue;
                bool peak;
                if (F == 1) peak = (v[u] == v[u]);
                else if (k == 0) peak = v[u] >= rgt[u];
                else if (k == F - 1) peak = v[u] > lft[u];
                else peak = v[u] > lft[u] && v[u] >= rgt[u];
                if (!peak) continue;
                if (n_loc == TK && !better(v[u], k, mv(TK - 1), mk(TK - 1))) continue;
                if (in_mask(md, grid_f(f0, df, k), v[u])) continue;
                int p = n_loc < TK ? n_loc++ : TK - 1;
                while (p > 0 && better(v[u], k, mv(p - 1), mk(p - 1))) {
                    mv(p) = mv(p - 1);
                    mk(p) = mk(p - 1);
                    --p;
                }
                mv(p) = v[u];
                mk(p) = k;
            }
        }
    }
    int slot = 0;
    const int am = block_best<NW>(bq, bk, wq, wk, slot);
    slot ^= 1;
    if (threadIdx.x == 0) po.argmax[c] = (am == 0x7fffffff) ? -1 : am;
    // top_k rounds take the best head among the threads' lists: the top_k of all maxima in rank
    // order.
    int count = 0, head = 0;
    for (int p = 0; p < top_k && ok; ++p) {
        const int kk = block_best<NW>(head < n_loc ? mv(head) : NAN,
                                      head < n_loc ? mk(head) : 0x7fffffff, wq, wk, slot);
        slot ^= 1;
        if (kk == 0x7fffffff) break;
        if (head < n_loc && mk(head) == kk) ++head;  // grid indices belong to one thread each
        if (threadIdx.x == 0) chosen[count] = kk;
        ++count;
    }
    if (threadIdx.x == 0) {
        po.npk[c] = count;
        for (int p = 0; p < count; ++p) {
            const int k = chosen[p];
            int a = k - 1, b = k + 1;
            if (F == 1) { a = 0; b = 0; }
            else if (k == 0) { a = 0; b = 1; }
            else if (k == F - 1) { a = F - 2; b = F - 1; }
            const double lo = grid_f(f0, df, a), hi = grid_f(f0, df, b);
            po.peak_k[(int64_t)c * top_k + p] = k;
            po.win[((int64_t)c * top_k + p) * 2 + 0] = lo;
            po.win[((int64_t)c * top_k + p) * 2 + 1] = (hi - lo) / (double)(n_fine - 1);
        }
    }
}

// --------------------------------------------------------------------------------------------
// Best-of: highest refined score outside every mask, ties to the lower frequency then the lower
// peak rank; without a refined candidate, the coarse argmax; without that, an empty result.
// --------------------------------------------------------------------------------------------

constexpr int kBestBlock = 256;

__global__ void __launch_bounds__(kBestBlock)
best_kernel(const CurveParams* __restrict__ cp, const double* __restrict__ coarse,
            const double* __restrict__ coarse2, int F,
            const double* __restrict__ fine, const double* __restrict__ fine2, int top_k,
            int n_fine, int score_kind, double f0, double df, MaskDev md, PeakOut po,
            DevResult* __restrict__ res) {
    __shared__ double sq[kBestBlock], sf[kBestBlock];
    __shared__ int ss[kBestBlock];
    const int c = blockIdx.x;
    const CurveParams P = cp[c];
    const int npk = (top_k > 0 && n_fine > 0 && P.status == 0) ? po.npk[c] : 0;
    const int64_t S = (int64_t)top_k * n_fine;
    double bq = NAN, bf = INFINITY;
    int bs = 0x7fffffff;
    for (int s = threadIdx.x; s < npk * n_fine; s += kBestBlock) {
        const double v = fine[(int64_t)c * S + s];
        if (!(v == v)) continue;
        const int p = s / n_fine, m = s - p * n_fine;
        const double* w = po.win + ((int64_t)c * top_k + p) * 2;
        const double fr = __dadd_rn(w[0], __dmul_rn((double)m, w[1]));
        bool b = !(bq == bq) || v > bq || (v == bq && (fr < bf || (fr == bf && s < bs)));
        if (b && !in_mask(md, fr, v)) { bq = v; bf = fr; bs = s; }
    }
    sq[threadIdx.x] = bq;
    sf[threadIdx.x] = bf;
    ss[threadIdx.x] = bs;
    __syncthreads();
    for (int h = kBestBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double v = sq[threadIdx.x + h], fr = sf[threadIdx.x + h];
            const int s = ss[threadIdx.x + h];
            const double cq = sq[threadIdx.x], cf = sf[threadIdx.x];
            const int cs = ss[threadIdx.x];
            bool b = (v == v) &&
                     (!(cq == cq) || v > cq || (v == cq && (fr < cf || (fr == cf && s < cs))));
            if (b) { sq[threadIdx.x] = v; sf[threadIdx.x] = fr; ss[threadIdx.x] = s; }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    DevResult r;
    r.sigma_y = P.sigma_y;
    r.sigma_t = P.sigma_t > 0.0 ? P.sigma_t : NAN;  // the rule flag until the prologue ran
    r.psnr = P.psnr;
    r.n = P.n;
    r.status = P.status;
    r.reserved = 0;
    r.n_peaks = npk;
    const int am = (P.status == 0) ? po.argmax[c] : -1;
    r.coarse_argmax = am;
    r.coarse_best = (am >= 0) ? coarse[(int64_t)c * F + am] : NAN;
    if (P.status != 0 || ((npk == 0 || ss[0] == 0x7fffffff) && am < 0)) {
        r.f_best = r.period = r.score = r.score_qmi = r.score_nckp = NAN;
        r.coarse_index = r.peak_rank = r.fine_index = -1;
    } else if (npk == 0 || ss[0] == 0x7fffffff) {
        r.f_best = grid_f(f0, df, am);
        r.period = 1.0 / r.f_best;
        r.score = r.coarse_best;
        r.coarse_index = am;
        r.peak_rank = -1;
        r.fine_index = -1;
        const double other = coarse2 ? coarse2[(int64_t)c * F + am] : NAN;
        r.score_qmi = score_kind == 0 ? r.coarse_best : other;
        r.score_nckp = score_kind == 0 ? other : r.coarse_best;
    } else {
        const int s = ss[0];
        const int p = s / n_fine, m = s - p * n_fine;
        r.f_best = sf[0];
        r.period = 1.0 / r.f_best;
        r.score = sq[0];
        const double other = fine2 ? fine2[(int64_t)c * S + s] : NAN;
        r.score_qmi = score_kind == 0 ? sq[0] : other;
        r.score_nckp = score_kind == 0 ? other : sq[0];
        r.coarse_index = po.peak_k[(int64_t)c * top_k + p];
        r.peak_rank = p;
        r.fine_index = m;
    }
    res[c] = r;
}

}  // namespace

hipError_t launch_peaks(hipStream_t st, const CurveParams* cp, int n_curves, const double* coarse,
                        int n_coarse, double f0, double df, int top_k, int n_fine,
                        const MaskDev& md, const PeakOut& po) {
    if (n_curves <= 0) return hipSuccess;
    // A launch of few curves (single-curve calls, serving batches) is one block per curve on a
    // mostly idle chip: wider blocks there scan the grid in fewer steps, while their per-thread
    // peak lists still fit the default 64 KiB of dynamic LDS.
    const int tk = top_k > 0 ? top_k : 1;
    const size_t per_thread = (size_t)tk * (sizeof(double) + sizeof(int));
    if (n_curves < 128 && (size_t)kPeakBlockWide * per_thread <= 64 * 1024) {
        peaks_kernel<kPeakBlockWide><<<n_curves, kPeakBlockWide, kPeakBlockWide * per_thread,
                                       st>>>(cp, coarse, n_coarse, f0, df, top_k, n_fine, md, po);
    } else {
        peaks_kernel<kPeakBlock><<<n_curves, kPeakBlock, kPeakBlock * per_thread, st>>>(
            cp, coarse, n_coarse, f0, df, top_k, n_fine, md, po);
    }
    return hipGetLastError();
}

hipError_t launch_best(hipStream_t st, const CurveParams* cp, int n_curves, const double* coarse,
                       const double* coarse2, int n_coarse, const double* fine,
                       const double* fine2, int top_k, int n_fine, int score_kind, double f0,
                       double df, const MaskDev& md, const PeakOut& po, DevResult* res) {
    if (n_curves <= 0) return hipSuccess;
    best_kernel<<<n_curves, kBestBlock, 0, st>>>(cp, coarse, coarse2, n_coarse, fine, fine2, top_k,
                                                  n_fine, score_kind, f0, df, md, po, res);
    return hipGetLastError();
}

}  // namespace qmi
