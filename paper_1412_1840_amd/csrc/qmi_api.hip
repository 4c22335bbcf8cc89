// Host runtime and C ABI of libqmi (declared in include/qmi.h): context, validation, batch
// planning under the HBM budget, kernel launches, optional hipGraph replay, the discriminator
// and the continuous-batching serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qmi.h"
#include "qmi_internal.h"

using namespace qmi;

namespace {

thread_local std::string g_create_error;

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Status {
    int code = QMI_OK;
    std::string msg;
};

}  // namespace

struct qmi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    size_t allocated = 0;
    std::string err;
    bool use_graph = true;
    int64_t tile = 0;
    int64_t serve_batch_items = 0;  // QMI_OPT_SERVE_BATCH_ITEMS
    qmi_stats stats{};
    std::vector<hipEvent_t> ev;  // timing events (pairs: before/after each pair launch)
    int ev_used = 0;
    // Device buffers, grown on demand.
    enum {
        kT, kY, kE, kCP, kOrder, kRowStart, kK, kR, kRP, kRD, kKS, kCoarse, kCoarse2, kFine, kFine2,
        kIps, kPeakK, kNpk, kWin, kArgmax, kRes, kFreqs, kProbe, kTS, kYS, kBandT, kBandCnt,
        kBandId, kS, kTrials, kTrialK, kPOff, kPStIn, kPCnt, kPSt, kPDet, kPTo, kPYo, kPEo,
        kPPer, kPart, kNumBufs
    };
    Buf bufs[kNumBufs];
    static_assert(kNumBufs <= 64, "one bit per buffer in in_use");
    uint64_t in_use = 0;  // bit per buffer ensured by the current operation
    // Scratch mode (qmi_periodogram_noalloc): the current call takes its buffers from the
    // device's static scratch array by bump allocation instead of from bufs.
    char* ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;
    void* ws_ptr[kNumBufs] = {};
    // Graph cache (device section of one planned group).
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint64_t> graph_key;
    // Autotuner: pair-kernel variant per length bucket (-1: not tuned yet).
    int tuned[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    // Spurious-period masks applied by the selection kernels (qmi_set_masks).
    qmi::MaskDev masks{};
    // Serving.
    struct Serve;
    std::unique_ptr<Serve> serve;
    std::mutex call_mu;  // serialises device calls between the serving thread and the caller
};

// Scratch memory of qmi_periodogram_noalloc: one static array per device, resolved once per
// device (hipGetSymbolAddress, with that device current) when the first context on it is created.
// In host code the array's name is only a stand-in; its device address is g_scratch[device].
static __device__ __align__(256) unsigned char scratch[QMI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Resolves the device address of the scratch array on the current device (once per device).
hipError_t resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch[device] = p;
    return e;
}

void set_err(qmi_ctx* ctx, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_error = buf;
}

#define HIP_OK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            set_err(ctx, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,  \
                    __LINE__);                                                             \
            return (e_ == hipErrorOutOfMemory) ? QMI_ENOMEM : QMI_EDEVICE;                  \
        }                                                                                  \
    } while (0)

void drop_graph(qmi_ctx* ctx) {
    // Any captured graph refers to buffer addresses that are about to change.
    if (ctx->graph_exec) {
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
    }
    if (ctx->graph) {
        (void)hipGraphDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    ctx->graph_key.clear();
}

int free_buf(qmi_ctx* ctx, int id) {
    Buf& b = ctx->bufs[id];
    if (!b.p) return QMI_OK;
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    HIP_OK(ctx, hipFree(b.p));
    ctx->allocated -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
    drop_graph(ctx);
    return QMI_OK;
}

// Buffers ensured since the last begin_use() are in use by the current operation; the others
// hold stale contents of earlier operations and may be released to stay inside the budget.
void begin_use(qmi_ctx* ctx) { ctx->in_use = 0; }

int ensure(qmi_ctx* ctx, int id, size_t bytes) {
    Buf& b = ctx->bufs[id];
    if (bytes == 0) bytes = 256;
    ctx->in_use |= 1ull << id;
    if (b.bytes >= bytes) return QMI_OK;
    // Some headroom for the next call, and at least twice the old size when a buffer grows, so
    // that a run of calls on curves of increasing length reallocates (and synchronises the
    // device in hipFree) only a logarithmic number of times.
    size_t want = std::max(bytes + bytes / 8, 2 * b.bytes);
    if (ctx->allocated - b.bytes + want > ctx->budget) {
        // Release buffers the current operation does not use before giving up.
        for (int k = 0; k < qmi_ctx::kNumBufs; ++k)
            if (!(ctx->in_use & (1ull << k))) {
                const int rc = free_buf(ctx, k);
                if (rc) return rc;
            }
    }
    if (ctx->allocated - b.bytes + want > ctx->budget) want = bytes;
    if (ctx->allocated - b.bytes + want > ctx->budget) {
        set_err(ctx, "HBM budget exceeded: need %zu more bytes (budget %zu)",
                want - b.bytes, ctx->budget);
        return QMI_ENOMEM;
    }
    if (b.p) {
        const int rc = free_buf(ctx, id);
        if (rc) return rc;
    }
    HIP_OK(ctx, hipMalloc(&b.p, want));
    b.bytes = want;
    ctx->allocated += want;
    return QMI_OK;
}

template <typename T>
T* dptr(qmi_ctx* ctx, int id) {
    return reinterpret_cast<T*>(ctx->ws_base ? ctx->ws_ptr[id] : ctx->bufs[id].p);
}

// A buffer of the current call: the context's own (grown on demand, see ensure), or in scratch
// mode the next 256-byte aligned piece of the scratch array.  Scratch mode never allocates.
int acquire(qmi_ctx* ctx, int id, size_t bytes) {
    if (!ctx->ws_base) return ensure(ctx, id, bytes);
    if (bytes == 0) bytes = 256;
    const size_t at = (ctx->ws_used + 255) / 256 * 256;
    if (at > ctx->ws_size || bytes > ctx->ws_size - at) {
        set_err(ctx, "the call needs more than the %zu bytes of scratch memory available to "
                "qmi_periodogram_noalloc", ctx->ws_size);
        return QMI_ENOMEM;
    }
    ctx->ws_ptr[id] = ctx->ws_base + at;
    ctx->ws_used = at + bytes;
    return QMI_OK;
}

int scratch_for_device(qmi_ctx* ctx, void** base) {
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) p = g_scratch[ctx->device];
    }
    if (!p) {
        set_err(ctx, "the scratch array of device %d was not resolved", ctx->device);
        return QMI_EDEVICE;
    }
    *base = p;
    return QMI_OK;
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int check_kernel_params(qmi_ctx* ctx, const qmi_kernel_params* kp) {
    if (!kp) { set_err(ctx, "kernel params is NULL"); return QMI_EINVAL; }
    if ((!(kp->sigma_t > 0.0) || !std::isfinite(kp->sigma_t)) &&
        kp->sigma_t != QMI_SIGMA_T_SKEWNESS) {
        set_err(ctx, "sigma_t must be finite and > 0 or QMI_SIGMA_T_SKEWNESS (got %g)",
                kp->sigma_t);
        return QMI_EINVAL;
    }
    if (kp->sigma_t == QMI_SIGMA_T_SKEWNESS && !(kp->skew_lambda == 0.0 && kp->skew_mu == 0.0) &&
        !(kp->skew_lambda > 0.0 && std::isfinite(kp->skew_lambda) && kp->skew_mu >= 0.0 &&
          std::isfinite(kp->skew_mu))) {
        set_err(ctx, "the sigma_t rule needs skew_lambda > 0 and skew_mu >= 0 (got %g, %g)",
                kp->skew_lambda, kp->skew_mu);
        return QMI_EINVAL;
    }
    if (!(kp->sigma_y > 0.0 && std::isfinite(kp->sigma_y)) && kp->sigma_y != QMI_SIGMA_SILVERMAN &&
        kp->sigma_y != QMI_SIGMA_MEDIAN_ERR) {
        set_err(ctx, "sigma_y must be > 0 or a QMI_SIGMA_* rule (got %g)", kp->sigma_y);
        return QMI_EINVAL;
    }
    if (kp->precision != QMI_PREC_MIXED && kp->precision != QMI_PREC_FP64 &&
        kp->precision != QMI_PREC_FOLD32) {
        set_err(ctx, "unknown precision %d", kp->precision);
        return QMI_EINVAL;
    }
    return QMI_OK;
}

int check_batch(qmi_ctx* ctx, const qmi_batch* b, bool need_e) {
    if (!b) { set_err(ctx, "batch is NULL"); return QMI_EINVAL; }
    if (b->n_curves < 0) { set_err(ctx, "n_curves < 0"); return QMI_EINVAL; }
    if (b->n_curves == 0) return QMI_OK;
    if (!b->offsets || !b->t || !b->y) {
        set_err(ctx, "batch offsets, t and y must not be NULL");
        return QMI_EINVAL;
    }
    if (b->offsets[0] != 0) { set_err(ctx, "offsets[0] must be 0"); return QMI_EINVAL; }
    for (int32_t k = 0; k < b->n_curves; ++k)
        if (b->offsets[k + 1] < b->offsets[k]) {
            set_err(ctx, "offsets must be non-decreasing (curve %d)", k);
            return QMI_EINVAL;
        }
    if (need_e && !b->e) {
        set_err(ctx, "this call needs error bars (batch e is NULL)");
        return QMI_EINVAL;
    }
    return QMI_OK;
}

// Host-side per-curve status from the lengths (and, for host arrays, the sample values).
int32_t host_curve_status(const qmi_batch* b, int32_t k, bool host_arrays) {
    const int64_t a = b->offsets[k], n = b->offsets[k + 1] - a;
    if (n < 2 || n > QMI_MAX_N) return QMI_EINVAL;
    if (host_arrays) {
        for (int64_t i = a; i < a + n; ++i) {
            if (!std::isfinite(b->t[i]) || !std::isfinite(b->y[i])) return QMI_EINVAL;
            if (b->e && !std::isfinite(b->e[i])) return QMI_EINVAL;
        }
    }
    return QMI_OK;
}

// A contiguous group of curves [c0, c1) processed by one device section.
struct Group {
    int32_t c0, c1;
    int64_t s0, s1;  // sample range
};

// Bytes of device memory one curve needs besides the fixed per-call buffers.
size_t curve_bytes(int64_t n, int64_t F1, int64_t F2, bool fp64, bool ips, bool two_scores) {
    const int64_t npad = round_up(std::max<int64_t>(n, 1), kPass);
    const size_t rs = fp64 ? 8 : 4;
    size_t b = 0;
    b += (size_t)n * 3 * 8;                      // t, y, e
    b += (size_t)n * (size_t)npad * rs;          // K
    b += (size_t)npad * 8;                       // rp (FP64)
    b += (size_t)n * 8;                          // rd
    b += (size_t)((n + 8 * (fp64 ? 16 : 32) - 1) / (8 * (fp64 ? 16 : 32))) * 8 * n * rs;  // ks
    b += sizeof(CurveParams) + 64;
    b += (size_t)F1 * 8 * (two_scores ? 2 : 1);  // coarse / periodogram scores
    b += (size_t)F2 * 8 * 2;                     // fine scores
    if (ips) b += (size_t)F1 * 24;
    b += (size_t)QMI_MAX_TOPK * 32 + sizeof(DevResult);
    return b;
}

struct CallSpec {
    bool noalloc;          // buffers from the device's scratch array (qmi_periodogram_noalloc)
    bool dev_inputs;       // batch arrays are device pointers
    bool dev_outputs;      // score/ips/coarse outputs are device pointers
    bool periodogram;      // caller list (true) or coarse-to-fine search (false)
    const qmi_kernel_params* kp;
    // periodogram
    const double* freqs;
    int32_t n_freq;
    int32_t score;
    double* score_out;
    double* ips_out;
    double* ip_y_out;
    int32_t* status_out;
    // search
    const qmi_search* search;
    qmi_result* out;
    double* coarse_out;
    // bands method (search == nullptr, periodogram == false)
    const qmi_bands* bands;
    double* trials_out;
    double* scores_out;
};

// Per-curve device bytes of the bands method's own buffers (time-ordered copies, band times,
// spectral windows, trial lists).
size_t bands_bytes(int64_t n, const qmi_bands& bp) {
    // Band rows are as long as the group's longest curve needs; count the longest possible.
    const int64_t stride = (QMI_MAX_N + bp.n_bands - 1) / bp.n_bands;
    size_t b = (size_t)n * 16;
    b += (size_t)bp.n_keep * (size_t)(stride * 8 + 8);
    b += (size_t)bp.n_keep * (size_t)bp.n_grid * 8;
    b += (size_t)bp.n_keep * (size_t)bp.n_trials * 12;
    return b;
}

int plan_groups(qmi_ctx* ctx, const qmi_batch* b, const CallSpec& cs, std::vector<Group>& groups) {
    const bool fp64 = cs.kp->precision == QMI_PREC_FP64;
    const qmi_bands* bp = cs.bands;
    const int64_t F1 = cs.periodogram ? cs.n_freq
                       : bp ? (int64_t)bp->n_keep * bp->n_trials : cs.search->n_coarse;
    const int64_t F2 = (cs.periodogram || bp) ? 0 : (int64_t)cs.search->top_k * cs.search->n_fine;
    const bool two = !cs.periodogram;
    const size_t fixed = 1 << 20;
    if (ctx->budget <= fixed) {
        set_err(ctx, "HBM budget too small");
        return QMI_ENOMEM;
    }
    // Buffers may carry 1/8 of growth headroom (see ensure), so a group is sized to fit even when
    // every buffer it uses has it.
    const size_t avail = (ctx->budget - fixed) / 9 * 8;
    Group g{0, 0, 0, 0};
    size_t used = 0;
    for (int32_t k = 0; k < b->n_curves; ++k) {
        const int64_t n = b->offsets[k + 1] - b->offsets[k];
        const int64_t nn = std::min<int64_t>(n, QMI_MAX_N);
        const size_t need = curve_bytes(nn, F1, F2, fp64, cs.ips_out != nullptr, two) +
                            (bp ? bands_bytes(nn, *bp) : 0);
        if (need > avail) {
            set_err(ctx, "curve %d (N=%lld) needs %zu bytes, more than the HBM budget %zu", k,
                    (long long)n, need, ctx->budget);
            return QMI_ENOMEM;
        }
        if (used + need > avail && g.c1 > g.c0) {
            groups.push_back(g);
            g = Group{k, k, b->offsets[k], b->offsets[k]};
            used = 0;
        }
        used += need;
        g.c1 = k + 1;
        g.s1 = b->offsets[k + 1];
    }
    if (g.c1 > g.c0) groups.push_back(g);
    return QMI_OK;
}

void record(qmi_ctx* ctx) {
    if (ctx->ev_used >= (int)ctx->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        ctx->ev.push_back(e);
    }
    (void)hipEventRecord(ctx->ev[ctx->ev_used++], ctx->stream);
}

template <typename R>
int run_group(qmi_ctx* ctx, const qmi_batch* b, const CallSpec& cs, const Group& g,
              std::vector<int32_t>& pair_event_idx) {
    begin_use(ctx);
    const int32_t nc = g.c1 - g.c0;
    const int64_t ns = g.s1 - g.s0;
    const bool fp64 = std::is_same<R, double>::value;
    const qmi_kernel_params* kp = cs.kp;

    // Per-curve parameters and layout.
    std::vector<CurveParams> cp(nc);
    std::vector<int32_t> order(nc);
    std::vector<int64_t> row_start(nc);
    int64_t koff = 0, poff = 0, ksoff = 0, rows = 0, pieces = 0;
    constexpr int kPassR = kWaves * rows_per_wave<R>();
    int max_n = 2, max_pieces = 0;
    for (int32_t i = 0; i < nc; ++i) {
        const int32_t k = g.c0 + i;
        const int64_t a = b->offsets[k], n = b->offsets[k + 1] - a;
        CurveParams& p = cp[i];
        std::memset(&p, 0, sizeof(p));
        p.status = host_curve_status(b, k, !cs.dev_inputs);
        p.off = a - g.s0;
        p.n = (int32_t)std::min<int64_t>(n, QMI_MAX_N);
        p.has_e = b->e != nullptr;
        p.sigma_t = kp->sigma_t;
        p.sigma_y_rule = kp->sigma_y;
        p.sigma_y = NAN;
        if (p.status == QMI_OK) {
            p.npad = (int32_t)round_up(p.n, kPass);
            p.koff = koff;
            p.poff = poff;
            p.ksoff = ksoff;
            koff += (int64_t)p.n * p.npad;
            poff += p.npad;
            ksoff += (int64_t)((p.n + kPassR - 1) / kPassR) * kWaves * p.n;
            const int nbp = (p.n + kPassR - 1) / kPassR;
            p.pqoff = pieces;
            pieces += (int64_t)nbp * (nbp + 1) / 2;
            max_pieces = std::max(max_pieces, nbp * (nbp + 1) / 2);
            row_start[i] = rows;
            rows += p.n;
            max_n = std::max(max_n, p.n);
        } else {
            row_start[i] = rows;
        }
        order[i] = i;
    }
    // Largest work first: the dispatcher hands out work items in order.
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        const int64_t na = cp[a].status ? 0 : cp[a].n, nb = cp[c].status ? 0 : cp[c].n;
        return na > nb;
    });

    const qmi_bands* bp = cs.bands;
    const bool search = !cs.periodogram && !bp;
    const int64_t F1 = cs.periodogram ? cs.n_freq
                       : bp ? (int64_t)bp->n_keep * bp->n_trials : cs.search->n_coarse;
    const int top_k = search ? cs.search->top_k : 0;
    const int n_fine = search ? cs.search->n_fine : 0;
    const bool refine = search && top_k > 0 && n_fine > 0;
    const int64_t F2 = refine ? (int64_t)top_k * n_fine : 0;
    const int score_kind = cs.periodogram ? cs.score : bp ? bp->score : cs.search->score;

    int rc;
#define ENSURE(id, bytes) \
    if ((rc = acquire(ctx, id, (bytes))) != QMI_OK) return rc
    if (!cs.dev_inputs) {
        ENSURE(qmi_ctx::kT, ns * 8);
        ENSURE(qmi_ctx::kY, ns * 8);
        if (b->e) ENSURE(qmi_ctx::kE, ns * 8);
    }
    ENSURE(qmi_ctx::kCP, nc * sizeof(CurveParams));
    ENSURE(qmi_ctx::kOrder, nc * sizeof(int32_t));
    ENSURE(qmi_ctx::kRowStart, nc * sizeof(int64_t));
    ENSURE(qmi_ctx::kK, std::max<int64_t>(koff, 1) * sizeof(R));
    ENSURE(qmi_ctx::kRP, std::max<int64_t>(poff, 1) * 8);
    ENSURE(qmi_ctx::kRD, std::max<int64_t>(ns, 1) * 8);
    ENSURE(qmi_ctx::kKS, std::max<int64_t>(ksoff, 1) * sizeof(R));
    if (!(cs.periodogram && cs.dev_outputs)) ENSURE(qmi_ctx::kCoarse, nc * F1 * 8);
    if (!cs.periodogram) ENSURE(qmi_ctx::kCoarse2, nc * F1 * 8);
    if (refine) {
        ENSURE(qmi_ctx::kFine, nc * F2 * 8);
        ENSURE(qmi_ctx::kFine2, nc * F2 * 8);
    }
    if (cs.ips_out && !cs.dev_outputs) ENSURE(qmi_ctx::kIps, nc * F1 * 24);
    if (bp) {
        const int64_t stride = (max_n + bp->n_bands - 1) / bp->n_bands;
        const int64_t nkt = (int64_t)nc * bp->n_keep;
        ENSURE(qmi_ctx::kTS, std::max<int64_t>(ns, 1) * 8);
        ENSURE(qmi_ctx::kYS, std::max<int64_t>(ns, 1) * 8);
        ENSURE(qmi_ctx::kBandT, nkt * stride * 8);
        ENSURE(qmi_ctx::kBandCnt, nkt * 4);
        ENSURE(qmi_ctx::kBandId, nkt * 4);
        ENSURE(qmi_ctx::kS, nkt * bp->n_grid * 8);
        ENSURE(qmi_ctx::kTrials, nc * F1 * 8);
        ENSURE(qmi_ctx::kTrialK, nc * F1 * 4);
    }
    if (!cs.periodogram) {
        ENSURE(qmi_ctx::kPeakK, nc * std::max(top_k, 1) * sizeof(int32_t));
        ENSURE(qmi_ctx::kNpk, nc * sizeof(int32_t));
        ENSURE(qmi_ctx::kWin, nc * std::max(top_k, 1) * 16);
        ENSURE(qmi_ctx::kArgmax, nc * sizeof(int32_t));
        ENSURE(qmi_ctx::kRes, nc * sizeof(DevResult));
    }
    if (cs.periodogram && !cs.dev_inputs) ENSURE(qmi_ctx::kFreqs, F1 * 8);
#undef ENSURE
    // A launch with fewer (curve, 64-frequency tile) items than this cannot fill the chip's 512
    // workgroup slots several times over; it runs one (pass, column segment) piece per workgroup
    // instead, with the pieces' sums in a scratch buffer (same bits either way).
    constexpr int64_t kSplitBelow = 2048;
    constexpr int64_t kSplitMaxBytes = int64_t(256) << 20;
    const int64_t tiles1 = (F1 + 63) / 64, tiles2 = (F2 + 63) / 64;
    const int64_t part_bytes = pieces * std::max(F1, F2) * 24;
    bool split1 = max_pieces > 1 && nc * tiles1 < kSplitBelow;
    bool split2 = refine && max_pieces > 1 && nc * tiles2 < kSplitBelow;
    if ((split1 || split2) &&
        (part_bytes > kSplitMaxBytes || (size_t)part_bytes > ctx->budget / 8 ||
         acquire(ctx, qmi_ctx::kPart, part_bytes) != QMI_OK)) {
        split1 = split2 = false;
        ctx->err.clear();
    }
    double* dpart = (split1 || split2) ? dptr<double>(ctx, qmi_ctx::kPart) : nullptr;

    hipStream_t st = ctx->stream;
    const double* t = cs.dev_inputs ? b->t + g.s0 : dptr<double>(ctx, qmi_ctx::kT);
    const double* y = cs.dev_inputs ? b->y + g.s0 : dptr<double>(ctx, qmi_ctx::kY);
    const double* e = b->e ? (cs.dev_inputs ? b->e + g.s0 : dptr<double>(ctx, qmi_ctx::kE))
                           : nullptr;
    if (!cs.dev_inputs) {
        HIP_OK(ctx, hipMemcpyAsync((void*)t, b->t + g.s0, ns * 8, hipMemcpyHostToDevice, st));
        HIP_OK(ctx, hipMemcpyAsync((void*)y, b->y + g.s0, ns * 8, hipMemcpyHostToDevice, st));
        if (e)
            HIP_OK(ctx, hipMemcpyAsync((void*)e, b->e + g.s0, ns * 8, hipMemcpyHostToDevice, st));
    }
    CurveParams* dcp = dptr<CurveParams>(ctx, qmi_ctx::kCP);
    int32_t* dorder = dptr<int32_t>(ctx, qmi_ctx::kOrder);
    int64_t* drow = dptr<int64_t>(ctx, qmi_ctx::kRowStart);
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    HIP_OK(ctx, hipMemcpyAsync(dcp, cp.data(), nc * sizeof(CurveParams), h2d, st));
    HIP_OK(ctx, hipMemcpyAsync(dorder, order.data(), nc * sizeof(int32_t), h2d, st));
    HIP_OK(ctx, hipMemcpyAsync(drow, row_start.data(), nc * sizeof(int64_t), h2d, st));
    const double* dfreqs = nullptr;
    if (cs.periodogram) {
        if (cs.dev_inputs) {
            dfreqs = cs.freqs;
        } else {
            dfreqs = dptr<double>(ctx, qmi_ctx::kFreqs);
            HIP_OK(ctx, hipMemcpyAsync((void*)dfreqs, cs.freqs, F1 * 8, hipMemcpyHostToDevice, st));
        }
    }

    R* K = dptr<R>(ctx, qmi_ctx::kK);
    double* rp = dptr<double>(ctx, qmi_ctx::kRP);
    double* rd = dptr<double>(ctx, qmi_ctx::kRD);
    R* ks = dptr<R>(ctx, qmi_ctx::kKS);

    FreqPlan fp{};
    PairOut po{};
    double* coarse = nullptr;
    double* coarse2 = nullptr;
    if (cs.periodogram) {
        fp.kind = 1;
        fp.count = (int32_t)F1;
        fp.list = dfreqs;
        coarse = cs.dev_outputs ? cs.score_out + (int64_t)g.c0 * F1
                                : dptr<double>(ctx, qmi_ctx::kCoarse);
        po.score = coarse;
        po.score2 = nullptr;
        po.ips = cs.ips_out ? (cs.dev_outputs ? cs.ips_out + (int64_t)g.c0 * F1 * 3
                                              : dptr<double>(ctx, qmi_ctx::kIps))
                            : nullptr;
        po.score_kind = score_kind;
    } else if (bp) {
        fp.kind = 3;
        fp.count = (int32_t)F1;
        fp.stride = (int32_t)F1;
        fp.list = dptr<double>(ctx, qmi_ctx::kTrials);
        coarse = dptr<double>(ctx, qmi_ctx::kCoarse);
        coarse2 = dptr<double>(ctx, qmi_ctx::kCoarse2);
        po.score = coarse;
        po.score2 = coarse2;
        po.ips = nullptr;
        po.score_kind = score_kind;
    } else {
        const qmi_search* s = cs.search;
        fp.kind = 0;
        fp.count = s->n_coarse;
        fp.f0 = s->f_min;
        fp.df = s->n_coarse > 1 ? (s->f_max - s->f_min) / (double)(s->n_coarse - 1) : 0.0;
        coarse = dptr<double>(ctx, qmi_ctx::kCoarse);
        coarse2 = dptr<double>(ctx, qmi_ctx::kCoarse2);
        po.score = coarse;
        po.score2 = coarse2;
        po.ips = nullptr;
        po.score_kind = score_kind;
    }
    PeakOut pk{};
    double* fine = nullptr;
    double* fine2 = nullptr;
    FreqPlan ff{};
    if (!cs.periodogram) {
        pk = PeakOut{dptr<int32_t>(ctx, qmi_ctx::kPeakK), dptr<int32_t>(ctx, qmi_ctx::kNpk),
                     dptr<double>(ctx, qmi_ctx::kWin), dptr<int32_t>(ctx, qmi_ctx::kArgmax)};
        if (refine) {
            fine = dptr<double>(ctx, qmi_ctx::kFine);
            fine2 = dptr<double>(ctx, qmi_ctx::kFine2);
            ff.kind = 2;
            ff.count = (int32_t)F2;
            ff.n_fine = n_fine;
            ff.top_k = top_k;
            ff.win = pk.win;
            ff.npk = pk.npk;
        }
    }
    DevResult* dres = cs.periodogram ? nullptr : dptr<DevResult>(ctx, qmi_ctx::kRes);
    BandsDev bd{};
    if (bp) {
        bd.f_lo = bp->f_lo;
        bd.df = (bp->f_hi - bp->f_lo) / (double)(bp->n_grid - 1);
        bd.n_grid = bp->n_grid;
        bd.n_bands = bp->n_bands;
        bd.n_keep = bp->n_keep;
        bd.n_trials = bp->n_trials;
        bd.stride = std::max(1, (max_n + bp->n_bands - 1) / bp->n_bands);
        bd.ts = dptr<double>(ctx, qmi_ctx::kTS);
        bd.ys = dptr<double>(ctx, qmi_ctx::kYS);
        bd.band_t = dptr<double>(ctx, qmi_ctx::kBandT);
        bd.band_cnt = dptr<int32_t>(ctx, qmi_ctx::kBandCnt);
        bd.band_id = dptr<int32_t>(ctx, qmi_ctx::kBandId);
        bd.S = dptr<double>(ctx, qmi_ctx::kS);
        bd.trials = dptr<double>(ctx, qmi_ctx::kTrials);
        bd.trial_k = dptr<int32_t>(ctx, qmi_ctx::kTrialK);
    }

    // Pair-kernel variant: forced by QMI_OPT_TILE, else the autotuned choice for this length
    // bucket; until the bucket has been tuned (see the end of this function), variant 1 (4 waves
    // per SIMD, 64-column chunks), the fastest on every length mix measured.
    std::vector<int32_t> lens;
    for (int32_t i = 0; i < nc; ++i)
        if (cp[i].status == QMI_OK) lens.push_back(cp[i].n);
    int bucket = 0;
    if (!lens.empty()) {
        std::nth_element(lens.begin(), lens.begin() + lens.size() / 2, lens.end());
        const int med = lens[lens.size() / 2];
        while (bucket < 7 && (192 << bucket) <= med) ++bucket;
    }
    const int nvar = pair_variants<R>();
    int variant = nvar > 1 ? 1 : 0;
    const bool fold32 = kp->precision == QMI_PREC_FOLD32;
    if (fold32) variant = kVariantFold32;
    else if (ctx->tile > 0) variant = (int)std::min<int64_t>(ctx->tile - 1, nvar - 1);
    else if (!fp64 && ctx->tuned[bucket] >= 0) variant = ctx->tuned[bucket];
    double group_items = 0.0;
    for (int32_t i = 0; i < nc; ++i)
        if (cp[i].status == QMI_OK) group_items += 0.5 * cp[i].n * (cp[i].n - 1.0) * (double)F1;
    const bool tune_now = !fp64 && !fold32 && ctx->tile == 0 && ctx->tuned[bucket] < 0 &&
                          nvar > 1 && !ctx->ws_base && group_items > 2e9;
    ctx->stats.pair_variant = variant;

    const bool skew_default = kp->skew_lambda == 0.0 && kp->skew_mu == 0.0;
    const double skew_lambda = skew_default ? QMI_SKEW_LAMBDA : kp->skew_lambda;
    const double skew_mu = skew_default ? QMI_SKEW_MU : kp->skew_mu;

    // The device section: every kernel of the call, and the timing events around the pair kernels.
    // It contains no copies or allocations, so it can be captured into a hipGraph and replayed.
    auto section = [&](bool events) -> int {
        auto rec = [&]() {
            if (events) record(ctx);
        };
        rec();  // device section start
        HIP_OK(ctx, launch_prologue(st, dcp, nc, max_n, t, y, e, skew_lambda, skew_mu));
        HIP_OK(ctx, launch_gram<R>(st, dcp, nc, rows, drow, y, K, rp, rd));
        HIP_OK(ctx, launch_gram_finalize<R>(st, dcp, nc, rd, rp));
        HIP_OK(ctx, launch_ksum<R>(st, dcp, nc, max_n, K, ks));
        if (bp) HIP_OK(ctx, launch_bands(st, dcp, nc, max_n, t, y, bd));
        if (events) pair_event_idx.push_back(ctx->ev_used);
        rec();
        {
            PairOut pc1 = po;
            pc1.part = split1 ? dpart : nullptr;
            // Per-curve lists whose last tile would hold only one or two slots (the bands
            // method's 450 trials): the main launch stops before that tile, and a kernel with one
            // row per lane takes its slots (FP32 path).
            FreqPlan fpm = fp;
            int rem_slot0 = -1;
            if constexpr (sizeof(R) == 4) {
                const int full = fp.count / kLanes, rem = fp.count % kLanes;
                if (fp.kind == 3 && variant != kVariantFold32 && full > 0 && rem > 0 &&
                    rem <= kRemSlots) {
                    fpm.tile_cap = full;
                    rem_slot0 = full * kLanes;
                }
            }
            HIP_OK(ctx, launch_pairs<R>(st, dcp, dorder, nc, fpm, t, K, rd, rp, ks, pc1, variant,
                                        split1 ? max_pieces : 0));
            if constexpr (sizeof(R) == 4) {
                if (rem_slot0 >= 0)
                    HIP_OK(ctx, launch_pairs_rows(st, dcp, dorder, nc, fp, rem_slot0, t, K, rd,
                                                  pc1));
            }
        }
        rec();
        if (bp) {
            HIP_OK(ctx, launch_bands_best(st, dcp, nc, coarse, coarse2, score_kind, bd,
                                          ctx->masks, dres));
        } else if (!cs.periodogram) {
            const qmi_search* s = cs.search;
            HIP_OK(ctx, launch_peaks(st, dcp, nc, coarse, s->n_coarse, fp.f0, fp.df, top_k,
                                     std::max(n_fine, 2), ctx->masks, pk));
            if (refine) {
                PairOut fo{fine, fine2, nullptr, score_kind, 0, split2 ? dpart : nullptr};
                if (events) pair_event_idx.push_back(ctx->ev_used);
                rec();
                HIP_OK(ctx,
                       launch_pairs<R>(st, dcp, dorder, nc, ff, t, K, rd, rp, ks, fo, variant,
                                       split2 ? max_pieces : 0));
                rec();
            }
            HIP_OK(ctx, launch_best(st, dcp, nc, coarse, coarse2, s->n_coarse, fine, fine2,
                                    refine ? top_k : 0, refine ? n_fine : 0, score_kind, fp.f0,
                                    fp.df, ctx->masks, pk, dres));
        }
        rec();  // device section end
        return QMI_OK;
    };

    // Graph replay: only for a call that is one group (event indices then start at 0), and not
    // in scratch mode (a capture and its instantiation allocate).
    bool ran = false;
    if (ctx->use_graph && ctx->ev_used == 0 && !ctx->ws_base) {
        auto u = [](const void* p) { return (uint64_t)(uintptr_t)p; };
        auto dbits = [](double v) { uint64_t b; std::memcpy(&b, &v, 8); return b; };
        std::vector<uint64_t> key = {
            (uint64_t)fp64, (uint64_t)cs.periodogram, (uint64_t)nc, (uint64_t)rows,
            (uint64_t)max_n, (uint64_t)F1, (uint64_t)F2, (uint64_t)top_k, (uint64_t)n_fine,
            (uint64_t)score_kind, (uint64_t)variant, dbits(fp.f0), dbits(fp.df),
            dbits(skew_lambda), dbits(skew_mu), u(st), u(t), u(y),
            u(e), u(dcp),
            u(dorder), u(drow), u(K), u(rp), u(rd), u(ks), u(dfreqs), u(coarse), u(coarse2),
            u(po.ips), u(fine), u(fine2), u(pk.peak_k), u(pk.npk), u(pk.win), u(pk.argmax),
            u(dres), (uint64_t)(bp != nullptr), dbits(bd.f_lo), dbits(bd.df),
            (uint64_t)bd.n_grid, (uint64_t)bd.n_bands, (uint64_t)bd.n_keep, (uint64_t)bd.n_trials,
            (uint64_t)bd.stride, u(bd.ts), u(bd.ys), u(bd.band_t), u(bd.band_cnt), u(bd.band_id),
            u(bd.S), u(bd.trials), u(bd.trial_k)};
        if (ctx->graph_exec && key == ctx->graph_key) {
            record(ctx);
            HIP_OK(ctx, hipGraphLaunch(ctx->graph_exec, st));
            record(ctx);
            ran = true;
            ctx->stats.used_graph = 1;
        } else {
            if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
            if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
            ctx->graph_exec = nullptr;
            ctx->graph = nullptr;
            ctx->graph_key.clear();
            // The captured section holds kernel launches only (no events, copies or allocations).
            bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
            int rc_sec = QMI_OK;
            hipGraph_t graph = nullptr;
            if (ok) {
                rc_sec = section(false);
                const bool ended = hipStreamEndCapture(st, &graph) == hipSuccess;
                hipGraphExec_t exec = nullptr;
                ok = rc_sec == QMI_OK && ended && graph &&
                     hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
                if (ok) {
                    ctx->graph = graph;
                    ctx->graph_exec = exec;
                    ctx->graph_key = key;
                    record(ctx);
                    HIP_OK(ctx, hipGraphLaunch(exec, st));
                    record(ctx);
                    ran = true;
                    ctx->stats.used_graph = 1;
                }
            }
            if (!ok) {
                // Capture is not available for this section: run eagerly from now on.  A stream
                // left in a failed capture is replaced when the context owns it.
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                ctx->use_graph = false;
                ctx->err.clear();
                if (ctx->own_stream) {
                    (void)hipStreamDestroy(ctx->stream);
                    HIP_OK(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
                    st = ctx->stream;
                }
            }
        }
    }
    if (!ran) {
        // Scratch mode records no timing events (their creation allocates).
        const int rc_sec = section(!ctx->ws_base);
        if (rc_sec != QMI_OK) return rc_sec;
    }

    // Results back to the caller.
    if (cs.periodogram) {
        if (!cs.dev_outputs) {
            HIP_OK(ctx, hipMemcpyAsync(cs.score_out + (int64_t)g.c0 * F1, coarse, nc * F1 * 8,
                                       hipMemcpyDeviceToHost, st));
            if (cs.ips_out)
                HIP_OK(ctx, hipMemcpyAsync(cs.ips_out + (int64_t)g.c0 * F1 * 3, po.ips,
                                           nc * F1 * 24, hipMemcpyDeviceToHost, st));
        }
        std::vector<CurveParams> cpo(nc);
        HIP_OK(ctx, hipMemcpyAsync(cpo.data(), dcp, nc * sizeof(CurveParams),
                                   hipMemcpyDeviceToHost, st));
        HIP_OK(ctx, hipStreamSynchronize(st));
        for (int32_t i = 0; i < nc; ++i) {
            if (cs.ip_y_out) cs.ip_y_out[g.c0 + i] = cpo[i].status ? NAN : cpo[i].ipy;
            if (cs.status_out) cs.status_out[g.c0 + i] = cpo[i].status;
        }
        // Curves rejected on the host were never given to the kernels' outputs.
        if (!cs.dev_outputs) {
            for (int32_t i = 0; i < nc; ++i)
                if (cp[i].status != QMI_OK) {
                    for (int64_t f = 0; f < F1; ++f) {
                        cs.score_out[(int64_t)(g.c0 + i) * F1 + f] = NAN;
                        if (cs.ips_out)
                            for (int q = 0; q < 3; ++q)
                                cs.ips_out[((int64_t)(g.c0 + i) * F1 + f) * 3 + q] = NAN;
                    }
                }
        }
    } else {
        static_assert(sizeof(DevResult) == sizeof(qmi_result), "result layout");
        HIP_OK(ctx, hipMemcpyAsync(cs.out + g.c0, dptr<DevResult>(ctx, qmi_ctx::kRes),
                                   nc * sizeof(DevResult), hipMemcpyDeviceToHost, st));
        if (cs.coarse_out) {
            if (cs.dev_outputs)
                HIP_OK(ctx, hipMemcpyAsync(cs.coarse_out + (int64_t)g.c0 * F1, coarse, nc * F1 * 8,
                                           hipMemcpyDeviceToDevice, st));
            else
                HIP_OK(ctx, hipMemcpyAsync(cs.coarse_out + (int64_t)g.c0 * F1, coarse, nc * F1 * 8,
                                           hipMemcpyDeviceToHost, st));
        }
        if (bp && cs.trials_out)
            HIP_OK(ctx, hipMemcpyAsync(cs.trials_out + (int64_t)g.c0 * F1, bd.trials,
                                       nc * F1 * 8, hipMemcpyDeviceToHost, st));
        if (bp && cs.scores_out)
            HIP_OK(ctx, hipMemcpyAsync(cs.scores_out + (int64_t)g.c0 * F1, coarse, nc * F1 * 8,
                                       hipMemcpyDeviceToHost, st));
        HIP_OK(ctx, hipStreamSynchronize(st));
        if (bp && (cs.trials_out || cs.scores_out)) {
            // Empty trial slots are never scored: report them as NaN in both outputs.
            std::vector<double> tr;
            const double* trp = cs.trials_out ? cs.trials_out + (int64_t)g.c0 * F1 : nullptr;
            if (!trp) {
                tr.resize((size_t)nc * F1);
                HIP_OK(ctx, hipMemcpy(tr.data(), bd.trials, nc * F1 * 8, hipMemcpyDeviceToHost));
                trp = tr.data();
            }
            if (cs.scores_out)
                for (int64_t q = 0; q < (int64_t)nc * F1; ++q)
                    if (!(trp[q] == trp[q])) cs.scores_out[(int64_t)g.c0 * F1 + q] = NAN;
        }
        for (int32_t i = 0; i < nc; ++i) {
            qmi_result& rr = cs.out[g.c0 + i];
            if (cp[i].status != QMI_OK) {
                // The kernels skipped this curve; make its record explicit.
                rr.status = cp[i].status;
                rr.n = cp[i].n;
            }
            if (cp[i].status != QMI_OK) rr.sigma_t = NAN;
            if (rr.status != QMI_OK) {
                rr.f_best = rr.period = rr.score = rr.score_qmi = rr.score_nckp = NAN;
                rr.coarse_best = NAN;
                rr.coarse_index = rr.peak_rank = rr.fine_index = rr.coarse_argmax = -1;
                rr.n_peaks = 0;
            }
            const int64_t n = b->offsets[g.c0 + i + 1] - b->offsets[g.c0 + i];
            rr.n = (int32_t)n;
            if (rr.status == QMI_OK)
                ctx->stats.pair_items += (double)n * (double)(n - 1) / 2.0 *
                                         (double)(bp ? (int64_t)rr.n_peaks
                                                     : F1 + (int64_t)rr.n_peaks * n_fine);
        }
    }
    if (cs.periodogram) {
        for (int32_t i = 0; i < nc; ++i) {
            const int64_t n = b->offsets[g.c0 + i + 1] - b->offsets[g.c0 + i];
            if (cp[i].status == QMI_OK)
                ctx->stats.pair_items += (double)n * (double)(n - 1) / 2.0 * (double)F1;
        }
    }
    if (tune_now) {
        // Time the four variants (2 or 4 waves per SIMD, 64- or 32-column chunks; they give the
        // same bits, so tuning never changes a result) on the largest curves of this group (the
        // first in LPT order) over a slice of the same frequency plan, into a scratch output, and
        // keep the fastest for this length bucket.
        const int pc = std::min(nc, 48);
        FreqPlan probe = fp;
        probe.count = (int32_t)std::min<int64_t>(F1, 64 * 24);
        // The kernel writes slot s of curve c (a curve id, not its rank in the work order) at
        // c * count + s, so the scratch output must cover every curve id of the group.
        int rc2 = ensure(ctx, qmi_ctx::kProbe, (size_t)nc * probe.count * 8);
        if (rc2 != QMI_OK) return rc2;
        PairOut pout{dptr<double>(ctx, qmi_ctx::kProbe), nullptr, nullptr, score_kind, 0};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_OK(ctx, hipEventCreate(&e0));
        HIP_OK(ctx, hipEventCreate(&e1));
        float best_ms = 0.f;
        int best_v = 0;
        for (int v = 0; v < nvar; ++v) {
            HIP_OK(ctx,
                   launch_pairs<R>(st, dcp, dorder, pc, probe, t, K, rd, rp, ks, pout, v, 0));
            HIP_OK(ctx, hipEventRecord(e0, st));
            for (int rep = 0; rep < 2; ++rep)
                HIP_OK(ctx,
                       launch_pairs<R>(st, dcp, dorder, pc, probe, t, K, rd, rp, ks, pout, v, 0));
            HIP_OK(ctx, hipEventRecord(e1, st));
            HIP_OK(ctx, hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(ctx, hipEventElapsedTime(&ms, e0, e1));
            if (v == 0 || ms < best_ms) {
                best_ms = ms;
                best_v = v;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->tuned[bucket] = best_v;
    }
    (void)fp64;
    return QMI_OK;
}

int run_call(qmi_ctx* ctx, const qmi_batch* b, const CallSpec& cs) {
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    ctx->err.clear();
    int rc = check_kernel_params(ctx, cs.kp);
    if (rc) return rc;
    rc = check_batch(ctx, b, cs.kp->sigma_y == QMI_SIGMA_MEDIAN_ERR);
    if (rc) return rc;
    if (cs.periodogram) {
        if (cs.n_freq < 1 || !cs.freqs || !cs.score_out) {
            set_err(ctx, "periodogram needs n_freq >= 1, freqs and score_out");
            return QMI_EINVAL;
        }
        if (cs.score != QMI_SCORE_CS_QMI && cs.score != QMI_SCORE_NCKP) {
            set_err(ctx, "unknown score %d", cs.score);
            return QMI_EINVAL;
        }
        if (!cs.dev_inputs)
            for (int32_t q = 0; q < cs.n_freq; ++q)
                if (!std::isfinite(cs.freqs[q]) || cs.freqs[q] < 0.0) {
                    set_err(ctx, "frequency %d is not finite and >= 0", q);
                    return QMI_EINVAL;
                }
    } else if (cs.bands) {
        const qmi_bands* p = cs.bands;
        if (!cs.out) { set_err(ctx, "out must not be NULL"); return QMI_EINVAL; }
        if (!(p->f_lo > 0.0) || !(p->f_hi > p->f_lo) || !std::isfinite(p->f_hi) ||
            p->n_grid < 2 || p->n_grid > (1 << 24) || p->n_bands < 1 ||
            p->n_bands > QMI_MAX_BANDS || p->n_keep < 1 || p->n_keep > p->n_bands ||
            p->n_trials < 1 || p->n_trials > QMI_MAX_TRIALS) {
            set_err(ctx, "bad bands parameters (f %g..%g, n_grid %d, n_bands %d, n_keep %d, "
                    "n_trials %d)", p->f_lo, p->f_hi, p->n_grid, p->n_bands, p->n_keep,
                    p->n_trials);
            return QMI_EINVAL;
        }
        if (p->score != QMI_SCORE_CS_QMI && p->score != QMI_SCORE_NCKP) {
            set_err(ctx, "unknown score %d", p->score);
            return QMI_EINVAL;
        }
    } else {
        const qmi_search* s = cs.search;
        if (!s || !cs.out) { set_err(ctx, "search and out must not be NULL"); return QMI_EINVAL; }
        if (!(s->f_min >= 0.0) || !(s->f_max > s->f_min) || !std::isfinite(s->f_max)) {
            set_err(ctx, "need 0 <= f_min < f_max (got %g, %g)", s->f_min, s->f_max);
            return QMI_EINVAL;
        }
        if (s->n_coarse < 1 || s->n_coarse > (1 << 26) || s->top_k < 0 ||
            s->top_k > QMI_MAX_TOPK || s->n_fine < 0 || s->n_fine == 1 ||
            s->n_fine > (1 << 20)) {
            set_err(ctx, "bad search sizes (n_coarse %d, top_k %d, n_fine %d)", s->n_coarse,
                    s->top_k, s->n_fine);
            return QMI_EINVAL;
        }
        if (s->score != QMI_SCORE_CS_QMI && s->score != QMI_SCORE_NCKP) {
            set_err(ctx, "unknown score %d", s->score);
            return QMI_EINVAL;
        }
    }
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (b->n_curves == 0) return QMI_OK;
    HIP_OK(ctx, hipSetDevice(ctx->device));
    std::vector<Group> groups;
    if (cs.noalloc) {
        // The whole batch is one group, its buffers in the device's scratch array.
        void* base = nullptr;
        rc = scratch_for_device(ctx, &base);
        if (rc) return rc;
        groups.push_back(Group{0, b->n_curves, 0, b->offsets[b->n_curves]});
        ctx->ws_base = static_cast<char*>(base);
        ctx->ws_size = QMI_NOALLOC_SCRATCH_BYTES;
        ctx->ws_used = 0;
    } else {
        rc = plan_groups(ctx, b, cs, groups);
        if (rc) return rc;
    }
    struct ScratchOff {
        qmi_ctx* c;
        ~ScratchOff() { c->ws_base = nullptr; }
    } scratch_off{ctx};
    ctx->ev_used = 0;
    std::vector<int32_t> pair_ev;
    for (const Group& g : groups) {
        rc = (cs.kp->precision == QMI_PREC_FP64) ? run_group<double>(ctx, b, cs, g, pair_ev)
                                                 : run_group<float>(ctx, b, cs, g, pair_ev);
        if (rc) return rc;
    }
    // Timing from the events (all complete: every group synchronised).
    float ms = 0.f;
    for (int32_t idx : pair_ev) {
        if (hipEventElapsedTime(&ms, ctx->ev[idx], ctx->ev[idx + 1]) == hipSuccess)
            ctx->stats.pair_kernel_ms += ms;
        ctx->stats.pair_launches += 1;
    }
    if (ctx->ev_used >= 2 &&
        hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[ctx->ev_used - 1]) == hipSuccess)
        ctx->stats.device_ms = ms;
    return QMI_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// Serving loop
// ------------------------------------------------------------------------------------------------

struct qmi_ctx::Serve {
    qmi_kernel_params kp{};
    qmi_search search{};
    size_t admit_budget = 0;
    int32_t max_batch = 256;
    int32_t max_inflight = 2;
    double max_items = 0.0;  // pair x frequency items per launch (0: no bound)
    struct Req {
        std::vector<double> t, y, e;
        bool has_e = false;
        uint64_t tag = 0;
        double items = 0.0;  // its pair x frequency items (coarse grid and refinement)
    };
    struct Done {
        qmi_result r;
        uint64_t tag;
    };
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Req> queue;
    std::deque<Done> done;
    size_t queued_bytes = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<qmi_ctx*> lanes;  // one private context (and stream) per in-flight launch
};

namespace {

size_t request_bytes(const qmi_search& s, int64_t n) {
    return curve_bytes(n, s.n_coarse, (int64_t)s.top_k * s.n_fine, false, false, true);
}

void serve_worker(qmi_ctx* ctx, int lane) {
    qmi_ctx::Serve* S = ctx->serve.get();
    qmi_ctx* lc = S->lanes[lane];
    for (;;) {
        std::vector<qmi_ctx::Serve::Req> take;
        size_t take_bytes = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop && S->queue.empty()) return;
            // Admit requests in arrival order while they fit this lane's share of the budget and
            // the launch's work bound (so that a request arriving meanwhile waits for at most
            // one bounded launch of some lane).
            const size_t share = S->admit_budget / (size_t)S->max_inflight;
            double take_items = 0.0;
            while (!S->queue.empty() && (int32_t)take.size() < S->max_batch) {
                size_t rb = request_bytes(S->search, (int64_t)S->queue.front().t.size());
                if (!take.empty() && take_bytes + rb > share) break;
                const double it = S->queue.front().items;
                if (!take.empty() && S->max_items > 0.0 && take_items + it > S->max_items) break;
                take_items += it;
                take_bytes += rb;
                take.push_back(std::move(S->queue.front()));
                S->queue.pop_front();
                S->queued_bytes -= rb;
            }
        }
        // Pack and run on this lane's context (its own stream), overlapping other lanes.
        std::vector<int64_t> off(take.size() + 1, 0);
        for (size_t i = 0; i < take.size(); ++i) off[i + 1] = off[i] + (int64_t)take[i].t.size();
        std::vector<double> t(off.back()), y(off.back()), e(off.back());
        bool all_e = true;
        for (size_t i = 0; i < take.size(); ++i) {
            std::copy(take[i].t.begin(), take[i].t.end(), t.begin() + off[i]);
            std::copy(take[i].y.begin(), take[i].y.end(), y.begin() + off[i]);
            if (take[i].has_e) std::copy(take[i].e.begin(), take[i].e.end(), e.begin() + off[i]);
            all_e = all_e && take[i].has_e;
        }
        qmi_batch b{(int32_t)take.size(), off.data(), t.data(), y.data(),
                    all_e ? e.data() : nullptr};
        std::vector<qmi_result> res(take.size());
        int rc = qmi_best_period(lc, &b, &S->kp, &S->search, res.data(), nullptr);
        std::lock_guard<std::mutex> lk(S->mu);
        for (size_t i = 0; i < take.size(); ++i) {
            if (rc != QMI_OK) {
                std::memset(&res[i], 0, sizeof(qmi_result));
                res[i].status = rc;
                res[i].f_best = res[i].period = res[i].score = NAN;
            }
            S->done.push_back({res[i], take[i].tag});
        }
        S->done_cv.notify_all();
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------

extern "C" {

int qmi_create(qmi_ctx** out, int hip_device, size_t hbm_budget_bytes, void* hip_stream) {
    if (!out) {
        set_err(nullptr, "out is NULL");
        return QMI_EINVAL;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        set_err(nullptr, "no HIP device available (%s)", hipGetErrorString(e));
        return QMI_EDEVICE;
    }
    if (hip_device < 0 || hip_device >= ndev) {
        set_err(nullptr, "device %d out of range (%d devices)", hip_device, ndev);
        return QMI_EINVAL;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
        set_err(nullptr, "hipSetDevice(%d) failed", hip_device);
        return QMI_EDEVICE;
    }
    e = resolve_scratch(hip_device);
    if (e != hipSuccess) {
        set_err(nullptr, "hipGetSymbolAddress(scratch) on device %d failed: %s", hip_device,
                hipGetErrorString(e));
        return QMI_EDEVICE;
    }
    std::unique_ptr<qmi_ctx> ctx(new (std::nothrow) qmi_ctx());
    if (!ctx) {
        set_err(nullptr, "out of host memory");
        return QMI_EINTERNAL;
    }
    ctx->device = hip_device;
    if (hip_stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            set_err(nullptr, "hipStreamCreate failed");
            return QMI_EDEVICE;
        }
        ctx->own_stream = true;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        set_err(nullptr, "hipMemGetInfo failed");
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        return QMI_EDEVICE;
    }
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
    *out = ctx.release();
    return QMI_OK;
}

void qmi_destroy(qmi_ctx* ctx) {
    if (!ctx) return;
    if (ctx->serve) qmi_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    for (auto& b : ctx->bufs)
        if (b.p) (void)hipFree(b.p);
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* qmi_last_error(const qmi_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int qmi_set_option(qmi_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return QMI_EINVAL;
    switch (option) {
        case QMI_OPT_USE_GRAPH: ctx->use_graph = value != 0; return QMI_OK;
        case QMI_OPT_TILE: ctx->tile = value; return QMI_OK;
        case QMI_OPT_SYNC: return QMI_OK;
        case QMI_OPT_SERVE_BATCH_ITEMS:
            if (value < 0) break;
            ctx->serve_batch_items = value;
            return QMI_OK;
        default: break;
    }
    set_err(ctx, "unknown option %d or bad value %lld", option, (long long)value);
    return QMI_EINVAL;
}

int qmi_get_stats(const qmi_ctx* ctx, qmi_stats* out) {
    if (!ctx || !out) return QMI_EINVAL;
    *out = ctx->stats;
    return QMI_OK;
}

int qmi_set_masks(qmi_ctx* ctx, const qmi_mask* masks, int32_t n_masks) {
    if (!ctx) return QMI_EINVAL;
    if (n_masks < 0 || n_masks > QMI_MAX_MASKS || (n_masks > 0 && !masks)) {
        set_err(ctx, "qmi_set_masks: need 0 <= n_masks <= %d and a table", QMI_MAX_MASKS);
        return QMI_EINVAL;
    }
    if (ctx->serve) {
        set_err(ctx, "qmi_set_masks: serving is running");
        return QMI_EINVAL;
    }
    qmi::MaskDev md{};
    for (int i = 0; i < n_masks; ++i) {
        const qmi_mask& m = masks[i];
        if (!(std::isfinite(m.period) && m.period > 0.0 && std::isfinite(m.sigma) &&
              m.sigma > 0.0 && std::isfinite(m.amplitude))) {
            set_err(ctx, "qmi_set_masks: mask %d needs a finite positive period and sigma and a "
                    "finite amplitude", i);
            return QMI_EINVAL;
        }
        md.period[i] = m.period;
        md.sigma[i] = m.sigma;
        md.amp[i] = m.amplitude;
    }
    md.n = n_masks;
    // A captured graph holds the previous table in its kernel arguments.
    drop_graph(ctx);
    ctx->masks = md;
    return QMI_OK;
}

int qmi_periodogram(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                    const double* freqs, int32_t n_freq, int32_t score, double* score_out,
                    double* ips_out, double* ip_y_out, int32_t* status_out) {
    if (!ctx) return QMI_EINVAL;
    CallSpec cs{};
    cs.dev_inputs = false;
    cs.dev_outputs = false;
    cs.periodogram = true;
    cs.kp = kp;
    cs.freqs = freqs;
    cs.n_freq = n_freq;
    cs.score = score;
    cs.score_out = score_out;
    cs.ips_out = ips_out;
    cs.ip_y_out = ip_y_out;
    cs.status_out = status_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_periodogram_dev(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                        const double* freqs, int32_t n_freq, int32_t score, double* score_out,
                        double* ips_out, double* ip_y_out, int32_t* status_out) {
    if (!ctx) return QMI_EINVAL;
    CallSpec cs{};
    cs.dev_inputs = true;
    cs.dev_outputs = true;
    cs.periodogram = true;
    cs.kp = kp;
    cs.freqs = freqs;
    cs.n_freq = n_freq;
    cs.score = score;
    cs.score_out = score_out;
    cs.ips_out = ips_out;
    cs.ip_y_out = ip_y_out;
    cs.status_out = status_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_periodogram_noalloc(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                            const double* freqs, int32_t n_freq, int32_t score, double* score_out,
                            double* ips_out, double* ip_y_out, int32_t* status_out) {
    if (!ctx) return QMI_EINVAL;
    CallSpec cs{};
    cs.noalloc = true;
    cs.dev_inputs = true;
    cs.dev_outputs = true;
    cs.periodogram = true;
    cs.kp = kp;
    cs.freqs = freqs;
    cs.n_freq = n_freq;
    cs.score = score;
    cs.score_out = score_out;
    cs.ips_out = ips_out;
    cs.ip_y_out = ip_y_out;
    cs.status_out = status_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_best_period(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                    const qmi_search* search, qmi_result* out, double* coarse_out) {
    if (!ctx) return QMI_EINVAL;
    CallSpec cs{};
    cs.dev_inputs = false;
    cs.dev_outputs = false;
    cs.periodogram = false;
    cs.kp = kp;
    cs.search = search;
    cs.out = out;
    cs.coarse_out = coarse_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_bands_best_period(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                          const qmi_bands* bands, qmi_result* out, double* trials_out,
                          double* scores_out) {
    if (!ctx) return QMI_EINVAL;
    if (!bands) {
        set_err(ctx, "bands must not be NULL");
        return QMI_EINVAL;
    }
    CallSpec cs{};
    cs.dev_inputs = false;
    cs.dev_outputs = false;
    cs.periodogram = false;
    cs.kp = kp;
    cs.bands = bands;
    cs.out = out;
    cs.trials_out = trials_out;
    cs.scores_out = scores_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

namespace {

// Uploads a host batch (arrays, offsets) and the per-curve host statuses; returns max N of the
// valid curves through *max_n.
int upload_batch(qmi_ctx* ctx, const qmi_batch* b, const std::vector<int32_t>& status,
                 int* max_n) {
    const int32_t nc = b->n_curves;
    const int64_t ns = b->offsets[nc];
    int rc;
    if ((rc = ensure(ctx, qmi_ctx::kT, std::max<int64_t>(ns, 1) * 8)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kY, std::max<int64_t>(ns, 1) * 8)) != QMI_OK) return rc;
    if (b->e && (rc = ensure(ctx, qmi_ctx::kE, std::max<int64_t>(ns, 1) * 8)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPOff, (nc + 1) * 8)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPStIn, nc * 4)) != QMI_OK) return rc;
    hipStream_t st = ctx->stream;
    HIP_OK(ctx, hipMemcpyAsync(dptr<double>(ctx, qmi_ctx::kT), b->t, ns * 8,
                               hipMemcpyHostToDevice, st));
    HIP_OK(ctx, hipMemcpyAsync(dptr<double>(ctx, qmi_ctx::kY), b->y, ns * 8,
                               hipMemcpyHostToDevice, st));
    if (b->e)
        HIP_OK(ctx, hipMemcpyAsync(dptr<double>(ctx, qmi_ctx::kE), b->e, ns * 8,
                                   hipMemcpyHostToDevice, st));
    HIP_OK(ctx, hipMemcpyAsync(dptr<int64_t>(ctx, qmi_ctx::kPOff), b->offsets, (nc + 1) * 8,
                               hipMemcpyHostToDevice, st));
    HIP_OK(ctx, hipMemcpyAsync(dptr<int32_t>(ctx, qmi_ctx::kPStIn), status.data(), nc * 4,
                               hipMemcpyHostToDevice, st));
    int mx = 1;
    for (int32_t k = 0; k < nc; ++k)
        if (status[k] == QMI_OK)
            mx = std::max<int>(mx, (int)(b->offsets[k + 1] - b->offsets[k]));
    *max_n = mx;
    return QMI_OK;
}

int preprocess_call(qmi_ctx* ctx, const qmi_batch* b, const qmi_preprocess_params* pp,
                    int64_t* offsets_out, double* t_out, double* y_out, double* e_out,
                    int32_t* status_out, uint8_t* detrended_out) {
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    ctx->err.clear();
    if (!pp || !offsets_out || !t_out || !y_out) {
        set_err(ctx, "params, offsets_out, t_out and y_out must not be NULL");
        return QMI_EINVAL;
    }
    int rc = check_batch(ctx, b, pp->error_cut || pp->detrend);
    if (rc) return rc;
    if (b->e && !e_out) {
        set_err(ctx, "e_out must not be NULL when the batch has error bars");
        return QMI_EINVAL;
    }
    if (pp->min_samples < 2 || pp->min_samples > QMI_MAX_N) {
        set_err(ctx, "min_samples must be in [2, %d] (got %d)", QMI_MAX_N, pp->min_samples);
        return QMI_EINVAL;
    }
    const int32_t nc = b->n_curves;
    offsets_out[0] = 0;
    if (nc == 0) return QMI_OK;
    const int64_t ns = b->offsets[nc];
    std::vector<int32_t> st_in(nc);
    for (int32_t k = 0; k < nc; ++k) {
        st_in[k] = host_curve_status(b, k, true);
        if (st_in[k] == QMI_OK && pp->detrend)
            for (int64_t i = b->offsets[k]; i < b->offsets[k + 1]; ++i)
                if (!(b->e[i] > 0.0)) st_in[k] = QMI_EINVAL;  // chi^2 weights need e > 0
    }
    HIP_OK(ctx, hipSetDevice(ctx->device));
    begin_use(ctx);
    int max_n = 0;
    if ((rc = upload_batch(ctx, b, st_in, &max_n)) != QMI_OK) return rc;
    const int ids[] = {qmi_ctx::kPTo, qmi_ctx::kPYo, qmi_ctx::kPEo};
    for (int id : ids)
        if ((rc = ensure(ctx, id, std::max<int64_t>(ns, 1) * 8)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPCnt, nc * 4)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPSt, nc * 4)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPDet, nc)) != QMI_OK) return rc;
    PrepDev pd{};
    pd.error_cut = pp->error_cut ? 1 : 0;
    pd.detrend = pp->detrend ? 1 : 0;
    pd.min_samples = pp->min_samples;
    pd.status_in = dptr<int32_t>(ctx, qmi_ctx::kPStIn);
    pd.counts = dptr<int32_t>(ctx, qmi_ctx::kPCnt);
    pd.status = dptr<int32_t>(ctx, qmi_ctx::kPSt);
    pd.detrended = dptr<uint8_t>(ctx, qmi_ctx::kPDet);
    pd.t_out = dptr<double>(ctx, qmi_ctx::kPTo);
    pd.y_out = dptr<double>(ctx, qmi_ctx::kPYo);
    pd.e_out = dptr<double>(ctx, qmi_ctx::kPEo);
    hipStream_t st = ctx->stream;
    HIP_OK(ctx, launch_prep(st, nc, dptr<int64_t>(ctx, qmi_ctx::kPOff),
                            dptr<double>(ctx, qmi_ctx::kT), dptr<double>(ctx, qmi_ctx::kY),
                            b->e ? dptr<double>(ctx, qmi_ctx::kE) : nullptr, pd));
    std::vector<int32_t> cnt(nc), stt(nc);
    std::vector<uint8_t> det(nc);
    std::vector<double> ht(ns), hy(ns), he(b->e ? ns : 0);
    HIP_OK(ctx, hipMemcpyAsync(cnt.data(), pd.counts, nc * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipMemcpyAsync(stt.data(), pd.status, nc * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipMemcpyAsync(det.data(), pd.detrended, nc, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipMemcpyAsync(ht.data(), pd.t_out, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipMemcpyAsync(hy.data(), pd.y_out, ns * 8, hipMemcpyDeviceToHost, st));
    if (b->e)
        HIP_OK(ctx, hipMemcpyAsync(he.data(), pd.e_out, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipStreamSynchronize(st));
    // Dense output: each accepted curve's kept samples; rejected curves keep none.
    int64_t o = 0;
    for (int32_t k = 0; k < nc; ++k) {
        const int64_t a = b->offsets[k];
        const int64_t m = stt[k] == QMI_OK ? cnt[k] : 0;
        std::memcpy(t_out + o, ht.data() + a, m * 8);
        std::memcpy(y_out + o, hy.data() + a, m * 8);
        if (b->e) std::memcpy(e_out + o, he.data() + a, m * 8);
        o += m;
        offsets_out[k + 1] = o;
        if (status_out) status_out[k] = stt[k];
        if (detrended_out) detrended_out[k] = det[k];
    }
    return QMI_OK;
}

int whiten_call(qmi_ctx* ctx, const qmi_batch* b, const double* periods, int32_t window,
                double* y_out, int32_t* status_out) {
    std::lock_guard<std::mutex> lk(ctx->call_mu);
    ctx->err.clear();
    int rc = check_batch(ctx, b, false);
    if (rc) return rc;
    if (!periods || !y_out || window < 1) {
        set_err(ctx, "periods and y_out must not be NULL and window must be >= 1");
        return QMI_EINVAL;
    }
    const int32_t nc = b->n_curves;
    if (nc == 0) return QMI_OK;
    const int64_t ns = b->offsets[nc];
    std::vector<int32_t> st_in(nc);
    for (int32_t k = 0; k < nc; ++k) {
        st_in[k] = host_curve_status(b, k, true);
        if (!(periods[k] > 0.0) || !std::isfinite(periods[k])) st_in[k] = QMI_EINVAL;
    }
    HIP_OK(ctx, hipSetDevice(ctx->device));
    begin_use(ctx);
    int max_n = 0;
    if ((rc = upload_batch(ctx, b, st_in, &max_n)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPYo, std::max<int64_t>(ns, 1) * 8)) != QMI_OK) return rc;
    if ((rc = ensure(ctx, qmi_ctx::kPPer, nc * 8)) != QMI_OK) return rc;
    hipStream_t st = ctx->stream;
    double* dper = dptr<double>(ctx, qmi_ctx::kPPer);
    double* dy = dptr<double>(ctx, qmi_ctx::kPYo);
    HIP_OK(ctx, hipMemcpyAsync(dper, periods, nc * 8, hipMemcpyHostToDevice, st));
    HIP_OK(ctx, launch_whiten(st, nc, max_n, dptr<int64_t>(ctx, qmi_ctx::kPOff),
                              dptr<double>(ctx, qmi_ctx::kT), dptr<double>(ctx, qmi_ctx::kY), dper,
                              window, dptr<int32_t>(ctx, qmi_ctx::kPStIn), dy));
    HIP_OK(ctx, hipMemcpyAsync(y_out, dy, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(ctx, hipStreamSynchronize(st));
    for (int32_t k = 0; k < nc; ++k) {
        if (st_in[k] != QMI_OK)
            for (int64_t i = b->offsets[k]; i < b->offsets[k + 1]; ++i) y_out[i] = NAN;
        if (status_out) status_out[k] = st_in[k];
    }
    return QMI_OK;
}

}  // namespace

int qmi_preprocess(qmi_ctx* ctx, const qmi_batch* batch, const qmi_preprocess_params* params,
                   int64_t* offsets_out, double* t_out, double* y_out, double* e_out,
                   int32_t* status_out, uint8_t* detrended_out) {
    if (!ctx) return QMI_EINVAL;
    try {
        return preprocess_call(ctx, batch, params, offsets_out, t_out, y_out, e_out, status_out,
                               detrended_out);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_whiten(qmi_ctx* ctx, const qmi_batch* batch, const double* periods, int32_t window,
               double* y_out, int32_t* status_out) {
    if (!ctx) return QMI_EINVAL;
    try {
        return whiten_call(ctx, batch, periods, window, y_out, status_out);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_best_period_dev(qmi_ctx* ctx, const qmi_batch* batch, const qmi_kernel_params* kp,
                        const qmi_search* search, qmi_result* out, double* coarse_out) {
    if (!ctx) return QMI_EINVAL;
    CallSpec cs{};
    cs.dev_inputs = true;
    cs.dev_outputs = true;
    cs.periodogram = false;
    cs.kp = kp;
    cs.search = search;
    cs.out = out;
    cs.coarse_out = coarse_out;
    try {
        return run_call(ctx, batch, cs);
    } catch (...) {
        set_err(ctx, "internal exception");
        return QMI_EINTERNAL;
    }
}

int qmi_discriminate(const qmi_result* best, int32_t n_curves, const double* psnr,
                     const qmi_thresholds* th, uint8_t* is_periodic) {
    if (n_curves < 0 || !th || !th->edges || !th->th || th->n_bins < 1 ||
        (th->score != QMI_SCORE_CS_QMI && th->score != QMI_SCORE_NCKP))
        return QMI_EINVAL;
    if (n_curves > 0 && (!best || !is_periodic)) return QMI_EINVAL;
    for (int32_t b = 0; b < th->n_bins; ++b)
        if (!(th->edges[b] <= th->edges[b + 1])) return QMI_EINVAL;
    for (int32_t k = 0; k < n_curves; ++k) {
        const qmi_result& r = best[k];
        const double p = psnr ? psnr[k] : r.psnr;
        const double s = th->score == QMI_SCORE_CS_QMI ? r.score_qmi : r.score_nckp;
        uint8_t v = QMI_UNDECIDED;
        if (r.status == QMI_OK && std::isfinite(s) && p == p) {
            for (int32_t b = 0; b < th->n_bins; ++b)
                if (th->edges[b] <= p && p < th->edges[b + 1]) {
                    v = s > th->th[b] ? QMI_PERIODIC : QMI_NOT_PERIODIC;
                    break;
                }
        }
        is_periodic[k] = v;
    }
    return QMI_OK;
}

int qmi_calibrate(const double* scores, const double* psnr, const uint8_t* truth, int32_t n,
                  const double* edges, int32_t n_bins, int32_t n_points, double* th_out,
                  double* f1_out, double* precision_out, double* recall_out) {
    if (n < 0 || n_bins < 1 || n_points < 1 || !edges || !th_out) return QMI_EINVAL;
    if (n > 0 && (!scores || !psnr || !truth)) return QMI_EINVAL;
    for (int32_t b = 0; b < n_bins; ++b)
        if (!(edges[b] <= edges[b + 1])) return QMI_EINVAL;
    std::vector<double> s;
    std::vector<uint8_t> lab;
    for (int32_t b = 0; b < n_bins; ++b) {
        s.clear();
        lab.clear();
        for (int32_t k = 0; k < n; ++k) {
            const double p = psnr[k];
            if (edges[b] <= p && p < edges[b + 1] && scores[k] == scores[k]) {
                s.push_back(scores[k]);
                lab.push_back(truth[k] ? 1 : 0);
            }
        }
        double th = INFINITY, f1 = 0.0, pr = 0.0, rc = 0.0;
        if (!s.empty()) {
            const double lo = *std::min_element(s.begin(), s.end());
            const double hi = *std::max_element(s.begin(), s.end());
            int64_t pos = 0;
            for (uint8_t v : lab) pos += v;
            if (pos == 0) {
                th = hi;
            } else {
                // Sort by score so each threshold's counts come from one pointer sweep.
                std::vector<size_t> idx(s.size());
                for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
                std::sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return s[a] < s[c]; });
                const double step = n_points > 1 ? (hi - lo) / (double)(n_points - 1) : 0.0;
                size_t below = 0;       // curves with score <= threshold
                int64_t pos_below = 0;  // periodic curves among them
                bool have = false;
                for (int32_t j = 0; j < n_points; ++j) {
                    const double c = n_points > 1 ? lo + (double)j * step : lo;
                    while (below < idx.size() && s[idx[below]] <= c) {
                        pos_below += lab[idx[below]];
                        ++below;
                    }
                    const int64_t tp = pos - pos_below;
                    const int64_t fp = (int64_t)(idx.size() - below) - tp;
                    const int64_t fn = pos_below;
                    const double p = (tp + fp) ? (double)tp / (double)(tp + fp) : 0.0;
                    const double r = (tp + fn) ? (double)tp / (double)(tp + fn) : 0.0;
                    const double den = 1.0 * p + r;
                    const double f = den == 0.0 ? 0.0 : 2.0 * p * r / den;
                    if (!have || f > f1) {
                        have = true;
                        f1 = f;
                        th = c;
                        pr = p;
                        rc = r;
                    }
                }
            }
        }
        th_out[b] = th;
        if (f1_out) f1_out[b] = f1;
        if (precision_out) precision_out[b] = pr;
        if (recall_out) recall_out[b] = rc;
    }
    return QMI_OK;
}

int qmi_serve_start(qmi_ctx* ctx, const qmi_kernel_params* kp, const qmi_search* search,
                    size_t admit_budget_bytes, int32_t max_batch, int32_t max_inflight) {
    if (!ctx || !kp || !search || max_batch < 1 || max_inflight < 1 || max_inflight > 8)
        return QMI_EINVAL;
    if (ctx->serve) {
        set_err(ctx, "serving already started");
        return QMI_EINVAL;
    }
    int rc = check_kernel_params(ctx, kp);
    if (rc) return rc;
    auto S = std::make_unique<qmi_ctx::Serve>();
    S->kp = *kp;
    S->search = *search;
    S->admit_budget = admit_budget_bytes ? admit_budget_bytes : ctx->budget / 2;
    S->max_batch = max_batch;
    S->max_inflight = max_inflight;
    S->max_items = ctx->serve_batch_items > 0 ? (double)ctx->serve_batch_items : 0.0;
    const size_t lane_budget = ctx->budget / (size_t)max_inflight;
    for (int i = 0; i < max_inflight; ++i) {
        qmi_ctx* lc = nullptr;
        rc = qmi_create(&lc, ctx->device, lane_budget, nullptr);
        if (rc) {
            set_err(ctx, "serving lane %d: %s", i, qmi_last_error(nullptr));
            for (qmi_ctx* c : S->lanes) qmi_destroy(c);
            return rc;
        }
        // Serving batches differ in composition, so a captured graph would almost never be
        // replayed: the lanes launch eagerly.
        lc->use_graph = false;
        lc->masks = ctx->masks;
        S->lanes.push_back(lc);
    }
    ctx->serve = std::move(S);
    for (int i = 0; i < max_inflight; ++i)
        ctx->serve->workers.emplace_back(serve_worker, ctx, i);
    return QMI_OK;
}

int qmi_submit(qmi_ctx* ctx, const double* t, const double* y, const double* e, int32_t n,
               uint64_t tag) {
    if (!ctx || !t || !y || n < 0) return QMI_EINVAL;
    qmi_ctx::Serve* S = ctx->serve.get();
    if (!S) {
        set_err(ctx, "serving not started");
        return QMI_EINVAL;
    }
    const size_t rb = request_bytes(S->search, n);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return QMI_EINVAL;
        if (S->queued_bytes + rb > S->admit_budget && !S->queue.empty()) return QMI_EAGAIN;
        qmi_ctx::Serve::Req r;
        r.t.assign(t, t + n);
        r.y.assign(y, y + n);
        if (e) {
            r.e.assign(e, e + n);
            r.has_e = true;
        }
        r.tag = tag;
        r.items = 0.5 * (double)n * (double)(n - 1) *
                  ((double)S->search.n_coarse + (double)S->search.top_k * S->search.n_fine);
        S->queue.push_back(std::move(r));
        S->queued_bytes += rb;
    }
    S->cv.notify_one();
    return QMI_OK;
}

int qmi_poll(qmi_ctx* ctx, qmi_result* out, uint64_t* tags, int32_t max, int32_t timeout_us) {
    if (!ctx || max < 0 || (max > 0 && (!out || !tags))) return QMI_EINVAL;
    qmi_ctx::Serve* S = ctx->serve.get();
    if (!S) return QMI_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_us > 0)
        S->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us),
                            [&] { return !S->done.empty(); });
    int32_t k = 0;
    while (k < max && !S->done.empty()) {
        out[k] = S->done.front().r;
        tags[k] = S->done.front().tag;
        S->done.pop_front();
        ++k;
    }
    return k;
}

int qmi_serve_stop(qmi_ctx* ctx) {
    if (!ctx || !ctx->serve) return QMI_EINVAL;
    qmi_ctx::Serve* S = ctx->serve.get();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto& th : S->workers) th.join();
    for (qmi_ctx* c : S->lanes) qmi_destroy(c);
    ctx->serve.reset();
    return QMI_OK;
}

}  // extern "C"
