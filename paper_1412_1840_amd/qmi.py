"""Python binding of libqmi (the C ABI in include/qmi.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts numpy arrays or
torch tensors to pointers and back.  It raises if libqmi.so has not been built - there is no
fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmi.so")

OK = 0
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
EDEGENERATE = -4
EAGAIN = -5
EINTERNAL = -6

SIGMA_SILVERMAN = -1.0
SIGMA_MEDIAN_ERR = -2.0
SIGMA_T_SKEWNESS = -1.0
SKEW_LAMBDA = 0.1
SKEW_MU = 12.0
SCORE_QMI = 0
SCORE_NCKP = 1
PREC_MIXED = 0
PREC_FP64 = 1
PREC_FOLD32 = 2  # precision control only: phase fold in FP32
OPT_USE_GRAPH = 1
OPT_TILE = 2
OPT_SERVE_BATCH_ITEMS = 4
NOT_PERIODIC, PERIODIC, UNDECIDED = 0, 1, 255
MAX_N = 8192
MAX_TOPK = 32
MAX_BANDS = 32
MAX_TRIALS = 1024
MAX_MASKS = 32
NOALLOC_SCRATCH_BYTES = 64 << 20

SYMBOLS = ("qmi_create", "qmi_destroy", "qmi_last_error", "qmi_set_option", "qmi_get_stats",
           "qmi_periodogram", "qmi_best_period", "qmi_periodogram_dev", "qmi_best_period_dev",
           "qmi_periodogram_noalloc",
           "qmi_discriminate", "qmi_calibrate", "qmi_serve_start", "qmi_submit", "qmi_poll",
           "qmi_serve_stop", "qmi_bands_best_period", "qmi_preprocess", "qmi_whiten",
           "qmi_set_masks")
SNR_EDGES = (0.0, 1.5, 2.0, 2.5, 3.5, 5.0, 10.0, 20.0, math.inf)


class QMIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libqmi error %d: %s" % (code, msg))
        self.code = code


class Batch(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("t", ctypes.c_void_p), ("y", ctypes.c_void_p), ("e", ctypes.c_void_p)]


class KernelParams(ctypes.Structure):
    _fields_ = [("sigma_t", ctypes.c_double), ("sigma_y", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("skew_lambda", ctypes.c_double), ("skew_mu", ctypes.c_double)]


class Search(ctypes.Structure):
    _fields_ = [("f_min", ctypes.c_double), ("f_max", ctypes.c_double),
                ("n_coarse", ctypes.c_int32), ("top_k", ctypes.c_int32),
                ("n_fine", ctypes.c_int32), ("score", ctypes.c_int32)]


class Bands(ctypes.Structure):
    _fields_ = [("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double),
                ("n_grid", ctypes.c_int32), ("n_bands", ctypes.c_int32),
                ("n_keep", ctypes.c_int32), ("n_trials", ctypes.c_int32),
                ("score", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PreprocessParams(ctypes.Structure):
    _fields_ = [("error_cut", ctypes.c_int32), ("min_samples", ctypes.c_int32),
                ("detrend", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Mask(ctypes.Structure):
    _fields_ = [("period", ctypes.c_double), ("sigma", ctypes.c_double),
                ("amplitude", ctypes.c_double)]


# Centres of the spurious-period masks of Sec. 6.1 (days), in the order of the paper's table: the
# solar day, the synodic month, the tropical year, the survey's mean span, then their aliases.
SPURIOUS_PERIODS = (1.0, 29.5305, 365.24, 2335.0, 0.4917, 0.5086, 0.9672, 1.0351, 0.9973,
                    1.0027, 27.31, 32.13, 315.65, 432.63)


def spurious_masks(amplitude: float, span: float = 2335.0, width: float = 0.5):
    """(period, sigma, amplitude) for every period of the table of Sec. 6.1.  The paper does not
    publish its widths and amplitudes; sigma = width * P^2 / span is `width` Fourier resolution
    elements 1/span mapped to period, and the amplitude is in units of the searched score."""
    return [(p, width * p * p / span, float(amplitude)) for p in SPURIOUS_PERIODS]


class Thresholds(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("score", ctypes.c_int32),
                ("edges", ctypes.POINTER(ctypes.c_double)), ("th", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("pair_kernel_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("pair_items", ctypes.c_double), ("pair_launches", ctypes.c_int32),
                ("used_graph", ctypes.c_int32), ("pair_variant", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


RESULT_DTYPE = np.dtype([("f_best", "f8"), ("period", "f8"), ("score", "f8"), ("score_qmi", "f8"),
                         ("score_nckp", "f8"), ("sigma_y", "f8"), ("psnr", "f8"),
                         ("coarse_best", "f8"), ("coarse_index", "i4"), ("peak_rank", "i4"),
                         ("fine_index", "i4"), ("coarse_argmax", "i4"), ("n_peaks", "i4"),
                         ("n", "i4"), ("status", "i4"), ("reserved", "i4"),
                         ("sigma_t", "f8")])
assert RESULT_DTYPE.itemsize == 104

_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded libqmi.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # When PyTorch is present its HIP runtime must be the one in the process: load it first so
        # that libqmi binds to the same libamdhip64 (two runtimes in one process do not share
        # devices).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqmi.so is not built (%s); run python -m "
                               "paper_1412_1840_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, V, I32, I64, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.qmi_create.argtypes = [P(V), ctypes.c_int, ctypes.c_size_t, V]
        L.qmi_create.restype = ctypes.c_int
        L.qmi_destroy.argtypes = [V]
        L.qmi_destroy.restype = None
        L.qmi_last_error.argtypes = [V]
        L.qmi_last_error.restype = ctypes.c_char_p
        L.qmi_set_option.argtypes = [V, I32, I64]
        L.qmi_get_stats.argtypes = [V, P(Stats)]
        L.qmi_set_masks.argtypes = [V, V, I32]
        L.qmi_set_masks.restype = ctypes.c_int
        for name in ("qmi_periodogram", "qmi_periodogram_dev", "qmi_periodogram_noalloc"):
            f = getattr(L, name)
            f.argtypes = [V, P(Batch), P(KernelParams), V, I32, I32, V, V, V, V]
            f.restype = ctypes.c_int
        for name in ("qmi_best_period", "qmi_best_period_dev"):
            f = getattr(L, name)
            f.argtypes = [V, P(Batch), P(KernelParams), P(Search), V, V]
            f.restype = ctypes.c_int
        L.qmi_bands_best_period.argtypes = [V, P(Batch), P(KernelParams), P(Bands), V, V, V]
        L.qmi_bands_best_period.restype = ctypes.c_int
        L.qmi_preprocess.argtypes = [V, P(Batch), P(PreprocessParams), V, V, V, V, V, V]
        L.qmi_preprocess.restype = ctypes.c_int
        L.qmi_whiten.argtypes = [V, P(Batch), V, I32, V, V]
        L.qmi_whiten.restype = ctypes.c_int
        L.qmi_discriminate.argtypes = [V, I32, V, P(Thresholds), V]
        L.qmi_discriminate.restype = ctypes.c_int
        L.qmi_calibrate.argtypes = [V, V, V, I32, V, I32, I32, V, V, V, V]
        L.qmi_calibrate.restype = ctypes.c_int
        L.qmi_serve_start.argtypes = [V, P(KernelParams), P(Search), ctypes.c_size_t, I32, I32]
        L.qmi_submit.argtypes = [V, V, V, V, I32, ctypes.c_uint64]
        L.qmi_poll.argtypes = [V, V, V, I32, I32]
        L.qmi_serve_stop.argtypes = [V]
        _LIB = L
    return _LIB


def _addr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel_params(sigma_t: float, sigma_y: float = SIGMA_SILVERMAN,
                  precision: int = PREC_MIXED, skew_lambda: float = SKEW_LAMBDA,
                  skew_mu: float = SKEW_MU) -> KernelParams:
    """sigma_t > 0 explicit, or SIGMA_T_SKEWNESS with the rule's constants."""
    return KernelParams(float(sigma_t), float(sigma_y), int(precision), 0, float(skew_lambda),
                        float(skew_mu))


def search(f_min: float, f_max: float, n_coarse: int, top_k: int = 10, n_fine: int = 1000,
           score: int = SCORE_QMI) -> Search:
    return Search(float(f_min), float(f_max), int(n_coarse), int(top_k), int(n_fine), int(score))


def discriminate(results: np.ndarray, edges: Sequence[float], th: Sequence[float],
                 score: int = SCORE_QMI, psnr: Optional[np.ndarray] = None) -> np.ndarray:
    """Periodic / non-periodic / undecided per curve (host-only; needs no device)."""
    res = np.ascontiguousarray(results, dtype=RESULT_DTYPE)
    e = _f64(edges)
    t = _f64(th)
    if len(e) != len(t) + 1:
        raise ValueError("edges must have one more entry than th")
    T = Thresholds(len(t), int(score), e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    out = np.zeros(len(res), np.uint8)
    p = None if psnr is None else _f64(psnr)
    rc = lib().qmi_discriminate(res.ctypes.data, len(res), _addr(p), ctypes.byref(T),
                                out.ctypes.data)
    if rc != OK:
        raise QMIError(rc, "bad threshold table")
    return out


def calibrate(scores, psnr, truth, edges: Sequence[float] = SNR_EDGES, n_points: int = 5000):
    """Per-bin F1-maximising thresholds (host-only): dict of th, f1, precision, recall."""
    sc = _f64(scores)
    ps = _f64(psnr)
    tr = np.ascontiguousarray(truth, dtype=np.uint8)
    e = _f64(edges)
    nb = len(e) - 1
    out = {k: np.zeros(nb) for k in ("th", "f1", "precision", "recall")}
    rc = lib().qmi_calibrate(sc.ctypes.data, ps.ctypes.data, tr.ctypes.data, len(sc), e.ctypes.data,
                             nb, int(n_points), out["th"].ctypes.data, out["f1"].ctypes.data,
                             out["precision"].ctypes.data, out["recall"].ctypes.data)
    if rc != OK:
        raise QMIError(rc, "bad calibration arguments")
    return out


class Context:
    """A libqmi context on one HIP device (its own stream unless ``stream`` is given)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream: Optional[int] = None):
        h = ctypes.c_void_p()
        rc = lib().qmi_create(ctypes.byref(h), int(device), int(budget_bytes),
                              ctypes.c_void_p(stream) if stream else None)
        if rc != OK:
            raise QMIError(rc, lib().qmi_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().qmi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int):
        if rc != OK:
            raise QMIError(rc, lib().qmi_last_error(self._h).decode())

    def set_option(self, option: int, value: int):
        self._check(lib().qmi_set_option(self._h, int(option), int(value)))

    def set_masks(self, masks=None):
        """Spurious-period masks [(period, sigma, amplitude), ...] for the searches that follow
        (None or [] removes them)."""
        masks = list(masks or [])
        arr = (Mask * max(len(masks), 1))(*[Mask(*map(float, m)) for m in masks])
        self._check(lib().qmi_set_masks(self._h, ctypes.addressof(arr) if masks else None,
                                        len(masks)))

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().qmi_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    # ---------------------------------------------------------------- host arrays
    @staticmethod
    def _batch(offsets, t, y, e):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        b = Batch(len(off) - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                  _addr(t), _addr(y), _addr(e))
        return b, off

    def periodogram(self, offsets, t, y, e, freqs, sigma_t: float,
                    sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                    precision: int = PREC_MIXED, want_ips: bool = False):
        """Scores [n_curves, n_freq] (and V_J, IP_t, V_C [n_curves, n_freq, 3], IP_y, status)."""
        t, y = _f64(t), _f64(y)
        e = None if e is None else _f64(e)
        f = _f64(freqs)
        b, off = self._batch(offsets, t, y, e)
        nc = b.n_curves
        out = np.empty((nc, len(f)))
        ips = np.empty((nc, len(f), 3)) if want_ips else None
        ipy = np.empty(nc)
        st = np.empty(nc, np.int32)
        kp = kernel_params(sigma_t, sigma_y, precision)
        self._check(lib().qmi_periodogram(self._h, ctypes.byref(b), ctypes.byref(kp), f.ctypes.data,
                                          len(f), int(score), out.ctypes.data, _addr(ips),
                                          ipy.ctypes.data, st.ctypes.data))
        return out, ips, ipy, st

    def best_period(self, offsets, t, y, e, sigma_t: float, f_min: float, f_max: float,
                    n_coarse: int, top_k: int = 10, n_fine: int = 1000,
                    sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                    precision: int = PREC_MIXED, want_coarse: bool = False):
        t, y = _f64(t), _f64(y)
        e = None if e is None else _f64(e)
        b, off = self._batch(offsets, t, y, e)
        res = np.zeros(b.n_curves, RESULT_DTYPE)
        coarse = np.empty((b.n_curves, n_coarse)) if want_coarse else None
        kp = kernel_params(sigma_t, sigma_y, precision)
        s = search(f_min, f_max, n_coarse, top_k, n_fine, score)
        self._check(lib().qmi_best_period(self._h, ctypes.byref(b), ctypes.byref(kp),
                                          ctypes.byref(s), res.ctypes.data, _addr(coarse)))
        return res, coarse

    # ------------------------------------------------------- device (torch) tensors
    def bands_best_period(self, offsets, t, y, e, sigma_t: float, n_keep: int = 3,
                          n_trials: int = 150, n_bands: int = 10, f_lo: float = 0.00125,
                          f_hi: float = 3.0, n_grid: int = 30000,
                          sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                          precision: int = PREC_MIXED):
        """Best period over the bands method's trial frequencies: (results, trials, scores),
        trials and scores of shape [n_curves, n_keep * n_trials] (NaN: empty)."""
        t, y = _f64(t), _f64(y)
        e = None if e is None else _f64(e)
        b, off = self._batch(offsets, t, y, e)
        res = np.zeros(b.n_curves, RESULT_DTYPE)
        trials = np.empty((b.n_curves, n_keep * n_trials))
        scores = np.empty((b.n_curves, n_keep * n_trials))
        kp = kernel_params(sigma_t, sigma_y, precision)
        bp = Bands(float(f_lo), float(f_hi), int(n_grid), int(n_bands), int(n_keep),
                   int(n_trials), int(score), 0)
        self._check(lib().qmi_bands_best_period(self._h, ctypes.byref(b), ctypes.byref(kp),
                                                ctypes.byref(bp), res.ctypes.data,
                                                trials.ctypes.data, scores.ctypes.data))
        return res, trials, scores

    def preprocess(self, offsets, t, y, e, error_cut: bool = True, min_samples: int = 50,
                   detrend: bool = True):
        """Sec. 5.2 preprocessing: (offsets, t, y, e, status, detrended) of the new batch."""
        t, y = _f64(t), _f64(y)
        e = None if e is None else _f64(e)
        b, off = self._batch(offsets, t, y, e)
        nc = b.n_curves
        oo = np.zeros(nc + 1, np.int64)
        to, yo = np.empty(len(t)), np.empty(len(t))
        eo = None if e is None else np.empty(len(t))
        st = np.zeros(nc, np.int32)
        det = np.zeros(nc, np.uint8)
        pp = PreprocessParams(int(bool(error_cut)), int(min_samples), int(bool(detrend)), 0)
        self._check(lib().qmi_preprocess(self._h, ctypes.byref(b), ctypes.byref(pp), oo.ctypes.data,
                                         to.ctypes.data, yo.ctypes.data, _addr(eo), st.ctypes.data,
                                         det.ctypes.data))
        m = int(oo[-1])
        return oo, to[:m], yo[:m], (None if eo is None else eo[:m]), st, det.astype(bool)

    def whiten(self, offsets, t, y, periods, window: int = 30):
        """Sec. 7.1 whitening at the given per-curve periods: (y_whitened, status)."""
        t, y = _f64(t), _f64(y)
        b, off = self._batch(offsets, t, y, None)
        p = _f64(periods)
        if len(p) != b.n_curves:
            raise ValueError("one period per curve")
        out = np.empty(len(y))
        st = np.zeros(b.n_curves, np.int32)
        self._check(lib().qmi_whiten(self._h, ctypes.byref(b), p.ctypes.data, int(window),
                                     out.ctypes.data, st.ctypes.data))
        return out, st

    def periodogram_dev(self, offsets, t, y, e, freqs, score_out, sigma_t: float,
                        sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                        precision: int = PREC_MIXED, ips_out=None):
        """t, y, e, freqs, score_out, ips_out: float64 CUDA tensors; offsets on the host."""
        b, off = self._batch(offsets, t, y, e)
        ipy = np.empty(b.n_curves)
        st = np.empty(b.n_curves, np.int32)
        kp = kernel_params(sigma_t, sigma_y, precision)
        self._check(lib().qmi_periodogram_dev(self._h, ctypes.byref(b), ctypes.byref(kp),
                                              _addr(freqs), int(freqs.numel()), int(score),
                                              _addr(score_out), _addr(ips_out), ipy.ctypes.data,
                                              st.ctypes.data))
        return ipy, st

    def periodogram_noalloc(self, offsets, t, y, e, freqs, score_out, sigma_t: float,
                            sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                            precision: int = PREC_MIXED, ips_out=None):
        """periodogram_dev computed in the library's fixed scratch area (no device allocation
        during the call; at most NOALLOC_SCRATCH_BYTES of intermediate tables)."""
        b, off = self._batch(offsets, t, y, e)
        ipy = np.empty(b.n_curves)
        st = np.empty(b.n_curves, np.int32)
        kp = kernel_params(sigma_t, sigma_y, precision)
        self._check(lib().qmi_periodogram_noalloc(self._h, ctypes.byref(b), ctypes.byref(kp),
                                                  _addr(freqs), int(freqs.numel()), int(score),
                                                  _addr(score_out), _addr(ips_out),
                                                  ipy.ctypes.data, st.ctypes.data))
        return ipy, st

    def best_period_dev(self, offsets, t, y, e, sigma_t: float, f_min: float, f_max: float,
                        n_coarse: int, top_k: int = 10, n_fine: int = 1000,
                        sigma_y: float = SIGMA_SILVERMAN, score: int = SCORE_QMI,
                        precision: int = PREC_MIXED, coarse_out=None):
        b, off = self._batch(offsets, t, y, e)
        res = np.zeros(b.n_curves, RESULT_DTYPE)
        kp = kernel_params(sigma_t, sigma_y, precision)
        s = search(f_min, f_max, n_coarse, top_k, n_fine, score)
        self._check(lib().qmi_best_period_dev(self._h, ctypes.byref(b), ctypes.byref(kp),
                                              ctypes.byref(s), res.ctypes.data,
                                              _addr(coarse_out)))
        return res

    # ------------------------------------------------------------------- serving
    def serve_start(self, sigma_t: float, f_min: float = 1e-3, f_max: float = 10.0,
                    n_coarse: int = 20000,
                    top_k: int = 10, n_fine: int = 1000, sigma_y: float = SIGMA_SILVERMAN,
                    score: int = SCORE_QMI, admit_budget_bytes: int = 0, max_batch: int = 256,
                    max_inflight: int = 2, max_batch_items: float = 0):
        """max_batch_items > 0 bounds each launch's pair x frequency items."""
        self.set_option(OPT_SERVE_BATCH_ITEMS, int(max_batch_items))
        kp = kernel_params(sigma_t, sigma_y, PREC_MIXED)
        s = search(f_min, f_max, n_coarse, top_k, n_fine, score)
        self._check(lib().qmi_serve_start(self._h, ctypes.byref(kp), ctypes.byref(s),
                                          int(admit_budget_bytes), int(max_batch),
                                          int(max_inflight)))

    def submit(self, t, y, e, tag: int) -> bool:
        """True if admitted, False if the admission budget is full (try again later)."""
        t, y = _f64(t), _f64(y)
        e = None if e is None else _f64(e)
        rc = lib().qmi_submit(self._h, t.ctypes.data, y.ctypes.data, _addr(e), len(t), int(tag))
        if rc == EAGAIN:
            return False
        self._check(rc)
        return True

    def poll(self, max_results: int = 256, timeout_us: int = 0):
        res = np.zeros(max_results, RESULT_DTYPE)
        tags = np.zeros(max_results, np.uint64)
        k = lib().qmi_poll(self._h, res.ctypes.data, tags.ctypes.data, int(max_results),
                           int(timeout_us))
        if k < 0:
            self._check(k)
        return res[:k], tags[:k]

    def serve_stop(self):
        self._check(lib().qmi_serve_stop(self._h))
