"""Test infrastructure only: the plain FP64 CPU oracle of the kernelised-periodogram period search.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import this module.  It
shares no code with the HIP library (``paper_1412_1840_amd``) and never imports it.

Citations are to Protopapas et al., "A novel, fully automated pipeline for period estimation in
the EROS 2 data set" (arXiv:1412.1840).  The pair sums are in ``qmi_oracle.c``; this module holds
the kernel-width rules, the score formulas, the coarse-to-fine search and the discriminator, each
written plainly in FP64 from its definition.

Readings of points the paper leaves open (kept identical in the HIP library, which implements them
separately):

* the score searched by default is the Cauchy-Schwarz quadratic mutual information built from the
  same pair sums as the CKP (Sec. 3): QMI = ln V_J + ln V_M - 2 ln V_C;
* sums include the diagonal i = j, as the CKP definition (Sec. 3) is written;
* sigma_y defaults to Silverman's rule 0.9 min(s, IQR/1.34) N^(-1/5) with s on N-1 and
  linear-interpolation quartiles; IQR = 0 falls back to s; s = 0 is degenerate.  The paper's own
  rule sigma_y = median(error bars) (Sec. 3) is the alternative;
* sigma_t is a caller value, or the skewness rule of Sec. 3 with the quartiles of its footnote
  (halves without the middle value for odd N) and S = 0 when Q3 = Q1;
* peaks of the coarse periodogram are its local maxima (q_k > q_{k-1} and q_k >= q_{k+1}; the first
  point needs q_0 >= q_1, the last q_{F-1} > q_{F-2}), ranked by value with ties to lower k;
* each kept peak k is refined on n_fine evenly spaced points of [f_{k-1}, f_{k+1}] (clamped to the
  grid's ends); the best is the highest refined score, ties to the lower frequency, then the lower
  peak rank;
* pSNR = 0.7413 iqr(y) / (alpha median(e)) with alpha = 1 (Sec. 5.2); the eight SNR bins of the
  threshold table of Sec. 4.1 are half-open [a, b); a curve is periodic iff score > th(bin).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SIGMA_SILVERMAN = -1.0
SIGMA_MEDIAN_ERR = -2.0
SCORE_QMI = 0
SCORE_NCKP = 1

SNR_EDGES = (0.0, 1.5, 2.0, 2.5, 3.5, 5.0, 10.0, 20.0, math.inf)
UNDECIDED = 255


class Degenerate(ValueError):
    """The kernel-width rule gives zero (e.g. all magnitudes equal)."""


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        src = os.path.join(HERE, "qmi_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            from . import build_oracle  # noqa: WPS433  (builds the checker, test-side only)
            build_oracle.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_batch_ips.argtypes = [ctypes.c_int64, P(ctypes.c_int64), P(ctypes.c_double),
                                         P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                         P(ctypes.c_int64), P(ctypes.c_double), ctypes.c_int,
                                         P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                         P(ctypes.c_double), ctypes.c_int]
        lib.oracle_batch_ips.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def threads(n_threads: int = 0) -> int:
    return int(_lib().oracle_threads(int(n_threads)))


# ------------------------------------------------------------------------------------------
# Order statistics (written out; linear interpolation between order statistics)
# ------------------------------------------------------------------------------------------

def quantile(x: np.ndarray, p: float) -> float:
    """Quantile by linear interpolation between the order statistics at position (N-1) p."""
    s = sorted(float(v) for v in x)
    n = len(s)
    h = (n - 1) * p
    lo = int(math.floor(h))
    hi = min(lo + 1, n - 1)
    return s[lo] + (h - lo) * (s[hi] - s[lo])


def median(x: np.ndarray) -> float:
    s = sorted(float(v) for v in x)
    n = len(s)
    if n % 2:
        return s[n // 2]
    return 0.5 * (s[n // 2 - 1] + s[n // 2])


def iqr(x: np.ndarray) -> float:
    return quantile(x, 0.75) - quantile(x, 0.25)


# ------------------------------------------------------------------------------------------
# Kernel widths (Sec. 3: sigma_y from the error bars; sigma_t a free parameter in [0.1, 0.6])
# ------------------------------------------------------------------------------------------

def silverman_sigma(y: np.ndarray) -> float:
    n = len(y)
    mean = sum(float(v) for v in y) / n
    s = math.sqrt(sum((float(v) - mean) ** 2 for v in y) / (n - 1)) if n > 1 else 0.0
    if s == 0.0:
        raise Degenerate("Silverman's rule: zero sample deviation")
    q = iqr(y)
    spread = s if q == 0.0 else min(s, q / 1.34)
    return 0.9 * spread * n ** (-0.2)


def sigma_y_of(y: np.ndarray, e: Optional[np.ndarray], rule: float) -> float:
    """sigma_y > 0 explicit; -1 Silverman; -2 median of the error bars (Sec. 3)."""
    if rule > 0:
        return float(rule)
    if rule == SIGMA_SILVERMAN:
        return silverman_sigma(y)
    if rule == SIGMA_MEDIAN_ERR:
        if e is None:
            raise ValueError("median-error-bar rule needs error bars")
        m = median(e)
        if not m > 0:
            raise Degenerate("median error bar is not positive")
        return m
    raise ValueError("unknown sigma_y rule %r" % rule)


# ------------------------------------------------------------------------------------------
# sigma_t from the skewness of the magnitudes (Sec. 3, the skewness rule and its quartile
# estimator of the skewness; in the paper's source text this passage is commented out, while the
# published text and the caption of its sigma_t example figure still describe the per-curve choice)
# ------------------------------------------------------------------------------------------

SIGMA_T_SKEWNESS = -1.0
SKEW_LAMBDA = 0.1  # the constants the paper reports for EROS-2
SKEW_MU = 12.0


def hinge_quartiles(x: np.ndarray) -> Tuple[float, float, float]:
    """Q1, Q2, Q3 as the paper's footnote defines them: Q2 is the median, Q1 and Q3 the medians of
    the first and second half of the rank-ordered values.  For odd N the middle value belongs to
    neither half (the halves are the N // 2 lowest and the N // 2 highest values)."""
    s = sorted(float(v) for v in x)
    n = len(s)
    h = n // 2
    if h == 0:
        return s[0], s[0], s[0]
    return median(s[:h]), median(s), median(s[n - h:])


def bowley_skewness(x: np.ndarray) -> float:
    """Quartile estimator of the skewness S = (Q3 + Q1 - 2 Q2) / (Q3 - Q1), in [-1, 1]; 0 when
    Q3 = Q1 (no spread between the quartiles; the estimator is then 0 / 0)."""
    q1, q2, q3 = hinge_quartiles(x)
    if q3 == q1:
        return 0.0
    return (q3 + q1 - 2.0 * q2) / (q3 - q1)


def sigma_t_skewness(y: np.ndarray, lam: float = SKEW_LAMBDA, mu: float = SKEW_MU) -> float:
    """sigma_t = lambda + 0.5 exp(-mu S^2): about lambda + 0.5 for symmetric magnitude
    distributions, down to lambda for very skewed ones (eclipsing binaries)."""
    S = bowley_skewness(y)
    return lam + 0.5 * math.exp(-mu * S * S)


def sigma_t_of(y: np.ndarray, sigma_t: float, lam: float = SKEW_LAMBDA,
               mu: float = SKEW_MU) -> float:
    """sigma_t > 0 explicit; SIGMA_T_SKEWNESS the skewness rule."""
    if sigma_t > 0:
        return float(sigma_t)
    if sigma_t == SIGMA_T_SKEWNESS:
        return sigma_t_skewness(y, lam, mu)
    raise ValueError("unknown sigma_t rule %r" % sigma_t)


# ------------------------------------------------------------------------------------------
# Information potentials and scores
# ------------------------------------------------------------------------------------------

@dataclass
class IPs:
    vj: np.ndarray  # joint information potential V_J(f)
    ipt: np.ndarray  # marginal information potential of the warped times IP_t(f)
    vc: np.ndarray  # cross information potential V_C(f)
    ipy: float  # marginal information potential of the magnitudes (Sec. 3)
    n: int
    sigma_t: float
    sigma_y: float


def information_potentials(t, y, sigma_t: float, sigma_y: float, freqs, mode: int = 1,
                           n_threads: int = 0) -> IPs:
    """V_J, IP_t, V_C at each frequency and IP_y, all pairs in FP64 (C part, ``mode`` 0 = plain
    double loop, 1 = i<j doubled plus the closed-form diagonal)."""
    res = batch_information_potentials([np.asarray(t, np.float64)], [np.asarray(y, np.float64)],
                                       [sigma_t], [sigma_y], [np.asarray(freqs, np.float64)],
                                       mode, n_threads)
    return res[0]


def batch_information_potentials(ts: Sequence[np.ndarray], ys: Sequence[np.ndarray],
                                 sigma_t: Sequence[float], sigma_y: Sequence[float],
                                 freqs: Sequence[np.ndarray], mode: int = 1,
                                 n_threads: int = 0) -> List[IPs]:
    nc = len(ts)
    offsets = np.zeros(nc + 1, np.int64)
    offsets[1:] = np.cumsum([len(x) for x in ts])
    foff = np.zeros(nc + 1, np.int64)
    foff[1:] = np.cumsum([len(f) for f in freqs])
    t = np.ascontiguousarray(np.concatenate(ts) if nc else np.zeros(0), np.float64)
    y = np.ascontiguousarray(np.concatenate(ys) if nc else np.zeros(0), np.float64)
    f = np.ascontiguousarray(np.concatenate(freqs) if nc else np.zeros(0), np.float64)
    st = np.ascontiguousarray(sigma_t, np.float64)
    sy = np.ascontiguousarray(sigma_y, np.float64)
    vj = np.zeros(len(f))
    ipt = np.zeros(len(f))
    vc = np.zeros(len(f))
    ipy = np.zeros(nc)
    D = ctypes.c_double
    rc = _lib().oracle_batch_ips(nc, _ptr(offsets, ctypes.c_int64), _ptr(t, D), _ptr(y, D),
                                 _ptr(st, D), _ptr(sy, D), _ptr(foff, ctypes.c_int64), _ptr(f, D),
                                 int(mode), _ptr(vj, D), _ptr(ipt, D), _ptr(vc, D), _ptr(ipy, D),
                                 int(n_threads))
    if rc != 0:
        raise ValueError("oracle_batch_ips failed (%d)" % rc)
    out = []
    for c in range(nc):
        a, b = foff[c], foff[c + 1]
        out.append(IPs(vj[a:b].copy(), ipt[a:b].copy(), vc[a:b].copy(), float(ipy[c]),
                       len(ts[c]), float(st[c]), float(sy[c])))
    return out


def qmi(ips: IPs) -> np.ndarray:
    """Cauchy-Schwarz QMI = ln(V_J V_M / V_C^2), V_M = IP_y IP_t, evaluated in FP64."""
    vm = ips.ipy * ips.ipt
    return np.log(ips.vj) + np.log(vm) - 2.0 * np.log(ips.vc)


def ckp(ips: IPs) -> np.ndarray:
    """CKP (Sec. 3) = (1/N^2) sum_ij (G_sy(dy) - IP_y) G^P = V_J - IP_y IP_t."""
    return ips.vj - ips.ipy * ips.ipt


def nckp(ips: IPs) -> np.ndarray:
    """Normalised CKP (Sec. 3): sqrt(N sigma_t) / IP_y * CKP."""
    return math.sqrt(ips.n * ips.sigma_t) / ips.ipy * ckp(ips)


def score_of(ips: IPs, score: int) -> np.ndarray:
    return qmi(ips) if score == SCORE_QMI else nckp(ips)


# ------------------------------------------------------------------------------------------
# Coarse-to-fine search (the CKP is maximised over frequency for fixed widths, Sec. 3; trial
# frequencies are the highest local maxima of a spectrum, as in the bands method of Sec. 3.1)
# ------------------------------------------------------------------------------------------

def linear_grid(f_lo: float, f_hi: float, n: int) -> np.ndarray:
    """n evenly spaced points, f_k = f_lo + k * ((f_hi - f_lo) / (n - 1)), from k (no running sum)."""
    if n == 1:
        return np.array([f_lo])
    step = (f_hi - f_lo) / (n - 1)
    return np.array([f_lo + float(k) * step for k in range(n)])


def local_maxima(q: np.ndarray) -> List[int]:
    F = len(q)
    if F == 1:
        return [0] if q[0] == q[0] else []
    peaks = []
    for k in range(F):
        if k == 0:
            ok = q[0] >= q[1]
        elif k == F - 1:
            ok = q[k] > q[k - 1]
        else:
            ok = q[k] > q[k - 1] and q[k] >= q[k + 1]
        if ok:
            peaks.append(k)
    return peaks


def top_peaks(q: np.ndarray, top_k: int) -> List[int]:
    peaks = local_maxima(q)
    peaks.sort(key=lambda k: (-q[k], k))
    return peaks[:top_k]


def fine_window(coarse: np.ndarray, k: int) -> Tuple[float, float]:
    """[f_{k-1}, f_{k+1}]; at the ends of the grid [f_0, f_1] and [f_{F-2}, f_{F-1}]."""
    F = len(coarse)
    if F == 1:
        return float(coarse[0]), float(coarse[0])
    if k == 0:
        return float(coarse[0]), float(coarse[1])
    if k == F - 1:
        return float(coarse[F - 2]), float(coarse[F - 1])
    return float(coarse[k - 1]), float(coarse[k + 1])


# ------------------------------------------------------------------------------------------
# Spurious-period filter (Sec. 6.1 and its table of spurious periods)
# ------------------------------------------------------------------------------------------
# Readings: a mask is a Gaussian in period, A exp(-(P - P_k)^2 / (2 sigma_k^2)), whose amplitude
# A is in units of the searched score; a candidate (period P = 1/f, score s) falls inside it when
# s < A exp(...), and a candidate inside any mask takes no part in the selection.  In the
# coarse-to-fine search that means: the coarse argmax, the local maxima kept for refinement (the
# local-maximum test itself still compares raw neighbours) and the best refined point are taken
# over candidates outside every mask; in the bands method the best trial is.  With no candidate
# left the result is empty (NaN).  The paper publishes the mask centres (its table) but not their
# widths or amplitudes; the default width below is our own: half of one Fourier resolution
# element 1/T of the survey span, mapped to period (sigma_k = 0.5 P_k^2 / T).

SOLAR_DAY = 1.0
SYNODIC_MONTH = 29.5305
TROPICAL_YEAR = 365.24
EROS_SPAN = 2335.0  # average time span of the survey's lightcurves (table of Sec. 6.1)

# The table of Sec. 6.1, in its order: the four base periods, then their aliases as printed.
SPURIOUS_PERIODS = (1.0, 29.5305, 365.24, 2335.0, 0.4917, 0.5086, 0.9672, 1.0351, 0.9973,
                    1.0027, 27.31, 32.13, 315.65, 432.63)


def spurious_masks(amplitude: float, span: float = EROS_SPAN,
                   width: float = 0.5) -> List[Tuple[float, float, float]]:
    """(P_k, sigma_k, A) for every period of the table, sigma_k = width P_k^2 / span."""
    return [(p, width * p * p / span, float(amplitude)) for p in SPURIOUS_PERIODS]


def in_mask(f: float, s: float, masks) -> bool:
    """True when the candidate (1/f, s) lies under any mask (Sec. 6.1)."""
    if not masks:
        return False
    P = math.inf if f == 0 else 1.0 / f
    for pk, sk, ak in masks:
        d = P - pk
        if s < ak * math.exp(-(d * d) / (2.0 * sk * sk)):
            return True
    return False


@dataclass
class SearchResult:
    f_best: float
    score: float  # the searched score at f_best
    qmi: float
    nckp: float
    coarse_index: int  # k of the refined peak that holds the best (or the coarse argmax)
    peak_rank: int
    fine_index: int
    coarse_argmax: int
    n_peaks: int
    sigma_y: float
    ipy: float
    coarse_scores: np.ndarray
    fine_scores: Optional[np.ndarray]  # [n_peaks, n_fine]
    peaks: Optional[List[int]] = None  # the refined peaks' k, in rank order


def best_period(t, y, e, sigma_t: float, sigma_y_rule: float, f_min: float, f_max: float,
                n_coarse: int, top_k: int, n_fine: int, score: int = SCORE_QMI,
                mode: int = 1, n_threads: int = 0, masks=()) -> SearchResult:
    """Coarse-to-fine search (Sec. 3, with the trial-selection rules listed at the top of this
    module); candidates under a spurious-period mask (Sec. 6.1) are left out of every selection.
    NaN scores never rank."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    sy = sigma_y_of(y, None if e is None else np.asarray(e, np.float64), sigma_y_rule)
    sigma_t = sigma_t_of(y, sigma_t)
    grid = linear_grid(f_min, f_max, n_coarse)
    ips = information_potentials(t, y, sigma_t, sy, grid, mode, n_threads)
    q = score_of(ips, score)
    q_all = (qmi(ips), nckp(ips))

    def usable(f, v):
        return v == v and not in_mask(f, v, masks)

    cand = [k for k in range(n_coarse) if usable(grid[k], q[k])]
    arg = min(cand, key=lambda k: (-q[k], k)) if cand else -1

    def coarse_result(n_peaks, fq, peaks=None):
        if arg < 0:
            return SearchResult(math.nan, math.nan, math.nan, math.nan, -1, -1, -1, -1, n_peaks,
                                sy, ips.ipy, q, fq, peaks)
        return SearchResult(float(grid[arg]), float(q[arg]), float(q_all[0][arg]),
                            float(q_all[1][arg]), arg, -1, -1, arg, n_peaks, sy, ips.ipy, q, fq,
                            peaks)

    if top_k <= 0 or n_fine <= 0:
        return coarse_result(0, None)
    peaks = [k for k in local_maxima(q) if usable(grid[k], q[k])]
    peaks.sort(key=lambda k: (-q[k], k))
    peaks = peaks[:top_k]
    if not peaks:
        return coarse_result(0, None)
    fine_f = [linear_grid(*fine_window(grid, k), n_fine) for k in peaks]
    fips = information_potentials(t, y, sigma_t, sy, np.concatenate(fine_f), mode, n_threads)
    fq = score_of(fips, score).reshape(len(peaks), n_fine)
    fq_all = (qmi(fips).reshape(len(peaks), n_fine), nckp(fips).reshape(len(peaks), n_fine))
    best = None
    for rank, k in enumerate(peaks):
        for m in range(n_fine):
            if not usable(fine_f[rank][m], fq[rank, m]):
                continue
            key = (-fq[rank, m], fine_f[rank][m], rank, m)
            if best is None or key < best[0]:
                best = (key, rank, m)
    if best is None:
        return coarse_result(len(peaks), fq, peaks)
    _, rank, m = best
    return SearchResult(float(fine_f[rank][m]), float(fq[rank, m]), float(fq_all[0][rank, m]),
                        float(fq_all[1][rank, m]), peaks[rank], rank, m, arg, len(peaks), sy,
                        ips.ipy, q, fq, peaks)


# ------------------------------------------------------------------------------------------
# Discrimination (Sec. 4.1 threshold procedure and decision rule; Sec. 5.2 pSNR; Sec. 3.2 scores)
# ------------------------------------------------------------------------------------------

def psnr(y: np.ndarray, e: np.ndarray, alpha: float = 1.0) -> float:
    """pseudo signal-to-noise ratio 0.7413 iqr(y) / (alpha med(e)) (Sec. 5.2)."""
    return 0.7413 * iqr(y) / (alpha * median(e))


def snr_bin(p: float, edges: Sequence[float] = SNR_EDGES) -> int:
    """Index b with edges[b] <= p < edges[b+1]; -1 when p is outside every bin or NaN."""
    for b in range(len(edges) - 1):
        if edges[b] <= p < edges[b + 1]:
            return b
    return -1


def discriminate(score: float, p: float, th: Sequence[float],
                 edges: Sequence[float] = SNR_EDGES) -> int:
    """1 if score > th(bin of p) (strict, Sec. 4.1), 0 if not, UNDECIDED without a bin/score."""
    b = snr_bin(p, edges)
    if b < 0 or not (score == score):
        return UNDECIDED
    return 1 if score > th[b] else 0


def f_beta(p: float, r: float, beta: float = 1.0) -> float:
    """F-score (Sec. 3.2) with the standard beta^2 p + r denominator (identical for beta = 1)."""
    den = beta * beta * p + r
    return 0.0 if den == 0 else (1.0 + beta * beta) * p * r / den


def precision_recall(pred: Sequence[bool], truth: Sequence[bool]) -> Tuple[float, float]:
    tp = sum(1 for a, b in zip(pred, truth) if a and b)
    fp = sum(1 for a, b in zip(pred, truth) if a and not b)
    fn = sum(1 for a, b in zip(pred, truth) if (not a) and b)
    p = tp / (tp + fp) if tp + fp else 0.0
    r = tp / (tp + fn) if tp + fn else 0.0
    return p, r


def calibrate_thresholds(scores: Sequence[float], psnrs: Sequence[float],
                         truth: Sequence[bool], edges: Sequence[float] = SNR_EDGES,
                         n_points: int = 5000) -> Dict[str, list]:
    """Per SNR bin, the F1-maximising threshold over n_points evenly spaced values in
    [min score, max score] of that bin (Sec. 4.1).  Ties go to the lowest threshold.  A bin with no
    periodic member gets th = max score (nothing above it), an empty bin th = +inf."""
    nb = len(edges) - 1
    th, fs, ps, rs = [], [], [], []
    for b in range(nb):
        idx = [i for i in range(len(scores)) if snr_bin(psnrs[i], edges) == b and
               scores[i] == scores[i]]
        if not idx:
            th.append(math.inf); fs.append(0.0); ps.append(0.0); rs.append(0.0)
            continue
        s = [float(scores[i]) for i in idx]
        lab = [bool(truth[i]) for i in idx]
        if not any(lab):
            th.append(max(s)); fs.append(0.0); ps.append(0.0); rs.append(0.0)
            continue
        cand = linear_grid(min(s), max(s), n_points) if n_points > 1 else np.array([min(s)])
        best = None
        for c in cand:
            pred = [v > c for v in s]
            p, r = precision_recall(pred, lab)
            f = f_beta(p, r, 1.0)
            if best is None or f > best[0]:
                best = (f, float(c), p, r)
        fs.append(best[0]); th.append(best[1]); ps.append(best[2]); rs.append(best[3])
    return {"th": th, "f1": fs, "precision": ps, "recall": rs}


# ------------------------------------------------------------------------------------------
# Trial frequencies by the bands method (Sec. 3.1) and the best period over them
# ------------------------------------------------------------------------------------------
# Readings where the paper leaves points open (the HIP library implements the same ones):
# * samples are taken in time order (stable: equal times keep their input order);
# * the derivative d_i = (y_{i+1} - y_i) / (t_{i+1} - t_i) belongs to sample i; a pair with equal
#   times contributes nothing;
# * the 10 equal-count bands split the samples by magnitude rank (stable in time order): sample
#   of rank r is in band floor(10 r / N); D_j sums |d_i| in time order;
# * bands are ranked by D_j descending, ties to the lower band;
# * the spectral-window grid is linear with n_grid points (30 000 by default: spacing ~1e-4 1/d,
#   about a quarter of the Fourier resolution of a 2500-day baseline);
# * the N_t highest local maxima of S_j use the local-maximum and tie rules of the search; a
#   maximum whose period satisfies |P - 1| < 1e-4 is dropped before the N_t are counted;
# * the trial list is band by band in rank order, maxima by rank (duplicates across bands kept);
# * the best trial is the highest score, ties to the lower frequency, then the earlier trial.

BANDS_F_LO = 0.00125
BANDS_F_HI = 3.0
BANDS_GRID = 30000


def bands_ranked(t, y, n_bands: int = 10) -> Tuple[np.ndarray, List[np.ndarray], List[float]]:
    """Time-ordered samples, the band members (indices into the time order, increasing) and D_j.

    Returns (order, members, D) where members[j] and D[j] belong to band j (j = 0 .. n_bands-1;
    band 0 holds the smallest magnitudes)."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    n = len(t)
    order = np.argsort(t, kind="stable")
    ts, ys = t[order], y[order]
    rank = np.empty(n, np.int64)
    rank[np.argsort(ys, kind="stable")] = np.arange(n)
    band = (rank * n_bands) // n
    D = [0.0] * n_bands
    for i in range(n - 1):
        dt = ts[i + 1] - ts[i]
        if dt != 0.0:
            D[int(band[i])] += abs((ys[i + 1] - ys[i]) / dt)
    members = [np.nonzero(band == j)[0] for j in range(n_bands)]
    return order, members, D


def spectral_window(times: np.ndarray, freqs: np.ndarray) -> np.ndarray:
    """S(f) = |sum_i exp(2 pi i f t_i)|^2 (Sec. 3.1, the spectral window of the band's times)."""
    x = np.outer(np.asarray(freqs, np.float64), np.asarray(times, np.float64))
    p = x - np.rint(x)  # the phase in cycles; exp(2 pi i x) = exp(2 pi i p)
    c = np.cos(2.0 * np.pi * p).sum(axis=1)
    s = np.sin(2.0 * np.pi * p).sum(axis=1)
    return c * c + s * s


def bands_trial_frequencies(t, y, n_keep: int = 3, n_trials: int = 150,
                            f_lo: float = BANDS_F_LO, f_hi: float = BANDS_F_HI,
                            n_grid: int = BANDS_GRID, n_bands: int = 10) -> Dict[str, object]:
    """The N_b N_t trial frequencies of the bands method (Sec. 3.1)."""
    order, members, D = bands_ranked(t, y, n_bands)
    ts = np.asarray(t, np.float64)[order]
    ranked = sorted(range(n_bands), key=lambda j: (-D[j], j))[:n_keep]
    grid = linear_grid(f_lo, f_hi, n_grid)
    trials, per_band = [], []
    for j in ranked:
        S = spectral_window(ts[members[j]], grid)
        peaks = [k for k in local_maxima(S) if not abs(1.0 / grid[k] - 1.0) < 1e-4]
        peaks.sort(key=lambda k: (-S[k], k))
        kept = peaks[:n_trials]
        per_band.append(kept)
        trials += [float(grid[k]) for k in kept]
    return {"bands": ranked, "D": D, "grid_index": per_band, "freqs": np.array(trials)}


def bands_best_period(t, y, e, sigma_t: float, sigma_y_rule: float, n_keep: int = 3,
                      n_trials: int = 150, score: int = SCORE_QMI, n_grid: int = BANDS_GRID,
                      n_threads: int = 0, masks=()) -> Dict[str, object]:
    """The score at every trial frequency and the best trial (Sec. 3.1 followed by Sec. 3),
    leaving out trials under a spurious-period mask (Sec. 6.1)."""
    tr = bands_trial_frequencies(t, y, n_keep, n_trials, n_grid=n_grid)
    f = tr["freqs"]
    sy = sigma_y_of(np.asarray(y, np.float64), None if e is None else np.asarray(e, np.float64),
                    sigma_y_rule)
    sigma_t = sigma_t_of(np.asarray(y, np.float64), sigma_t)
    if len(f) == 0:
        return dict(tr, scores=np.zeros(0), best=-1, f_best=math.nan, score=math.nan, sigma_y=sy)
    ips = information_potentials(t, y, sigma_t, sy, f, 1, n_threads)
    q = score_of(ips, score)
    best = None
    for i in range(len(f)):
        if not (q[i] == q[i]) or in_mask(f[i], q[i], masks):
            continue
        key = (-q[i], f[i], i)
        if best is None or key < best:
            best = key
    b = -1 if best is None else best[2]
    return dict(tr, scores=q, best=b, f_best=math.nan if b < 0 else float(f[b]),
                score=math.nan if b < 0 else float(q[b]), sigma_y=sy)


# ------------------------------------------------------------------------------------------
# Preprocessing (Sec. 5.2) and whitening for multimode search (Sec. 7.1)
# ------------------------------------------------------------------------------------------
# Readings: the error-bar statistics are the mean and the standard deviation with N - 1; a sample
# is kept iff e_i < mean + 3 std, except that when all error bars are equal nothing is an outlier
# and every sample is kept; a curve left with fewer than min_samples samples is rejected.  The
# chi^2 line minimises sum (a0 + a1 t_i - y_i)^2 / e_i^2; it is subtracted (a0 + a1 t) when the
# Pearson correlation between the magnitudes and the fitted line exceeds 0.5.  Whitening folds
# with the period P0 (phase t/P0 - floor(t/P0)), orders the samples by phase (stable), takes as
# template at folded position i the mean of the w = min(30, N) samples at positions i - w//2 ..
# i - w//2 + w - 1 (cyclically: the folded curve is periodic), subtracts it, and returns the
# samples in their input order.

def error_bar_cut(e, k_sigma: float = 3.0) -> np.ndarray:
    """Boolean mask of the samples kept by the error-bar cut (Sec. 5.2)."""
    e = np.asarray(e, np.float64)
    n = len(e)
    if n == 0 or all(v == e[0] for v in e):
        return np.ones(n, bool)
    mean = 0.0
    for v in e:
        mean += v
    mean /= n
    ss = 0.0
    for v in e:
        ss += (v - mean) * (v - mean)
    sd = math.sqrt(ss / (n - 1)) if n > 1 else 0.0
    thr = mean + k_sigma * sd
    return np.array([v < thr for v in e])


def chi2_line(t, y, e) -> Tuple[float, float]:
    """(a0, a1) minimising sum (a0 + a1 t_i - y_i)^2 / e_i^2, from the normal equations."""
    S = Sx = Sy = Sxx = Sxy = 0.0
    for ti, yi, ei in zip(t, y, e):
        w = 1.0 / (ei * ei)
        S += w
        Sx += w * ti
        Sy += w * yi
        Sxx += w * ti * ti
        Sxy += w * ti * yi
    den = S * Sxx - Sx * Sx
    a1 = (S * Sxy - Sx * Sy) / den if den != 0.0 else 0.0
    a0 = (Sy - a1 * Sx) / S
    return a0, a1


def pearson(x, y) -> float:
    n = len(x)
    mx = sum(x) / n
    my = sum(y) / n
    sxy = sum((a - mx) * (b - my) for a, b in zip(x, y))
    sxx = sum((a - mx) * (a - mx) for a in x)
    syy = sum((b - my) * (b - my) for b in y)
    return sxy / math.sqrt(sxx * syy) if sxx > 0.0 and syy > 0.0 else 0.0


def preprocess(t, y, e, min_samples: int = 50, min_corr: float = 0.5) -> Dict[str, object]:
    """Error-bar cut, minimum length, then the chi^2 linear detrending (Sec. 5.2)."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    e = np.asarray(e, np.float64)
    keep = error_bar_cut(e)
    t, y, e = t[keep], y[keep], e[keep]
    if len(t) < min_samples:
        return {"t": t, "y": y, "e": e, "ok": False, "detrended": False, "line": (0.0, 0.0)}
    a0, a1 = chi2_line(t, y, e)
    fit = a0 + a1 * t
    r = pearson(fit, y)
    detrended = r > min_corr
    if detrended:
        y = y - fit
    return {"t": t, "y": y, "e": e, "ok": True, "detrended": bool(detrended), "line": (a0, a1),
            "corr": r}


def whiten(t, y, period: float, window: int = 30) -> np.ndarray:
    """The curve minus its folded moving-average template (Sec. 7.1), in input order."""
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    n = len(t)
    x = t / period
    phase = x - np.floor(x)
    order = np.argsort(phase, kind="stable")
    ys = y[order]
    w = min(window, n)
    out = np.empty(n)
    for i in range(n):
        s = 0.0
        for m in range(w):
            s += ys[(i - w // 2 + m) % n]
        out[order[i]] = ys[i] - s / w
    return out
