"""Seeded synthetic lightcurves shaped like the EROS-2 survey data.

This module only makes input data. It holds none of the periodogram's arithmetic, so both the
HIP path and the CPU oracle can be fed from it without sharing any method code.

Every curve is drawn from its own ``numpy.random.Generator(PCG64(SeedSequence([config_id, k])))``,
so curve ``k`` of a workload is the same whatever batch it is generated in.

Workloads (names follow the sizes they describe):

* ``single_sinusoid``   N=200, t ~ U[0, 2500] d sorted, y = 0.3 sin(2 pi t / 3.7) + N(0, 0.1^2),
  e = 0.1; 5000-point grid on [1e-3, 10] d^-1.
* ``survey_batch``      N ~ U{300..1000}; seasonal cadence over 2500 d (about half of each year
  observed, one visit per night with +-0.15 d jitter); even k periodic (sinusoid, sawtooth or
  two-dip eclipse, period log-uniform on [0.1, 500] d, amplitude U[0.05, 1] mag, SNR U[0.5, 10]);
  odd k non-periodic (white noise plus Ornstein-Uhlenbeck red noise).  The survey's baseline of
  about 2500 d at about 1.2 samples per night (Sec. 4.2 "Efficiency as a function of parameters")
  and mean lengths of 430 / 780 samples (Sec. 5.1) set these shapes.
* ``long_baseline``     same generator over 7000 d, periods log-uniform on [0.05, 10] d, N = 1000.
* ``serving_stream``    survey mix with N = round(lognormal(ln 500, 0.5)) resampled into [50, 2000].
* ``survey_stream``     N = round(lognormal(ln 500, 0.4)) resampled into [100, 1500]; only
  k mod 100 == 0 is periodic (1 %).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterable, List, Optional, Sequence

import numpy as np

# Configuration ids used as the first word of each curve's SeedSequence.
CFG_SINGLE_SINUSOID = 0
CFG_SURVEY_BATCH = 1
CFG_LONG_BASELINE = 2
CFG_SERVING_STREAM = 3
CFG_SURVEY_STREAM = 4

SHAPES = ("sinusoid", "sawtooth", "eclipse")


@dataclasses.dataclass
class Curve:
    """One lightcurve: times (days), magnitudes and error bars, plus the generator's truth."""

    t: np.ndarray
    y: np.ndarray
    e: np.ndarray
    periodic: bool
    period: float = float("nan")
    shape: str = "noise"
    snr: float = float("nan")

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


@dataclasses.dataclass
class Batch:
    """A CSR-packed batch: curve k is samples [offsets[k], offsets[k+1])."""

    offsets: np.ndarray  # int64 [n_curves + 1]
    t: np.ndarray  # float64 [total]
    y: np.ndarray
    e: np.ndarray
    periodic: np.ndarray  # bool [n_curves]
    period: np.ndarray  # float64 [n_curves] (nan for non-periodic)

    @property
    def n_curves(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def curve(self, k: int) -> Curve:
        a, b = int(self.offsets[k]), int(self.offsets[k + 1])
        return Curve(self.t[a:b], self.y[a:b], self.e[a:b], bool(self.periodic[k]),
                     float(self.period[k]))


def pack(curves: Sequence[Curve]) -> Batch:
    lens = np.array([c.n for c in curves], dtype=np.int64)
    offsets = np.zeros(len(curves) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    cat = lambda name: (np.concatenate([getattr(c, name) for c in curves]).astype(np.float64)
                        if curves else np.zeros(0))
    return Batch(offsets, cat("t"), cat("y"), cat("e"),
                 np.array([c.periodic for c in curves], dtype=bool),
                 np.array([c.period for c in curves], dtype=np.float64))


def rng_for(config_id: int, k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(k)])))


# --------------------------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------------------------

def seasonal_times(rng: np.random.Generator, n: int, baseline: float = 2500.0,
                   season_len: float = 182.6, jitter: float = 0.15) -> np.ndarray:
    """Nightly visits inside an observing season of ``season_len`` days per year.

    A season offset o ~ U[0, 365.25) is drawn; night d (integer day in [0, baseline)) is observable
    when (d - o) mod 365.25 < season_len.  N nights are drawn without replacement (with replacement
    when N exceeds the observable nights) and each visit is at d + 0.5 + U(-jitter, jitter).
    """
    o = rng.uniform(0.0, 365.25)
    days = np.arange(int(baseline), dtype=np.float64)
    nights = days[np.mod(days - o, 365.25) < season_len]
    replace = n > nights.shape[0]
    d = rng.choice(nights, size=n, replace=replace)
    t = d + 0.5 + rng.uniform(-jitter, jitter, size=n)
    return np.sort(t)


def wrapped_gaussian(phase: np.ndarray, mu: float, w: float) -> np.ndarray:
    """Unit-height Gaussian dip centred at ``mu`` on the unit circle of phase."""
    d = np.mod(phase - mu + 0.5, 1.0) - 0.5
    return np.exp(-0.5 * (d / w) ** 2)


def periodic_signal(rng: np.random.Generator, t: np.ndarray, period: float,
                    shape: str) -> np.ndarray:
    phi = t / period + rng.uniform(0.0, 1.0)
    if shape == "sinusoid":
        return np.sin(2.0 * np.pi * phi)
    if shape == "sawtooth":
        return 2.0 * np.mod(phi, 1.0) - 1.0
    if shape == "eclipse":
        w = rng.uniform(0.02, 0.08)
        d2 = rng.uniform(0.3, 1.0)
        return -(wrapped_gaussian(phi, 0.0, w) + d2 * wrapped_gaussian(phi, 0.5, w))
    raise ValueError(shape)


def ou_noise(rng: np.random.Generator, t: np.ndarray, tau: float, sigma: float) -> np.ndarray:
    """Stationary Ornstein-Uhlenbeck (continuous AR(1)) process sampled exactly at sorted times."""
    x = np.empty_like(t)
    if t.shape[0] == 0:
        return x
    x[0] = rng.normal(0.0, sigma)
    dt = np.diff(t)
    a = np.exp(-dt / tau)
    innov = rng.normal(0.0, 1.0, size=dt.shape[0]) * sigma * np.sqrt(1.0 - a * a)
    for k in range(dt.shape[0]):
        x[k + 1] = a[k] * x[k] + innov[k]
    return x


def log_uniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def bounded_lognormal_length(rng: np.random.Generator, median: float, sigma_ln: float,
                             lo: int, hi: int) -> int:
    while True:
        n = int(round(rng.lognormal(math.log(median), sigma_ln)))
        if lo <= n <= hi:
            return n


def survey_curve(rng: np.random.Generator, n: int, periodic: bool, baseline: float = 2500.0,
                 p_range=(0.1, 500.0)) -> Curve:
    """One curve of the survey mix (periodic or white + red noise) on a seasonal cadence."""
    t = seasonal_times(rng, n, baseline=baseline)
    if periodic:
        shape = SHAPES[int(rng.integers(0, 3))]
        period = log_uniform(rng, *p_range)
        amp = rng.uniform(0.05, 1.0)
        snr = rng.uniform(0.5, 10.0)
        s = amp * periodic_signal(rng, t, period, shape)
        rms = float(np.sqrt(np.mean((s - s.mean()) ** 2)))
        sigma_n = rms / snr
        y = s + rng.normal(0.0, sigma_n, size=n)
        e = np.full(n, sigma_n)
        return Curve(t, y, e, True, period, shape, snr)
    sigma_w = rng.uniform(0.02, 0.3)
    tau = log_uniform(rng, 1.0, 300.0)
    sigma_r = sigma_w * rng.uniform(0.5, 2.0)
    y = rng.normal(0.0, sigma_w, size=n) + ou_noise(rng, t, tau, sigma_r)
    e = np.full(n, sigma_w)
    return Curve(t, y, e, False)


# --------------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------------

def single_sinusoid(k: int = 0, n: int = 200) -> Curve:
    rng = rng_for(CFG_SINGLE_SINUSOID, k)
    t = np.sort(rng.uniform(0.0, 2500.0, size=n))
    y = 0.3 * np.sin(2.0 * np.pi * t / 3.7) + rng.normal(0.0, 0.1, size=n)
    return Curve(t, y, np.full(n, 0.1), True, 3.7, "sinusoid", 3.0)


def survey_batch_curve(k: int, n: Optional[int] = None) -> Curve:
    rng = rng_for(CFG_SURVEY_BATCH, k)
    n_draw = int(rng.integers(300, 1001))
    return survey_curve(rng, n if n is not None else n_draw, periodic=(k % 2 == 0))


def long_baseline_curve(k: int) -> Curve:
    rng = rng_for(CFG_LONG_BASELINE, k)
    return survey_curve(rng, 1000, periodic=(k % 2 == 0), baseline=7000.0, p_range=(0.05, 10.0))


def serving_curve(k: int) -> Curve:
    rng = rng_for(CFG_SERVING_STREAM, k)
    n = bounded_lognormal_length(rng, 500.0, 0.5, 50, 2000)
    return survey_curve(rng, n, periodic=(k % 2 == 0))


def survey_stream_curve(k: int) -> Curve:
    rng = rng_for(CFG_SURVEY_STREAM, k)
    n = bounded_lognormal_length(rng, 500.0, 0.4, 100, 1500)
    return survey_curve(rng, n, periodic=(k % 100 == 0))


def make_batch(kind: str, indices: Iterable[int], n: Optional[int] = None) -> Batch:
    fn = {
        "single_sinusoid": lambda k: single_sinusoid(k) if n is None else single_sinusoid(k, n),
        "survey_batch": lambda k: survey_batch_curve(k, n),
        "long_baseline": long_baseline_curve,
        "serving_stream": serving_curve,
        "survey_stream": survey_stream_curve,
    }[kind]
    return pack([fn(int(k)) for k in indices])


def poisson_arrivals(seed: int, n: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of ``n`` requests at ``rate_per_s``."""
    rng = rng_for(1000 + CFG_SERVING_STREAM, seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


# Search and kernel settings of the workloads above (frequencies in 1/day).
WORKLOADS = {
    "single_sinusoid": dict(f_min=1e-3, f_max=10.0, n_coarse=5000, top_k=0, n_fine=0, sigma_t=0.3),
    "survey_batch": dict(f_min=1e-3, f_max=10.0, n_coarse=20000, top_k=10, n_fine=1000, sigma_t=0.3),
    "long_baseline": dict(f_min=1e-3, f_max=20.0, n_coarse=20000, top_k=10, n_fine=1000, sigma_t=0.3),
    "serving_stream": dict(f_min=1e-3, f_max=10.0, n_coarse=20000, top_k=10, n_fine=1000, sigma_t=0.3),
    "survey_stream": dict(f_min=1e-3, f_max=10.0, n_coarse=30000, top_k=10, n_fine=1000, sigma_t=0.3),
}


def curves_of(batch: Batch) -> List[Curve]:
    return [batch.curve(k) for k in range(batch.n_curves)]
