"""Pins of the oracle's preprocessing (Sec. 5.2) and whitening (Sec. 7.1) against library routines
and properties fixed by the mathematics (no GPU)."""
import math

import numpy as np

import oracle as O
from paper_1412_1840_amd import synth


def test_error_bar_cut_matches_numpy_statistics():
    rng = np.random.default_rng(1)
    for n in (5, 60, 1000):
        e = rng.lognormal(np.log(0.1), 0.3, n)
        e[rng.integers(0, n, 2)] *= 20.0
        thr = np.mean(e) + 3.0 * np.std(e, ddof=1)
        keep = O.error_bar_cut(e)
        assert np.array_equal(keep, e < thr)
    # equal error bars: no outliers
    assert O.error_bar_cut(np.full(40, 0.07)).all()


def test_chi2_line_matches_weighted_polyfit():
    rng = np.random.default_rng(2)
    t = np.sort(rng.uniform(0, 2500, 400))
    e = rng.uniform(0.02, 0.3, 400)
    y = 0.3 - 2e-4 * t + rng.normal(0, 1, 400) * e
    a0, a1 = O.chi2_line(t, y, e)
    b1, b0 = np.polyfit(t, y, 1, w=1.0 / e)  # polyfit weights multiply the residuals
    assert abs(a1 - b1) <= 1e-9 * abs(b1) and abs(a0 - b0) <= 1e-9 * abs(b0)
    # exact on a noiseless line
    a0, a1 = O.chi2_line(t, 1.5 + 3e-3 * t, e)
    assert abs(a0 - 1.5) < 1e-10 and abs(a1 - 3e-3) < 1e-14


def test_pearson_matches_numpy():
    rng = np.random.default_rng(3)
    x, y = rng.normal(size=200), rng.normal(size=200)
    y += 0.5 * x
    assert abs(O.pearson(x, y) - np.corrcoef(x, y)[0, 1]) < 1e-12


def test_detrending_applies_to_trends_only():
    rng = np.random.default_rng(4)
    t = np.sort(rng.uniform(0, 2500, 300))
    e = rng.uniform(0.05, 0.15, 300)
    trend = O.preprocess(t, 0.1 + 4e-4 * t + rng.normal(0, 0.05, 300), e)
    assert trend["ok"] and trend["detrended"]
    # after subtraction the weighted line through the residuals is flat
    b0, b1 = O.chi2_line(trend["t"], trend["y"], trend["e"])
    assert abs(b1) < 1e-12 and abs(b0) < 1e-9
    flat = O.preprocess(t, rng.normal(0, 0.05, 300), e)
    assert flat["ok"] and not flat["detrended"]
    short = O.preprocess(t[:49], rng.normal(0, 0.05, 49), e[:49])
    assert not short["ok"]


def test_whitening_definition_cases():
    rng = np.random.default_rng(5)
    t = rng.uniform(0, 100, 57)
    # constant magnitudes whiten to zero; a window as long as the curve subtracts the mean
    assert np.all(O.whiten(t, np.full(57, 3.25), 2.2) == 0.0)
    y = rng.normal(size=57)
    np.testing.assert_allclose(O.whiten(t, y, 2.2, window=57), y - y.mean(), atol=1e-14)
    # a window of one sample subtracts the sample itself
    assert np.all(O.whiten(t, y, 2.2, window=1) == 0.0)
    # brute force for a small window: template = mean of the cyclic neighbours in phase order
    ph = t / 2.2 - np.floor(t / 2.2)
    order = np.argsort(ph, kind="stable")
    w = O.whiten(t, y, 2.2, window=4)
    for pos, i in enumerate(order):
        nb = [order[(pos + d) % 57] for d in (-2, -1, 0, 1)]
        assert abs(w[i] - (y[i] - np.mean(y[nb]))) < 1e-14


def test_whitening_removes_the_folded_signal_and_exposes_a_second_mode():
    """Two sinusoids of incommensurate periods on the survey cadence: the search finds the
    stronger one, whitening with it leaves the weaker one as the best period (Sec. 7.1).  Expected,
    not proven; holds for this seed."""
    rng = synth.rng_for(88, 0)
    t = synth.seasonal_times(rng, 500)
    p0, p1 = 2.7183, 11.31
    y = 1.0 * np.sin(2 * math.pi * t / p0) + 0.5 * np.sin(2 * math.pi * t / p1 + 1.0)
    y = y + rng.normal(0, 0.05, len(t))
    kw = dict(f_min=1e-3, f_max=1.0, n_coarse=4000, top_k=3, n_fine=100)
    r0 = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, **kw)
    assert abs(r0.f_best - 1 / p0) < 2e-4
    yw = O.whiten(t, y, 1.0 / r0.f_best)
    # the folded template absorbs most of mode 0: the whitened scatter is that of mode 1 + noise
    assert np.std(yw) < 0.6
    r1 = O.best_period(t, yw, None, 0.3, O.SIGMA_SILVERMAN, **kw)
    assert abs(r1.f_best - 1 / p1) < 2e-4
