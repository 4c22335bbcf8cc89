"""Pins of the oracle's bands method (Sec. 3.1) against closed forms and properties fixed by the
mathematics (no GPU): the Dirichlet-kernel spectral window of evenly spaced times, equal-count
magnitude bands, the derivative ranking of a densely sampled sinusoid (its per-band share of the
total variation follows from the arcsine distribution of sin), the one-day rejection, order
invariance and recovery of a noiseless sinusoid's frequency.
"""
import math

import numpy as np

import oracle as O
from paper_1412_1840_amd import synth


def test_spectral_window_of_evenly_spaced_times_is_a_dirichlet_kernel():
    """t_i = t0 + i d (i < M): |sum e^{2 pi i f t_i}|^2 = sin^2(pi f M d) / sin^2(pi f d)."""
    rng = np.random.default_rng(1)
    for M, d, t0 in ((7, 1.0, 0.0), (40, 0.37, 123.25), (123, 2.5, -50.0)):
        t = t0 + d * np.arange(M)
        f = rng.uniform(0.001, 3.0, 200)
        want = np.sin(math.pi * f * M * d) ** 2 / np.sin(math.pi * f * d) ** 2
        np.testing.assert_allclose(O.spectral_window(t, f), want, rtol=1e-9, atol=1e-9)
        # at f d integer every term is 1
        assert abs(O.spectral_window(t, np.array([1.0 / d]))[0] - M * M) < 1e-8 * M * M


def test_bands_are_equal_count_and_ordered_by_magnitude():
    rng = np.random.default_rng(2)
    for n in (10, 11, 37, 600, 1001):
        t = rng.uniform(0, 2500, n)
        y = rng.normal(0, 1, n)
        order, members, D = O.bands_ranked(t, y, 10)
        ys = y[order]
        counts = [len(m) for m in members]
        assert sum(counts) == n and max(counts) - min(counts) <= 1
        assert sorted(np.concatenate(members).tolist()) == list(range(n))
        for j in range(9):
            if len(members[j]) and len(members[j + 1]):
                assert ys[members[j]].max() <= ys[members[j + 1]].min()
        assert np.all(np.diff(t[order]) >= 0)


def test_band_derivative_sums_follow_the_arcsine_law_for_a_dense_sinusoid():
    """y = sin(2 pi t / P) on a fine regular grid (many periods): the band of magnitudes [a, b]
    collects 2 (b - a) of variation per period, and the equal-count band edges are quantiles of
    sin of a uniform phase, q(p) = sin(pi (p - 1/2)).  So D_j is proportional to the band's width,
    the central bands rank first and the extreme ones last."""
    P, dt, n_per = 3.7, 0.01, 200
    t = np.arange(0.0, P * n_per, dt)
    y = np.sin(2 * math.pi * t / P)
    _, _, D = O.bands_ranked(t, y, 10)
    edges = np.sin(math.pi * (np.arange(11) / 10.0 - 0.5))
    width = np.diff(edges)
    share = np.array(D) / np.sum(D)
    np.testing.assert_allclose(share, width / width.sum(), rtol=2e-2)
    ranked = sorted(range(10), key=lambda j: (-D[j], j))
    assert set(ranked[:2]) == {4, 5} and set(ranked[-2:]) == {0, 9}


def test_one_day_period_is_rejected():
    """Nightly sampling at the same hour: every band's window peaks at f = 1/d; no trial may have
    |1/f - 1| < 1e-4."""
    rng = np.random.default_rng(3)
    nights = np.sort(rng.choice(2500, 600, replace=False)).astype(float)
    t = nights + 0.4 + rng.uniform(-0.01, 0.01, 600)
    y = rng.normal(0, 0.1, 600)
    grid = O.linear_grid(O.BANDS_F_LO, O.BANDS_F_HI, O.BANDS_GRID)
    S = O.spectral_window(t, grid)
    k1 = int(np.argmin(np.abs(grid - 1.0)))
    assert S[k1] > 0.5 * 600 ** 2  # the one-day alias dominates the window
    tr = O.bands_trial_frequencies(t, y, n_keep=3, n_trials=150)
    f = tr["freqs"]
    assert len(f) == 450
    assert not np.any(np.abs(1.0 / f - 1.0) < 1e-4)


def test_trials_do_not_depend_on_sample_order():
    c = synth.survey_batch_curve(4, n=300)
    a = O.bands_trial_frequencies(c.t, c.y)
    p = np.random.default_rng(5).permutation(c.n)
    b = O.bands_trial_frequencies(c.t[p], c.y[p])
    assert a["bands"] == b["bands"] and np.array_equal(a["freqs"], b["freqs"])


def test_trials_are_the_highest_local_maxima_of_each_window():
    """Brute force on a small grid: the trials of each kept band are exactly the n_trials largest
    local maxima of the band's window outside the one-day window."""
    c = synth.survey_batch_curve(6, n=120)
    n_grid = 3000
    tr = O.bands_trial_frequencies(c.t, c.y, n_keep=2, n_trials=25, n_grid=n_grid)
    order, members, D = O.bands_ranked(c.t, c.y, 10)
    ts = c.t[order]
    grid = O.linear_grid(O.BANDS_F_LO, O.BANDS_F_HI, n_grid)
    for j, ks in zip(tr["bands"], tr["grid_index"]):
        S = O.spectral_window(ts[members[j]], grid)
        interior = [k for k in range(1, n_grid - 1) if S[k] > S[k - 1] and S[k] >= S[k + 1]]
        ends = ([0] if S[0] >= S[1] else []) + ([n_grid - 1] if S[-1] > S[-2] else [])
        cand = [k for k in sorted(interior + ends) if abs(1 / grid[k] - 1) >= 1e-4]
        want = sorted(cand, key=lambda k: (-S[k], k))[:25]
        assert ks == want


def test_noiseless_sinusoid_frequency_is_among_trials_and_best():
    """A noiseless sinusoid sampled on the survey cadence: its frequency (within a grid step) is a
    trial of the first band and the best trial by QMI.  Expected, not proven; holds for this
    seed."""
    rng = synth.rng_for(77, 0)
    t = synth.seasonal_times(rng, 500)
    f0 = 0.5371
    y = np.sin(2 * math.pi * f0 * t)
    step = (O.BANDS_F_HI - O.BANDS_F_LO) / (O.BANDS_GRID - 1)
    tr = O.bands_trial_frequencies(t, y)
    assert np.min(np.abs(tr["freqs"][:150] - f0)) <= step
    r = O.bands_best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN)
    assert abs(r["f_best"] - f0) <= step


def test_curves_shorter_than_the_band_count():
    """With N < n_bands some bands are empty: their window is identically zero, whose only local
    maximum (by the tie rules) is the first grid point."""
    t = np.array([10.0, 11.3, 17.9])
    y = np.array([0.1, 0.5, 0.2])
    tr = O.bands_trial_frequencies(t, y, n_keep=4, n_trials=3, n_grid=500)
    order, members, D = O.bands_ranked(t, y, 10)
    assert sorted(len(m) for m in members) == [0] * 7 + [1] * 3
    for j, ks in zip(tr["bands"], tr["grid_index"]):
        if len(members[j]) == 0:
            assert ks == [0]
