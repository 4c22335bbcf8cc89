"""Pins of the oracle's spurious-period filter (Sec. 6.1) against the alias formulas of the table of
spurious periods, the half width of a Gaussian, and the selection properties the filter must have
(no GPU)."""
import math

import numpy as np

import oracle as O
from paper_1412_1840_amd import synth


def test_table_aliases_follow_from_the_base_periods():
    """Every alias of the table is (1/P_a +- 1/P_b)^-1 (or with 2/P_d) of the base periods; the
    printed values agree with those formulas to 0.1% and within half of a default mask's sigma
    (the four-digit rounding of the sub-day aliases is that large; the table prints 27.31 for the
    sidereal month, whose formula gives 27.32, and its last two entries imply spans of 2325 and
    2345 d rather than 2335)."""
    Pd, Pm, Py, T = O.SOLAR_DAY, O.SYNODIC_MONTH, O.TROPICAL_YEAR, O.EROS_SPAN
    assert O.SPURIOUS_PERIODS[:4] == (Pd, Pm, Py, T)
    derived = [1 / (2 / Pd + 1 / Pm), 1 / (2 / Pd - 1 / Pm), 1 / (1 / Pd + 1 / Pm),
               1 / (1 / Pd - 1 / Pm), 1 / (1 / Pd + 1 / Py), 1 / (1 / Pd - 1 / Py),
               1 / (1 / Pm + 1 / Py), 1 / (1 / Pm - 1 / Py), 1 / (1 / Py + 1 / T),
               1 / (1 / Py - 1 / T)]
    masks = O.spurious_masks(1.0)
    for printed, want, (pk, sk, _) in zip(O.SPURIOUS_PERIODS[4:], derived, masks[4:]):
        assert pk == printed
        assert abs(printed - want) <= 1e-3 * want, (printed, want)
        assert abs(printed - want) <= 0.5 * sk, (printed, want, sk)
    # the lunar day and the sidereal day are the textbook values
    assert abs(derived[3] - 1.0351) < 1e-4 and abs(derived[4] - 0.99727) < 1e-5


def test_mask_is_a_gaussian_of_the_stated_half_width():
    """At the centre a candidate is inside iff its score is below the amplitude; at the half width
    at half maximum, sigma sqrt(2 ln 2), iff below half of it."""
    pk, sk, ak = 29.5305, 0.4, 2.0
    m = [(pk, sk, ak)]
    assert O.in_mask(1 / pk, 1.999, m) and not O.in_mask(1 / pk, 2.001, m)
    h = sk * math.sqrt(2 * math.log(2))
    for P in (pk - h, pk + h):
        assert O.in_mask(1 / P, 0.999, m) and not O.in_mask(1 / P, 1.001, m)
    # far from the centre nothing positive is inside
    assert not O.in_mask(1 / (pk + 40 * sk), 1e-300, m)
    assert not O.in_mask(1.0, 0.5, [])


def _curve(seed=3, n=160):
    rng = synth.rng_for(seed, 0)
    t = synth.seasonal_times(rng, n, baseline=800.0)
    y = np.sin(2 * math.pi * t / 2.37) + 0.6 * np.sin(2 * math.pi * t / 0.731 + 0.4)
    return t, y + rng.normal(0, 0.2, n)


KW = dict(f_min=0.01, f_max=2.0, n_coarse=1500, top_k=4, n_fine=40)


def test_no_or_zero_amplitude_masks_change_nothing():
    t, y = _curve()
    a = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, **KW)
    b = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, masks=O.spurious_masks(0.0), **KW)
    for f in ("f_best", "score", "coarse_index", "peak_rank", "fine_index", "coarse_argmax",
              "n_peaks"):
        assert getattr(a, f) == getattr(b, f), f


def test_masked_search_selects_the_best_unmasked_candidates():
    """A mask over the unmasked best period with an amplitude above every score: the coarse
    argmax, the refined peaks and the best refined point are each the best of the candidates
    outside the mask; everything ranked above them lies inside it."""
    t, y = _curve()
    a = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, **KW)
    P0 = 1 / a.f_best
    amp = 10 * float(np.nanmax(a.coarse_scores))
    masks = [(P0, 0.02 * P0, amp)]
    b = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, masks=masks, **KW)
    assert not O.in_mask(b.f_best, b.score, masks) and abs(1 / b.f_best - P0) > 0.05 * P0
    grid = O.linear_grid(KW["f_min"], KW["f_max"], KW["n_coarse"])
    q = b.coarse_scores
    np.testing.assert_array_equal(q, a.coarse_scores)  # the periodogram itself is not masked
    inside = np.array([O.in_mask(f, v, masks) for f, v in zip(grid, q)])
    assert inside.any() and not inside[b.coarse_argmax]
    assert np.all(inside[q > q[b.coarse_argmax]])
    # the refined peaks: unmasked local maxima, the top_k of them by score
    loc = [k for k in range(1, len(q) - 1) if q[k] > q[k - 1] and q[k] >= q[k + 1]]
    free = sorted((k for k in loc if not inside[k]), key=lambda k: (-q[k], k))
    assert b.n_peaks == KW["top_k"] and b.coarse_index in free[:KW["top_k"]]
    # the best refined point beats every unmasked refined point of every kept peak
    assert b.fine_scores.shape == (KW["top_k"], KW["n_fine"])
    sy = O.sigma_y_of(y, None, O.SIGMA_SILVERMAN)
    for rank, k in enumerate(free[:KW["top_k"]]):
        lo, hi = O.fine_window(grid, k)
        fine = O.linear_grid(lo, hi, KW["n_fine"])
        # row `rank` holds the window of the rank-th unmasked peak
        want = O.qmi(O.information_potentials(t, y, 0.3, sy, fine))
        np.testing.assert_array_equal(b.fine_scores[rank], want)
        for m, f in enumerate(fine):
            v = b.fine_scores[rank, m]
            if not O.in_mask(f, v, masks):
                assert v <= b.score


def test_everything_masked_gives_an_empty_result():
    t, y = _curve(n=60)
    kw = dict(KW, n_coarse=200)
    masks = [(1.0, 1e6, 1e30)]  # one mask wider than the grid, above every score
    r = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, masks=masks, **kw)
    assert math.isnan(r.f_best) and math.isnan(r.score) and r.coarse_argmax == -1
    assert r.n_peaks == 0
    rb = O.bands_best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, n_trials=20, n_grid=2000,
                             masks=masks)
    assert rb["best"] == -1 and math.isnan(rb["f_best"]) and len(rb["scores"]) > 0


def test_masked_bands_best_is_the_best_unmasked_trial():
    t, y = _curve()
    a = O.bands_best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, n_trials=30, n_grid=4000)
    P0 = 1 / a["f_best"]
    masks = [(P0, 0.01 * P0, 10 * float(np.nanmax(a["scores"])))]
    b = O.bands_best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, n_trials=30, n_grid=4000,
                            masks=masks)
    assert np.array_equal(a["freqs"], b["freqs"]) and np.array_equal(a["scores"], b["scores"])
    f, q = b["freqs"], b["scores"]
    inside = np.array([O.in_mask(x, v, masks) for x, v in zip(f, q)])
    assert inside[a["best"]] and not inside[b["best"]]
    assert np.all(inside[q > q[b["best"]]])
