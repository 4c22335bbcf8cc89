"""Parity of the preprocessing (qmi_preprocess, Sec. 5.2) and whitening (qmi_whiten, Sec. 7.1)
kernels with the FP64 oracle, and the two-level multimode search they enable.

The keep / reject / detrend decisions compare FP64 statistics whose summation orders differ
(a block tree on the GPU, a running sum in the oracle); the inputs keep every decision far from
its threshold, so the decisions must agree exactly.  Kept samples are copies (exact); a detrended
magnitude differs by the rounding of the fitted line (1e-12 absolute).  Whitening uses the same
operations in the same order on both sides and must agree bit for bit.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1412_1840_amd import qmi, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    with qmi.Context(0) as c:
        yield c


def _prep_curves():
    rng = np.random.default_rng(11)
    out = []
    for k in range(24):
        n = int(rng.integers(30, 900))
        t = np.sort(rng.uniform(0, 2500, n))
        e = rng.lognormal(np.log(0.08), 0.25, n)
        if k % 3 == 0:
            e[rng.choice(n, 3, replace=False)] *= 25.0  # outliers
        y = rng.normal(0, 1, n) * e
        if k % 2 == 0:
            y = y + (3e-4 if k % 4 == 0 else -2e-4) * t  # a trend
        if k % 5 == 0:
            y = y + 0.4 * np.sin(2 * math.pi * t / 5.3)
        out.append(synth.Curve(t, y, e, False))
    out[5].e = np.full(out[5].n, 0.1)  # equal error bars: nothing is an outlier
    return out


def test_preprocess_matches_oracle(ctx):
    curves = _prep_curves()
    b = synth.pack(curves)
    oo, to, yo, eo, st, det = ctx.preprocess(b.offsets, b.t, b.y, b.e)
    for k, c in enumerate(curves):
        ref = O.preprocess(c.t, c.y, c.e)
        a, z = oo[k], oo[k + 1]
        if not ref["ok"]:
            assert st[k] == qmi.EINVAL and z == a, k
            continue
        assert st[k] == 0 and det[k] == ref["detrended"], k
        assert np.array_equal(to[a:z], ref["t"]) and np.array_equal(eo[a:z], ref["e"]), k
        np.testing.assert_allclose(yo[a:z], ref["y"], rtol=0, atol=1e-12)
    assert sum(det) > 0 and sum(st != 0) > 0  # both branches exercised


def test_preprocess_options_and_invalid_input(ctx):
    curves = _prep_curves()[:6]
    bad = curves[2]
    bad.y = bad.y.copy()
    bad.y[1] = np.nan
    b = synth.pack(curves)
    oo, to, yo, eo, st, det = ctx.preprocess(b.offsets, b.t, b.y, b.e, error_cut=False,
                                             detrend=False, min_samples=2)
    assert st[2] == qmi.EINVAL and oo[3] == oo[2]
    for k, c in enumerate(curves):
        if k == 2:
            continue
        a, z = oo[k], oo[k + 1]
        assert np.array_equal(to[a:z], c.t) and np.array_equal(yo[a:z], c.y) and not det[k]
    with pytest.raises(qmi.QMIError):
        ctx.preprocess(b.offsets, b.t, b.y, None)  # the cut needs error bars
    with pytest.raises(qmi.QMIError):
        ctx.preprocess(b.offsets, b.t, b.y, b.e, min_samples=1)


@pytest.mark.parametrize("window", [30, 1, 7])
def test_whiten_matches_oracle_bitwise(ctx, window):
    curves = [synth.survey_batch_curve(k, n=n) for k, n in
              enumerate([2, 3, 29, 30, 31, 257, 600, 1000])]
    periods = np.array([0.731, 2.5, 11.0, 3.3, 0.2, 47.0, 1.0001, 123.4])
    b = synth.pack(curves)
    yw, st = ctx.whiten(b.offsets, b.t, b.y, periods, window=window)
    assert np.all(st == 0)
    for k, c in enumerate(curves):
        ref = O.whiten(c.t, c.y, periods[k], window=window)
        assert np.array_equal(yw[b.offsets[k]:b.offsets[k + 1]], ref), k


def test_whiten_maximum_length_and_bad_period(ctx):
    rng = synth.rng_for(99, 2)
    t = synth.seasonal_times(rng, 8192, baseline=30000.0)
    y = np.sin(2 * math.pi * t / 2.9) + rng.normal(0, 0.3, 8192)
    t2, y2 = t[:100], y[:100]
    b = synth.pack([synth.Curve(t, y, np.ones_like(t), True),
                    synth.Curve(t2, y2, np.ones_like(t2), True)])
    yw, st = ctx.whiten(b.offsets, b.t, b.y, [2.9, -1.0])
    assert st[0] == 0 and st[1] == qmi.EINVAL
    assert np.array_equal(yw[:8192], O.whiten(t, y, 2.9))
    assert np.all(np.isnan(yw[8192:]))


def test_two_mode_search_through_whitening(ctx):
    """Search, whiten at the found period, search again: the second search finds the weaker mode,
    as the oracle's does (Sec. 7.1)."""
    rng = synth.rng_for(88, 0)
    t = synth.seasonal_times(rng, 500)
    p0, p1 = 2.7183, 11.31
    y = np.sin(2 * math.pi * t / p0) + 0.5 * np.sin(2 * math.pi * t / p1 + 1.0)
    y = y + rng.normal(0, 0.05, len(t))
    kw = dict(f_min=1e-3, f_max=1.0, n_coarse=4000, top_k=3, n_fine=100)
    r0, _ = ctx.best_period([0, len(t)], t, y, None, 0.3, **kw)
    assert abs(r0["f_best"][0] - 1 / p0) < 2e-4
    yw, st = ctx.whiten([0, len(t)], t, y, [r0["period"][0]])
    ref0 = O.best_period(t, y, None, 0.3, O.SIGMA_SILVERMAN, **kw)
    if r0["f_best"][0] == ref0.f_best:
        assert np.array_equal(yw, O.whiten(t, y, 1.0 / ref0.f_best))
    r1, _ = ctx.best_period([0, len(t)], t, yw, None, 0.3, **kw)
    assert abs(r1["f_best"][0] - 1 / p1) < 2e-4
