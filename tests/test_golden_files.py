"""The stored oracle searches (tests/golden/*_oracle.json, written by make_survey_parity.py) agree
with the generator and with the oracle as it stands (no GPU): every record belongs to the curve
the generator makes for its index, the search parameters are the workload's, and the cheapest
stored curves of each workload, searched again by the oracle, give the same grid indices."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1412_1840_amd import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MAKE = {"survey_batch": synth.survey_batch_curve, "survey_stream": synth.survey_stream_curve,
        "long_baseline": synth.long_baseline_curve}


def _load(workload):
    return json.load(open(os.path.join(HERE, "%s_oracle.json" % workload)))


@pytest.mark.parametrize("workload", sorted(MAKE))
def test_records_belong_to_the_generated_curves(workload):
    g = _load(workload)
    wl = synth.WORKLOADS[workload]
    assert g["workload"] == workload and g["sigma_t"] == wl["sigma_t"]
    for key in ("f_min", "f_max", "n_coarse", "top_k", "n_fine"):
        assert g["search"][key] == wl[key], key
    ks = [r["k"] for r in g["curves"]]
    assert ks == list(range(len(ks))) and len(ks) >= 8
    for r in g["curves"]:
        c = MAKE[workload](r["k"])
        assert r["n"] == c.n and r["periodic"] == bool(c.periodic), r["k"]
        assert 0 <= r["coarse_index"] < wl["n_coarse"] and 0 <= r["fine_index"] < wl["n_fine"]
        assert 0 <= r["peak_rank"] < r["n_peaks"] <= wl["top_k"]


@pytest.mark.parametrize("sigma_t", [0.1, 0.6])
def test_long_baseline_width_variants_belong_to_the_generated_curves(sigma_t):
    """The stored long-baseline searches at the other two widths of the precision study."""
    path = os.path.join(HERE, "long_baseline_st%g_oracle.json" % sigma_t)
    if not os.path.exists(path):
        pytest.skip("not written yet")
    g = json.load(open(path))
    wl = synth.WORKLOADS["long_baseline"]
    assert g["workload"] == "long_baseline" and g["sigma_t"] == sigma_t
    for key in ("f_min", "f_max", "n_coarse", "top_k", "n_fine"):
        assert g["search"][key] == wl[key], key
    ks = [r["k"] for r in g["curves"]]
    assert ks == list(range(len(ks))) and len(ks) >= 8
    for r in g["curves"]:
        c = synth.long_baseline_curve(r["k"])
        assert r["n"] == c.n and r["periodic"] == bool(c.periodic), r["k"]
        assert 0 <= r["coarse_index"] < wl["n_coarse"] and 0 <= r["fine_index"] < wl["n_fine"]


@pytest.mark.parametrize("workload", ["survey_batch", "survey_stream"])
def test_cheapest_stored_searches_are_reproduced_by_the_oracle(workload):
    g = _load(workload)
    recs = sorted(g["curves"], key=lambda r: (r["n"], r["k"]))[:2]
    kw = {key: g["search"][key] for key in ("f_min", "f_max", "n_coarse", "top_k", "n_fine")}
    for r in recs:
        c = MAKE[workload](r["k"])
        o = O.best_period(c.t, c.y, c.e, g["sigma_t"], O.SIGMA_SILVERMAN, **kw)
        got = (o.coarse_index, o.peak_rank, o.fine_index, o.coarse_argmax, o.n_peaks)
        want = (r["coarse_index"], r["peak_rank"], r["fine_index"], r["coarse_argmax"],
                r["n_peaks"])
        assert got == want, (workload, r["k"])
        assert o.f_best == r["f_best"]
        # the oracle's threaded sums may be added in another order: scores to FP64 rounding
        assert abs(o.score - r["score"]) <= 1e-9 * abs(r["score"])
        assert o.sigma_y == pytest.approx(r["sigma_y"], rel=1e-14)


def test_stored_precision_values_are_the_oracles():
    """long_baseline_precision_oracle.npz (the benchmark's precision reference): the frequencies
    follow the precision study's sample of the same curves, and the oracle recomputes a slice of
    the stored values."""
    import sys
    sys.path.insert(0, HERE)
    import make_precision_golden as M

    g = np.load(os.path.join(HERE, "long_baseline_precision_oracle.npz"))
    assert list(g["widths"]) == [0.3, 0.1, 0.6] and list(g["k"]) == list(range(M.N_CURVES))
    for k in range(M.N_CURVES):
        c = synth.long_baseline_curve(k)
        np.testing.assert_array_equal(g["freqs"][k], M.freq_sample(k, c))
    for k, st in ((0, 0.3), (3, 0.1), (6, 0.6)):
        c = synth.long_baseline_curve(k)
        sel = [0, 100, 230, 255]
        r = O.information_potentials(c.t, c.y, st, O.silverman_sigma(c.y), g["freqs"][k][sel])
        tag = "%g" % st
        np.testing.assert_allclose(r.vj, g["vj_" + tag][k][sel], rtol=1e-12)
        np.testing.assert_allclose(r.vc, g["vc_" + tag][k][sel], rtol=1e-12)
        np.testing.assert_allclose(O.qmi(r), g["qmi_" + tag][k][sel], rtol=1e-9, atol=1e-14)
