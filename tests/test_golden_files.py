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
