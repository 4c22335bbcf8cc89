"""Writes <workload>_oracle.json: the FP64 oracle's full coarse-to-fine search of the first curves
of a workload (survey_batch: 20 000 coarse + 10 x 1000 refined frequencies on [1e-3, 10] 1/d;
long_baseline: the same on [1e-3, 20] 1/d over a 7000-day baseline; survey_stream: 30 000 coarse +
10 x 1000 refined on [1e-3, 10] 1/d; Silverman sigma_y; sigma_t = the workload's 0.3 unless a
fourth argument gives another, which goes into <workload>_st<sigma_t>_oracle.json), for the GPU
parity tests of the best period at full size.

    python tests/golden/make_survey_parity.py [n_curves] [threads] [workload] [sigma_t]

Calls only oracle/ (and the seeded input generator).  About 35 s per survey curve on 8 cores.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1412_1840_amd import synth  # noqa: E402


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    workload = sys.argv[3] if len(sys.argv) > 3 else "survey_batch"
    wl = synth.WORKLOADS[workload]
    sigma_t = float(sys.argv[4]) if len(sys.argv) > 4 else wl["sigma_t"]
    make = {"survey_batch": synth.survey_batch_curve, "long_baseline": synth.long_baseline_curve,
            "survey_stream": synth.survey_stream_curve}[workload]
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    name = (workload if sigma_t == wl["sigma_t"] else "%s_st%g" % (workload, sigma_t))
    out_path = os.path.join(HERE, "%s_oracle.json" % name)
    records = []
    if os.path.exists(out_path):
        records = json.load(open(out_path))["curves"]
    done = {r["k"] for r in records}
    for k in range(n):
        if k in done:
            continue
        c = make(k)
        t0 = time.time()
        r = O.best_period(c.t, c.y, c.e, sigma_t, O.SIGMA_SILVERMAN, n_threads=threads, **kw)
        fq = np.sort(r.fine_scores.ravel())[::-1]
        cq = r.coarse_scores
        peaks = O.top_peaks(cq, kw["top_k"] + 1)
        pk_gaps = [float(cq[peaks[i]] - cq[peaks[i + 1]]) for i in range(len(peaks) - 1)]
        records.append({
            "k": k, "n": c.n, "periodic": bool(c.periodic), "period_true": c.period,
            "f_best": r.f_best, "score": r.score, "qmi": r.qmi, "nckp": r.nckp,
            "coarse_index": r.coarse_index, "peak_rank": r.peak_rank,
            "fine_index": r.fine_index, "coarse_argmax": r.coarse_argmax,
            "n_peaks": r.n_peaks, "sigma_y": r.sigma_y,
            "best_gap": float(fq[0] - fq[1]),          # refined best minus runner-up
            "min_peak_gap": float(min(pk_gaps[:kw["top_k"]]) if pk_gaps else np.inf),
            "coarse_best": float(cq[r.coarse_argmax]),
        })
        records.sort(key=lambda x: x["k"])
        with open(out_path + ".tmp", "w") as f:
            json.dump({"workload": workload, "search": kw, "sigma_t": sigma_t,
                       "sigma_y": "silverman", "curves": records}, f, indent=1)
        os.replace(out_path + ".tmp", out_path)
        print("curve %d N=%d done in %.1f s" % (k, c.n, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
