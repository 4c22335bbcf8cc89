"""Writes long_baseline_precision_oracle.npz: the FP64 oracle's information potentials of the
first 16 curves of the long-baseline workload (7000-day baselines, N = 1000, frequencies to 20 1/d)
at 256 frequencies each (224 random points of the 20 000-point grid on [1e-3, 20] 1/d plus 32
around the generating frequency of the periodic half; the precision study's sample), for
sigma_t 0.3, 0.1 and 0.6 with Silverman's sigma_y.  The benchmark's precision leg compares the
GPU's mixed and FP64 paths with these stored values.

    python tests/golden/make_precision_golden.py [threads]

Calls only oracle/ (and the seeded input generator).  About 100 core-seconds.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1412_1840_amd import synth  # noqa: E402

N_CURVES = 16
WIDTHS = (0.3, 0.1, 0.6)


def freq_sample(k, c, n_random=224, n_window=32):
    wl = synth.WORKLOADS["long_baseline"]
    grid = O.linear_grid(wl["f_min"], wl["f_max"], wl["n_coarse"])
    rng = np.random.default_rng([4242, k])
    idx = np.sort(rng.choice(len(grid), n_random + (0 if c.periodic else n_window),
                             replace=False))
    f = list(grid[idx])
    if c.periodic:
        f0 = 1.0 / c.period
        half = 2.0 * (grid[1] - grid[0])
        f += list(np.linspace(f0 - half, f0 + half, n_window))
    return np.asarray(f)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    curves = [synth.long_baseline_curve(k) for k in range(N_CURVES)]
    freqs = np.stack([freq_sample(k, c) for k, c in enumerate(curves)])
    sy = [O.silverman_sigma(c.y) for c in curves]
    out = {"freqs": freqs, "widths": np.asarray(WIDTHS), "k": np.arange(N_CURVES)}
    for st in WIDTHS:
        refs = O.batch_information_potentials([c.t for c in curves], [c.y for c in curves],
                                              [st] * N_CURVES, sy, list(freqs), 1, threads)
        tag = "%g" % st
        out["vj_" + tag] = np.stack([r.vj for r in refs])
        out["ipt_" + tag] = np.stack([r.ipt for r in refs])
        out["vc_" + tag] = np.stack([r.vc for r in refs])
        out["ipy_" + tag] = np.array([r.ipy for r in refs])
        out["qmi_" + tag] = np.stack([O.qmi(r) for r in refs])
        print("sigma_t %g done" % st, flush=True)
    np.savez_compressed(os.path.join(HERE, "long_baseline_precision_oracle.npz"), **out)


if __name__ == "__main__":
    main()
