#!/usr/bin/env python3
"""Throughput of the kernelised-periodogram period search on one MI355X.

A step is one full coarse-to-fine search (prologue, magnitude Gram matrix, 20k-frequency coarse
periodogram, top-10 peak selection, 10 x 1000 refinement, best-of) over a resident batch of 4096
seeded survey-like lightcurves (N uniform in 300..1000, half periodic).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload survey_batch]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "lightcurves/sec (N~600, 20k freqs) vs plain; Gpairs/s % VALU peak; p99 ms"

# VALU roofline of the pair sums (derived from unit counts): each pair x frequency
# item needs 5 FP32 VALU operations and one v_exp_f32 at a quarter of the FP32 rate (4 slots):
# 256 CUs x 64 FP32 lanes x 2.4 GHz / 9 slots.
PEAK_ITEMS_PER_S = 256 * 64 * 2.4e9 / 9.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="survey_batch")
    ap.add_argument("--n-curves", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=16,
                    help="curves timed one per call for the plain per-curve path (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=8,
                    help="curves of the CPU-oracle baseline sample (0: skip)")
    ap.add_argument("--cpu-freqs", type=int, default=512)
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d "
              "requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1412_1840_amd import qmi, synth

    wl = synth.WORKLOADS[a.workload]
    batch = synth.make_batch(a.workload, range(a.n_curves))
    nc = batch.n_curves
    dev = torch.device("cuda:0")
    T = torch.from_numpy(batch.t).to(dev)
    Y = torch.from_numpy(batch.y).to(dev)
    E = torch.from_numpy(batch.e).to(dev)
    stream = torch.cuda.current_stream()
    ctx = qmi.Context(0, stream=stream.cuda_stream)
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    st_ = wl["sigma_t"]

    def step():
        return ctx.best_period_dev(batch.offsets, T, Y, E, st_, **kw)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pair_ms = 0.0
    items = 0.0
    launches = 0
    for _ in range(a.steps):
        res = step()
        s = ctx.stats()
        pair_ms += s["pair_kernel_ms"]
        items += s["pair_items"]
        launches += s["pair_launches"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = int(np.sum(res["status"] == 0))
    value = nc * a.steps / dt
    ms_per_step = 1e3 * dt / a.steps
    achieved = items / (pair_ms * 1e-3) if pair_ms > 0 else float("nan")
    items_per_curve = items / a.steps / max(ok, 1)

    # Plain per-curve path: one curve per call, same search, on the same context.
    plain = None
    if a.plain_sample > 0:
        ks = list(range(min(a.plain_sample, nc)))
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for k in ks:
            lo, hi = int(batch.offsets[k]), int(batch.offsets[k + 1])
            ctx.best_period_dev([0, hi - lo], T[lo:hi], Y[lo:hi], E[lo:hi], st_, **kw)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - p0
        pitems = sum(float(n) * (n - 1) / 2.0 for n in np.diff(batch.offsets)[ks])
        bitems = sum(float(n) * (n - 1) / 2.0 for n in np.diff(batch.offsets))
        # Scale the sample to the batch by pair work, so that the ratio compares like with like.
        plain_value = nc / (pdt * bitems / pitems)
        plain = {"value": plain_value, "sample_curves": len(ks), "speedup": value / plain_value}

    cpu = None
    if a.cpu_sample > 0:
        import oracle as O

        ks = list(range(min(a.cpu_sample, nc)))
        fr = O.linear_grid(wl["f_min"], wl["f_max"], a.cpu_freqs)
        cs = [batch.curve(k) for k in ks]
        threads = O.threads()
        c0 = time.perf_counter()
        O.batch_information_potentials([c.t for c in cs], [c.y for c in cs], [st_] * len(cs),
                                       [O.silverman_sigma(c.y) for c in cs], [fr] * len(cs), 1)
        cdt = time.perf_counter() - c0
        citems = sum(c.n * (c.n - 1) / 2.0 * len(fr) for c in cs)
        cpu = {"value": (citems / cdt) / items_per_curve, "unit": "lightcurves/s",
               "cores": threads, "kind": "oracle",
               "sample": "FP64 oracle pair sums of %d curves x %d coarse frequencies (%.3g pair*f "
                         "items in %.1f s = %.3g items/s), scaled by the %.3g items one curve of "
                         "the workload needs" % (len(cs), len(fr), citems, cdt, citems / cdt,
                                                 items_per_curve)}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "lightcurves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 fold and scores)",
        "data": "synthetic",
        "config": {"workload": "%s: %d lightcurves, N uniform 300..1000, %d coarse + %dx%d fine "
                               "frequencies on [%g, %g] 1/d, sigma_t %g, Silverman sigma_y"
                               % (a.workload, nc, wl["n_coarse"], wl["top_k"], wl["n_fine"],
                                  wl["f_min"], wl["f_max"], st_),
                   "n_curves": nc, "samples": int(batch.offsets[-1])},
        "gpairs_per_s": items / a.steps / (dt / a.steps) / 1e9,
        "roofline": {"bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_ITEMS_PER_S / 1e9,
                     "unit": "G pair*freq items/s", "frac": achieved / PEAK_ITEMS_PER_S,
                     "traffic": None,
                     "kernel": "pairs_kernel<float>", "launches": launches,
                     "avg_launch_ms": pair_ms / max(launches, 1)},
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
