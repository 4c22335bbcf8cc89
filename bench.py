#!/usr/bin/env python3
"""Throughput of the kernelised-periodogram period search on one MI355X.

A step is one full coarse-to-fine search (prologue, magnitude Gram matrix, 20k-frequency coarse
periodogram, top-10 peak selection, 10 x 1000 refinement, best-of) over a resident batch of 4096
seeded survey-like lightcurves (N uniform in 300..1000, half periodic).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload survey_batch]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "lightcurves/sec (N~600, 20k freqs) vs plain; Gpairs/s % VALU peak; p99 ms"

# VALU roofline of the pair sums, from unit counts: each pair x frequency item needs 6 FP32 VALU
# instructions (a multiply and two FMAs for the squared half-angle sine, two adds and an FMA for
# the three accumulations) and one v_exp_f32.  The VALU issues one FP32 instruction per lane per
# clock (packed FP32 is not used), 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, and in the pair body the
# exp overlaps the other VALU work (the valu_rates probe measures the body at 90% of this bound, far
# above the 8-slot count of an exp at its own half rate), so the ceiling is 6 issue slots per item.
PEAK_ITEMS_PER_S = 256 * 64 * 2.4e9 / 6.0
# FP32 flops per item (FMA = 2) against MI355X's published FP32 vector peak, which counts packed
# (two-wide) FP32 instructions.
FLOP_PER_ITEM = 10.0
PUBLISHED_FP32_FLOPS = 157.3e12


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
    ap.add_argument("--cpu-freqs", type=int, default=4096,
                    help="coarse frequencies of the CPU-oracle sample (about 10 s on 16 cores)")
    ap.add_argument("--no-probe", action="store_true", help="skip the VALU rate probe")
    ap.add_argument("--serve-requests", type=int, default=5000,
                    help="measured requests per serving load (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="Poisson arrival rate as a fraction of the measured batch throughput")
    ap.add_argument("--serve-batch", type=int, default=256)
    ap.add_argument("--serve-inflight", type=int, default=4)
    ap.add_argument("--serve-items", type=float, default=1e10,
                    help="pair x frequency items per serving launch (0: no bound)")
    ap.add_argument("--serve-sweep", default="0.25,0.5,0.8",
                    help="comma-separated loads (fractions of the saturated serving throughput, "
                         "measured first; empty: one load, --serve-load of the batch rate)")
    ap.add_argument("--serve-warmup", type=int, default=500,
                    help="requests served first and left out of the latency statistics")
    ap.add_argument("--tile", type=int, default=0,
                    help="force pair-kernel variant k-1 (0: autotuned)")
    ap.add_argument("--no-graph-check", action="store_true")
    ap.add_argument("--fp64-curves", type=int, default=256,
                    help="curves of the all-FP64 path timing (0: skip)")
    ap.add_argument("--metric-point-steps", type=int, default=2,
                    help="timed steps of the same search with every curve at N = 600 (0: skip)")
    ap.add_argument("--bands-steps", type=int, default=2,
                    help="timed calls of the bands-method front end on the same batch (0: skip)")
    ap.add_argument("--precision", type=int, default=1,
                    help="compare the mixed and FP64 paths with the stored FP64 oracle values of "
                         "16 long-baseline curves (0: skip)")
    ap.add_argument("--length-sweep", default="",
                    help="comma-separated curve lengths: print the pair kernel's rate per length "
                         "(survey-batch generator at fixed N, 20 000 + 10 x 1000 frequencies) as "
                         "JSON lines and exit")
    ap.add_argument("--survey-curves", type=int, default=16384,
                    help="survey-stream curves timed in batches of 2048 with host inputs (0: skip)")
    return ap.parse_args()


def serving(qmi, synth, wl, st_, rate, n_req, max_batch, inflight, warmup=0, curves=None,
            max_items=0):
    """Poisson stream of single-curve requests (serving-stream lengths, survey mix and search)
    into the continuous-batching loop; latency = completion (poll) - arrival, host clock.
    rate = inf submits every request at once (saturated throughput).  The first ``warmup``
    requests are served but left out of the statistics."""
    import threading

    if curves is None:
        curves = [synth.serving_curve(k) for k in range(n_req)]
    arrivals = (np.zeros(n_req) if not np.isfinite(rate)
                else synth.poisson_arrivals(0, n_req, rate))
    ctx = qmi.Context(0)
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    ctx.serve_start(st_, max_batch=max_batch, max_inflight=inflight, max_batch_items=max_items,
                    **kw)
    t_arr = np.zeros(n_req)
    t_done = np.full(n_req, np.nan)
    status = np.zeros(n_req, np.int32)
    t0 = time.perf_counter()

    def submitter():
        for k, c in enumerate(curves[:n_req]):
            delay = t0 + arrivals[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            t_arr[k] = time.perf_counter()
            while not ctx.submit(c.t, c.y, c.e, tag=k):
                time.sleep(0.0005)

    th = threading.Thread(target=submitter)
    th.start()
    got = 0
    deadline = t0 + arrivals[-1] + 120.0 + (n_req / 50.0 if not np.isfinite(rate) else 0.0)
    next_note = 5000
    while got < n_req and time.perf_counter() < deadline:
        res, tags = ctx.poll(256, 2000)
        now = time.perf_counter()
        for r, tg in zip(res, tags):
            t_done[int(tg)] = now
            status[int(tg)] = r["status"]
        got += len(tags)
        if got >= next_note:
            print("serving: %d of %d requests done after %.1f s" % (got, n_req, now - t0),
                  file=sys.stderr, flush=True)
            next_note += 5000
    th.join()
    ctx.serve_stop()
    ctx.close()
    lat = (t_done - t_arr) * 1e3
    ok = np.isfinite(lat)
    ok[:warmup] = False
    # Throughput over the measured requests: from the first measured arrival to the last
    # completion.
    t_first = t_arr[warmup] if warmup < n_req else t0
    span = np.nanmax(t_done[warmup:]) - t_first
    return {"requests": n_req, "warmup_requests": warmup, "completed": int(ok.sum()),
            "arrival_rate_per_s": None if not np.isfinite(rate) else rate,
            "p50_ms": float(np.percentile(lat[ok], 50)),
            "p99_ms": float(np.percentile(lat[ok], 99)),
            "max_ms": float(np.max(lat[ok])), "throughput_per_s": float(ok.sum() / span),
            "max_batch": max_batch, "max_inflight": inflight, "max_batch_items": max_items,
            "lengths": "round(lognormal(ln 500, 0.5)) in [50, 2000]",
            "bad_status": int(np.sum(status != 0))}


def synth_curve(workload, k):
    from paper_1412_1840_amd import synth

    return {"survey_batch": synth.survey_batch_curve, "long_baseline": synth.long_baseline_curve,
            "serving_stream": synth.serving_curve,
            "survey_stream": synth.survey_stream_curve}[workload](k)


def classification_report(qmi, res, truth):
    """Thresholds per SNR bin calibrated (F1-maximising sweep, Sec. 4.1) on the curves with
    k mod 4 in {0, 1}, evaluated on the others: per bin and overall precision, recall, F1 and hit
    rate (periodic, classified periodic and period recovered within 1 / (2T), over all periodic
    curves; Sec. 3.2)."""
    nc = len(truth)
    is_per = np.array([c.periodic for c in truth])
    rec = np.array([bool(c.periodic) and abs(res["f_best"][k] - 1.0 / c.period)
                    <= 0.5 / float(c.t.max() - c.t.min()) for k, c in enumerate(truth)])
    train = np.array([k % 4 < 2 for k in range(nc)])
    cal = qmi.calibrate(res["score_qmi"][train], res["psnr"][train], is_per[train])
    th = [float(x) if np.isfinite(x) else 1e300 for x in cal["th"]]
    dec = qmi.discriminate(res, qmi.SNR_EDGES, th) == qmi.PERIODIC
    test = ~train

    def quality(sel):
        tp = int(np.sum(dec & is_per & sel))
        fp = int(np.sum(dec & ~is_per & sel))
        fn = int(np.sum(~dec & is_per & sel))
        tps = int(np.sum(dec & rec & sel))
        n_per = int(np.sum(is_per & sel))
        p = tp / (tp + fp) if tp + fp else None
        r = tp / (tp + fn) if tp + fn else None
        f1 = (2 * p * r / (p + r)) if p and r else None
        return {"curves": int(np.sum(sel)), "periodic": n_per, "precision": p, "recall": r,
                "f1": f1, "hit_rate": tps / n_per if n_per else None}

    edges = list(qmi.SNR_EDGES)
    bins = np.array([np.searchsorted(edges, v, side="right") - 1 if np.isfinite(v) else -1
                     for v in res["psnr"]])
    per_bin = []
    for b in range(len(edges) - 1):
        q = quality(test & (bins == b))
        q["bin"] = [edges[b], edges[b + 1] if np.isfinite(edges[b + 1]) else None]
        q["threshold"] = th[b] if th[b] < 1e300 else None
        per_bin.append(q)
    return {"score": "qmi", "calibrated_on": "k mod 4 in {0,1}", "evaluated_on": "k mod 4 in {2,3}",
            "overall": quality(test), "per_snr_bin": per_bin}


def kernel_code_digest(root=ROOT):
    """sha256 of the pair kernel's sources (csrc/qmi_kernels.hip, then csrc/qmi_internal.h) with
    comments and white space removed, so that editing a comment keeps recorded counters valid."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in ("qmi_kernels.hip", "qmi_internal.h"):
        with open(os.path.join(root, "paper_1412_1840_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(workload, n_curves, variant):
    """HBM bytes per pair-kernel launch from the committed counter summary, or None unless the
    counters were taken on this workload, this variant and the current kernel code."""
    path = os.path.join(ROOT, "profiles", "pairs_kernel_survey_batch_4096_traffic.txt")
    if workload != "survey_batch" or n_curves != 4096 or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    digest = kernel_code_digest()
    if kv.get("kernel_source_sha256") != digest or int(kv.get("variant", -99)) != variant:
        return None
    return float(kv["bytes_per_launch"])


def valu_probe():
    import subprocess

    exe = os.path.join(ROOT, "paper_1412_1840_amd", "valu_rates")
    if not os.path.exists(exe):
        return None
    try:
        out = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                             timeout=120)
        return json.loads(out.stdout.strip().splitlines()[-1]) if out.returncode == 0 else None
    except Exception:
        return None


def precision_report(qmi, synth):
    """The mixed and FP64 paths against stored FP64 oracle values (tests/golden/
    long_baseline_precision_oracle.npz, written by make_precision_golden.py from the oracle): 16
    long-baseline curves (7000-day baselines, N = 1000) at 256 frequencies up to 20 1/d, for
    sigma_t 0.3, 0.1 and 0.6.  QMI error |dQMI| / max(|QMI_ref|, 1e-3 max |QMI_ref|) per curve,
    max and p99.9 over all points; largest relative error of V_J, IP_t, V_C."""
    path = os.path.join(ROOT, "tests", "golden", "long_baseline_precision_oracle.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    curves = [synth.long_baseline_curve(int(k)) for k in g["k"]]
    freqs = g["freqs"]
    out = {"workload": "long_baseline: first %d curves, N = 1000, 7000-day baselines, %d "
                       "frequencies each on [1e-3, 20] 1/d" % (len(curves), freqs.shape[1]),
           "reference": "stored FP64 oracle values", "by_sigma_t": {}}
    ctx = qmi.Context(0)
    for st in g["widths"]:
        tag = "%g" % st
        rq = g["qmi_" + tag]
        rv = (g["vj_" + tag], g["ipt_" + tag], g["vc_" + tag])
        rec = {}
        for name, prec in (("mixed", qmi.PREC_MIXED), ("fp64", qmi.PREC_FP64)):
            qe, ve = [], []
            for k, c in enumerate(curves):
                sc, ips, _, status = ctx.periodogram([0, c.n], c.t, c.y, c.e, freqs[k], float(st),
                                                     precision=prec, want_ips=True)
                den = np.maximum(np.abs(rq[k]), 1e-3 * np.max(np.abs(rq[k])))
                qe.append(np.abs(sc[0] - rq[k]) / den)
                ve.append(max(float(np.max(np.abs(ips[0, :, i] / rv[i][k] - 1.0)))
                              for i in range(3)))
            q = np.concatenate(qe)
            rec[name] = {"qmi_err_max": float(q.max()),
                         "qmi_err_p999": float(np.quantile(q, 0.999)),
                         "v_rel_err_max": float(max(ve)), "points": int(q.size)}
        out["by_sigma_t"][tag] = rec
    ctx.close()
    return out


def survey_report(qmi, synth, n_curves, batch=2048):
    """Survey-scale stream (survey-stream workload: N lognormal(ln 500, 0.4) in [100, 1500], 1%
    periodic, 30 000 coarse + 10 x 1000 refined frequencies): n_curves curves in batches with host
    inputs (copies included), wall time; lightcurves per hour and the VALU roofline fraction on
    wall time."""
    wl = synth.WORKLOADS["survey_stream"]
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    batches = [synth.make_batch("survey_stream", range(a, min(a + batch, n_curves)))
               for a in range(0, n_curves, batch)]
    ctx = qmi.Context(0)
    ctx.best_period(batches[0].offsets, batches[0].t, batches[0].y, batches[0].e,
                    wl["sigma_t"], **kw)  # warm-up (and autotune)
    t0 = time.perf_counter()
    items = 0.0
    ok = 0
    for b in batches:
        res, _ = ctx.best_period(b.offsets, b.t, b.y, b.e, wl["sigma_t"], **kw)
        items += ctx.stats()["pair_items"]
        ok += int(np.sum(res["status"] == 0))
    dt = time.perf_counter() - t0
    ctx.close()
    return {"curves": n_curves, "batch": batch, "host_inputs": True, "status_ok": ok,
            "value": n_curves / dt * 3600.0, "unit": "lightcurves/hour",
            "gpairs_per_s": items / dt / 1e9, "roofline_frac_wall": items / dt / PEAK_ITEMS_PER_S}


def length_sweep(qmi, synth, lengths, tile=0):
    """Pair-kernel rate by curve length: a resident batch of equal-length curves of the survey
    generator (enough of them for at least ~2e13 pair x frequency items, at most 4096), the
    coarse-to-fine search of the survey batch, HIP-event time of the pair launches."""
    import torch

    wl = synth.WORKLOADS["survey_batch"]
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    dev = torch.device("cuda:0")
    for n in lengths:
        per_curve = n * (n - 1) / 2.0 * (wl["n_coarse"] + wl["top_k"] * wl["n_fine"])
        nc = int(max(64, min(4096, math.ceil(2e13 / per_curve))))
        b = synth.make_batch("survey_batch", range(nc), n=n)
        T, Y, E = (torch.from_numpy(x).to(dev) for x in (b.t, b.y, b.e))
        ctx = qmi.Context(0, stream=torch.cuda.current_stream().cuda_stream)
        ctx.set_option(qmi.OPT_USE_GRAPH, 0)
        if tile:
            ctx.set_option(qmi.OPT_TILE, tile)
        ctx.best_period_dev(b.offsets, T, Y, E, wl["sigma_t"], **kw)  # warm-up (and autotune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.best_period_dev(b.offsets, T, Y, E, wl["sigma_t"], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = ctx.stats()
        rate = s["pair_items"] / (s["pair_kernel_ms"] * 1e-3)
        print(json.dumps({"n": n, "curves": nc, "pair_items": s["pair_items"],
                          "pair_kernel_ms": s["pair_kernel_ms"], "items_per_s": rate,
                          "frac_of_peak": rate / PEAK_ITEMS_PER_S, "variant": s["pair_variant"],
                          "wall_items_per_s": s["pair_items"] / dt,
                          "lightcurves_per_s": nc / dt}), flush=True)
        ctx.close()
        del T, Y, E


def roofline_object(achieved, probe, pair_ms, launches, traffic, variant):
    """The pair kernel against the 6-slot VALU issue bound, with the rates the probe measured in
    this run beside it: the kernel's own column body (as compiled and with the exp-interleaving
    hint), one exp with 6 and 7 independent FMAs, exp and FMA alone."""
    measured = None
    best = None
    if probe:
        mix = probe.get("mix_items_per_s", {})
        measured = {"pair_body": probe.get("pair_items_per_s"),
                    "pair_body_interleaved": probe.get("pair_hint_items_per_s"),
                    "mix_1exp_6fma": mix.get("6"), "mix_1exp_7fma": mix.get("7"),
                    "exp_alone": probe.get("exp_per_s"), "fma_alone": probe.get("fma_per_s"),
                    "clock_mhz_reported": probe.get("clock_mhz")}
        cands = [v for k, v in measured.items()
                 if k.startswith(("pair", "mix_1exp_6")) and v]
        best = max(cands) if cands else None
    return {"bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_ITEMS_PER_S / 1e9,
            "unit": "G pair*freq items/s", "frac": achieved / PEAK_ITEMS_PER_S,
            "peak_basis": "6 FP32 VALU issue slots per item, 256 CUs x 64 lanes x 2.4 GHz",
            "best_measured_ceiling": best and best / 1e9,
            "frac_of_best_measured": best and achieved / best,
            "measured_rates_per_s": measured,
            "fp32_flop_per_item": FLOP_PER_ITEM,
            "frac_of_published_fp32_peak": achieved * FLOP_PER_ITEM / PUBLISHED_FP32_FLOPS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
            "kernel": "pairs_kernel<float>", "variant": variant, "launches": launches,
            "avg_launch_ms": pair_ms / max(launches, 1)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d "
              "requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.length_sweep:
        from paper_1412_1840_amd import qmi, synth

        length_sweep(qmi, synth, [int(x) for x in a.length_sweep.split(",")], a.tile)
        return
    probe = None if a.no_probe else valu_probe()
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
    # The timed steps run the device section eagerly so that HIP events around each pair-kernel
    # launch give its duration (at seconds per step, graph replay would change nothing measurable);
    # graph replay is measured separately below and used by the serving loop.
    ctx.set_option(qmi.OPT_USE_GRAPH, 0)
    if a.tile:
        ctx.set_option(qmi.OPT_TILE, a.tile)
    kw = dict(f_min=wl["f_min"], f_max=wl["f_max"], n_coarse=wl["n_coarse"], top_k=wl["top_k"],
              n_fine=wl["n_fine"])
    st_ = wl["sigma_t"]

    def step():
        return ctx.best_period_dev(batch.offsets, T, Y, E, st_, **kw)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    print("bench: %d warm-up steps done" % a.warmup, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pair_ms = 0.0
    items = 0.0
    launches = 0
    for i in range(a.steps):
        res = step()
        s = ctx.stats()
        pair_ms += s["pair_kernel_ms"]
        items += s["pair_items"]
        launches += s["pair_launches"]
        if (i + 1) % 5 == 0:
            print("bench: %d of %d timed steps done" % (i + 1, a.steps), file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = int(np.sum(res["status"] == 0))
    variant = s["pair_variant"]
    # The same step replayed from a captured hipGraph (first call captures, second replays).
    graph = None
    if not a.no_graph_check:
        ctx.set_option(qmi.OPT_USE_GRAPH, 1)
        step()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        res_g = step()
        torch.cuda.synchronize()
        graph = {"ms_per_step": 1e3 * (time.perf_counter() - g0),
                 "used": ctx.stats()["used_graph"],
                 "same_results": bool(np.array_equal(res_g, res))}
    value = nc * a.steps / dt
    ms_per_step = 1e3 * dt / a.steps
    achieved = items / (pair_ms * 1e-3) if pair_ms > 0 else float("nan")
    items_per_curve = items / a.steps / max(ok, 1)

    # Plain per-curve path: one curve per call, same search, on the same context.
    plain = None
    if a.plain_sample > 0:
        ks = list(range(min(a.plain_sample, nc)))
        # One untimed single-curve call first, on the sample's longest curve: it sizes the
        # context's buffers for this launch form (the piece sums, the K table), as a long run of
        # per-curve calls would have them; allocation is not part of the path.
        kmax = max(ks, key=lambda k: int(batch.offsets[k + 1] - batch.offsets[k]))
        lo, hi = int(batch.offsets[kmax]), int(batch.offsets[kmax + 1])
        ctx.best_period_dev([0, hi - lo], T[lo:hi], Y[lo:hi], E[lo:hi], st_, **kw)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        call_ms = []
        for k in ks:
            lo, hi = int(batch.offsets[k]), int(batch.offsets[k + 1])
            c0 = time.perf_counter()
            ctx.best_period_dev([0, hi - lo], T[lo:hi], Y[lo:hi], E[lo:hi], st_, **kw)
            call_ms.append(1e3 * (time.perf_counter() - c0))
        torch.cuda.synchronize()
        pdt = time.perf_counter() - p0
        pitems = sum(float(n) * (n - 1) / 2.0 for n in np.diff(batch.offsets)[ks])
        bitems = sum(float(n) * (n - 1) / 2.0 for n in np.diff(batch.offsets))
        # Scale the sample to the batch by pair work, so that the ratio compares like with like.
        plain_value = nc / (pdt * bitems / pitems)
        plain = {"value": plain_value, "sample_curves": len(ks), "speedup": value / plain_value,
                 "call_p50_ms": float(np.percentile(call_ms, 50)),
                 "call_p99_ms": float(np.percentile(call_ms, 99))}

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
        # The same oracle on one thread (first curve, 64 of the frequencies).
        f1 = fr[:64]
        c1 = time.perf_counter()
        O.batch_information_potentials([cs[0].t], [cs[0].y], [st_], [O.silverman_sigma(cs[0].y)],
                                       [f1], 1, 1)
        c1dt = time.perf_counter() - c1
        items1 = cs[0].n * (cs[0].n - 1) / 2.0 * len(f1)
        cpu = {"value": (citems / cdt) / items_per_curve, "unit": "lightcurves/s",
               "cores": threads, "kind": "oracle",
               "single_thread_value": (items1 / c1dt) / items_per_curve,
               "single_thread_items_per_s": items1 / c1dt,
               "sample": "FP64 oracle pair sums of %d curves x %d coarse frequencies (%.3g pair*f "
                         "items in %.1f s = %.3g items/s), scaled by the %.3g items one curve of "
                         "the workload needs" % (len(cs), len(fr), citems, cdt, citems / cdt,
                                                 items_per_curve)}

    # The metric's own point: every curve of the batch generator at N = 600, 20 000 coarse
    # frequencies plus the refinement, timed like the main steps.
    metric_point = None
    if a.metric_point_steps > 0 and a.workload == "survey_batch":
        mb = synth.make_batch(a.workload, range(a.n_curves), n=600)
        MT = torch.from_numpy(mb.t).to(dev)
        MY = torch.from_numpy(mb.y).to(dev)
        ME = torch.from_numpy(mb.e).to(dev)
        ctx.best_period_dev(mb.offsets, MT, MY, ME, st_, **kw)
        torch.cuda.synchronize()
        m0 = time.perf_counter()
        mitems = 0.0
        for _ in range(a.metric_point_steps):
            ctx.best_period_dev(mb.offsets, MT, MY, ME, st_, **kw)
            mitems += ctx.stats()["pair_items"]
        torch.cuda.synchronize()
        mdt = time.perf_counter() - m0
        metric_point = {"n": 600, "n_curves": mb.n_curves,
                        "value": mb.n_curves * a.metric_point_steps / mdt,
                        "unit": "lightcurves/s", "gpairs_per_s": mitems / mdt / 1e9,
                        "roofline_frac_wall": mitems / mdt / PEAK_ITEMS_PER_S}
        del MT, MY, ME

    # The all-FP64 path (QMI_PREC_FP64) on the first curves of the batch: the cost of full
    # precision against the mixed path timed above.
    fp64 = None
    if a.fp64_curves > 0:
        k64 = min(a.fp64_curves, nc)
        o64 = batch.offsets[:k64 + 1]
        s64 = int(o64[-1])
        ctx.best_period_dev(o64, T[:s64], Y[:s64], E[:s64], st_, precision=qmi.PREC_FP64, **kw)
        torch.cuda.synchronize()
        d0 = time.perf_counter()
        ctx.best_period_dev(o64, T[:s64], Y[:s64], E[:s64], st_, precision=qmi.PREC_FP64, **kw)
        torch.cuda.synchronize()
        d64 = time.perf_counter() - d0
        i64 = ctx.stats()["pair_items"]
        fp64 = {"curves": k64, "value": k64 / d64, "unit": "lightcurves/s",
                "gpairs_per_s": i64 / d64 / 1e9,
                "mixed_over_fp64": (items / (dt)) / (i64 / d64)}

    # Bands-method front end (Sec. 3.1: 3 bands x 150 trial frequencies instead of the coarse
    # grid and refinement) on the same batch, and the period recovery of both front ends against
    # the generator's truth: a periodic curve's period counts as recovered when the best frequency
    # lies within half a Fourier resolution element, 1 / (2 T), of the generating one.
    bands = None
    if a.bands_steps > 0 and a.workload in ("survey_batch", "long_baseline", "serving_stream",
                                             "survey_stream"):
        hb = synth.make_batch(a.workload, range(a.n_curves))
        bctx = qmi.Context(0)
        bctx.bands_best_period(hb.offsets, hb.t, hb.y, hb.e, st_)  # warm-up (and autotune)
        b0 = time.perf_counter()
        bitems = 0.0
        for _ in range(a.bands_steps):
            bres, _, _ = bctx.bands_best_period(hb.offsets, hb.t, hb.y, hb.e, st_)
            bitems += bctx.stats()["pair_items"]
        bdt = time.perf_counter() - b0
        bctx.close()
        truth = [synth_curve(a.workload, k) for k in range(nc)]
        per = [k for k, c in enumerate(truth) if c.periodic]

        def recovered(r, k):
            c = truth[k]
            span = float(c.t.max() - c.t.min())
            return bool(abs(r["f_best"][k] - 1.0 / c.period) <= 0.5 / span)

        in_range = [k for k in per if 1.0 / truth[k].period >= 0.00125 and
                    1.0 / truth[k].period <= 3.0]
        bands = {"value": nc * a.bands_steps / bdt, "unit": "lightcurves/s",
                 "ms_per_step": 1e3 * bdt / a.bands_steps,
                 "host_inputs": True,
                 "gpairs_per_s": bitems / bdt / 1e9,
                 "trials_per_curve": "3 bands x 150 local maxima of the spectral window on 30000 "
                                     "points of [0.00125, 3] 1/d",
                 "periodic_curves": len(per),
                 "recovered_bands": sum(recovered(bres, k) for k in per) / max(len(per), 1),
                 "recovered_coarse_to_fine": sum(recovered(res, k) for k in per)
                 / max(len(per), 1),
                 "periodic_in_bands_range": len(in_range),
                 "recovered_bands_in_range": sum(recovered(bres, k) for k in in_range)
                 / max(len(in_range), 1),
                 "recovered_coarse_to_fine_in_range": sum(recovered(res, k) for k in in_range)
                 / max(len(in_range), 1)}

    # Classification quality of the discriminator (Sec. 4.1) against the generator's truth.
    classification = None
    if a.workload in ("survey_batch", "long_baseline", "serving_stream", "survey_stream"):
        classification = classification_report(
            qmi, res, [synth_curve(a.workload, k) for k in range(nc)])

    precision = precision_report(qmi, synth) if a.precision else None
    print("bench: precision leg done", file=sys.stderr, flush=True)
    survey = survey_report(qmi, synth, a.survey_curves) if a.survey_curves > 0 else None
    print("bench: survey-stream leg done", file=sys.stderr, flush=True)

    serve = None
    sweep = None
    if a.serve_requests > 0 and a.serve_sweep:
        n_req = a.serve_requests + a.serve_warmup
        curves = [synth.serving_curve(k) for k in range(n_req)]
        sat = serving(qmi, synth, wl, st_, float("inf"), n_req, a.serve_batch, a.serve_inflight,
                      warmup=a.serve_warmup, curves=curves, max_items=a.serve_items)
        print("serving saturated: %.1f requests/s" % sat["throughput_per_s"], file=sys.stderr,
              flush=True)
        sweep = {"saturated": sat, "loads": []}
        for load in [float(x) for x in a.serve_sweep.split(",")]:
            r = serving(qmi, synth, wl, st_, load * sat["throughput_per_s"], n_req, a.serve_batch,
                        a.serve_inflight, warmup=a.serve_warmup, curves=curves,
                        max_items=a.serve_items)
            r["load"] = load
            print("serving at %.2f of saturation: p50 %.1f ms p99 %.1f ms, %.1f requests/s"
                  % (load, r["p50_ms"], r["p99_ms"], r["throughput_per_s"]), file=sys.stderr,
                  flush=True)
            sweep["loads"].append(r)
        serve = min(sweep["loads"], key=lambda r: abs(r["load"] - 0.5))
    elif a.serve_requests > 0:
        serve = serving(qmi, synth, wl, st_, a.serve_load * value,
                        a.serve_requests + a.serve_warmup, a.serve_batch, a.serve_inflight,
                        warmup=a.serve_warmup, max_items=a.serve_items)

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
        "roofline": roofline_object(achieved, probe, pair_ms, launches,
                                    measured_traffic(a.workload, nc, variant), variant),
        "graph": graph,
        "bands": bands,
        "metric_point": metric_point,
        "fp64_path": fp64,
        "classification": classification,
        "precision": precision,
        "survey_stream": survey,
        "plain": plain,
        "serving": serve,
        "serving_sweep": sweep,
        "p99_ms": serve and serve["p99_ms"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
