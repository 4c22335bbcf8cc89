"""Survey-scale streaming: lightcurves from a source are searched in large batches through
qmi_best_period, with a checkpoint after every batch so that an interrupted run resumes where it
stopped and produces the same bytes as an uninterrupted one.

Layout of an output directory:

* ``results.bin``      one ``qmi.RESULT_DTYPE`` record (104 bytes) per curve, in curve order;
* ``checkpoint.json``  the run's configuration, the number of curves whose records are in
                       ``results.bin``, that file's length at that point, and running totals
                       (pair items, pair-kernel and wall time).

A batch is appended and flushed to disk before the checkpoint that covers it is written (to a
temporary file, flushed, then renamed over the old one), so the checkpoint never points past data
that is on disk.  On resume, bytes of ``results.bin`` beyond the checkpointed length (a batch
written after the last checkpoint) are cut off and that batch is searched again.

Batches are generated on a producer thread while the device works on the previous one (the
library call releases the GIL).  Batch size is a number of curves, chosen large enough that a
batch fills every compute unit through the tail of the coarse and the refinement launches; the
pair-kernel variant is chosen by the library's autotuner for the batch's length bucket.  With
spurious-period masks (Sec. 6.1) every search of the run leaves out candidates under a mask; the
masks are part of the run's configuration.

    python -m paper_1412_1840_amd.survey --out DIR --curves 125000 [--batch 2048] [--first 0]
        [--spurious-amplitude A [--spurious-width W]]
"""
from __future__ import annotations

import argparse
import json
import os
import queue
import sys
import threading
import time
from typing import Callable, Optional

import numpy as np

from . import synth

CHECKPOINT = "checkpoint.json"
RESULTS = "results.bin"


def _fsync_write(path: str, data: bytes) -> None:
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(data)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


class SurveyRunner:
    """Streams curves ``first .. first + n_curves - 1`` of ``source`` through ``compute``.

    ``source(k) -> synth.Curve``; ``compute(batch) -> (results, stats)`` where ``results`` is a
    ``qmi.RESULT_DTYPE`` array of the batch's curves and ``stats`` a dict with ``pair_items`` and
    ``pair_kernel_ms`` (the default runs qmi_best_period on device ``device``).
    """

    def __init__(self, out_dir: str, n_curves: int, source: Callable[[int], synth.Curve],
                 source_name: str, search: dict, sigma_t: float, batch_curves: int = 2048,
                 first: int = 0, device: int = 0, compute=None, result_dtype=None,
                 masks=None):
        if n_curves < 0 or batch_curves < 1:
            raise ValueError("n_curves must be >= 0 and batch_curves >= 1")
        self.out_dir = out_dir
        self.n_curves = int(n_curves)
        self.first = int(first)
        self.source = source
        self.batch_curves = int(batch_curves)
        self.config = {"source": source_name, "first": self.first, "n_curves": self.n_curves,
                       "sigma_t": float(sigma_t), "search": dict(search),
                       "batch_curves": self.batch_curves}
        self.masks = [tuple(float(v) for v in m) for m in (masks or [])]
        if self.masks:
            self.config["masks"] = [list(m) for m in self.masks]
        self.search = dict(search)
        self.sigma_t = float(sigma_t)
        self.device = device
        self._compute = compute
        self._ctx = None
        if result_dtype is None:
            from . import qmi
            result_dtype = qmi.RESULT_DTYPE
        self.dtype = np.dtype(result_dtype)

    # ---------------------------------------------------------------- state on disk
    def _load(self) -> dict:
        path = os.path.join(self.out_dir, CHECKPOINT)
        if not os.path.exists(path):
            return {"config": self.config, "done": 0, "bytes": 0, "pair_items": 0.0,
                    "pair_kernel_ms": 0.0, "wall_s": 0.0, "batches": 0}
        with open(path) as f:
            ck = json.load(f)
        if ck["config"] != self.config:
            raise ValueError("checkpoint in %s was written by a different run configuration: %s"
                             % (self.out_dir, ck["config"]))
        return ck

    def _save(self, ck: dict) -> None:
        _fsync_write(os.path.join(self.out_dir, CHECKPOINT),
                     json.dumps(ck, indent=1).encode())

    # ---------------------------------------------------------------- compute
    def _default_compute(self, batch: synth.Batch):
        from . import qmi
        if self._ctx is None:
            self._ctx = qmi.Context(self.device)
            # Batches differ in composition, so a captured graph would never be replayed; eager
            # launches also let the library time the pair kernels.
            self._ctx.set_option(qmi.OPT_USE_GRAPH, 0)
            self._ctx.set_masks(self.masks)
        s = self.search
        res, _ = self._ctx.best_period(batch.offsets, batch.t, batch.y, batch.e, self.sigma_t,
                                       f_min=s["f_min"], f_max=s["f_max"],
                                       n_coarse=s["n_coarse"], top_k=s["top_k"],
                                       n_fine=s["n_fine"])
        return res, self._ctx.stats()

    def close(self):
        if self._ctx is not None:
            self._ctx.close()
            self._ctx = None

    # ---------------------------------------------------------------- run
    def run(self, max_batches: Optional[int] = None, log=None) -> dict:
        """Searches the remaining curves (at most ``max_batches`` batches); returns the
        checkpoint dictionary with the running totals."""
        os.makedirs(self.out_dir, exist_ok=True)
        ck = self._load()
        res_path = os.path.join(self.out_dir, RESULTS)
        # Drop anything written after the last checkpoint.
        mode = "r+b" if os.path.exists(res_path) else "w+b"
        with open(res_path, mode) as f:
            f.truncate(ck["bytes"])
        compute = self._compute or self._default_compute
        starts = list(range(ck["done"], self.n_curves, self.batch_curves))
        if max_batches is not None:
            starts = starts[:max(0, int(max_batches))]
        q: "queue.Queue" = queue.Queue(maxsize=2)
        stop = threading.Event()

        def producer():
            try:
                for s0 in starts:
                    if stop.is_set():
                        return
                    s1 = min(s0 + self.batch_curves, self.n_curves)
                    curves = [self.source(self.first + k) for k in range(s0, s1)]
                    q.put((s0, s1, synth.pack(curves)))
                q.put(None)
            except BaseException as exc:  # surfaced on the consumer side
                q.put(exc)

        th = threading.Thread(target=producer, daemon=True)
        th.start()
        try:
            with open(res_path, "ab") as out:
                # A batch's wall time runs from the end of the previous one (or the start), so
                # that time spent waiting for the producer is counted.
                t0 = time.perf_counter()
                while True:
                    item = q.get()
                    if item is None:
                        break
                    if isinstance(item, BaseException):
                        raise item
                    s0, s1, batch = item
                    assert s0 == ck["done"], (s0, ck["done"])
                    res, stats = compute(batch)
                    res = np.ascontiguousarray(res, dtype=self.dtype)
                    if len(res) != s1 - s0:
                        raise RuntimeError("compute returned %d results for %d curves"
                                           % (len(res), s1 - s0))
                    out.write(res.tobytes())
                    out.flush()
                    os.fsync(out.fileno())
                    t1 = time.perf_counter()
                    dt, t0 = t1 - t0, t1
                    ck["done"] = s1
                    ck["bytes"] += res.nbytes
                    ck["batches"] += 1
                    ck["pair_items"] += float(stats.get("pair_items", 0.0))
                    ck["pair_kernel_ms"] += float(stats.get("pair_kernel_ms", 0.0))
                    ck["wall_s"] += dt
                    self._save(ck)
                    if log:
                        log("batch %d: curves %d..%d done (%d of %d) in %.2f s, %.3g pair items"
                            % (ck["batches"], s0, s1 - 1, s1, self.n_curves, dt,
                               float(stats.get("pair_items", 0.0))))
        finally:
            stop.set()
            # Unblock a producer waiting on a full queue, then let it finish.
            while th.is_alive():
                try:
                    q.get_nowait()
                except queue.Empty:
                    pass
                th.join(timeout=0.05)
        return ck

    def results(self) -> np.ndarray:
        """The records written so far (curve order)."""
        path = os.path.join(self.out_dir, RESULTS)
        ck = self._load()
        with open(path, "rb") as f:
            data = f.read(ck["bytes"])
        return np.frombuffer(data, dtype=self.dtype)


SOURCES = {
    "survey_stream": synth.survey_stream_curve,
    "survey_batch": synth.survey_batch_curve,
    "serving_stream": synth.serving_curve,
    "long_baseline": synth.long_baseline_curve,
}

# VALU issue bound of the pair sums: 256 CUs x 64 FP32 lanes x 2.4 GHz / 6 FP32 VALU instructions
# per pair x frequency item (the exp overlaps them).
PEAK_ITEMS_PER_S = 256 * 64 * 2.4e9 / 6.0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--source", default="survey_stream", choices=sorted(SOURCES))
    ap.add_argument("--curves", type=int, default=125000)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--max-batches", type=int, default=None)
    ap.add_argument("--device", type=int, default=0)
    ap.add_argument("--spurious-amplitude", type=float, default=None,
                    help="mask the table of spurious periods (Sec. 6.1) at this amplitude, in "
                         "units of the searched score")
    ap.add_argument("--spurious-width", type=float, default=0.5,
                    help="mask sigma in Fourier resolution elements of a 2335-day span")
    a = ap.parse_args(argv)
    wl = synth.WORKLOADS[a.source]
    search = {k: wl[k] for k in ("f_min", "f_max", "n_coarse", "top_k", "n_fine")}
    masks = None
    if a.spurious_amplitude is not None:
        from . import qmi
        masks = qmi.spurious_masks(a.spurious_amplitude, width=a.spurious_width)
    run = SurveyRunner(a.out, a.curves, SOURCES[a.source], a.source, search, wl["sigma_t"],
                       batch_curves=a.batch, first=a.first, device=a.device, masks=masks)

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    try:
        ck = run.run(max_batches=a.max_batches, log=log)
    finally:
        run.close()
    elapsed = time.perf_counter() - t0
    res = run.results()
    summary = {
        "source": a.source, "curves_done": ck["done"], "curves_total": a.curves,
        "batches": ck["batches"], "wall_s_total": ck["wall_s"], "this_call_s": elapsed,
        "curves_per_hour": 3600.0 * ck["done"] / ck["wall_s"] if ck["wall_s"] > 0 else None,
        "pair_items": ck["pair_items"],
        "pair_items_per_s": ck["pair_items"] / ck["wall_s"] if ck["wall_s"] > 0 else None,
        "roofline_frac_wall": (ck["pair_items"] / ck["wall_s"] / PEAK_ITEMS_PER_S
                               if ck["wall_s"] > 0 else None),
        "roofline_frac_kernel": (ck["pair_items"] / (ck["pair_kernel_ms"] * 1e-3)
                                 / PEAK_ITEMS_PER_S if ck["pair_kernel_ms"] > 0 else None),
        "bad_status": int(np.sum(res["status"] != 0)),
    }
    print(json.dumps(summary), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
