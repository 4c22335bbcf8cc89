"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances, derived from the arithmetic: the mixed-precision path evaluates each
kernel value in FP32 (argument error ~ a few ulp of log2(e)/sigma_t^2, exp2 ~1 ulp) and sums short
runs in FP32 before folding into FP64, so the three information potentials carry relative errors of
order 1e-7; the score target is the per-frequency QMI relative error <= 1e-4, measured against
max(|QMI_ref(f)|, 1e-3 max_f |QMI_ref|).  The FP64 path must agree to 1e-10.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1412_1840_amd import qmi, synth

pytestmark = pytest.mark.gpu

QMI_TOL = 1e-4
V_RTOL = 2e-6


@pytest.fixture(scope="module")
def ctx():
    with qmi.Context(0) as c:
        yield c


def floor_rel(got, ref):
    ref = np.asarray(ref)
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.abs(np.asarray(got) - ref) / den


def pack(curves):
    b = synth.pack(curves)
    return b


def oracle_ips(c, freqs, st=0.3, rule=O.SIGMA_SILVERMAN):
    sy = O.sigma_y_of(c.y, c.e, rule)
    return O.information_potentials(c.t, c.y, st, sy, freqs, mode=1)


RAGGED_N = [2, 3, 37, 64, 255, 256, 257, 300, 513, 600]


def test_periodogram_ragged_sizes(ctx):
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate(RAGGED_N)]
    b = pack(curves)
    freqs = np.concatenate([[0.0, 1.0, 1 / 3.7], O.linear_grid(1e-3, 10.0, 297)])  # 300: 4 tiles + 44
    sc, ips, ipy, st = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3, want_ips=True)
    assert np.all(st == 0)
    worst = 0.0
    for k, c in enumerate(curves):
        ref = oracle_ips(c, freqs)
        # IP_y sums the FP32-rounded Gram values in FP64: relative error ~ 2^-24 / sqrt(N^2).
        np.testing.assert_allclose(ipy[k], ref.ipy, rtol=1e-7)
        ev = [np.max(np.abs(ips[k, :, q] / r - 1)) for q, r in enumerate((ref.vj, ref.ipt, ref.vc))]
        err = floor_rel(sc[k], O.qmi(ref))
        print("N=%d V rel err %.2e %.2e %.2e  QMI floor-rel err max %.2e (f=0: %.2e abs)"
              % (c.n, ev[0], ev[1], ev[2], err.max(), abs(sc[k, 0])))
        worst = max(worst, err.max())
    for k, c in enumerate(curves):
        ref = oracle_ips(c, freqs)
        np.testing.assert_allclose(ips[k, :, 0], ref.vj, rtol=V_RTOL)
        np.testing.assert_allclose(ips[k, :, 1], ref.ipt, rtol=V_RTOL)
        np.testing.assert_allclose(ips[k, :, 2], ref.vc, rtol=V_RTOL)
        assert floor_rel(sc[k], O.qmi(ref)).max() <= QMI_TOL, c.n
        # f = 0: every kernel value is exactly 1, every FP32 partial sum is exact (integers, or
        # bit-identical to the precomputed K sums), so QMI(0) = 0 up to FP64 rounding.
        assert abs(sc[k, 0]) <= 1e-12, (c.n, sc[k, 0])
    print("worst QMI rel err %.3g" % worst)


def test_nckp_score(ctx):
    """nCKP = sqrt(N sigma_t) / IP_y (V_J - V_M) is a difference: where V_J and V_M nearly cancel
    its relative error is that of the V's times (V_J + V_M) / |V_J - V_M|.  The bar: relative error
    <= 1e-4 wherever |V_J - V_M| >= 1e-2 (V_J + V_M) (not cancellation-dominated), and everywhere
    an absolute error within the V's own bar, 2 V_RTOL sqrt(N sigma_t) / IP_y (V_J + V_M)."""
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate([90, 400, 777, 1200])]
    b = pack(curves)
    freqs = np.concatenate([O.linear_grid(1e-3, 10.0, 130),
                            1.0 / np.array([c.period for c in curves if c.periodic])])
    sc, _, _, st = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3, score=qmi.SCORE_NCKP)
    strict_points = 0
    for k, c in enumerate(curves):
        ips = oracle_ips(c, freqs)
        ref = O.nckp(ips)
        vm = ips.ipy * ips.ipt
        scale = math.sqrt(c.n * 0.3) / ips.ipy
        strict = np.abs(ips.vj - vm) >= 1e-2 * (ips.vj + vm)
        strict_points += int(strict.sum())
        rel = np.abs(sc[k] - ref) / np.abs(ref)
        assert rel[strict].max(initial=0.0) <= 1e-4, (c.n, rel[strict].max(initial=0.0))
        assert np.all(np.abs(sc[k] - ref) <= 2 * V_RTOL * scale * (ips.vj + vm)), c.n
    assert strict_points >= 50


@pytest.mark.parametrize("st_", [0.1, 0.6])
def test_other_kernel_widths(ctx, st_):
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate([150, 333])]
    b = pack(curves)
    freqs = O.linear_grid(1e-3, 10.0, 200)
    sc, ips, _, _ = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, st_, want_ips=True)
    for k, c in enumerate(curves):
        ref = oracle_ips(c, freqs, st=st_)
        assert floor_rel(sc[k], O.qmi(ref)).max() <= QMI_TOL
        np.testing.assert_allclose(ips[k, :, 2], ref.vc, rtol=5 * V_RTOL)


def test_fp64_path(ctx):
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate([5, 129, 300])]
    b = pack(curves)
    freqs = O.linear_grid(1e-3, 10.0, 100)
    sc, ips, ipy, st = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3,
                                       precision=qmi.PREC_FP64, want_ips=True)
    for k, c in enumerate(curves):
        ref = oracle_ips(c, freqs)
        # FP64 throughout: library exp/sincospi (~1 ulp) and a different summation order.
        np.testing.assert_allclose(ips[k, :, 0], ref.vj, rtol=1e-11)
        np.testing.assert_allclose(ips[k, :, 1], ref.ipt, rtol=1e-11)
        np.testing.assert_allclose(ips[k, :, 2], ref.vc, rtol=1e-11)
        assert floor_rel(sc[k], O.qmi(ref)).max() <= 1e-9


def test_sigma_rules(ctx):
    c = synth.survey_batch_curve(4, n=222)
    b = pack([c])
    freqs = O.linear_grid(1e-3, 10.0, 70)
    for rule in (O.SIGMA_MEDIAN_ERR, 0.137):
        sc, _, _, st = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3, sigma_y=rule)
        ref = oracle_ips(c, freqs, rule=rule)
        assert floor_rel(sc[0], O.qmi(ref)).max() <= QMI_TOL


def test_per_curve_status_and_neighbours(ctx):
    good = synth.survey_batch_curve(1, n=120)
    nan_t = synth.survey_batch_curve(2, n=50)
    nan_t.t = nan_t.t.copy()
    nan_t.t[7] = np.nan
    flat = synth.survey_batch_curve(3, n=40)
    flat.y = np.full(40, 17.0)
    one = synth.survey_batch_curve(5, n=1)
    empty = synth.Curve(np.zeros(0), np.zeros(0), np.zeros(0), False)
    curves = [good, nan_t, flat, one, empty, good]
    b = pack(curves)
    freqs = O.linear_grid(1e-3, 10.0, 65)
    sc, ips, ipy, st = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3, want_ips=True)
    assert list(st) == [0, qmi.EINVAL, qmi.EDEGENERATE, qmi.EINVAL, qmi.EINVAL, 0]
    for k in (1, 2, 3, 4):
        assert np.all(np.isnan(sc[k])) and np.isnan(ipy[k])
    ref = O.qmi(oracle_ips(good, freqs))
    assert floor_rel(sc[0], ref).max() <= QMI_TOL
    assert np.array_equal(sc[0], sc[5])


def test_call_level_errors_leave_outputs_untouched(ctx):
    c = synth.survey_batch_curve(1, n=50)
    b = pack([c])
    out = np.full((1, 3), 7.0)
    kp = qmi.kernel_params(-0.5)  # sigma_t <= 0 and not a rule
    bb, off = ctx._batch(b.offsets, b.t, b.y, b.e)
    f = np.array([0.1, 0.2, 0.3])
    rc = qmi.lib().qmi_periodogram(ctx._h, bb, kp, f.ctypes.data, 3, 0, out.ctypes.data, None,
                                   None, None)
    assert rc == qmi.EINVAL and np.all(out == 7.0)
    assert b"sigma_t" in qmi.lib().qmi_last_error(ctx._h)
    with pytest.raises(qmi.QMIError):
        ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, 1.0, 0.5, 100)  # f_max <= f_min
    with pytest.raises(qmi.QMIError):
        ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, 0.0, 1.0, 100, top_k=qmi.MAX_TOPK + 1)
    with pytest.raises(qmi.QMIError):
        ctx.periodogram(b.offsets, b.t, b.y, None, f, 0.3, sigma_y=qmi.SIGMA_MEDIAN_ERR)
    res, _ = ctx.best_period([0], np.zeros(0), np.zeros(0), None, 0.3, 0.0, 1.0, 10)
    assert len(res) == 0


def test_sample_order_and_batch_composition(ctx):
    c = synth.survey_batch_curve(6, n=301)
    p = np.random.default_rng(0).permutation(c.n)
    cp = synth.Curve(c.t[p], c.y[p], c.e[p], c.periodic)
    freqs = O.linear_grid(1e-3, 10.0, 128)
    alone, _, _, _ = ctx.periodogram([0, c.n], c.t, c.y, c.e, freqs, 0.3)
    perm, _, _, _ = ctx.periodogram([0, c.n], cp.t, cp.y, cp.e, freqs, 0.3)
    assert floor_rel(perm[0], alone[0]).max() <= 2 * QMI_TOL
    others = [synth.survey_batch_curve(k, n=n) for k, n in ((10, 900), (11, 77), (12, 513))]
    b = pack([others[0], c, others[1], others[2]])
    mixed, _, _, _ = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3)
    assert np.array_equal(mixed[1], alone[0])  # bitwise: per-curve work is batch independent


SEARCH = dict(f_min=1e-3, f_max=10.0, n_coarse=400, top_k=5, n_fine=50)


def _near_tie(ref: O.SearchResult) -> bool:
    q = np.sort(ref.fine_scores.ravel())[::-1] if ref.fine_scores is not None else None
    return q is not None and len(q) > 1 and (q[0] - q[1]) <= 1e-6 * abs(q[0])


def test_best_period_parity(ctx):
    curves = [synth.survey_batch_curve(k, n=n) for k, n in
              enumerate([60, 97, 128, 200, 257, 311, 380, 400])]
    b = pack(curves)
    res, coarse = ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **SEARCH)
    mism = []
    for k, c in enumerate(curves):
        ref = O.best_period(c.t, c.y, c.e, 0.3, O.SIGMA_SILVERMAN, **SEARCH)
        r = res[k]
        assert r["status"] == 0
        assert floor_rel(coarse[k], ref.coarse_scores).max() <= QMI_TOL
        assert r["sigma_y"] == pytest.approx(ref.sigma_y, rel=1e-13)
        assert r["n_peaks"] == ref.n_peaks
        same = (r["coarse_argmax"] == ref.coarse_argmax and r["coarse_index"] == ref.coarse_index
                and r["peak_rank"] == ref.peak_rank and r["fine_index"] == ref.fine_index)
        if not same:
            mism.append((k, _near_tie(ref)))
            continue
        assert r["f_best"] == ref.f_best  # same index -> the same FP64 grid point
        assert abs(r["score"] - ref.score) <= QMI_TOL * abs(ref.score)
        assert abs(r["score_nckp"] - ref.nckp) <= 1e-3 * abs(ref.nckp) + 1e-9
        assert r["period"] == pytest.approx(1.0 / ref.f_best, rel=1e-15)
    assert all(tie for _, tie in mism), mism


def test_single_sinusoid_workload_full_periodogram(ctx):
    """The plain one-curve workload: N = 200 times on [0, 2500] d, y = 0.3 sin(2 pi t / 3.7) plus
    noise, the full 5000-point QMI periodogram on [1e-3, 10] 1/d (mixed and FP64) and its best
    period (the coarse argmax), against the oracle at every frequency."""
    c = synth.single_sinusoid()
    wl = synth.WORKLOADS["single_sinusoid"]
    grid = O.linear_grid(wl["f_min"], wl["f_max"], wl["n_coarse"])
    ref = O.information_potentials(c.t, c.y, wl["sigma_t"], O.silverman_sigma(c.y), grid)
    rq = O.qmi(ref)
    for prec, tol in ((qmi.PREC_MIXED, QMI_TOL), (qmi.PREC_FP64, 1e-10)):
        sc, ips, _, st = ctx.periodogram([0, c.n], c.t, c.y, c.e, grid, wl["sigma_t"],
                                         precision=prec, want_ips=True)
        assert st[0] == 0
        assert floor_rel(sc[0], rq).max() <= tol
    kw = {k: wl[k] for k in ("f_min", "f_max", "n_coarse", "top_k", "n_fine")}
    res, coarse = ctx.best_period([0, c.n], c.t, c.y, c.e, wl["sigma_t"], want_coarse=True, **kw)
    best = O.best_period(c.t, c.y, c.e, wl["sigma_t"], O.SIGMA_SILVERMAN, **kw)
    assert res[0]["coarse_argmax"] == best.coarse_argmax == int(np.argmax(rq))
    assert res[0]["f_best"] == grid[best.coarse_argmax]
    # No recovery claim: the 2e-3 1/d grid step is five times the 1/2500 d peak width, so the
    # grid can miss the generating frequency's peak (here the maximum falls on half of it).


def test_best_period_without_refinement_and_nckp_search(ctx):
    c = synth.single_sinusoid()
    kw = dict(f_min=1e-3, f_max=10.0, n_coarse=1500, top_k=0, n_fine=0)
    res, _ = ctx.best_period([0, c.n], c.t, c.y, c.e, 0.3, **kw)
    ref = O.best_period(c.t, c.y, c.e, 0.3, O.SIGMA_SILVERMAN, **kw)
    assert res[0]["coarse_argmax"] == ref.coarse_argmax and res[0]["peak_rank"] == -1
    assert res[0]["f_best"] == ref.f_best
    kw = dict(f_min=1e-3, f_max=2.0, n_coarse=300, top_k=3, n_fine=40, score=O.SCORE_NCKP)
    res, _ = ctx.best_period([0, c.n], c.t, c.y, c.e, 0.3, **kw)
    ref = O.best_period(c.t, c.y, c.e, 0.3, O.SIGMA_SILVERMAN, **kw)
    assert res[0]["coarse_index"] == ref.coarse_index and res[0]["fine_index"] == ref.fine_index


def test_full_size_survey_curve_sampled(ctx):
    """A survey-batch curve at full size (N = 1000, 20k coarse + 10 x 1000 fine, the launch the
    benchmark times): sampled coarse scores against the oracle, and the peak/best logic of the
    oracle applied to the GPU's own coarse scores."""
    c = synth.survey_batch_curve(2, n=1000)
    kw = synth.WORKLOADS["survey_batch"]
    args = dict(f_min=kw["f_min"], f_max=kw["f_max"], n_coarse=kw["n_coarse"], top_k=kw["top_k"],
                n_fine=kw["n_fine"])
    res, coarse = ctx.best_period([0, c.n], c.t, c.y, c.e, 0.3, want_coarse=True, **args)
    r = res[0]
    grid = O.linear_grid(args["f_min"], args["f_max"], args["n_coarse"])
    idx = np.unique(np.concatenate([np.random.default_rng(1).integers(0, len(grid), 40),
                                    [0, len(grid) - 1, r["coarse_argmax"]]]))
    ref = O.qmi(oracle_ips(c, grid[idx]))
    assert floor_rel(coarse[0, idx], ref).max() <= QMI_TOL
    peaks = O.top_peaks(coarse[0], args["top_k"])
    assert r["n_peaks"] == len(peaks)
    assert r["coarse_index"] == peaks[r["peak_rank"]]
    assert r["coarse_argmax"] == int(np.argmax(coarse[0]))
    lo, hi = O.fine_window(grid, int(r["coarse_index"]))
    f_expect = O.linear_grid(lo, hi, args["n_fine"])[r["fine_index"]]
    assert r["f_best"] == f_expect
    q = O.qmi(oracle_ips(c, [r["f_best"]]))[0]
    assert abs(r["score"] - q) <= QMI_TOL * abs(q)


def test_long_baseline_high_frequency_fold(ctx):
    """7000-day baseline at frequencies up to 20 / day: f t reaches 1.4e5 cycles, the FP64 fold
    must keep the phase exact enough for the same 1e-4 QMI bar."""
    c = synth.long_baseline_curve(0)
    freqs = np.concatenate([O.linear_grid(19.5, 20.0, 96), O.linear_grid(1e-3, 20.0, 64)])
    sc, _, _, _ = ctx.periodogram([0, c.n], c.t, c.y, c.e, freqs, 0.3)
    ref = O.qmi(oracle_ips(c, freqs))
    assert floor_rel(sc[0], ref).max() <= QMI_TOL


def test_maximum_length(ctx):
    rng = np.random.default_rng(9)
    n = qmi.MAX_N
    t = np.sort(rng.uniform(0, 2500, n))
    y = 0.2 * np.sin(2 * np.pi * t / 1.37) + rng.normal(0, 0.1, n)
    freqs = np.array([1 / 1.37, 0.01, 3.3])
    sc, _, _, st = ctx.periodogram([0, n], t, y, None, freqs, 0.3)
    assert st[0] == 0
    ref = O.qmi(O.information_potentials(t, y, 0.3, O.silverman_sigma(y), freqs))
    assert floor_rel(sc[0], ref).max() <= QMI_TOL
    t2 = np.concatenate([t, [2600.0]])
    y2 = np.concatenate([y, [0.0]])
    sc2, _, _, st2 = ctx.periodogram([0, n + 1], t2, y2, None, freqs, 0.3)
    assert st2[0] == qmi.EINVAL and np.all(np.isnan(sc2[0]))


def test_device_pointer_variants(ctx):
    import torch

    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate([90, 260, 41])]
    b = pack(curves)
    freqs = O.linear_grid(1e-3, 10.0, 150)
    host, _, _, _ = ctx.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    T, Y, E, Fq = dev(b.t), dev(b.y), dev(b.e), dev(freqs)
    out = torch.empty((b.n_curves, len(freqs)), dtype=torch.float64, device="cuda")
    ctx.periodogram_dev(b.offsets, T, Y, E, Fq, out, 0.3)
    assert np.array_equal(out.cpu().numpy(), host)
    res_h, coarse_h = ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **SEARCH)
    cd = torch.empty((b.n_curves, SEARCH["n_coarse"]), dtype=torch.float64, device="cuda")
    res_d = ctx.best_period_dev(b.offsets, T, Y, E, 0.3, coarse_out=cd, **SEARCH)
    assert np.array_equal(res_d, res_h)
    assert np.array_equal(cd.cpu().numpy(), coarse_h)
    st = ctx.stats()
    assert st["device_ms"] > 0 and st["pair_items"] > 0
    if not st["used_graph"]:
        assert st["pair_launches"] == 2 and st["pair_kernel_ms"] > 0
    with qmi.Context(0) as eager:
        eager.set_option(qmi.OPT_USE_GRAPH, 0)
        eager.best_period_dev(b.offsets, T, Y, E, 0.3, coarse_out=cd, **SEARCH)
        st = eager.stats()
        assert st["used_graph"] == 0 and st["pair_launches"] == 2 and st["pair_kernel_ms"] > 0


def test_graph_replay_matches_eager(ctx):
    """The device section captured once and replayed on new data of the same shape gives the eager
    results bit for bit, with eager work on another context between the replays."""
    ns = [120, 333, 257]
    A = pack([synth.survey_batch_curve(k, n=n) for k, n in enumerate(ns)])
    B = pack([synth.survey_batch_curve(k + 50, n=n) for k, n in enumerate(ns)])
    with qmi.Context(0) as eager:
        eager.set_option(qmi.OPT_USE_GRAPH, 0)
        ref = {}
        for name, b in (("A", A), ("B", B)):
            ref[name] = eager.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **SEARCH)
            assert eager.stats()["used_graph"] == 0
    other = synth.survey_batch_curve(99, n=64)
    with qmi.Context(0) as g:
        for name in ("A", "B", "A", "B", "A"):
            b = A if name == "A" else B
            res, coarse = g.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **SEARCH)
            assert g.stats()["used_graph"] == 1
            assert np.array_equal(res, ref[name][0])
            assert np.array_equal(coarse, ref[name][1])
            ctx.periodogram([0, other.n], other.t, other.y, other.e, [0.1, 0.2], 0.3)


def test_serving_results_equal_alone(ctx):
    """Continuous batching: requests submitted while others run are admitted into overlapping
    launches; every result equals the same curve searched alone."""
    import time

    curves = [synth.serving_curve(k) for k in range(40)]
    kw = dict(f_min=1e-3, f_max=10.0, n_coarse=600, top_k=4, n_fine=64)
    alone = []
    for c in curves[:6]:
        r, _ = ctx.best_period([0, c.n], c.t, c.y, c.e, 0.3, **kw)
        alone.append(r[0])
    batch = pack(curves)
    mixed, _ = ctx.best_period(batch.offsets, batch.t, batch.y, batch.e, 0.3, **kw)
    for k in range(6):
        assert np.array_equal(mixed[k], alone[k])
    # unbounded launches of up to 8 requests on 3 lanes, then launches bounded to about two
    # requests' pair work on 4 lanes
    for max_batch, inflight, items in ((8, 3, 0), (64, 4, 2.5e8)):
        with qmi.Context(0) as srv:
            srv.serve_start(0.3, max_batch=max_batch, max_inflight=inflight,
                            max_batch_items=items, **kw)
            got = {}
            for k, c in enumerate(curves):
                while not srv.submit(c.t, c.y, c.e, tag=k):
                    res, tags = srv.poll(64, 1000)
                    got.update({int(t): r for t, r in zip(tags, res)})
                if k % 7 == 0:
                    time.sleep(0.002)
            t0 = time.time()
            while len(got) < len(curves) and time.time() - t0 < 60:
                res, tags = srv.poll(64, 10000)
                got.update({int(t): r for t, r in zip(tags, res)})
            srv.serve_stop()
        assert len(got) == len(curves)
        for k in range(len(curves)):
            assert np.array_equal(got[k], mixed[k]), (items, k)


def test_one_piece_per_workgroup_launches_give_the_same_bits(ctx):
    """A call with too few (curve, 64-frequency tile) items to fill the chip runs one (pass, column
    segment) piece per workgroup and adds the pieces' sums in an epilogue kernel; a large enough
    batch runs every piece of a (curve, tile) in one workgroup.  Both add the pieces in the same
    order, so a curve's coarse periodogram and search result are the same bits either way."""
    ns = [1000, 257, 600, 513, 300, 900, 777, 2, 256, 1500]
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate(ns)]
    kw = dict(f_min=1e-3, f_max=10.0, n_coarse=20000, top_k=10, n_fine=1000)
    b = pack(curves)
    big, cbig = ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
    for k, c in enumerate(curves):
        r, cc = ctx.best_period([0, c.n], c.t, c.y, c.e, 0.3, want_coarse=True, **kw)
        assert np.array_equal(cc[0], cbig[k], equal_nan=True), k
        assert r.tobytes() == big[k:k + 1].tobytes(), k
    # refinement windows and periodograms of both kinds, mixed and FP64
    freqs = O.linear_grid(1e-3, 10.0, 1500)
    many = pack([synth.survey_batch_curve(k, n=300 + 7 * k) for k in range(90)])
    for prec in (qmi.PREC_MIXED, qmi.PREC_FP64):
        sc, ips, _, _ = ctx.periodogram(many.offsets, many.t, many.y, many.e, freqs, 0.3,
                                        precision=prec, want_ips=True)
        for k in (0, 41, 89):
            lo, hi = many.offsets[k], many.offsets[k + 1]
            s1, i1, _, _ = ctx.periodogram([0, hi - lo], many.t[lo:hi], many.y[lo:hi],
                                           many.e[lo:hi], freqs, 0.3, precision=prec,
                                           want_ips=True)
            assert np.array_equal(s1[0], sc[k]) and np.array_equal(i1[0], ips[k]), (prec, k)


def test_pair_kernel_variants_agree(ctx):
    """Every pair-kernel variant the autotuner can pick meets the oracle bar, and all four (2 or 4
    waves per SIMD, 64- or 32-column chunks) give identical bits, on lengths that end their passes
    and column segments inside a 32-column chunk and on both launch forms."""
    curves = [synth.survey_batch_curve(k, n=n) for k, n in enumerate([70, 300, 777, 529, 1100])]
    b = pack(curves)
    freqs = O.linear_grid(1e-3, 10.0, 190)
    refs = [O.qmi(oracle_ips(c, freqs)) for c in curves]
    out = {}
    with qmi.Context(0) as c2:
        for v in range(1, 5):
            c2.set_option(qmi.OPT_TILE, v)
            sc, _, _, _ = c2.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3)
            assert c2.stats()["pair_variant"] == v - 1
            out[v] = sc
            for k in range(len(curves)):
                assert floor_rel(sc[k], refs[k]).max() <= QMI_TOL, (v, k)
    for v in (2, 3, 4):
        assert np.array_equal(out[1], out[v]), v
    # the batched launch form (whole tiles per workgroup) gives the same bits in every variant
    many = [synth.survey_batch_curve(50 + k, n=300 + 37 * k) for k in range(40)]
    bm = pack(many)
    fm = O.linear_grid(1e-3, 10.0, 3300)
    outs = []
    with qmi.Context(0) as c3:
        for v in range(1, 5):
            c3.set_option(qmi.OPT_TILE, v)
            outs.append(c3.periodogram(bm.offsets, bm.t, bm.y, bm.e, fm, 0.3)[0])
    for v in (1, 2, 3):
        assert np.array_equal(outs[0], outs[v]), v


def test_autotune_on_batch_larger_than_probe(ctx):
    """The autotuner probes the largest curves of a batch on a slice of the frequency plan; with
    more curves than the probe uses, the probe's scratch output must still cover every curve id.
    The tuned result must match a forced default variant within the parity bar."""
    curves = [synth.survey_batch_curve(k, n=300 + (k % 7) * 13) for k in range(72)]
    b = pack(curves)
    kw = dict(f_min=1e-3, f_max=10.0, n_coarse=2400, top_k=2, n_fine=32)
    with qmi.Context(0) as tuned, qmi.Context(0) as fixed:
        fixed.set_option(qmi.OPT_TILE, 1)
        r_t, c_t = tuned.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
        r_f, c_f = fixed.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
        r_t2, c_t2 = tuned.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
    assert np.all(r_t["status"] == 0)
    for k in range(len(curves)):
        assert floor_rel(c_t[k], c_f[k]).max() <= QMI_TOL
        assert floor_rel(c_t2[k], c_f[k]).max() <= QMI_TOL


def _golden_search(workload, make):
    """GPU full-size search of the stored curves of a workload: (records, curves, results)."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "%s_oracle.json" % workload)
    if not os.path.exists(path):
        pytest.skip("no stored oracle search for %s" % workload)
    gold = json.load(open(path))
    recs = gold["curves"]
    curves = [make(r["k"]) for r in recs]
    b = pack(curves)
    with qmi.Context(0) as c2:
        res, _ = c2.best_period(b.offsets, b.t, b.y, b.e, gold["sigma_t"], **gold["search"])
    return gold, recs, curves, res


def _compare_best(gold, recs, curves, res, name):
    """Indices must agree; where the oracle's best and runner-up refined scores are within 1e-5
    of each other (a flat maximum: several grid points are correct), the GPU's choice must score
    within that margin of the best under the oracle."""
    exact, ties, bad = 0, [], []
    for r, c, g in zip(res, curves, recs):
        assert r["status"] == 0 and r["n_peaks"] == g["n_peaks"]
        assert r["sigma_y"] == pytest.approx(g["sigma_y"], rel=1e-13)
        same = (r["coarse_argmax"] == g["coarse_argmax"] and r["coarse_index"] == g["coarse_index"]
                and r["fine_index"] == g["fine_index"])
        if same:
            assert r["f_best"] == g["f_best"]
            assert abs(r["score"] - g["score"]) <= QMI_TOL * abs(g["score"])
            exact += 1
            continue
        q = O.qmi(O.information_potentials(c.t, c.y, gold["sigma_t"], g["sigma_y"],
                                           [r["f_best"]]))[0]
        if g["best_gap"] <= 1e-5 * abs(g["score"]) and q >= g["score"] * (1 - 1e-5):
            ties.append((g["k"], g["fine_index"], int(r["fine_index"])))
        else:
            bad.append((g["k"], dict(coarse=(g["coarse_index"], int(r["coarse_index"])),
                                     fine=(g["fine_index"], int(r["fine_index"])))))
    print("%s: %d of %d identical, %d flat-maximum ties %s" % (name, exact, len(recs), len(ties),
                                                               ties))
    assert not bad, bad
    assert exact + len(ties) == len(recs)


def test_survey_stream_best_period_matches_oracle_full_search():
    """The survey-stream workload's search (30 000 coarse + 10 x 1000 refined frequencies, N
    lognormal in [100, 1500]) against the stored FP64 oracle search of its first curves."""
    gold, recs, curves, res = _golden_search("survey_stream", synth.survey_stream_curve)
    _compare_best(gold, recs, curves, res, "survey stream")


def test_survey_batch_best_period_matches_oracle_full_search():
    """Full-size search (20 000 coarse + 10 x 1000 refined frequencies) of the stored curves of
    the survey batch against the FP64 oracle results (tests/golden/make_survey_parity.py), then
    the discriminator's decisions."""
    gold, recs, curves, res = _golden_search("survey_batch", synth.survey_batch_curve)
    _compare_best(gold, recs, curves, res, "survey batch")
    # Discriminator: thresholds calibrated by the oracle on its own scores of the curves with
    # k mod 4 in {0, 1}; then, for the other curves, the decision from the GPU result (score at
    # f_best, pSNR) against the oracle's decision.  Curves whose oracle score lies within the
    # score tolerance of their bin's threshold may go either way and are counted separately.
    psn = [O.psnr(c.y, c.e) for c in curves]
    for r, p in zip(res, psn):
        assert r["psnr"] == pytest.approx(p, rel=1e-12)
    train = [k for k, g in enumerate(recs) if g["k"] % 4 < 2]
    test = [k for k, g in enumerate(recs) if g["k"] % 4 >= 2]
    cal = O.calibrate_thresholds([recs[k]["score"] for k in train], [psn[k] for k in train],
                                 [recs[k]["periodic"] for k in train], n_points=5000)
    th = [x if math.isfinite(x) else 1e300 for x in cal["th"]]
    got = qmi.discriminate(res, O.SNR_EDGES, th)
    want = [O.discriminate(g["score"], p, th) for g, p in zip(recs, psn)]
    near = [k for k in test if O.snr_bin(psn[k]) >= 0 and
            abs(recs[k]["score"] - th[O.snr_bin(psn[k])]) <= QMI_TOL * abs(recs[k]["score"])]
    agree = sum(1 for k in test if got[k] == want[k])
    print("discriminator: %d of %d held-out curves agree (%d within the score tolerance of a "
          "threshold)" % (agree, len(test), len(near)))
    assert all(got[k] == want[k] for k in test if k not in near)


def test_empty_batches_on_every_entry_point(ctx):
    """A batch of zero curves is valid everywhere and produces empty outputs."""
    z = np.zeros(0)
    off = [0]
    sc, ips, ipy, st = ctx.periodogram(off, z, z, z, [0.1, 0.2], 0.3, want_ips=True)
    assert sc.shape == (0, 2) and ips.shape == (0, 2, 3) and st.shape == (0,)
    res, coarse = ctx.best_period(off, z, z, z, 0.3, want_coarse=True, **SEARCH)
    assert len(res) == 0 and coarse.shape == (0, SEARCH["n_coarse"])
    res, trials, scores = ctx.bands_best_period(off, z, z, z, 0.3)
    assert len(res) == 0 and trials.shape == (0, 450)
    oo, to, yo, eo, st, det = ctx.preprocess(off, z, z, z)
    assert list(oo) == [0] and len(to) == 0 and len(st) == 0
    yw, st = ctx.whiten(off, z, z, np.zeros(0))
    assert len(yw) == 0 and len(st) == 0
    assert len(qmi.discriminate(np.zeros(0, qmi.RESULT_DTYPE), O.SNR_EDGES, [0.5] * 8)) == 0


def test_benchmark_launch_configuration_sampled():
    """The benchmark's own call: all 4096 survey-batch curves in one qmi_best_period_dev launch
    sequence on device-resident inputs (XCD-grouped blocks, autotuned variant).  Sampled coarse
    scores of sampled curves against the oracle, and every curve that has a stored oracle search
    against it."""
    import json
    import os

    import torch

    b = synth.make_batch("survey_batch", range(4096))
    wl = synth.WORKLOADS["survey_batch"]
    kw = {k: wl[k] for k in ("f_min", "f_max", "n_coarse", "top_k", "n_fine")}
    dev = torch.device("cuda:0")
    T, Y, E = (torch.from_numpy(a).to(dev) for a in (b.t, b.y, b.e))
    coarse = torch.empty((4096, kw["n_coarse"]), dtype=torch.float64, device=dev)
    with qmi.Context(0) as c:
        c.best_period_dev(b.offsets, T, Y, E, wl["sigma_t"], **kw)  # first call tunes
        res = c.best_period_dev(b.offsets, T, Y, E, wl["sigma_t"], coarse_out=coarse, **kw)
        variant = c.stats()["pair_variant"]
    torch.cuda.synchronize()
    assert np.all(res["status"] == 0)
    print("variant %d" % variant)
    rng = np.random.default_rng(12)
    grid = O.linear_grid(kw["f_min"], kw["f_max"], kw["n_coarse"])
    for k in np.sort(rng.choice(4096, 24, replace=False)):
        cv = b.curve(int(k))
        idx = np.sort(rng.choice(len(grid), 48, replace=False))
        got = coarse[int(k), torch.from_numpy(idx).to(dev)].cpu().numpy()
        ref = O.qmi(oracle_ips(cv, grid[idx]))
        assert floor_rel(got, ref).max() <= QMI_TOL, k
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "survey_batch_oracle.json")
    gold = json.load(open(path))
    exact, ties = 0, []
    for g in gold["curves"]:
        r = res[g["k"]]
        if (r["coarse_index"], r["fine_index"]) == (g["coarse_index"], g["fine_index"]):
            assert r["f_best"] == g["f_best"]
            exact += 1
            continue
        # A flat maximum (the oracle's best and runner-up refined scores within 1e-5 of each
        # other) has several correct grid points: the GPU's choice must then score within that
        # margin of the best under the oracle, as in the other full-search comparisons.
        cv = b.curve(g["k"])
        q = O.qmi(O.information_potentials(cv.t, cv.y, gold["sigma_t"], g["sigma_y"],
                                           [r["f_best"]]))[0]
        assert g["best_gap"] <= 1e-5 * abs(g["score"]) and q >= g["score"] * (1 - 1e-5), g["k"]
        ties.append((g["k"], g["fine_index"], int(r["fine_index"])))
    print("benchmark launch: %d of %d stored searches identical, %d flat-maximum ties %s"
          % (exact, len(gold["curves"]), len(ties), ties))


def test_small_hbm_budget_splits_the_batch_into_groups():
    """A context whose HBM budget holds only a few curves at a time plans several groups (and
    reuses its buffers across them); the results equal those of one group, bit for bit, for the
    search, the periodogram and the bands front end.  A curve that alone exceeds the budget is a
    call-level QMI_ENOMEM."""
    curves = [synth.survey_batch_curve(k, n=n) for k, n in
              enumerate([300, 800, 120, 1000, 450, 640, 999, 301, 77])]
    b = pack(curves)
    kw = dict(f_min=1e-3, f_max=10.0, n_coarse=3000, top_k=3, n_fine=64)
    freqs = O.linear_grid(1e-3, 10.0, 700)
    with qmi.Context(0) as big, qmi.Context(0, budget_bytes=8 << 20) as small:
        for c in (big, small):  # one variant for both (the autotuner may not see every group)
            c.set_option(qmi.OPT_TILE, 2)
        r1, c1 = big.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
        r2, c2 = small.best_period(b.offsets, b.t, b.y, b.e, 0.3, want_coarse=True, **kw)
        assert r1.tobytes() == r2.tobytes() and np.array_equal(c1, c2)
        s1 = big.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3)[0]
        s2 = small.periodogram(b.offsets, b.t, b.y, b.e, freqs, 0.3)[0]
        assert np.array_equal(s1, s2)
        q1 = big.bands_best_period(b.offsets, b.t, b.y, b.e, 0.3, n_trials=40, n_grid=5000)
        q2 = small.bands_best_period(b.offsets, b.t, b.y, b.e, 0.3, n_trials=40, n_grid=5000)
        assert q1[0].tobytes() == q2[0].tobytes()
        assert np.array_equal(q1[1], q2[1], equal_nan=True)
    with qmi.Context(0, budget_bytes=3 << 20) as tiny:
        with pytest.raises(qmi.QMIError) as ei:
            tiny.best_period(b.offsets, b.t, b.y, b.e, 0.3, **kw)
        assert ei.value.code == qmi.ENOMEM
