"""Host logic of the survey streaming runner (batching, checkpoint and resume), with a stand-in
for the device call; the same runner on the GPU is covered at the end."""
import json
import os

import numpy as np
import pytest

from paper_1412_1840_amd import synth
from paper_1412_1840_amd.survey import CHECKPOINT, RESULTS, SurveyRunner

DT = np.dtype([("k", "<i8"), ("n", "<i4"), ("pad", "<i4"), ("mean_t", "<f8")])
SEARCH = dict(f_min=1e-3, f_max=10.0, n_coarse=256, top_k=2, n_fine=16)


def fake_compute(batch):
    n = np.diff(batch.offsets)
    r = np.zeros(batch.n_curves, DT)
    r["n"] = n
    r["mean_t"] = [batch.t[a:b].mean() for a, b in zip(batch.offsets[:-1], batch.offsets[1:])]
    return r, {"pair_items": float(np.sum(n * (n - 1) / 2)), "pair_kernel_ms": 1.0}


def runner(tmp, n=23, batch=5, compute=fake_compute, **kw):
    return SurveyRunner(str(tmp), n, synth.survey_stream_curve, "survey_stream", SEARCH, 0.3,
                        batch_curves=batch, compute=compute, result_dtype=DT, **kw)


def test_full_run_writes_every_curve_in_order(tmp_path):
    ck = runner(tmp_path).run()
    assert ck["done"] == 23 and ck["batches"] == 5
    res = runner(tmp_path).results()
    want = np.array([synth.survey_stream_curve(k).n for k in range(23)])
    assert np.array_equal(res["n"], want)
    assert os.path.getsize(tmp_path / RESULTS) == 23 * DT.itemsize


def test_resume_after_interruption_gives_identical_bytes(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    runner(a).run()
    ck = runner(b).run(max_batches=2)
    assert ck["done"] == 10
    ck = runner(b).run(max_batches=1)
    assert ck["done"] == 15
    runner(b).run()
    assert (a / RESULTS).read_bytes() == (b / RESULTS).read_bytes()


def test_bytes_past_the_checkpoint_are_discarded(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    runner(a).run()
    runner(b).run(max_batches=3)
    # A crash after a batch was appended but before its checkpoint: partial, stale bytes.
    with open(b / RESULTS, "ab") as f:
        f.write(b"\x7f" * (DT.itemsize * 3 + 5))
    runner(b).run()
    assert (a / RESULTS).read_bytes() == (b / RESULTS).read_bytes()


def test_failed_batch_leaves_a_consistent_checkpoint(tmp_path):
    calls = {"n": 0}

    def flaky(batch):
        calls["n"] += 1
        if calls["n"] == 3:
            raise RuntimeError("device lost")
        return fake_compute(batch)

    with pytest.raises(RuntimeError):
        runner(tmp_path, compute=flaky).run()
    ck = json.load(open(tmp_path / CHECKPOINT))
    assert ck["done"] == 10 and ck["bytes"] == 10 * DT.itemsize
    runner(tmp_path).run()
    ref = tmp_path / "ref"
    runner(ref).run()
    assert (ref / RESULTS).read_bytes() == (tmp_path / RESULTS).read_bytes()


def test_changed_configuration_is_refused(tmp_path):
    runner(tmp_path).run(max_batches=1)
    with pytest.raises(ValueError):
        runner(tmp_path, batch=7).run()
    with pytest.raises(ValueError):
        runner(tmp_path, n=30).run()


def test_masks_are_part_of_the_configuration(tmp_path):
    m = [(1.0, 1e-3, 0.5), (29.5305, 0.2, 0.5)]
    runner(tmp_path, masks=m).run(max_batches=1)
    ck = json.load(open(os.path.join(str(tmp_path), CHECKPOINT)))
    assert ck["config"]["masks"] == [list(x) for x in m]
    assert runner(tmp_path, masks=m).run()["done"] == 23
    with pytest.raises(ValueError):
        runner(tmp_path).run()  # the same run without masks is a different configuration
    with pytest.raises(ValueError):
        runner(tmp_path, masks=m[:1]).run()


def test_empty_and_single_curve_runs(tmp_path):
    assert runner(tmp_path / "e", n=0).run()["done"] == 0
    assert len(runner(tmp_path / "e", n=0).results()) == 0
    assert runner(tmp_path / "s", n=1, batch=64).run()["done"] == 1


@pytest.mark.gpu
def test_survey_runner_on_gpu_matches_one_call(tmp_path):
    """The streamed, interrupted and resumed run gives, bit for bit, the records of one
    qmi_best_period call over the same curves."""
    from paper_1412_1840_amd import qmi

    n = 40

    def run(d, **kw):
        r = SurveyRunner(str(d), n, synth.survey_stream_curve, "survey_stream", SEARCH, 0.3,
                         batch_curves=16)
        try:
            return r.run(**kw), r
        finally:
            r.close()

    run(tmp_path / "a", max_batches=1)
    ck, r = run(tmp_path / "a")
    assert ck["done"] == n and ck["pair_items"] > 0
    got = r.results()
    b = synth.pack([synth.survey_stream_curve(k) for k in range(n)])
    with qmi.Context(0) as ctx:
        want, _ = ctx.best_period(b.offsets, b.t, b.y, b.e, 0.3, **SEARCH)
    assert got.tobytes() == want.tobytes()


@pytest.mark.gpu
def test_survey_command_line(tmp_path, capsys):
    """python -m paper_1412_1840_amd.survey: the full survey-stream search on 40 curves in two
    invocations (the second resumes), ending with a summary line."""
    import json

    from paper_1412_1840_amd import survey

    out = str(tmp_path / "s")
    assert survey.main(["--out", out, "--curves", "40", "--batch", "16", "--max-batches", "1"]) == 0
    assert survey.main(["--out", out, "--curves", "40", "--batch", "16"]) == 0
    summary = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert summary["curves_done"] == 40 and summary["batches"] == 3 and summary["bad_status"] == 0
    assert summary["roofline_frac_kernel"] is not None


@pytest.mark.gpu
def test_survey_with_spurious_masks_matches_one_masked_call(tmp_path):
    """--spurious-amplitude: the run's records equal one qmi_best_period call over the same curves
    with the table's masks set."""
    from paper_1412_1840_amd import qmi, survey

    out = str(tmp_path / "m")
    assert survey.main(["--out", out, "--curves", "24", "--batch", "16", "--source",
                        "survey_batch", "--spurious-amplitude", "0.3",
                        "--spurious-width", "20"]) == 0
    got = np.fromfile(os.path.join(out, RESULTS), dtype=qmi.RESULT_DTYPE)
    wl = synth.WORKLOADS["survey_batch"]
    kw = {k: wl[k] for k in ("f_min", "f_max", "n_coarse", "top_k", "n_fine")}
    b = synth.pack([synth.survey_batch_curve(k) for k in range(24)])
    with qmi.Context(0) as ctx:
        ctx.set_masks(qmi.spurious_masks(0.3, width=20.0))
        want, _ = ctx.best_period(b.offsets, b.t, b.y, b.e, wl["sigma_t"], **kw)
        ctx.set_masks(None)
        plain, _ = ctx.best_period(b.offsets, b.t, b.y, b.e, wl["sigma_t"], **kw)
    assert got.tobytes() == want.tobytes()
    assert not np.array_equal(want["f_best"], plain["f_best"])  # the masks changed some result
