"""CPU-side checks of the C-ABI library: it loads, exports every symbol include/qmi.h declares,
its struct layouts match the header, and its host-only logic (the discriminator, argument
validation) behaves as documented.  No GPU compute is called here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1412_1840_amd import qmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmi.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(qmi_\w+)\s*\(", text,
                                 re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 14, names
    L = qmi.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(qmi.SYMBOLS)


def test_header_constants_match_binding():
    text = open(HEADER).read()

    def val(name):
        m = re.search(r"#define\s+%s\s+\(?(-?[0-9.]+)\)?" % name, text)
        return float(m.group(1))

    assert val("QMI_OK") == qmi.OK and val("QMI_EINVAL") == qmi.EINVAL
    assert val("QMI_EAGAIN") == qmi.EAGAIN and val("QMI_EDEVICE") == qmi.EDEVICE
    assert val("QMI_SIGMA_SILVERMAN") == qmi.SIGMA_SILVERMAN
    assert val("QMI_SIGMA_MEDIAN_ERR") == qmi.SIGMA_MEDIAN_ERR
    assert val("QMI_MAX_N") == qmi.MAX_N and val("QMI_MAX_TOPK") == qmi.MAX_TOPK
    assert val("QMI_UNDECIDED") == qmi.UNDECIDED
    assert val("QMI_MAX_BANDS") == qmi.MAX_BANDS and val("QMI_MAX_TRIALS") == qmi.MAX_TRIALS
    assert val("QMI_MAX_MASKS") == qmi.MAX_MASKS
    assert val("QMI_PREC_FOLD32") == qmi.PREC_FOLD32
    assert val("QMI_SIGMA_T_SKEWNESS") == qmi.SIGMA_T_SKEWNESS
    assert val("QMI_SKEW_LAMBDA") == qmi.SKEW_LAMBDA and val("QMI_SKEW_MU") == qmi.SKEW_MU
    m = re.search(r"#define\s+QMI_NOALLOC_SCRATCH_BYTES\s+\((\d+)u << (\d+)\)", text)
    assert (int(m.group(1)) << int(m.group(2))) == qmi.NOALLOC_SCRATCH_BYTES


def test_struct_sizes():
    assert ctypes.sizeof(qmi.Stats) == 40
    assert ctypes.sizeof(qmi.Batch) == 40
    assert ctypes.sizeof(qmi.KernelParams) == 40
    assert ctypes.sizeof(qmi.Search) == 32
    assert ctypes.sizeof(qmi.Thresholds) == 24
    assert ctypes.sizeof(qmi.Bands) == 40
    assert ctypes.sizeof(qmi.PreprocessParams) == 16
    assert ctypes.sizeof(qmi.Mask) == 24
    assert qmi.RESULT_DTYPE.itemsize == 104


def test_discriminate_matches_oracle_rule():
    rng = np.random.default_rng(3)
    n = 500
    res = np.zeros(n, qmi.RESULT_DTYPE)
    res["score_qmi"] = rng.uniform(0, 1.5, n)
    res["score_nckp"] = rng.uniform(0, 3, n)
    res["psnr"] = rng.uniform(-1, 30, n)
    res["status"] = np.where(rng.random(n) < 0.05, -4, 0)
    res["score_qmi"][::37] = np.nan
    res["psnr"][::41] = np.nan
    edges = list(O.SNR_EDGES)
    th = list(rng.uniform(0.2, 1.2, 8))
    th[2] = res["score_qmi"][5]  # an exact tie must be "not periodic" (strict >)
    for score, field in ((qmi.SCORE_QMI, "score_qmi"), (qmi.SCORE_NCKP, "score_nckp")):
        got = qmi.discriminate(res, edges, th, score=score)
        for k in range(n):
            want = (O.UNDECIDED if res["status"][k] != 0 else
                    O.discriminate(res[field][k], res["psnr"][k], th, edges))
            assert got[k] == want, (k, res[k])
    # caller-supplied pSNR overrides the result's
    p = np.full(n, 3.0)
    got = qmi.discriminate(res, edges, th, psnr=p)
    ok = (res["status"] == 0) & np.isfinite(res["score_qmi"])
    assert np.all(got[ok] == (res["score_qmi"][ok] > th[3]))


def test_discriminate_rejects_bad_tables():
    res = np.zeros(2, qmi.RESULT_DTYPE)
    with pytest.raises(qmi.QMIError):
        qmi.discriminate(res, [0.0, 2.0, 1.0], [0.1, 0.2])  # decreasing edges
    with pytest.raises(ValueError):
        qmi.discriminate(res, [0.0, 1.0], [0.1, 0.2])


def test_create_without_device_fails_cleanly():
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    with pytest.raises(qmi.QMIError) as ei:
        qmi.Context(0)
    assert ei.value.code == qmi.EDEVICE


def test_calibration_matches_oracle():
    rng = np.random.default_rng(7)
    n = 400
    truth = rng.random(n) < 0.5
    psnr = rng.uniform(0.2, 30, n)
    scores = np.where(truth, rng.normal(0.9, 0.35, n), rng.normal(0.35, 0.2, n))
    scores[::53] = np.nan
    for pts in (1, 2, 257, 5000):
        got = qmi.calibrate(scores, psnr, truth, n_points=pts)
        ref = O.calibrate_thresholds(list(scores), list(psnr), list(truth), n_points=pts)
        assert np.array_equal(got["th"], np.array(ref["th"])), pts
        assert np.array_equal(got["f1"], np.array(ref["f1"]))
        assert np.array_equal(got["precision"], np.array(ref["precision"]))
        assert np.array_equal(got["recall"], np.array(ref["recall"]))
    # empty bins and bins without periodic members
    got = qmi.calibrate([0.5, 0.7], [1.0, 1.2], [0, 0])
    assert got["th"][0] == 0.7 and got["f1"][0] == 0.0 and np.isinf(got["th"][1])


def test_spurious_table_of_the_binding_is_the_papers():
    """The binding's copy of the table of spurious periods (Sec. 6.1) and its default mask widths
    agree with the oracle's transcription."""
    assert qmi.SPURIOUS_PERIODS == O.SPURIOUS_PERIODS
    for amp, w in ((0.7, 0.5), (2.0, 20.0)):
        assert qmi.spurious_masks(amp, width=w) == O.spurious_masks(amp, width=w)
