"""qmi_periodogram_noalloc (the entry point for callers that cannot allocate device memory)
against qmi_periodogram_dev, through the C ABI: the same scores, V's, IP_y and statuses bit for
bit, on two calls in a row (the second smaller, so the scratch array holds the first call's
tables), on both launch forms of the pair kernel (a batch with enough frequency tiles to run whole
tiles per workgroup, and a small one that runs one piece per workgroup); and a batch too large for
the scratch array is refused before any device work, outputs untouched."""
import numpy as np
import pytest

from paper_1412_1840_amd import qmi, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _both(ctx, curves, freqs, st=0.3):
    b = synth.pack(curves)
    T, Y, E, F = _dev(b.t), _dev(b.y), _dev(b.e), _dev(freqs)
    nc, nf = b.n_curves, len(freqs)
    outs = []
    for call in (ctx.periodogram_dev, ctx.periodogram_noalloc):
        sc = torch.full((nc, nf), -7.0, dtype=torch.float64, device="cuda:0")
        ips = torch.full((nc, nf, 3), -7.0, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()  # the library works on its own stream
        ipy, status = call(b.offsets, T, Y, E, F, sc, st, ips_out=ips)
        torch.cuda.synchronize()
        outs.append((sc.cpu().numpy(), ips.cpu().numpy(), ipy, status))
    return outs


def _assert_same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_noalloc_matches_dev_entry_point_twice():
    print("noalloc: 24 curves x 5500 frequencies, then 3 curves x 1000", flush=True)
    with qmi.Context(0) as ctx:
        big = [synth.survey_batch_curve(k, n=300 + 17 * k) for k in range(24)]
        freqs = np.linspace(1e-3, 10.0, 5500)  # 24 x 86 tiles: whole tiles per workgroup
        ref, got = _both(ctx, big, freqs)
        assert np.all(ref[3] == 0)
        assert np.all(np.isfinite(ref[0]))
        _assert_same(ref, got)
        small = [synth.survey_batch_curve(100 + k, n=n) for k, n in enumerate((37, 300, 513))]
        freqs2 = np.concatenate([[0.0], np.linspace(1e-3, 5.0, 999)])  # few tiles: one piece each
        ref2, got2 = _both(ctx, small, freqs2)
        assert np.all(ref2[3] == 0)
        _assert_same(ref2, got2)
        assert np.max(np.abs(got2[0][:, 0])) < 1e-12  # QMI(0) = 0


def test_noalloc_refuses_a_batch_larger_than_its_scratch():
    print("noalloc: oversize batch", flush=True)
    with qmi.Context(0) as ctx:
        n = 4200  # one K table alone needs 4200 x 4352 x 4 bytes > 64 MiB
        c = synth.survey_batch_curve(0, n=n)
        b = synth.pack([c])
        T, Y, E = _dev(b.t), _dev(b.y), _dev(b.e)
        F = _dev(np.linspace(0.01, 1.0, 64))
        sc = torch.full((1, 64), -7.0, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        with pytest.raises(qmi.QMIError) as ei:
            ctx.periodogram_noalloc(b.offsets, T, Y, E, F, sc, 0.3)
        assert ei.value.code == qmi.ENOMEM and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert np.all(sc.cpu().numpy() == -7.0)
        # the context stays usable
        small = synth.pack([synth.survey_batch_curve(1, n=200)])
        sc1 = torch.zeros((1, 64), dtype=torch.float64, device="cuda:0")
        sc2 = torch.zeros((1, 64), dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        args = (small.offsets, _dev(small.t), _dev(small.y), _dev(small.e), F)
        ctx.periodogram_dev(*args, sc1, 0.3)
        ctx.periodogram_noalloc(*args, sc2, 0.3)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(sc1.cpu().numpy(), sc2.cpu().numpy())
