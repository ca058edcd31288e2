"""Maximum sizes (needs an MI355X): a single object on 10^8 bins (the largest
grid Section 4.10 evaluates) and a batch whose periodogram holds more than
2^31 bins, so that output offsets need 64 bits and grid launches fold into
two dimensions.  The oracle is evaluated at sampled (object, bin) pairs; the
sampled values are gathered on the device so that the multi-gigabyte
periodograms never cross to the host.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import (FP32_ATOL, assert_fp32_close, assert_fp64_close, cuda, dev,  # noqa: E402,F401
                             oracle, say)

pytestmark = pytest.mark.gpu


def test_single_object_1e8_bins(dev):
    w = synth.make_workload("single_4096")
    n_f = 100_000_000
    t, y = cuda(w.t, dev), cuda(w.y, dev)
    say(f"  single_4096 on {n_f} bins, FP32 form with periodogram, FP64 form peaks only")
    p32 = lsp.Periodogram(t, y, w.f_min, w.f_max, n_f, form=lsp.FORM_FP32P)
    p32()
    p64 = lsp.Periodogram(t, y, w.f_min, w.f_max, n_f, form=lsp.FORM_FP64, pgram=False)
    p64()
    torch.cuda.synchronize()
    k32, k64 = p32.peaks()[0], p64.peaks()[0]
    rng = np.random.default_rng(41)
    bins = np.unique(np.concatenate([rng.integers(0, n_f, 400), [0, n_f - 1],
                                     np.clip(k64["index"] + np.arange(-3, 4), 0, n_f - 1)]))
    got = p32.pgram[0][torch.as_tensor(bins, device=dev)].double().cpu().numpy()
    off = np.array([0, w.n_obs], dtype=np.int64)
    ora = oracle.eval_bins(off, w.t, w.y, w.f_min, w.f_max, n_f, np.zeros(len(bins), np.int64),
                           bins)
    err = assert_fp32_close(got, ora, "1e8 bins, sampled")
    say(f"    sampled max |dP| {err:.3g}; peaks fp32 {k32['index']} fp64 {k64['index']}")
    assert abs(int(k32["index"]) - int(k64["index"])) <= 1
    # the FP64 peak is the oracle's best bin in its neighbourhood
    nb = np.clip(k64["index"] + np.arange(-3, 4), 0, n_f - 1)
    ora_nb = oracle.eval_bins(off, w.t, w.y, w.f_min, w.f_max, n_f, np.zeros(7, np.int64), nb)
    assert nb[int(np.argmax(ora_nb))] == k64["index"]
    assert_fp64_close([k64["power"]], [ora_nb[int(np.argmax(ora_nb))]], "1e8 bins, peak power")


@pytest.mark.parametrize("schedule", (lsp.SCHED_GRID, lsp.SCHED_PERSISTENT))
def test_batch_beyond_2_31_bins(dev, schedule):
    # 2,200 objects x 1,000,000 bins = 2.2e9 bins (8.8 GB of FP32 periodogram):
    # objects from 2,148 on start past 2^31 in the output, and the grid launch
    # has 2.2e6 items, folded into a 2-D grid
    w = synth.make_workload("batch_10k", n_obj=2200)
    n_f = 1_000_000
    assert w.n_obj * n_f > 2 ** 31
    say(f"  batch of {w.n_obj} objects on {n_f} bins, schedule {schedule}")
    p = lsp.Periodogram(cuda(w.t, dev), cuda(w.y, dev), w.f_min, w.f_max, n_f,
                        offsets=cuda(w.offsets, dev, torch.int64), form=lsp.FORM_FP32P,
                        schedule=schedule)
    p()
    torch.cuda.synchronize()
    pk = p.peaks()
    rng = np.random.default_rng(43)
    objs = np.concatenate([rng.integers(0, w.n_obj, 150), rng.integers(2148, w.n_obj, 150),
                           [w.n_obj - 1, w.n_obj - 1, 0]])
    bins = np.concatenate([rng.integers(0, n_f, 300), [n_f - 1, 0, n_f - 1]])
    flat = torch.as_tensor(objs * n_f + bins, device=dev)
    got = p.pgram.view(-1)[flat].double().cpu().numpy()
    ora = oracle.eval_bins(w.offsets, w.t, w.y, w.f_min, w.f_max, n_f, objs, bins)
    err = assert_fp32_close(got, ora, "beyond 2^31 bins, sampled")
    say(f"    sampled max |dP| {err:.3g}")
    assert np.all(pk["status"] == 0)
    # whole periodograms of the last two objects (output offsets past 2^31)
    for o in (w.n_obj - 2, w.n_obj - 1):
        a, b = w.offsets[o], w.offsets[o + 1]
        ora_pg, ora_pk = oracle.single(w.t[a:b], w.y[a:b], w.f_min, w.f_max, n_f)
        row = p.pgram[o].double().cpu().numpy()
        assert_fp32_close(row, ora_pg, f"object {o} whole periodogram")
        i = int(pk["index"][o])
        assert abs(i - int(ora_pk["index"])) <= 1 or ora_pg[i] >= ora_pk["power"] - FP32_ATOL
