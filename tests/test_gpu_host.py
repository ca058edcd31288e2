"""Returning batch periodograms to host memory through the pinned-staging
pipeline (lsp_pipe_create / lsp_batch_to_host; Section 3.5), needs an MI355X.

The pipeline runs the same kernels with the whole batch's launch
configuration chunk by chunk, so its host arrays must equal lsp_batch's device
results copied back, bit for bit, whatever the stream count, staging size and
chunk size (pieces that do not divide a chunk, chunks that do not divide the
batch, several chunks per stream).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import cuda, dev, peak_ok, say  # noqa: E402,F401

pytestmark = pytest.mark.gpu

PIPES = [  # (streams, staging bytes, chunk bytes, copy threads)
    (1, 64 << 10, 256 << 10, 1),
    (3, 0, 1 << 20, 0),
    (8, 4 << 10, 64 << 10, 16),
]


def device_batch(dev, w, n_f, dy=None, method="standard", **kw):
    p = lsp.Periodogram(cuda(w.t, dev), cuda(w.y, dev), w.f_min, w.f_max, n_f,
                        offsets=cuda(w.offsets, dev, torch.int64), method=method,
                        dy=None if dy is None else cuda(dy, dev), **kw)
    p()
    torch.cuda.synchronize()
    return p.pgram.cpu().numpy(), p.peaks()


def host_batch(pipe, dev, w, n_f, dy=None, method="standard", **kw):
    say(f"  lsp_batch_to_host n_obj={w.n_obj} n_f={n_f} {method} {kw}")
    pg, pk = pipe.batch_to_host(cuda(w.offsets, dev, torch.int64), cuda(w.t, dev),
                                cuda(w.y, dev), w.f_min, w.f_max, n_f,
                                dy=None if dy is None else cuda(dy, dev), method=method, **kw)
    return pg, pk


@pytest.mark.parametrize("pipe_args", PIPES, ids=lambda a: "s%d" % a[0])
@pytest.mark.parametrize("form", (lsp.FORM_FP64, lsp.FORM_FP32P))
def test_to_host_equals_device_batch(dev, pipe_args, form):
    w = synth.make_workload("batch_10k", n_obj=37)
    pipe = lsp.HostPipe(*pipe_args)
    for dt in (lsp.PGRAM_F32, lsp.PGRAM_F64):
        ref, rk = device_batch(dev, w, 3001, form=form, pgram_dtype=dt)
        pg, pk = host_batch(pipe, dev, w, 3001, form=form, pgram_dtype=dt)
        assert np.array_equal(pg, ref)
        assert np.array_equal(pk.view(np.uint8), rk.view(np.uint8))
    # peaks only, then the periodogram only, on the same pipe
    _, pk = host_batch(pipe, dev, w, 3001, form=form, pgram=False)
    _, rk = device_batch(dev, w, 3001, form=form)
    assert np.array_equal(pk.view(np.uint8), rk.view(np.uint8))
    pg, pk = host_batch(pipe, dev, w, 3001, form=form, peaks=False)
    assert pk is None and np.array_equal(pg, device_batch(dev, w, 3001, form=form)[0])
    pipe.close()


def test_to_host_generalized_and_single_object(dev):
    w = synth.make_workload("batch_10k", n_obj=20, errors=True)
    pipe = lsp.HostPipe(2, 32 << 10, 128 << 10, 4)
    for form in (lsp.FORM_FP64, lsp.FORM_FP32P):
        ref, rk = device_batch(dev, w, 2500, dy=w.dy, method="generalized", form=form)
        pg, pk = host_batch(pipe, dev, w, 2500, dy=w.dy, method="generalized", form=form)
        assert np.array_equal(pg, ref)
        assert np.array_equal(pk.view(np.uint8), rk.view(np.uint8))
    one = w.subset(1)
    ref, rk = device_batch(dev, one, 40000, form=lsp.FORM_FP32P)
    pg, pk = host_batch(pipe, dev, one, 40000, form=lsp.FORM_FP32P)
    assert np.array_equal(pg, ref) and np.array_equal(pk.view(np.uint8), rk.view(np.uint8))
    pipe.close()


def test_to_host_large_batch(dev):
    # 2,000 objects x 100,000 bins: an 800 MB FP32 periodogram, 13 chunks of
    # 64 MiB over 3 streams
    w = synth.make_workload("batch_10k", n_obj=2000)
    pipe = lsp.HostPipe()
    pg, pk = host_batch(pipe, dev, w, w.n_f, form=lsp.FORM_FP32P)
    ref, rk = device_batch(dev, w, w.n_f, form=lsp.FORM_FP32P)
    assert np.array_equal(pg, ref)
    assert np.array_equal(pk.view(np.uint8), rk.view(np.uint8))
    pipe.close()


@pytest.mark.parametrize("method", ["standard", "generalized"])
def test_to_host_against_oracle(dev, method):
    """The host arrays themselves against the oracle's batch mode (Section
    3.5's returned periodograms, Section 3.4's peaks): every bin of 37 objects
    in both forms, FP64 within 1e-9 * max(P, 1e-3) and FP32 within 1e-3, with
    one pipe shape whose staging pieces and chunks divide nothing evenly."""
    import oracle

    gen = method == "generalized"
    w = synth.make_workload("batch_10k", n_obj=37, errors=gen)
    n_f = 3001
    if gen:
        ora_pg, ora_pk = oracle.gen_batch(w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, n_f)
    else:
        ora_pg, ora_pk = oracle.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, n_f)
    pipe = lsp.HostPipe(3, 24 << 10, 200 << 10, 5)
    for form, dt in ((lsp.FORM_FP64, lsp.PGRAM_F64), (lsp.FORM_FP32P, lsp.PGRAM_F32)):
        pg, pk = host_batch(pipe, dev, w, n_f, dy=w.dy if gen else None, method=method,
                            form=form, pgram_dtype=dt)
        err = np.abs(pg.astype(np.float64) - ora_pg)
        if form == lsp.FORM_FP64:
            assert np.all(err <= 1e-9 * np.maximum(ora_pg, 1e-3)), err.max()
        else:
            assert err.max() <= 1e-3
        for o in range(w.n_obj):
            if form == lsp.FORM_FP64:
                assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], 1e-9)
            else:
                assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], 2e-3, bins=1)
        assert np.array_equal(pk["status"], ora_pk["status"])
    pipe.close()
