"""lsp_batch_static -- lsp_batch without a workspace, for callers that cannot
allocate -- against lsp_batch through the C ABI (needs an MI355X).

Two calls in a row on the library's static scratch, the second on a smaller
input, each compared with lsp_batch on its own workspace: the periodograms and
peak records must be identical bit for bit (same kernels, same launch
configuration), in the FP32 and the FP64 form.  A call whose workspace would
exceed the static array is refused on the host with LSP_ESCRATCH.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(dev, n_obj, seed):
    w = synth.make_workload("batch_10k", n_obj=n_obj, seed=seed)
    return w, (torch.as_tensor(w.offsets, device=dev), torch.as_tensor(w.t, device=dev),
               torch.as_tensor(w.y, device=dev))


def _compare(dev, n_obj, seed, n_f, form, pgram_dtype):
    w, (off, t, y) = _inputs(dev, n_obj, seed)
    kw = dict(form=form, pgram_dtype=pgram_dtype)
    grid, opt = lsp.make_grid(w.f_min, w.f_max, n_f), lsp.make_options(**kw)
    need = lsp.workspace_bytes(w.n_obj, w.n_obs, grid, opt)
    assert 0 < need <= lsp.STATIC_SCRATCH_BYTES
    ref = lsp.Periodogram(t, y, w.f_min, w.f_max, n_f, offsets=off, pgram=True, peaks=True, **kw)
    ref()
    pdt = torch.float64 if pgram_dtype == lsp.PGRAM_F64 else torch.float32
    pg = torch.full((w.n_obj, n_f), -7.0, dtype=pdt, device=dev)
    pk = torch.zeros(w.n_obj * lsp.PEAK_BYTES, dtype=torch.uint8, device=dev)
    lsp.batch_static(off, t, y, w.f_min, w.f_max, n_f, pgram=pg, peaks=pk, **kw)
    torch.cuda.synchronize()
    assert torch.equal(pg.view(torch.uint8), ref.pgram.view(torch.uint8))
    assert torch.equal(pk, ref.peaks_raw)
    peaks = pk.cpu().numpy().view(lsp.PEAK_DTYPE)
    assert np.all(peaks["status"] == lsp.OBJ_OK) and np.all(peaks["index"] >= 0)
    return need


@pytest.mark.parametrize("form", [lsp.FORM_FP32P, lsp.FORM_FP64], ids=["fp32", "fp64"])
def test_static_scratch_matches_workspace_call_twice(dev, form):
    # a larger call, then a smaller one on the same static array
    need1 = _compare(dev, 1500, synth.SEED_BASE + 7001, 40_000, form, lsp.PGRAM_F32)
    need2 = _compare(dev, 200, synth.SEED_BASE + 7002, 9_000, form, lsp.PGRAM_F64)
    assert need2 < need1


def test_static_scratch_refuses_oversized_calls(dev):
    w, (off, t, y) = _inputs(dev, 10, synth.SEED_BASE + 7003)
    grid = lsp.make_grid(w.f_min, w.f_max, 250_000)
    opt = lsp.make_options(form=lsp.FORM_FP64)
    big = 200_000  # the FP64 form's per-tile records need ~1.6 GB: refused before any read
    assert lsp.workspace_bytes(big, w.n_obs, grid, opt) > lsp.STATIC_SCRATCH_BYTES
    peaks = torch.zeros(w.n_obj * lsp.PEAK_BYTES, dtype=torch.uint8, device=dev)
    st = lsp.lib().lsp_batch_static(ctypes.c_void_p(off.data_ptr()), big, w.n_obs,
                                    ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    ctypes.byref(grid), ctypes.byref(opt), None,
                                    ctypes.c_void_p(peaks.data_ptr()), None)
    assert st == lsp.ESCRATCH
    assert lsp.status_string(st).startswith("call exceeds the static scratch")
    # and a valid call afterwards still works
    _compare(dev, 50, synth.SEED_BASE + 7004, 5_000, lsp.FORM_FP32P, lsp.PGRAM_F32)
