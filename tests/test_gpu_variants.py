"""The FP32 form's read-path and seed-trig variants (Sections 3.6, 4.9 and
4.12 ask the same questions of shared memory and of the fast hardware sine)
against the oracle, through the C ABI (needs an MI355X).

Every variant computes the same sums, so each must meet the FP32 form's
bound (|dP| <= 1e-3 on the normalised power, peaks within one bin or an
oracle near-tie).  Reading the staged values from global memory instead of
LDS changes only where the same numbers come from, so LSP_OBS_DIRECT must
equal LSP_OBS_LDS bit for bit for each trig choice at the same K and waves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import (FP32_ATOL, assert_fp32_close, dev, oracle, peak_ok,  # noqa: E402,F401
                             run_batch, run_single, say)

pytestmark = pytest.mark.gpu

TRIGS = (lsp.TRIG_HW, lsp.TRIG_LIB, lsp.TRIG_POLY)


@pytest.mark.parametrize("k,waves", ((16, 1), (8, 4)))
def test_variants_batch(dev, k, waves):
    w = synth.make_workload("batch_10k", n_obj=24)
    ora_pg, ora_pk = oracle.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, 3000)
    for trig in TRIGS:
        got = {}
        for obs in (lsp.OBS_LDS, lsp.OBS_DIRECT):
            pg, pk = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, 3000,
                               form=lsp.FORM_FP32P, pgram_dtype=lsp.PGRAM_F64, k=k, waves=waves,
                               obs_read=obs, seed_trig=trig)
            err = assert_fp32_close(pg, ora_pg, f"obs={obs} trig={trig} k={k}")
            say(f"    obs={obs} trig={trig} k={k} waves={waves}: max |dP| {err:.3g}")
            for o in range(w.n_obj):
                assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], FP32_ATOL, 1)
            got[obs] = (pg, pk)
        assert np.array_equal(got[lsp.OBS_LDS][0], got[lsp.OBS_DIRECT][0])
        assert np.array_equal(got[lsp.OBS_LDS][1]["index"], got[lsp.OBS_DIRECT][1]["index"])


@pytest.mark.parametrize("t_split", (1, 8))
def test_variants_single_object(dev, t_split):
    w = synth.make_workload("single_4096")
    ora_pg, ora_pk = oracle.single(w.t, w.y, w.f_min, w.f_max, 20000)
    for obs, trig in ((lsp.OBS_DIRECT, lsp.TRIG_HW), (lsp.OBS_LDS, lsp.TRIG_POLY),
                      (lsp.OBS_DIRECT, lsp.TRIG_LIB)):
        pg, pk = run_single(dev, w.t, w.y, w.f_min, w.f_max, 20000, form=lsp.FORM_FP32P,
                            pgram_dtype=lsp.PGRAM_F64, t_split=t_split, obs_read=obs,
                            seed_trig=trig)
        err = assert_fp32_close(pg, ora_pg, f"single obs={obs} trig={trig} split={t_split}")
        say(f"    single obs={obs} trig={trig} split={t_split}: max |dP| {err:.3g}")
        assert peak_ok(ora_pg, ora_pk["index"], pk["index"], FP32_ATOL, 1)


def test_variants_edge_objects(dev):
    t0, y0, _ = synth.sine_object(120, 9)
    series = [(t0, y0), (np.zeros(0), np.zeros(0)), (np.array([2.0]), np.array([1.0])),
              (t0, np.full(120, 0.3)), (t0, np.where(np.arange(120) == 3, np.nan, y0)),
              (t0[:2], y0[:2])]
    off, t, y = synth.pack(series)
    ora_pg, ora_pk = oracle.batch(off, t, y, 1.0, 12.0, 1500)
    for trig in TRIGS:
        pg, pk = run_batch(dev, off, t, y, 1.0, 12.0, 1500, form=lsp.FORM_FP32P,
                           pgram_dtype=lsp.PGRAM_F64, obs_read=lsp.OBS_DIRECT, seed_trig=trig)
        assert_fp32_close(pg, ora_pg, f"edge objects trig={trig}")
        assert list(pk["status"]) == list(ora_pk["status"])
