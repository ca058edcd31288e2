"""Generalized periodogram (errors, floating mean; Section 4.11): HIP path vs
the oracle through the C ABI (needs an MI355X).

Tolerances are those of the standard periodogram:
  FP64 form : |P_gpu - P_ora| <= 1e-9 * max(P_ora, 1e-3) on the normalised power
  FP32 form : |P_gpu - P_ora| <= 1e-3 on the normalised power
  peaks     : FP64 form the oracle's index unless the oracle ties within 1e-9;
              FP32 form within one bin, or an oracle near-tie (1e-3).
The unnormalised power (half the chi^2 reduction) is compared after dividing
by half the object's weighted variance sum, which maps it onto the normalised
scale where these tolerances apply.

A three-point object has bins where the mean-removed cos and sin columns are
nearly parallel: the 2 x 2 moment matrix has condition number kappa^2 up to
~1e10 there, and any FP64 evaluation (the oracle's included) carries relative
error ~ eps * kappa^2.  For that object the FP64 bound gains
1e-14 * kappa^2 * max(P, 1e-3) (about 45 eps kappa^2), with kappa^2 computed
per bin by numpy from the weighted, mean-removed design.  (With two points the
mean-removed columns are always parallel; both sides drop that direction and
agree to the plain bound.)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as _oracle  # noqa: E402
from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import (FP32_ATOL, assert_fp32_close, assert_fp64_close, cuda, dev,  # noqa: E402,F401
                             oracle, peak_ok, say)

pytestmark = pytest.mark.gpu

FORMS = (lsp.FORM_FP64, lsp.FORM_FP32P)


def gen_batch(dev, off, t, y, dy, f_min, f_max, n_f, **kw):
    say(f"  gpu lsp_gen_batch n_obj={len(off) - 1} n_obs={len(t)} n_f={n_f} "
        f"dy={'yes' if dy is not None else 'unit'} {kw}")
    p = lsp.Periodogram(cuda(t, dev), cuda(y, dev), f_min, f_max, n_f,
                        offsets=cuda(off, dev, torch.int64), method="generalized",
                        dy=None if dy is None else cuda(dy, dev), **kw)
    p()
    torch.cuda.synchronize()
    pg = p.pgram.double().cpu().numpy() if p.pgram is not None else None
    return pg, p.peaks()


def gen_single(dev, t, y, dy, f_min, f_max, n_f, **kw):
    say(f"  gpu lsp_gen_single n_t={len(t)} n_f={n_f} {kw}")
    p = lsp.Periodogram(cuda(t, dev), cuda(y, dev), f_min, f_max, n_f, method="generalized",
                        dy=None if dy is None else cuda(dy, dev), **kw)
    p()
    torch.cuda.synchronize()
    pg = p.pgram[0].double().cpu().numpy() if p.pgram is not None else None
    return pg, p.peaks()[0]


def moment_condition(t, dy, freqs):
    """kappa^2 = lambda_max / lambda_min of the weighted, mean-removed [cos, sin]
    moment matrix at each frequency (cycles)."""
    w = 1.0 / dy ** 2
    w = w / w.sum()
    ph = 2 * np.pi * np.outer(freqs, t)
    c, s = np.cos(ph), np.sin(ph)
    c -= (c * w).sum(axis=1, keepdims=True)
    s -= (s * w).sum(axis=1, keepdims=True)
    m = np.empty((len(freqs), 2, 2))
    m[:, 0, 0] = (w * c * c).sum(axis=1)
    m[:, 1, 1] = (w * s * s).sum(axis=1)
    m[:, 0, 1] = m[:, 1, 0] = (w * c * s).sum(axis=1)
    ev = np.linalg.eigvalsh(m)
    return ev[:, 1] / np.maximum(ev[:, 0], 1e-300)


def check_rows(form, pg, pk, ora_pg, ora_pk, what, kappa2=None):
    if form == lsp.FORM_FP64:
        if kappa2 is None:
            assert_fp64_close(pg, ora_pg, what)
        else:
            both_nan = np.isnan(pg) & np.isnan(ora_pg)
            err = np.where(both_nan, 0.0, np.abs(pg - ora_pg))
            scale = np.maximum(np.abs(np.nan_to_num(ora_pg)), 1e-3)
            bad = ~(err <= (1e-9 + 1e-14 * kappa2) * scale)
            assert not bad.any(), f"{what}: {bad.sum()} bins off"
        tol, bins = 1e-9, 0
    else:
        err = assert_fp32_close(pg, ora_pg, what)
        say(f"    {what}: max |dP| {err:.3g}")
        tol, bins = FP32_ATOL, 1
    for o in range(len(pk)):
        assert pk["status"][o] == ora_pk["status"][o], (what, o)
        if ora_pk["status"][o] == _oracle.OK:
            assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], tol, bins), (what, o)
        else:
            assert pk["index"][o] == -1


@pytest.mark.parametrize("form", FORMS)
def test_gen_batch_with_errors(dev, form):
    # 24 objects of 50-1000 points; 3,000 bins span several tiles of either
    # form with a ragged last tile
    w = synth.make_workload("batch_10k", n_obj=24, errors=True)
    ora_pg, ora_pk = oracle.gen_batch(w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, 3000)
    pg, pk = gen_batch(dev, w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, 3000, form=form,
                       pgram_dtype=lsp.PGRAM_F64)
    check_rows(form, pg, pk, ora_pg, ora_pk, f"gen batch form={form}")


@pytest.mark.parametrize("form", FORMS)
def test_gen_unit_errors(dev, form):
    w = synth.make_workload("batch_10k", n_obj=12)
    ora_pg, ora_pk = oracle.gen_batch(w.offsets, w.t, w.y, None, w.f_min, w.f_max, 2100)
    pg, pk = gen_batch(dev, w.offsets, w.t, w.y, None, w.f_min, w.f_max, 2100, form=form,
                       pgram_dtype=lsp.PGRAM_F64)
    check_rows(form, pg, pk, ora_pg, ora_pk, f"gen unit errors form={form}")
    # dy = NULL and dy = 1 are the same computation
    pg1, pk1 = gen_batch(dev, w.offsets, w.t, w.y, np.ones(w.n_obs), w.f_min, w.f_max, 2100,
                         form=form, pgram_dtype=lsp.PGRAM_F64)
    assert np.array_equal(pg1, pg) and np.array_equal(pk1["index"], pk["index"])


@pytest.mark.parametrize("form", FORMS)
def test_gen_unnormalised(dev, form):
    w = synth.make_workload("batch_10k", n_obj=8, errors=True)
    ora_pg, _ = oracle.gen_batch(w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, 1500,
                                 normalize=False)
    pg, _ = gen_batch(dev, w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, 1500, form=form,
                      normalize=False, pgram_dtype=lsp.PGRAM_F64)
    for o in range(w.n_obj):
        a, b = w.offsets[o], w.offsets[o + 1]
        _, _, _, yy, _ = _oracle.gen_prep(w.t[a:b], w.y[a:b], w.dy[a:b])
        scale = 2.0 / yy
        what = f"gen unnormalised form={form} object {o}"
        if form == lsp.FORM_FP64:
            assert_fp64_close(pg[o] * scale, ora_pg[o] * scale, what)
        else:
            assert_fp32_close(pg[o] * scale, ora_pg[o] * scale, what)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("t_split", (0, 1, 8))
def test_gen_single_object(dev, form, t_split):
    # one 4,096-point object on 20,000 bins: the FP32 form's four-wave
    # single-object launch, unsplit (fix-up path) and split (combine path)
    if form == lsp.FORM_FP64 and t_split > 1:
        pytest.skip("the FP64 form has no observation split")
    w = synth.make_workload("single_4096", errors=True)
    n_f = 20000
    ora_pg, ora_pk = oracle.gen_single(w.t, w.y, w.dy, w.f_min, w.f_max, n_f)
    pg, pk = gen_single(dev, w.t, w.y, w.dy, w.f_min, w.f_max, n_f, form=form, t_split=t_split,
                        pgram_dtype=lsp.PGRAM_F64)
    check_rows(form, pg[None], np.array([pk]), ora_pg[None], np.array([ora_pk]),
               f"gen single form={form} t_split={t_split}")


@pytest.mark.parametrize("form", FORMS)
def test_gen_edge_objects(dev, form):
    rng = np.random.default_rng(17)
    t0, y0, _ = synth.sine_object(150, 3)
    d0 = rng.uniform(0.02, 0.1, 150)
    bad = lambda v, j, x: np.where(np.arange(len(v)) == j, x, v)  # noqa: E731
    series = [
        (t0, y0, d0),
        (np.zeros(0), np.zeros(0), np.zeros(0)),            # empty
        (np.array([5.0]), np.array([1.0]), np.array([0.1])),  # one point
        (t0[:2], y0[:2], d0[:2]),                            # two points
        (t0[:3], y0[:3], d0[:3]),                            # three points
        (t0, np.full(150, 0.4), d0),                         # no variance
        (t0, bad(y0, 4, np.nan), d0),                        # NaN magnitude
        (t0, y0, bad(d0, 9, 0.0)),                           # zero error
        (t0, y0, bad(d0, 9, -0.05)),                         # negative error
        (t0, y0, bad(d0, 9, np.inf)),                        # infinite error
        (t0, y0, bad(d0, 9, np.nan)),                        # NaN error
        (t0[:40], y0[:40], d0[:40]),                         # short, ordinary
    ]
    off = np.concatenate([[0], np.cumsum([len(s[0]) for s in series])]).astype(np.int64)
    t = np.concatenate([s[0] for s in series])
    y = np.concatenate([s[1] for s in series])
    dy = np.concatenate([s[2] for s in series])
    ora_pg, ora_pk = oracle.gen_batch(off, t, y, dy, 1.0, 12.0, 700)
    pg, pk = gen_batch(dev, off, t, y, dy, 1.0, 12.0, 700, form=form, pgram_dtype=lsp.PGRAM_F64)
    freqs = 1.0 + 11.0 / 700 * np.arange(700)
    kappa2 = np.zeros_like(ora_pg)
    for o in (4,):  # the three-point object
        a, b = off[o], off[o + 1]
        kappa2[o] = moment_condition(t[a:b], dy[a:b], freqs)
    check_rows(form, pg, pk, ora_pg, ora_pk, f"gen edge objects form={form}", kappa2)
    want = [_oracle.OK, _oracle.DEGENERATE, _oracle.DEGENERATE, _oracle.OK, _oracle.OK,
            _oracle.DEGENERATE] + [_oracle.NONFINITE] * 5 + [_oracle.OK]
    assert list(pk["status"]) == want


@pytest.mark.parametrize("form", FORMS)
def test_gen_ill_conditioned_bins(dev, form):
    # integer-day sampling: at f = 0, 1, 2, ... cycles/day every phase is
    # equal, only the offset survives and the power is 0; the FP32 form must
    # hand those bins to the FP64 fix-up (single object and batch alike)
    rng = np.random.default_rng(23)
    t = np.sort(rng.choice(np.arange(2000.0), 300, replace=False))
    y = 0.3 * np.sin(2 * np.pi * 0.37 * t) + rng.normal(0, 0.05, 300)
    dy = rng.uniform(0.03, 0.08, 300)
    ora_pg, ora_pk = oracle.gen_single(t, y, dy, 0.0, 3.0, 3000)
    assert ora_pg[0] == 0.0 and abs(ora_pg[1000]) < 1e-9 and abs(ora_pg[2000]) < 1e-9
    pg, pk = gen_single(dev, t, y, dy, 0.0, 3.0, 3000, form=form, pgram_dtype=lsp.PGRAM_F64)
    check_rows(form, pg[None], np.array([pk]), ora_pg[None], np.array([ora_pk]),
               f"gen ill-conditioned single form={form}")
    off = np.array([0, 300, 600], dtype=np.int64)
    pgb, pkb = gen_batch(dev, off, np.concatenate([t, t]), np.concatenate([y, -y]),
                         np.concatenate([dy, dy]), 0.0, 3.0, 3000, form=form,
                         pgram_dtype=lsp.PGRAM_F64)
    ora_b, ora_bk = oracle.gen_batch(off, np.concatenate([t, t]), np.concatenate([y, -y]),
                                     np.concatenate([dy, dy]), 0.0, 3.0, 3000)
    check_rows(form, pgb, pkb, ora_b, ora_bk, f"gen ill-conditioned batch form={form}")


def test_gen_single_4096_full_size_sampled(dev):
    # the benchmark's launch: one 4,096-point object with errors on 500,000
    # bins, FP32 form with the library's default configuration; sampled bins
    # against the oracle, and the peak against the FP64 form's on the same grid
    w = synth.make_workload("single_4096", errors=True)
    p32, k32 = gen_single(dev, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P)
    p64, k64 = gen_single(dev, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64,
                          pgram_dtype=lsp.PGRAM_F64)
    rng = np.random.default_rng(29)
    bins = np.unique(np.concatenate([rng.integers(0, w.n_f, 300), [0, w.n_f - 1],
                                     np.clip(k64["index"] + np.arange(-2, 3), 0, w.n_f - 1)]))
    off = np.array([0, w.n_obs], dtype=np.int64)
    ora = oracle.gen_eval_bins(off, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f,
                               np.zeros(len(bins), np.int64), bins)
    assert_fp64_close(p64[bins], ora, "gen single_4096 fp64 sampled")
    err = assert_fp32_close(p32[bins], ora, "gen single_4096 fp32 sampled")
    assert_fp32_close(p32, p64, "gen single_4096 fp32 vs fp64 whole grid")
    say(f"    sampled max |dP| fp32 {err:.3g}; peaks fp32 {k32['index']} fp64 {k64['index']}")
    assert peak_ok(p64, k64["index"], k32["index"], FP32_ATOL, 1)
    # the FP64 form's peak is the oracle's maximum over its neighbourhood
    nb = np.clip(k64["index"] + np.arange(-2, 3), 0, w.n_f - 1)
    ora_nb = oracle.gen_eval_bins(off, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f,
                                  np.zeros(5, np.int64), nb)
    assert nb[int(np.argmax(ora_nb))] == k64["index"]


def test_gen_batch_10k_full_size_sampled_objects(dev):
    # the whole batch_10k workload with errors, peaks only (the batch launch),
    # FP32 form; a sample of objects against the oracle's whole periodograms
    w = synth.make_workload("batch_10k", errors=True)
    _, pk = gen_batch(dev, w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, w.n_f,
                      form=lsp.FORM_FP32P, pgram=False)
    rng = np.random.default_rng(31)
    objs = np.sort(rng.choice(w.n_obj, 6, replace=False))
    for o in objs:
        a, b = w.offsets[o], w.offsets[o + 1]
        ora_pg, ora_pk = oracle.gen_single(w.t[a:b], w.y[a:b], w.dy[a:b], w.f_min, w.f_max,
                                           w.n_f)
        assert pk["status"][o] == _oracle.OK
        assert peak_ok(ora_pg, ora_pk["index"], pk["index"][o], FP32_ATOL, 1), o
        assert abs(pk["power"][o] - ora_pg[pk["index"][o]]) <= FP32_ATOL, o


@pytest.mark.parametrize("form", FORMS)
def test_gen_wide_error_range(dev, form):
    # errors spread over six decades (weights over twelve): the power is set
    # by the best-measured points, which the rescaled FP32 weights must keep
    rng = np.random.default_rng(47)
    w = synth.make_workload("batch_10k", n_obj=10)
    dy = 10.0 ** rng.uniform(-3.0, 3.0, w.n_obs)
    ora_pg, ora_pk = oracle.gen_batch(w.offsets, w.t, w.y, dy, w.f_min, w.f_max, 1800)
    pg, pk = gen_batch(dev, w.offsets, w.t, w.y, dy, w.f_min, w.f_max, 1800, form=form,
                       pgram_dtype=lsp.PGRAM_F64)
    check_rows(form, pg, pk, ora_pg, ora_pk, f"gen wide error range form={form}")


@pytest.mark.parametrize("form", FORMS)
def test_gen_rows(dev, form):
    # row mode of the generalized periodogram: whole-grid rows equal
    # lsp_gen_batch bit for bit; banded rows match the oracle on their bins
    w = synth.make_workload("batch_10k", n_obj=9, errors=True)
    n_f, bb = 2000, 250
    ref, rk = gen_batch(dev, w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, n_f, form=form,
                        pgram_dtype=lsp.PGRAM_F64)
    args = (cuda(w.offsets, dev, torch.int64), cuda(w.t, dev), cuda(w.y, dev), w.f_min, w.f_max,
            n_f)
    pg = torch.full((w.n_obj, n_f), -7.0, dtype=torch.float64, device=dev)
    r = lsp.Rows(*args, row_obj=torch.arange(w.n_obj, dtype=torch.int32, device=dev),
                 form=form, pgram=pg, pgram_dtype=lsp.PGRAM_F64, method="generalized",
                 dy=cuda(w.dy, dev))
    r()
    torch.cuda.synchronize()
    assert np.array_equal(pg.cpu().numpy(), ref)
    assert np.array_equal(r.peaks()["index"], rk["index"])
    ora_pg, _ = oracle.gen_batch(w.offsets, w.t, w.y, w.dy, w.f_min, w.f_max, n_f)
    row_obj = torch.tensor([2, 2, 5, 5, 7, 7], dtype=torch.int32, device=dev)
    row_band = torch.tensor([0, 3, 7, 1, 4, 6], dtype=torch.int32, device=dev)
    pg2 = torch.full((w.n_obj, n_f), -7.0, dtype=torch.float64, device=dev)
    r2 = lsp.Rows(*args, row_obj=row_obj, row_band=row_band, band_bins=bb, rows_per_group=2,
                  form=form, pgram=pg2, pgram_dtype=lsp.PGRAM_F64, method="generalized",
                  dy=cuda(w.dy, dev))
    r2()
    torch.cuda.synchronize()
    got = pg2.cpu().numpy()
    for o, b in zip(row_obj.tolist(), row_band.tolist()):
        sl = slice(b * bb, (b + 1) * bb)
        if form == lsp.FORM_FP64:
            assert_fp64_close(got[o, sl], ora_pg[o, sl], f"gen rows object {o} band {b}")
        else:
            assert_fp32_close(got[o, sl], ora_pg[o, sl], f"gen rows object {o} band {b}")
    untouched = np.ones((w.n_obj, n_f), dtype=bool)
    for o, b in zip(row_obj.tolist(), row_band.tolist()):
        untouched[o, b * bb:(b + 1) * bb] = False
    assert np.all(got[untouched] == -7.0)


def test_gen_plan_replays(dev):
    # a generalized call captured once as a HIP graph: every replay, with eager
    # work in between, reproduces the eager result bit for bit
    w = synth.make_workload("batch_10k", n_obj=16, errors=True)
    p = lsp.Periodogram(cuda(w.t, dev), cuda(w.y, dev), w.f_min, w.f_max, 3000,
                        offsets=cuda(w.offsets, dev, torch.int64), form=lsp.FORM_FP32P,
                        method="generalized", dy=cuda(w.dy, dev))
    p()
    torch.cuda.synchronize()
    eager, ek = p.pgram.clone(), p.peaks()
    plan = p.capture()
    for i in range(3):
        p.pgram.fill_(-1.0)
        torch.cuda.synchronize()
        plan()
        torch.cuda.synchronize()
        assert torch.equal(p.pgram, eager), f"replay {i}"
        assert np.array_equal(p.peaks()["index"], ek["index"])
        p()  # eager call between replays
        torch.cuda.synchronize()
