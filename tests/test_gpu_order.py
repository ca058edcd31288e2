"""Longest-first row order (lsp_row_order, LSP_ORDER_LPT) through the C ABI
(needs an MI355X).

  * The permutation: every row exactly once; position s of the descending
    order in XCD s % 8's run, the runs contiguous and balanced.  With
    observation counts below 1,024 (compared exactly) each run must equal the
    descending order dealt round-robin; above, each entry may differ from it
    only within a bucket (1/64 of an octave).  Rows with no work (invalid
    objects, negative bands) come after every other row, empty objects' rows
    among the cheapest.
  * The order changes no result: periodograms and peaks are bitwise equal
    under input and longest-first order for the FP32 form (persistent and grid
    schedules), the FP64 form, both generalized forms, row mode, and replays
    of a captured graph.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_04006_amd import lsp, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _runs(n_rows):
    """Contiguous, balanced runs of the 8 XCDs (the first n_rows % 8 one longer)."""
    base, rem = divmod(n_rows, 8)
    sizes = [base + (x < rem) for x in range(8)]
    starts = np.concatenate([[0], np.cumsum(sizes)])
    return [(int(starts[x]), int(starts[x + 1])) for x in range(8)]


def _perm(dev, n_t, **kw):
    off = np.concatenate([[0], np.cumsum(n_t)]).astype(np.int64)
    say(f"lsp_row_order n_obj={len(n_t)} {sorted(kw)}")
    perm = lsp.row_order(torch.as_tensor(off, device=dev), **kw)
    torch.cuda.synchronize()
    return perm.cpu().numpy().astype(np.int64)


def _check_dealt(cost, perm, exact):
    n = len(cost)
    assert np.array_equal(np.sort(perm), np.arange(n)), "not a permutation"
    want = np.sort(cost)[::-1]
    for x, (a, b) in enumerate(_runs(n)):
        got = cost[perm[a:b]]
        ref = want[x::8]
        assert len(got) == len(ref)
        if exact:
            assert np.array_equal(got, ref), f"run {x}"
        else:
            assert np.all(np.abs(got - ref) <= np.maximum(got, ref) / 64.0), f"run {x}"


@pytest.mark.parametrize("n_obj", [1, 7, 8, 9, 1000, 20011])
def test_row_order_small_counts_exact(dev, n_obj):
    rng = np.random.default_rng(n_obj)
    n_t = rng.integers(0, 1024, size=n_obj)
    n_t[: min(3, n_obj)] = 0
    perm = _perm(dev, n_t)
    _check_dealt(n_t.astype(np.int64), perm, exact=True)


def test_row_order_large_counts_within_bucket(dev):
    rng = np.random.default_rng(11)
    n_t = np.exp(rng.uniform(0.0, np.log(3e9), size=5000)).astype(np.int64)
    n_t[:40] = rng.integers(1000, 1100, size=40)  # both sides of the exact range
    perm = _perm(dev, n_t)
    _check_dealt(n_t, perm, exact=False)


def test_row_order_rows_bands_and_invalid_rows(dev):
    rng = np.random.default_rng(12)
    n_obj = 300
    n_t = rng.integers(5, 900, size=n_obj)
    n_t[:4] = 0  # empty objects: rows that still write fill values
    # 8 (object, band) rows per object in shuffled order, some bands negative
    # and some objects out of range: rows with no work, which come after all
    # others (cost -1 here)
    row_obj = np.repeat(np.arange(n_obj), 8)
    row_band = np.tile(np.arange(8), n_obj)
    sh = rng.permutation(len(row_obj))
    row_obj, row_band = row_obj[sh], row_band[sh]
    row_band[rng.choice(len(row_band), 50, replace=False)] = -1
    row_obj[rng.choice(len(row_obj), 20, replace=False)] = n_obj + 5
    cost = np.where((row_band >= 0) & (row_obj < n_obj), n_t[np.minimum(row_obj, n_obj - 1)], -1)
    perm = _perm(dev, n_t, row_obj=torch.as_tensor(row_obj.astype(np.int32), device=dev),
                 row_band=torch.as_tensor(row_band.astype(np.int32), device=dev))
    _check_dealt(cost.astype(np.int64), perm, exact=True)
    # implicit rows: row r is object r / rows_per_group
    perm = _perm(dev, n_t, rows_per_group=3)
    _check_dealt(np.repeat(n_t, 3).astype(np.int64), perm, exact=True)


def _batch(dev, w, method, **kw):
    off = torch.as_tensor(w.offsets, device=dev)
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    dy = torch.as_tensor(w.dy, device=dev) if method == "generalized" else None
    p = lsp.Periodogram(t, y, w.f_min, w.f_max, 4000, offsets=off, unit=w.unit, method=method,
                        dy=dy, **kw)
    p()
    torch.cuda.synchronize()
    return p


@pytest.mark.parametrize("method", ["standard", "generalized"])
@pytest.mark.parametrize("form,schedule", [(lsp.FORM_FP32P, lsp.SCHED_PERSISTENT),
                                           (lsp.FORM_FP32P, lsp.SCHED_GRID),
                                           (lsp.FORM_FP64, lsp.SCHED_AUTO)])
def test_longest_first_changes_no_result(dev, method, form, schedule):
    w = synth.make_asteroids("asteroids_1k", n_obj=400)
    g = lsp.make_grid(w.f_min, w.f_max, 4000, w.unit)
    o = lsp.make_options(form=form, schedule=schedule, order=lsp.ORDER_LPT)
    d = lsp.describe_launch(w.n_obj, len(w.t), g, o, generalized=method == "generalized")
    assert d["order"] == lsp.ORDER_LPT
    say(f"order {method} form={form} schedule={schedule}: input vs longest first")
    runs = [_batch(dev, w, method, form=form, schedule=schedule, order=od,
                   pgram_dtype=lsp.PGRAM_F64) for od in (lsp.ORDER_INPUT, lsp.ORDER_LPT)]
    assert torch.equal(runs[0].pgram, runs[1].pgram)
    assert np.array_equal(runs[0].peaks(), runs[1].peaks())


def test_longest_first_row_mode_and_graph_replays(dev):
    w = synth.make_asteroids("asteroids_1k", n_obj=300)
    off = torch.as_tensor(w.offsets, device=dev)
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    n_f, band = 5000, 700
    rng = np.random.default_rng(3)
    row_obj = np.repeat(np.arange(w.n_obj), 3).astype(np.int32)
    row_band = rng.integers(-1, (n_f + band - 1) // band, size=len(row_obj)).astype(np.int32)
    res = []
    for od in (lsp.ORDER_INPUT, lsp.ORDER_LPT):
        say(f"row mode order={od}")
        pg = torch.full((w.n_obj, n_f), -1.0, dtype=torch.float32, device=dev)
        r = lsp.Rows(off, t, y, w.f_min, w.f_max, n_f, torch.as_tensor(row_obj, device=dev),
                     torch.as_tensor(row_band, device=dev), band_bins=band, rows_per_group=3,
                     unit=w.unit, pgram=pg, order=od)
        r()
        torch.cuda.synchronize()
        res.append((pg.clone(), r.peaks()))
    assert torch.equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    # a captured longest-first call replays to the eager result
    p = lsp.Periodogram(t, y, w.f_min, w.f_max, 3000, offsets=off, unit=w.unit,
                        form=lsp.FORM_FP32P, order=lsp.ORDER_LPT)
    p()
    torch.cuda.synchronize()
    ref_pg, ref_pk = p.pgram.clone(), p.peaks()
    plan = p.capture()
    for rep in range(3):
        p.pgram.fill_(-1.0)
        _ = (t * 2.0).sum().item()
        torch.cuda.synchronize()
        plan()
        torch.cuda.synchronize()
        assert torch.equal(p.pgram, ref_pg), f"replay {rep}"
        assert np.array_equal(p.peaks(), ref_pk)
    del plan


@pytest.mark.parametrize("form", [lsp.FORM_FP32P, lsp.FORM_FP64])
def test_rows_without_work(dev, form):
    """Row mode whose rows all have no work (every band negative): under
    longest-first order every XCD queue is empty; no bin is written and every
    group's peak is empty, as under input order."""
    w = synth.make_workload("batch_10k", n_obj=40)
    off = torch.as_tensor(w.offsets, device=dev)
    t = torch.as_tensor(w.t, device=dev)
    y = torch.as_tensor(w.y, device=dev)
    row_band = torch.full((w.n_obj * 4,), -1, dtype=torch.int32, device=dev)
    res = []
    for od in (lsp.ORDER_INPUT, lsp.ORDER_LPT):
        say(f"rows without work form={form} order={od}")
        pg = torch.full((w.n_obj, 3000), -1.0, dtype=torch.float32, device=dev)
        r = lsp.Rows(off, t, y, w.f_min, w.f_max, 3000, None, row_band, band_bins=750,
                     rows_per_group=4, form=form, pgram=pg, order=od)
        r()
        torch.cuda.synchronize()
        assert torch.all(pg == -1.0)
        res.append(r.peaks())
    # empty peaks carry NaN frequencies and periods: compare the records' bits
    assert res[0].tobytes() == res[1].tobytes()
    assert np.all(res[1]["index"] == -1)
