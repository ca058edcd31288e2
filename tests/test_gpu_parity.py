"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Tolerances
  FP64 form : |P_gpu - P_ora| <= 1e-9 * max(P_ora, 1e-3)   (relative 1e-9 on power,
              with an absolute floor where relative error is ill-posed, P -> 0)
  FP32 form : |P_gpu - P_ora| <= 1e-3 (absolute, on the normalised power)
  peaks     : FP64 form: same index as the oracle unless the oracle's powers at the
              two indices tie within the power tolerance; FP32 form: within one bin,
              or a near-tie in the oracle's own periodogram.
"""
import math
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as _oracle  # noqa: E402
from paper_2105_04006_amd import lsp, synth  # noqa: E402

pytestmark = pytest.mark.gpu


class _LoggedOracle:
    """The oracle, announcing each call so a stalled step is named in the log."""

    def __getattr__(self, name):
        fn = getattr(_oracle, name)
        if not callable(fn):
            return fn

        def call(*a, **k):
            say(f"  oracle.{name}")
            out = fn(*a, **k)
            say(f"  oracle.{name} done")
            return out

        return call


oracle = _LoggedOracle()

FP64_RTOL, FP64_FLOOR = 1e-9, 1e-3
FP32_ATOL = 1e-3


_T0 = time.time()


def say(msg):
    print(f"[{time.time() - _T0:8.2f}s] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def cuda(a, dev, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def run_batch(dev, off, t, y, f_min, f_max, n_f, **kw):
    say(f"  gpu lsp_batch n_obj={len(off) - 1} n_obs={len(t)} n_f={n_f} {kw}")
    p = lsp.Periodogram(cuda(t, dev), cuda(y, dev), f_min, f_max, n_f,
                        offsets=cuda(off, dev, torch.int64), **kw)
    p()
    torch.cuda.synchronize()
    pg = p.pgram.double().cpu().numpy() if p.pgram is not None else None
    return pg, p.peaks()


def run_single(dev, t, y, f_min, f_max, n_f, **kw):
    say(f"  gpu lsp_single n_t={len(t)} n_f={n_f} {kw}")
    p = lsp.Periodogram(cuda(t, dev), cuda(y, dev), f_min, f_max, n_f, **kw)
    p()
    torch.cuda.synchronize()
    pg = p.pgram[0].double().cpu().numpy() if p.pgram is not None else None
    return pg, p.peaks()[0]


def assert_fp64_close(gpu, ora, what):
    gpu, ora = np.asarray(gpu), np.asarray(ora)
    both_nan = np.isnan(gpu) & np.isnan(ora)
    err = np.where(both_nan, 0.0, np.abs(gpu - ora))
    tol = FP64_RTOL * np.maximum(np.abs(np.nan_to_num(ora)), FP64_FLOOR)
    bad = ~(err <= tol)
    assert not bad.any(), (f"{what}: {bad.sum()} bins off, worst rel "
                           f"{np.nanmax(err / np.maximum(np.abs(ora), FP64_FLOOR)):.3g}")


def assert_fp32_close(gpu, ora, what, atol=FP32_ATOL):
    gpu, ora = np.asarray(gpu), np.asarray(ora)
    both_nan = np.isnan(gpu) & np.isnan(ora)
    err = np.where(both_nan, 0.0, np.abs(gpu - ora))
    assert np.all(err <= atol), f"{what}: max |dP| = {np.nanmax(err):.3g}"
    return float(np.max(err)) if err.size else 0.0


def peak_ok(ora_row, i_ora, i_gpu, tol, bins=0):
    if i_gpu == i_ora or (bins and abs(int(i_gpu) - int(i_ora)) <= bins):
        return True
    return ora_row[i_gpu] >= ora_row[i_ora] - tol


# ---------------------------------------------------------------- small shapes

def test_single_small_fp64(dev):
    w = synth.make_workload("single_256")
    say(f"single_256 fp64 n_t={w.n_obs} n_f={w.n_f}")
    ora_pg, ora_pk = oracle.single(w.t, w.y, w.f_min, w.f_max, w.n_f)
    pg, pk = run_single(dev, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64,
                        pgram_dtype=lsp.PGRAM_F64)
    assert_fp64_close(pg, ora_pg, "single_256 fp64")
    assert pk["status"] == lsp.OBJ_OK
    assert peak_ok(ora_pg, ora_pk["index"], pk["index"], 1e-9)
    assert pk["freq"] == pytest.approx(oracle.grid_freq(w.f_min, w.f_max, w.n_f, pk["index"]),
                                       rel=1e-15)
    assert pk["period"] == pytest.approx(1.0 / pk["freq"], rel=1e-15)
    assert_fp64_close([pk["power"]], [ora_pg[pk["index"]]], "peak power")


def test_single_small_fp32p(dev):
    w = synth.make_workload("single_256")
    ora_pg, ora_pk = oracle.single(w.t, w.y, w.f_min, w.f_max, w.n_f)
    for rec in (lsp.REC_ROTATION, lsp.REC_CHEBYSHEV):
        for k in (4, 8, 16, 32):
            pg, pk = run_single(dev, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P, k=k,
                                recurrence=rec)
            err = assert_fp32_close(pg, ora_pg, f"single_256 fp32p k={k} rec={rec}")
            say(f"    max |dP| = {err:.3g} (bound {FP32_ATOL})")
            assert peak_ok(ora_pg, ora_pk["index"], pk["index"], 2 * FP32_ATOL, bins=1)


def test_batch_ragged_both_forms(dev):
    w = synth.make_workload("batch_10k", n_obj=40)
    n_f = 2500  # not a multiple of any tile size: ragged tail in every object
    say(f"batch40 n_obs={w.n_obs} n_f={n_f}")
    ora_pg, ora_pk = oracle.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, n_f)
    pg, pk = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, n_f, form=lsp.FORM_FP64,
                       pgram_dtype=lsp.PGRAM_F64)
    assert_fp64_close(pg, ora_pg, "batch fp64")
    for o in range(w.n_obj):
        assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], 1e-9)
    for sched in (lsp.SCHED_GRID, lsp.SCHED_PERSISTENT):
        pg, pk = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, n_f, form=lsp.FORM_FP32P,
                           schedule=sched)
        assert_fp32_close(pg, ora_pg, f"batch fp32p sched={sched}")
        for o in range(w.n_obj):
            assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], 2 * FP32_ATOL, bins=1)


def test_n_f_edges(dev):
    t, y, _ = synth.sine_object(300, 12)
    for n_f in (1, 63, 64, 65, 1023, 4097):
        say(f"n_f edge {n_f}")
        ora_pg, ora_pk = oracle.single(t, y, 1.0, 12.0, n_f)
        pg, pk = run_single(dev, t, y, 1.0, 12.0, n_f, form=lsp.FORM_FP64,
                            pgram_dtype=lsp.PGRAM_F64)
        assert_fp64_close(pg, ora_pg, f"n_f={n_f} fp64")
        assert pk["index"] == ora_pk["index"]
        pg, pk = run_single(dev, t, y, 1.0, 12.0, n_f, form=lsp.FORM_FP32P)
        assert_fp32_close(pg, ora_pg, f"n_f={n_f} fp32p")


# ------------------------------------------------------------------ edge cases

def _edge_series():
    rng = np.random.default_rng(1)
    good_t = np.sort(rng.uniform(0, 10, 12))
    good_y = rng.normal(size=12)
    t2, y2, _ = synth.sine_object(90, 4)
    return [
        (good_t, good_y),                                          # OK
        (np.array([1.0]), np.array([2.0])),                        # N_t = 1
        (np.zeros(0), np.zeros(0)),                                # empty
        (good_t, np.full(12, 0.1)),                                # no variance
        (good_t, np.where(np.arange(12) == 3, np.nan, good_y)),    # NaN magnitude
        (np.where(np.arange(12) == 5, np.inf, good_t), good_y),    # Inf time
        (t2, y2),                                                  # OK
        (np.array([0.3, 1.7]), np.array([1.0, 3.0])),              # N_t = 2: P = 1
        (np.array([0.1, 0.9, 2.3]), np.array([0.5, -1.0, 2.0])),   # N_t = 3
    ]


@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_edge_objects(dev, form):
    off, t, y = synth.pack(_edge_series())
    n_f = 300
    say(f"edge objects form={form}")
    ora_pg, ora_pk = oracle.batch(off, t, y, 0.5, 3.0, n_f)
    pg, pk = run_batch(dev, off, t, y, 0.5, 3.0, n_f, form=form, pgram_dtype=lsp.PGRAM_F64)
    assert list(pk["status"]) == list(ora_pk["status"])
    assert list(pk["index"][ora_pk["index"] < 0]) == list(ora_pk["index"][ora_pk["index"] < 0])
    if form == lsp.FORM_FP64:
        assert_fp64_close(pg, ora_pg, "edge fp64")
    else:
        assert_fp32_close(pg, ora_pg, "edge fp32p")
    ok = ora_pk["status"] == oracle.OK
    deg = ora_pk["status"] == oracle.DEGENERATE
    assert np.all(pk["power"][deg] == 0.0)
    assert np.all(np.isnan(pk["power"][~ok & ~deg]))
    assert np.all(np.isnan(pk["freq"][~ok]))


@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_bad_csr_range(dev, form):
    rng = np.random.default_rng(2)
    t = np.sort(rng.uniform(0, 20, 12))
    y = rng.normal(size=12)
    off = np.array([0, 5, 3, 12], dtype=np.int64)
    ora_pg, ora_pk = oracle.batch(off, t, y, 0.5, 3.0, 100)
    pg, pk = run_batch(dev, off, t, y, 0.5, 3.0, 100, form=form, pgram_dtype=lsp.PGRAM_F64)
    assert list(pk["status"]) == [lsp.OBJ_OK, lsp.OBJ_BADRANGE, lsp.OBJ_OK]
    assert np.all(np.isnan(pg[1]))
    tol_fn = assert_fp64_close if form == lsp.FORM_FP64 else assert_fp32_close
    tol_fn(pg[[0, 2]], ora_pg[[0, 2]], "bad-range neighbours")


@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_degenerate_frequencies_even_sampling(dev, form):
    """f = 0 and the Nyquist frequency of evenly sampled data make one shifted
    regressor vanish; the FP32 form must hand those bins to its FP64 fix-up.
    The 33 bins form a single tile, which holds those ill-conditioned bins, so
    the fix-up recomputes all of it in FP64 and stores each value rounded to
    FP32 (the FP32 form's output precision): the FP32 form is held to the FP64
    bound plus half an FP32 ulp, 1e-9 max(P, 1e-3) + 2^-24 P.  The bins' sum is
    1 (the sum rule pinned on the oracle), so it is within 32 (1e-9 + 2^-24)
    < 1e-6 of 1."""
    rng = np.random.default_rng(5)
    n = 64
    t = np.arange(n, dtype=np.float64)
    y = rng.normal(size=n)
    n_f = n // 2 + 1  # f_i = i / N, i = 0 .. N/2: includes 0 and Nyquist
    say(f"even sampling form={form}")
    ora_pg, _ = oracle.single(t, y, 0.0, (n_f) / n, n_f)
    pg, pk = run_single(dev, t, y, 0.0, n_f / n, n_f, form=form, pgram_dtype=lsp.PGRAM_F64)
    if form == lsp.FORM_FP64:
        assert_fp64_close(pg, ora_pg, "even sampling fp64")
    else:
        err = np.abs(pg - ora_pg)
        bound = FP64_RTOL * np.maximum(ora_pg, FP64_FLOOR) + 2.0 ** -24 * ora_pg
        assert np.all(err <= bound), f"even sampling fp32p: worst {np.max(err / bound):.3g} x bound"
    assert abs(pg[0]) < 1e-12
    assert np.sum(pg[1:]) == pytest.approx(1.0, abs=1e-6)  # Nyquist sum rule


@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_tiny_series(dev, form):
    rng = np.random.default_rng(9)
    series = [(np.sort(rng.uniform(0, 50, n)), rng.normal(size=n)) for n in (2, 2, 3, 3, 4, 5)]
    off, t, y = synth.pack(series)
    ora_pg, ora_pk = oracle.batch(off, t, y, 0.05, 5.0, 2000)
    pg, pk = run_batch(dev, off, t, y, 0.05, 5.0, 2000, form=form, pgram_dtype=lsp.PGRAM_F64)
    if form == lsp.FORM_FP64:
        assert_fp64_close(pg, ora_pg, "tiny fp64")
    else:
        assert_fp32_close(pg, ora_pg, "tiny fp32p")
    # two points fit any sinusoid exactly: P = 1 at every bin, within the bound of the form
    assert np.max(np.abs(pg[:2] - 1.0)) <= (1e-9 if form == lsp.FORM_FP64 else FP32_ATOL)


# --------------------------------------------------------------------- options

@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_options(dev, form):
    t, y, _ = synth.sine_object(200, 21)
    y = y + 3.0
    chk = assert_fp64_close if form == lsp.FORM_FP64 else assert_fp32_close
    say(f"options form={form}")
    ora_pg, _ = oracle.single(t, y, 1.0, 12.0, 3000, normalize=False)
    pg, _ = run_single(dev, t, y, 1.0, 12.0, 3000, form=form, normalize=False,
                       pgram_dtype=lsp.PGRAM_F64)
    if form == lsp.FORM_FP64:
        chk(pg, ora_pg, "P_LS")
    else:  # unnormalised power scales with S_yy: compare relative to its scale
        assert_fp32_close(pg / ora_pg.max(), ora_pg / ora_pg.max(), "P_LS (scaled)")
    ora_pg, _ = oracle.single(t, y - y.mean(), 1.0, 12.0, 3000, subtract_mean=False)
    pg, _ = run_single(dev, t, y - y.mean(), 1.0, 12.0, 3000, form=form, subtract_mean=False,
                       pgram_dtype=lsp.PGRAM_F64)
    chk(pg, ora_pg, "y as given")
    ora_pg, ora_pk = oracle.single(t, y, 2 * math.pi, 24 * math.pi, 3000, unit=oracle.ANGULAR)
    pg, pk = run_single(dev, t, y, 2 * math.pi, 24 * math.pi, 3000, form=form, unit=lsp.ANGULAR,
                        pgram_dtype=lsp.PGRAM_F64)
    chk(pg, ora_pg, "angular unit")
    assert pk["period"] == pytest.approx(2 * math.pi / pk["freq"], rel=1e-15)
    pg32, _ = run_single(dev, t, y, 1.0, 12.0, 3000, form=form, pgram_dtype=lsp.PGRAM_F32)
    pg64, _ = run_single(dev, t, y, 1.0, 12.0, 3000, form=form, pgram_dtype=lsp.PGRAM_F64)
    assert np.array_equal(pg32, pg64.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("form", [lsp.FORM_FP64, lsp.FORM_FP32P])
def test_peaks_only_and_determinism(dev, form):
    w = synth.make_workload("batch_10k", n_obj=64)
    args = (dev, w.offsets, w.t, w.y, w.f_min, w.f_max, 5000)
    pg1, pk1 = run_batch(*args, form=form)
    pg2, pk2 = run_batch(*args, form=form)
    _, pk3 = run_batch(*args, form=form, pgram=False)
    assert np.array_equal(pg1, pg2)
    assert np.array_equal(pk1, pk2)
    assert np.array_equal(pk1, pk3)


def test_batch_row_equals_single(dev):
    # Same launch shape on both sides (frequencies per lane, no splitting of
    # the observations): a batch row is then bit-identical to the single call.
    w = synth.make_workload("batch_10k", n_obj=5)
    for form, k in ((lsp.FORM_FP64, 2), (lsp.FORM_FP32P, 16)):
        kw = dict(form=form, t_split=1, k=k)
        if form == lsp.FORM_FP32P:
            kw["wave_split"] = lsp.WSPLIT_OFF
        pgb, pkb = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, 4000, **kw)
        for o in range(w.n_obj):
            t, y = w.obj(o)
            pgs, pks = run_single(dev, t, y, w.f_min, w.f_max, 4000, **kw)
            assert np.array_equal(pgs, pgb[o])
            assert pks["index"] == pkb["index"][o]


def test_fp32p_observation_split(dev):
    t, y, _ = synth.sine_object(3000, 33)
    ora_pg, ora_pk = oracle.single(t, y, 1.0, 12.0, 5000)
    for split in (1, 2, 5, 16):
        say(f"fp32p t_split={split}")
        pg, pk = run_single(dev, t, y, 1.0, 12.0, 5000, form=lsp.FORM_FP32P, t_split=split)
        assert_fp32_close(pg, ora_pg, f"t_split={split}")
        assert peak_ok(ora_pg, ora_pk["index"], pk["index"], 2 * FP32_ATOL, bins=1)


def test_fp32p_wave_split(dev):
    """The in-workgroup wave split (the waves of a workgroup share bins and
    take every W-th observation, sums added in LDS as a fixed tree): 2, 4 and
    8 waves, with and without the observation split, single object and batch,
    against the oracle."""
    t, y, _ = synth.sine_object(3000, 34)
    ora_pg, ora_pk = oracle.single(t, y, 1.0, 12.0, 5000)
    for waves, k, split in ((2, 16, 1), (4, 16, 1), (8, 16, 1), (8, 12, 1), (8, 8, 3), (4, 10, 2)):
        say(f"fp32p wave split: waves={waves} k={k} t_split={split}")
        pg, pk = run_single(dev, t, y, 1.0, 12.0, 5000, form=lsp.FORM_FP32P, waves=waves, k=k,
                            t_split=split, wave_split=lsp.WSPLIT_ON)
        assert_fp32_close(pg, ora_pg, f"waves={waves} k={k} split={split}")
        assert peak_ok(ora_pg, ora_pk["index"], pk["index"], 2 * FP32_ATOL, bins=1)
    w = synth.make_workload("batch_10k", n_obj=24)
    ora_pg, ora_pk = oracle.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, 3000)
    pg, pk = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, 3000, form=lsp.FORM_FP32P,
                       waves=8, k=16, wave_split=lsp.WSPLIT_ON)
    assert_fp32_close(pg, ora_pg, "batch, 8 waves")
    for o in range(w.n_obj):
        assert peak_ok(ora_pg[o], ora_pk["index"][o], pk["index"][o], 2 * FP32_ATOL, bins=1)


# -------------------------------------------------------------- full-size cases

def test_full_single_4096(dev):
    """The 4,096-point, 500,000-bin object at full size: the oracle is evaluated
    at 3,000 sampled bins plus the GPU's 64 strongest bins."""
    w = synth.make_workload("single_4096")
    say(f"single_4096 full n_f={w.n_f}")
    pg64, pk64 = run_single(dev, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64,
                            pgram_dtype=lsp.PGRAM_F64)
    pg32, pk32 = run_single(dev, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P,
                            recurrence=lsp.REC_ROTATION)
    pgc, pkc = run_single(dev, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P,
                          recurrence=lsp.REC_CHEBYSHEV)
    say(f"    rotation max |dP| vs fp64 {np.max(np.abs(pg32 - pg64)):.3g}, "
        f"chebyshev {np.max(np.abs(pgc - pg64)):.3g}")
    assert_fp32_close(pgc, pg64, "single_4096 chebyshev vs fp64 (all bins)")
    assert_fp32_close(pg32, pg64, "single_4096 rotation vs fp64 (all bins)")
    assert abs(int(pkc["index"]) - int(pk64["index"])) <= 1
    rng = np.random.default_rng(0)
    top = np.argsort(pg64)[-64:]
    bins = np.unique(np.concatenate([rng.integers(0, w.n_f, 3000), top,
                                     [0, w.n_f - 1, pk32["index"]]]))
    off = np.array([0, w.n_obs], dtype=np.int64)
    ora = oracle.eval_bins(off, w.t, w.y, w.f_min, w.f_max, w.n_f, np.zeros(len(bins), np.int64),
                           bins)
    assert_fp64_close(pg64[bins], ora, "single_4096 fp64 sampled")
    assert_fp32_close(pg32[bins], ora, "single_4096 fp32p sampled")
    assert_fp32_close(pg32, pg64, "single_4096 fp32p vs fp64 (all bins)")
    assert np.all((pg64 >= 0) & (pg64 <= 1 + 1e-12))
    ora_top = ora[np.searchsorted(bins, top)]
    assert top[np.argmax(ora_top)] == pk64["index"] or \
        pg64[pk64["index"]] - ora_top.max() <= 1e-9
    assert abs(int(pk32["index"]) - int(pk64["index"])) <= 1


def test_full_batch_10k_peaks(dev):
    """10,000 objects x 100,000 bins, peaks only: the FP32 form agrees with the
    FP64 GPU form on >= 99.9% of peaks (within one bin); both agree with the
    oracle on a seeded subset, whole periodograms for 8 objects."""
    w = synth.make_workload("batch_10k")
    say(f"batch_10k full n_obj={w.n_obj} n_obs={w.n_obs} n_f={w.n_f}")
    _, pk64 = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP64,
                        pgram=False)
    _, pk32 = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P,
                        pgram=False, schedule=lsp.SCHED_PERSISTENT, recurrence=lsp.REC_ROTATION)
    assert np.all(pk64["status"] == 0) and np.all(pk32["status"] == 0)
    agree = np.abs(pk32["index"] - pk64["index"]) <= 1
    assert agree.mean() >= 0.999, f"peak agreement {agree.mean():.4%}"
    assert np.all(np.abs(pk32["power"] - pk64["power"]) <= FP32_ATOL)
    _, pkc = run_batch(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, w.n_f, form=lsp.FORM_FP32P,
                       pgram=False, recurrence=lsp.REC_CHEBYSHEV)
    agree_c = np.abs(pkc["index"] - pk64["index"]) <= 1
    say(f"    peak agreement rotation {agree.mean():.5f} chebyshev {agree_c.mean():.5f}; max dP "
        f"{np.max(np.abs(pk32['power'] - pk64['power'])):.3g} / "
        f"{np.max(np.abs(pkc['power'] - pk64['power'])):.3g}")
    assert agree_c.mean() >= 0.999
    assert np.all(np.abs(pkc["power"] - pk64["power"]) <= FP32_ATOL)
    sub = w.subset(8)
    ora_pg, ora_pk = oracle.batch(sub.offsets, sub.t, sub.y, w.f_min, w.f_max, w.n_f,
                                  want_pgram=True)
    for o in range(8):
        assert peak_ok(ora_pg[o], ora_pk["index"][o], pk64["index"][o], 1e-9)
        assert_fp64_close([pk64["power"][o]], [ora_pg[o][pk64["index"][o]]], "peak power fp64")
        assert peak_ok(ora_pg[o], ora_pk["index"][o], pk32["index"][o], 2 * FP32_ATOL, bins=1)


def test_single_wide_grid_statuses(dev):
    """Objects that take the single-object default of eight waves sharing each
    tile (4,096 points, N_f = 5e5), but have no periodogram to compute: a NaN
    magnitude (NONFINITE: every bin NaN, no peak) and a constant series
    (DEGENERATE: every bin 0, no peak), written by the tile's owning wave;
    then a series whose sums the eight waves do add, checked on sampled bins
    against the oracle."""
    t, y, _ = synth.sine_object(4096, 77)
    n_f = 500_000
    d = lsp.describe_launch(1, len(t), lsp.make_grid(0.5, 24.0, n_f),
                            lsp.make_options(form=lsp.FORM_FP32P))
    assert (d["waves_per_wg"], d["wave_split"], d["t_split"]) == (8, lsp.WSPLIT_ON, 1)
    y_nan = y.copy()
    y_nan[1234] = np.nan
    for yy, status, fill in ((y_nan, lsp.OBJ_NONFINITE, np.nan),
                             (np.full_like(y, 0.25), lsp.OBJ_DEGENERATE, 0.0)):
        pg, pk = run_single(dev, t, yy, 0.5, 24.0, n_f, form=lsp.FORM_FP32P)
        assert pk["status"] == status and pk["index"] == -1
        if np.isnan(fill):
            assert np.all(np.isnan(pg))
        else:
            assert np.all(pg == fill)
    pg, pk = run_single(dev, t, y, 0.5, 24.0, n_f, form=lsp.FORM_FP32P)
    bins = np.unique(np.concatenate([np.arange(3, n_f, 4999), [pk["index"]]]))
    ora = oracle.eval_bins(np.array([0, len(t)], dtype=np.int64), t, y, 0.5, 24.0, n_f,
                           np.zeros(len(bins), np.int64), bins)
    assert_fp32_close(pg[bins], ora, "eight-wave single object, sampled bins")


def test_single_wide_grid_fixup_tiles(dev):
    """Evenly sampled 4,096-point object on [0, 2) c/d with 5e5 bins, run by
    the single-object default of eight waves sharing each 1,024-bin tile: f = 0
    and 1 (every phase an integer) and the Nyquist frequency 0.5 and 1.5 make
    a shifted regressor vanish, so the tiles holding those bins must be the
    ones the FP64 fix-up recomputes.  Those tiles match the FP64 form to its
    bound plus half an FP32 ulp (the fix-up stores FP32); every bin is within
    the FP32 bound of it."""
    rng = np.random.default_rng(13)
    n, n_f = 4096, 500_000
    t = np.arange(n, dtype=np.float64)
    y = rng.normal(size=n)
    d = lsp.describe_launch(1, n, lsp.make_grid(0.0, 2.0, n_f),
                            lsp.make_options(form=lsp.FORM_FP32P))
    assert (d["waves_per_wg"], d["wave_split"], d["tile_freqs"]) == (8, lsp.WSPLIT_ON, 1024)
    pg64, _ = run_single(dev, t, y, 0.0, 2.0, n_f, form=lsp.FORM_FP64, pgram_dtype=lsp.PGRAM_F64)
    pg32, _ = run_single(dev, t, y, 0.0, 2.0, n_f, form=lsp.FORM_FP32P, pgram_dtype=lsp.PGRAM_F64)
    assert_fp32_close(pg32, pg64, "even sampling, wide grid")
    ill = np.array([0, n_f // 4, n_f // 2, 3 * n_f // 4])  # f = 0, 0.5, 1, 1.5
    for i in ill:
        lo = (i // 1024) * 1024
        a, b = pg32[lo:lo + 1024], pg64[lo:lo + 1024]
        bound = 2.0 * FP64_RTOL * np.maximum(b, FP64_FLOOR) + 2.0 ** -24 * b
        assert np.all(np.abs(a - b) <= bound), f"tile of bin {i} not recomputed in FP64"
    assert pg32[0] < 1e-12 and pg64[0] < 1e-12
