"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest

import oracle
from oracle_pins import ALL_PINS


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(ora, pin):
    pin(ora)


def test_degenerate_and_bad_objects(ora):
    """Conventions where the paper is silent: N_t < 2 or no variance -> DEGENERATE
    (power 0, index -1); non-finite input -> NONFINITE; a broken CSR range ->
    BADRANGE (power NaN, index -1)."""
    rng = np.random.default_rng(1)
    good_t = np.sort(rng.uniform(0, 10, 12))
    good_y = rng.normal(size=12)
    series = [
        (good_t, good_y),
        (np.array([1.0]), np.array([2.0])),
        (np.zeros(0), np.zeros(0)),
        (good_t, np.full(12, 0.1)),
        (good_t, np.where(np.arange(12) == 3, np.nan, good_y)),
        (np.where(np.arange(12) == 5, np.inf, good_t), good_y),
    ]
    from paper_2105_04006_amd.synth import pack

    off, t, y = pack(series)
    pg, pk = ora.batch(off, t, y, 0.5, 3.0, 25)
    assert list(pk["status"]) == [oracle.OK, oracle.DEGENERATE, oracle.DEGENERATE,
                                  oracle.DEGENERATE, oracle.NONFINITE, oracle.NONFINITE]
    assert pk["index"][0] >= 0 and all(pk["index"][1:] == -1)
    assert np.all(pg[1:4] == 0.0) and np.all(pk["power"][1:4] == 0.0)
    assert np.all(np.isnan(pg[4:])) and np.all(np.isnan(pk["power"][4:]))
    bad = np.array([0, 5, 3, 12], dtype=np.int64)
    pg, pk = ora.batch(bad, t[:12], y[:12], 0.5, 3.0, 25)
    assert list(pk["status"]) == [oracle.OK, oracle.BADRANGE, oracle.OK]
    assert np.all(np.isnan(pg[1]))


def test_overlapping_ranges_are_independent(ora):
    """A malformed CSR array can make two valid ranges overlap; each object is
    still computed from its own range alone."""
    rng = np.random.default_rng(4)
    t = np.sort(rng.uniform(0, 20, 12))
    y = rng.normal(size=12)
    off = np.array([0, 10, 2, 3, 12], dtype=np.int64)  # objects 0 and 3 overlap
    pg, pk = ora.batch(off, t, y, 0.5, 3.0, 60)
    assert list(pk["status"]) == [oracle.OK, oracle.BADRANGE, oracle.DEGENERATE, oracle.OK]
    for o, (a, b) in ((0, (0, 10)), (3, (3, 12))):
        ps, _ = ora.single(t[a:b], y[a:b], 0.5, 3.0, 60)
        assert np.array_equal(ps, pg[o])


def test_batch_equals_single(ora):
    from paper_2105_04006_amd import synth

    w = synth.make_workload("batch_10k", n_obj=6)
    w_nf = 300
    pg, pk = ora.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, w_nf)
    for o in range(w.n_obj):
        t, y = w.obj(o)
        ps, ks = ora.single(t, y, w.f_min, w.f_max, w_nf)
        assert np.array_equal(ps, pg[o])
        assert ks["index"] == pk["index"][o]
    _, pk2 = ora.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, w_nf, want_pgram=False)
    assert np.array_equal(pk2["index"], pk["index"])
    assert np.array_equal(pk2["power"], pk["power"])


def test_thread_count_does_not_change_results(ora):
    from paper_2105_04006_amd import synth

    t, y, _ = synth.sine_object(200, 77)
    a, ka = ora.single(t, y, 1.0, 12.0, 500, threads=1)
    b, kb = ora.single(t, y, 1.0, 12.0, 500, threads=4)
    assert np.array_equal(a, b) and ka["index"] == kb["index"]


def test_eval_bins_matches_pgram(ora):
    from paper_2105_04006_amd import synth

    w = synth.make_workload("batch_10k", n_obj=4)
    pg, _ = ora.batch(w.offsets, w.t, w.y, w.f_min, w.f_max, 200)
    rng = np.random.default_rng(3)
    obj = rng.integers(0, 4, 30)
    bins = rng.integers(0, 200, 30)
    v = ora.eval_bins(w.offsets, w.t, w.y, w.f_min, w.f_max, 200, obj, bins)
    assert np.array_equal(v, pg[obj, bins])


def test_peak_record(ora):
    """The peak record carries the argmax index, its frequency and the period."""
    from paper_2105_04006_amd import synth

    t, y, f0 = synth.sine_object(256, 5)
    pg, pk = ora.single(t, y, 1.0, 12.0, 1000)
    assert pk["index"] == ora.argmax(pg)
    assert pk["freq"] == ora.grid_freq(1.0, 12.0, 1000, pk["index"])
    assert pk["period"] == pytest.approx(1.0 / pk["freq"], rel=1e-15)
    assert pk["power"] == pg[pk["index"]]
