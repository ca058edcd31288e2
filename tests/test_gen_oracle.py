"""The oracle's generalized periodogram against its pins, and its batch,
single and spot-check entry points against each other (CPU only)."""
import numpy as np
import pytest

import oracle
from gen_pins import GEN_PINS


@pytest.fixture(scope="module")
def ora():
    return oracle.Oracle()


@pytest.mark.parametrize("pin", GEN_PINS, ids=lambda f: f.__name__)
def test_gen_pin(ora, pin):
    pin(ora)


def _series(seed, sizes):
    rng = np.random.default_rng(seed)
    ts, ys, ds = [], [], []
    for n in sizes:
        t = np.sort(rng.uniform(0.0, 80.0, n))
        ts.append(t)
        ys.append(rng.normal(size=n) + np.sin(2 * np.pi * 0.21 * t))
        ds.append(rng.uniform(0.2, 1.5, n))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return off, np.concatenate(ts), np.concatenate(ys), np.concatenate(ds)


def test_gen_batch_equals_single(ora):
    off, t, y, dy = _series(3, [17, 0, 1, 40, 9])
    pg, pk = ora.gen_batch(off, t, y, dy, 0.05, 1.0, 37)
    for o in range(len(off) - 1):
        a, b = off[o], off[o + 1]
        ps, ks = ora.gen_single(t[a:b], y[a:b], dy[a:b], 0.05, 1.0, 37)
        assert np.array_equal(pg[o], ps, equal_nan=True)
        assert ks["index"] == pk[o]["index"] and ks["status"] == pk[o]["status"]
    assert pk[1]["status"] == oracle.DEGENERATE and pk[2]["status"] == oracle.DEGENERATE


def test_gen_eval_bins_and_threads(ora):
    off, t, y, dy = _series(5, [30, 25, 60])
    pg, _ = ora.gen_batch(off, t, y, None, 0.05, 1.0, 41, threads=1)
    pg4, _ = ora.gen_batch(off, t, y, None, 0.05, 1.0, 41, threads=4)
    assert np.array_equal(pg, pg4)
    obj = np.array([0, 2, 1, 2])
    bins = np.array([0, 40, 7, 13])
    v = ora.gen_eval_bins(off, t, y, None, 0.05, 1.0, 41, obj, bins)
    assert np.array_equal(v, pg[obj, bins])


def test_gen_bad_range(ora):
    off = np.array([0, 5, 3, 10], dtype=np.int64)
    t = np.linspace(0, 9, 10)
    y = np.sin(t)
    pg, pk = ora.gen_batch(off, t, y, None, 0.1, 1.0, 5)
    assert pk[1]["status"] == oracle.BADRANGE and np.all(np.isnan(pg[1]))
    assert pk[0]["status"] == oracle.OK and pk[2]["status"] == oracle.OK
