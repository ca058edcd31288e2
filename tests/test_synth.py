"""Seeded input generator: reproducible, exact sizes, the stated sampling model."""
import numpy as np

from paper_2105_04006_amd import synth


def test_seeds_reproduce_and_prefixes_agree():
    a = synth.make_workload("batch_10k", n_obj=200)
    b = synth.make_workload("batch_10k", n_obj=200)
    c = synth.make_workload("batch_10k", n_obj=50)
    assert np.array_equal(a.t, b.t) and np.array_equal(a.y, b.y)
    assert np.array_equal(a.offsets[:51], c.offsets)
    assert np.array_equal(a.t[: c.n_obs], c.t) and np.array_equal(a.y[: c.n_obs], c.y)
    d = synth.make_workload("batch_10k", n_obj=50, seed=1)
    assert not np.array_equal(c.t, d.t)


def test_sizes_gaps_and_order():
    w = synth.make_workload("batch_10k", n_obj=300)
    nt = w.n_t
    assert nt.min() >= 50 and nt.max() <= 1000 and w.offsets[0] == 0
    assert not synth.in_gap(w.t).any()
    assert w.t.min() >= 0.0 and w.t.max() < 3650.0
    for o in range(w.n_obj):
        assert np.all(np.diff(w.obj(o)[0]) >= 0.0)
    s = synth.make_workload("single_4096")
    assert s.n_obj == 1 and s.n_obs == 4096 and s.n_f == 500_000
    assert (s.f_min, s.f_max) == (0.5, 24.0)


def test_gap_fraction_matches_model():
    """Uniform over [0, 3650) minus the gaps: each allowed day equally likely."""
    w = synth.make_workload("batch_10k", n_obj=2000)
    m = np.mod(w.t, 365.0)
    frac_early = np.mean(m < 120.0)
    assert abs(frac_early - 120.0 / 245.0) < 0.005


def test_lsst_mixture_fractions():
    w = synth.make_workload("lsst_200k", n_obj=20000)
    frac = np.bincount(w.kind, minlength=3) / w.n_obj
    assert abs(frac[0] - 0.6) < 0.015 and abs(frac[1] - 0.3) < 0.015 and abs(frac[2] - 0.1) < 0.01
    assert np.all(np.isnan(w.true_freq[w.kind == synth.KIND_NOISE]))
    assert w.n_t.min() >= 20 and w.n_t.max() <= 500


def test_asteroid_population():
    w = synth.make_workload("asteroids_1k")
    n_t = np.diff(w.offsets)
    assert w.n_obj == 1000 and w.unit == 1 and w.dy is not None
    # log-normal number of observations, clipped to [10, 1500]
    assert n_t.min() >= 10 and n_t.max() <= 1500
    assert 90 <= np.median(n_t) <= 130
    assert 0.1 < np.mean(n_t < 50) < 0.3
    # times sorted within objects, inside three seasonal years
    for a, b in zip(w.offsets[:-1], w.offsets[1:]):
        assert np.all(np.diff(w.t[a:b]) >= 0)
    assert w.t.min() >= 0.0 and w.t.max() < synth.AST_SPAN_DAYS + 1.0
    assert not np.any(synth.in_gap(w.t))
    # survey pairs: a good share of points have a partner 30 minutes earlier
    d = np.concatenate([np.diff(w.t[a:b]) for a, b in zip(w.offsets[:-1], w.offsets[1:])])
    assert np.mean(np.abs(d - 30.0 / 1440.0) < 1e-9) > 0.2
    assert np.all(w.dy > 0)
    # light-curve frequency = twice the rotation frequency, in rad/day
    assert np.allclose(w.true_freq, 2.0 * 2.0 * np.pi * 24.0 / w.p_rot_hours)
    assert w.p_rot_hours.min() >= 2.0 and np.mean(w.p_rot_hours > 300.0) < 0.02
    # the first k objects do not depend on how many are drawn
    v = synth.make_workload("asteroids_1k", n_obj=77)
    n = v.n_obs
    assert np.array_equal(v.t, w.t[:n]) and np.array_equal(v.y, w.y[:n])
    assert np.array_equal(v.dy, w.dy[:n]) and np.array_equal(v.p_rot_hours, w.p_rot_hours[:77])
