"""Pins of the band-proposal feature reference (CPU only).

Each check rests on something other than the reference's own code: exact
values of constructed series, closed forms, and invariances of the
periodogram.
"""
import numpy as np
import pytest

import oracle
from oracle import features_ref as fr


def test_season_split():
    t = np.array([0.0, 1.0, 2.0, 70.0, 71.0, 200.0, 261.0, 262.0])
    assert fr.seasons(t, 60.0) == [(0, 3), (3, 5), (5, 6), (6, 8)]
    assert fr.seasons(t, 1e9) == [(0, 8)]
    assert fr.seasons(np.zeros(0)) == []
    # a gap of exactly `gap` does not start a season
    assert fr.seasons(np.array([0.0, 60.0, 120.5]), 60.0) == [(0, 2), (2, 3)]


def _even_season(n, dt, f0, t_start=0.0, phase=0.3):
    t = t_start + dt * np.arange(n)
    return t, np.sin(2 * np.pi * f0 * (t - t_start) + phase)


def test_coarse_peak_of_even_sinusoid_is_one():
    # n = 64 points at dt = 0.05: f = k / (n dt) = k * 0.3125 and the Nyquist
    # frequency is 10.  Grid [0, 10) with 8,192 bins has df = 10 / 8192, so
    # f = 0.3125 k is bin 256 k.  At a DFT frequency the sample mean of the
    # sinusoid is exactly zero and sum exp(2 i w t) = 0, so the normalised
    # power is exactly 1 there (the grid stops below the Nyquist frequency,
    # so no alias ties with it).
    n, dt, k = 64, 0.05, 9
    f0 = k / (n * dt)
    t, y = _even_season(n, dt, f0)
    c = fr.coarse(t, y, 0.0, 10.0)
    q = (256 * k) // fr.POOL
    assert c[q] == pytest.approx(1.0, abs=1e-12)
    assert int(np.argmax(c)) == q
    assert np.all(c <= 1.0 + 1e-12) and np.all(c >= 0.0)


def test_coarse_average_over_seasons_and_min_obs():
    n, dt, k = 64, 0.05, 9
    f0 = k / (n * dt)
    t1, y1 = _even_season(n, dt, f0)
    one = fr.coarse(t1, y1, 0.0, 40.0)
    # a second copy 500 units later is its own season with the same periodogram
    # (time-shift invariance), so the season average is unchanged
    t2, y2 = _even_season(n, dt, f0, t_start=500.0)
    two = fr.coarse(np.concatenate([t1, t2]), np.concatenate([y1, y2]), 0.0, 40.0)
    assert np.allclose(two, one, atol=1e-9)
    # a short trailing season (fewer than 8 points) is dropped; its values
    # average to zero, like the first season's, so the object mean is unchanged
    t3 = np.array([900.0, 901.0, 902.5])
    y3 = np.array([1.0, -2.0, 1.0])
    three = fr.coarse(np.concatenate([t1, t3]), np.concatenate([y1, y3]), 0.0, 40.0)
    assert np.allclose(three, one, rtol=0, atol=1e-12)
    # with no group of 8 points the coarse part is zero
    assert np.array_equal(fr.coarse(t3, y3, 0.0, 40.0), np.zeros(fr.COARSE))


def test_short_seasons_merge_into_groups():
    # seasons of 5, 5 and 12 points: the first two form one group of 10, the
    # third is a group of its own
    rng = np.random.default_rng(8)
    ta = np.sort(rng.uniform(0, 30, 5))
    tb = np.sort(rng.uniform(200, 230, 5))
    tc = np.sort(rng.uniform(400, 440, 12))
    t = np.concatenate([ta, tb, tc])
    y = rng.normal(size=len(t))
    assert fr.seasons(t) == [(0, 5), (5, 10), (10, 22)]
    assert fr.season_groups(t) == [(0, 10), (10, 22)]
    yc = y - y.mean()
    pg1, _ = oracle.single(t[:10], yc[:10], 1.0, 5.0, fr.COARSE_BINS, subtract_mean=False)
    pg2, _ = oracle.single(t[10:], yc[10:], 1.0, 5.0, fr.COARSE_BINS, subtract_mean=False)
    want = (pg1.reshape(-1, 8).max(1) + pg2.reshape(-1, 8).max(1)) / 2
    assert np.allclose(fr.coarse(t, y, 1.0, 5.0), want, rtol=0, atol=1e-15)
    # a short season at the end joins nothing and is dropped
    assert fr.season_groups(np.concatenate([t, [700.0, 701.0]])) == [(0, 10), (10, 22)]


def test_coarse_pooling_matches_per_bin_maxima():
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0, 50, 40))
    y = rng.normal(size=40)
    # one group: its mean is the object's mean, so this is the plain periodogram
    pg, _ = oracle.single(t, y, 1.0, 9.0, fr.COARSE_BINS)
    c = fr.coarse(t, y, 1.0, 9.0)
    for q in (0, 1, 511, 1023):
        assert c[q] == max(pg[8 * q:8 * q + 8])


def test_window_closed_forms():
    # evenly sampled, dt = 1 / f_p for probe p = 40: every phase is a whole
    # number of cycles, so the spectral window there is exactly 1
    p = 40
    dt = 1.0 / fr.PROBE_FREQS[p]
    n = 20
    t = dt * np.arange(n)
    y = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)  # two-point distribution
    w = fr.window(t, y, gap=1e9)
    assert w[11 + p] == pytest.approx(1.0, abs=1e-9)
    assert w[0] == pytest.approx(np.log10(20))
    assert w[1] == pytest.approx(np.log10(19 * dt))
    assert w[2] == 1 and w[3] == 1 and w[6] == 1.0
    assert w[4] == pytest.approx(np.log10(dt))
    assert w[5] == pytest.approx(0.0, abs=1e-12)
    assert w[7] == pytest.approx(0.0, abs=1e-12)      # sigma = 1
    assert w[8] == pytest.approx(0.0, abs=1e-12)      # symmetric
    assert w[9] == pytest.approx(-2.0, abs=1e-12)     # two-point: kurtosis 1
    assert w[10] == pytest.approx(1.0, abs=1e-12)
    # at a frequency that is a multiple of 1 / (n dt) (not of 1 / dt) the
    # window vanishes: probe in the middle of the range for a tailored dt
    f = fr.PROBE_FREQS[30]
    t2 = np.arange(n) / (f * n) * 3.0  # f = 3 / (n dt)... choose dt so f n dt = 3
    w2 = fr.window(t2, y, gap=1e9)
    assert w2[11 + 30] == pytest.approx(0.0, abs=1e-20)


def test_window_spacing_and_seasons():
    t = np.array([0.0, 1.0, 3.0, 100.0, 110.0])
    y = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    w = fr.window(t, y, gap=60.0, min_obs=3)
    assert w[2] == 2 and w[3] == 1
    within = np.array([1.0, 2.0, 10.0])
    assert w[4] == pytest.approx(np.log10(within.mean()))
    assert w[5] == pytest.approx(np.log10(within).std())
    assert w[6] == pytest.approx(3 / 5)


def test_bad_objects_have_zero_features():
    rng = np.random.default_rng(0)
    good_t = np.sort(rng.uniform(0, 30, 30))
    series = [(good_t, rng.normal(size=30)), (np.array([1.0]), np.array([2.0])),
              (good_t, np.full(30, 4.0)), (good_t, np.where(np.arange(30) == 2, np.nan, 1.0))]
    n_t = [len(s[0]) for s in series]
    off = np.concatenate([[0], np.cumsum(n_t)])
    t = np.concatenate([s[0] for s in series])
    y = np.concatenate([s[1] for s in series])
    f = fr.features(off, t, y, 1.0, 5.0)
    assert f.shape == (4, fr.DIM)
    assert np.any(f[0] != 0)
    assert np.all(f[1:] == 0)


def test_probe_frequencies_span_and_spacing():
    f = fr.PROBE_FREQS
    assert len(f) == fr.N_PROBES == fr.WINDOW - 11
    assert f[0] == pytest.approx(1e-3, rel=1e-12) and f[-1] == pytest.approx(30.0, rel=1e-12)
    r = f[1:] / f[:-1]
    assert np.allclose(r, r[0], rtol=1e-12)
