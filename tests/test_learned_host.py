"""Host-side logic of the learned path (CPU only): band geometry and the
fallback-threshold calibration."""
import numpy as np

from paper_2105_04006_amd import learned, lsp


def test_band_geometry():
    g = learned.BandGeometry(200_000, 64)
    assert g.band_bins == 3125 and g.band_bins * g.n_bands == 200_000
    g = learned.BandGeometry(1000, 64)
    # ceil(1000 / 64) = 16 bins per band: bands 0..62 cover the grid (the last
    # one holds 8 bins) and band 63 is empty, which row mode evaluates as nothing
    assert g.band_bins == 16 and 62 * 16 < 1000 <= 63 * 16


def _peaks(idx, power, status=None):
    p = np.zeros(len(idx), lsp.PEAK_DTYPE)
    p["index"] = idx
    p["power"] = power
    if status is not None:
        p["status"] = status
    return p


def test_calibrate_meets_target_with_fewest_fallbacks():
    rng = np.random.default_rng(0)
    n = 20000
    full = _peaks(rng.integers(0, 10**5, n), rng.uniform(0.2, 1, n))
    mass = rng.uniform(0.5, 1.0, n)
    refined_idx = full["index"].copy()
    # 2% misses, all with low proposal mass; 0.05% misses with high mass
    miss_low = rng.choice(n, 400, replace=False)
    mass[miss_low] = rng.uniform(0.0, 0.3, 400)
    refined_idx[miss_low] += 1000
    rest = np.setdiff1d(np.arange(n), miss_low)
    miss_high = rng.choice(rest, 10, replace=False)
    refined_idx[miss_high] += 5
    refined = _peaks(refined_idx, full["power"])
    mass_min, power_min, n_fb = learned.calibrate(refined, full, mass, target=0.999)
    fb = (mass < mass_min) | (refined["power"] < power_min)
    hit = np.abs(refined["index"] - full["index"]) <= 1
    recovered = np.mean(hit | fb)
    assert recovered >= 0.999
    assert n_fb == int(fb.sum())
    assert np.all(fb[miss_low])               # every low-mass miss falls back
    assert n_fb < 0.1 * n                     # ... without sending everything back


def test_calibrate_ignores_objects_without_peak():
    n = 1000
    full = _peaks(np.arange(n), np.ones(n), status=np.where(np.arange(n) < 10, 1, 0))
    refined = _peaks(np.arange(n), np.ones(n))
    mass = np.ones(n)
    mm, pm, n_fb = learned.calibrate(refined, full, mass)
    assert n_fb == 0


def _calibrate_by_loop(refined, full, mass, target, weights):
    """The threshold search written as the plain double loop."""
    ok = full["status"] == 0
    hit = ok & (np.abs(refined["index"] - full["index"]) <= 1)
    n = int(ok.sum())
    allowed = int(np.floor((1.0 - target) * n))
    pw = np.where(np.isfinite(refined["power"]), refined["power"], -1.0)
    q = np.linspace(0.0, 1.0, 101)
    m_grid = np.unique(np.concatenate([[0.0], np.quantile(mass[ok], q), [2.0]]))
    p_grid = np.unique(np.concatenate([[0.0], np.quantile(pw[ok], q), [2.0]]))
    best = (2.0, 2.0, n + 1, np.inf)
    for mm in m_grid:
        for pm in p_grid:
            fb = ok & ((mass < mm) | (pw < pm) | (refined["index"] < 0))
            miss = int((ok & ~hit & ~fb).sum())
            wt = float(weights[fb].sum())
            if miss <= allowed and wt < best[3]:
                best = (float(mm), float(pm), int(fb.sum()), wt)
    return best


def test_vectorised_calibration_equals_the_loop():
    rng = np.random.default_rng(4)
    n = 3000
    full = _peaks(rng.integers(0, 10**4, n), rng.uniform(0.1, 1, n),
                  status=(rng.random(n) < 0.02).astype(np.int32))
    idx = full["index"].copy()
    miss = rng.random(n) < 0.05
    idx[miss] += rng.integers(2, 50, miss.sum())
    idx[rng.random(n) < 0.01] = -1
    power = np.where(miss, rng.uniform(0.0, 0.6, n), full["power"])
    power[rng.random(n) < 0.01] = np.nan
    refined = _peaks(idx, power)
    mass = np.where(miss, rng.uniform(0, 0.7, n), rng.uniform(0.3, 1.0, n))
    for weights in (np.ones(n), rng.integers(20, 500, n).astype(np.float64)):
        for target in (0.99, 0.999):
            got = learned._calibrate(refined, full, mass, target, weights)
            want = _calibrate_by_loop(refined, full, mass, target, weights)
            assert got[:3] == want[:3] and abs(got[3] - want[3]) < 1e-6


def test_group_peaks_pick_highest_power_then_lowest_bin():
    index = np.array([[5, 9, 2], [7, -1, 3], [-1, -1, -1], [4, 8, 1]])
    power = np.array([[0.5, 0.9, 0.9], [0.2, 0.99, 0.1], [1.0, 1.0, 1.0], [0.3, 0.7, 0.8]])
    kept = np.array([[True, True, True], [True, True, False], [True, True, True],
                     [True, True, False]])
    pk = learned._group_peaks(index, power, kept)
    assert pk["index"].tolist() == [2, 7, -1, 8]   # tie 0.9 -> bin 2; -1 rows never win
    assert pk["power"][0] == 0.9 and np.isnan(pk["power"][2])
