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
