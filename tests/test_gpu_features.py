"""Band-proposal features (lsp_features) vs the FP64 feature reference (needs an MI355X).

Tolerances
  coarse part [0, 1024): |d| <= 1e-3, the FP32 form's bound on the normalised
                         power (max-pooling and averaging over groups are
                         1-Lipschitz in the max norm, so they do not enlarge it).
                         As in the main kernel, bins FP32 cannot resolve (N -
                         |sum exp(2iwt)| <= N/32, frequent in groups of 3-7
                         points) are recomputed in FP64, so the bound holds for
                         every group size.
  window part [1024, 1088): FP64 statistics and FP32 sin/cos of FP64-reduced
                         phases, stored as FP32: |d| <= 1e-6 * max(1, |ref|)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import features_ref  # noqa: E402
from paper_2105_04006_amd import lsp, synth  # noqa: E402
from test_gpu_parity import cuda, dev, say  # noqa: E402,F401

pytestmark = pytest.mark.gpu

COARSE_ATOL = 1e-3
WINDOW_RTOL = 1e-6


def gpu_features(dev, off, t, y, f_min, f_max, unit=lsp.CYCLES, **kw):
    say(f"  gpu lsp_features n_obj={len(off) - 1} n_obs={len(t)} {kw}")
    f = lsp.Features(cuda(off, dev, torch.int64), cuda(t, dev), cuda(y, dev), f_min, f_max,
                     unit=unit, **kw)
    out = f()
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def assert_features_close(got, ref, what, coarse_atol=COARSE_ATOL):
    c = np.abs(got[:, :lsp.FEAT_COARSE] - ref[:, :lsp.FEAT_COARSE])
    assert np.all(c <= coarse_atol), f"{what}: coarse max |d| = {c.max():.3g}"
    wg, wr = got[:, lsp.FEAT_COARSE:], ref[:, lsp.FEAT_COARSE:]
    err = np.abs(wg - wr) / np.maximum(1.0, np.abs(wr))
    bad = np.argwhere(~(err <= WINDOW_RTOL))
    assert len(bad) == 0, f"{what}: window features off at {bad[:5].tolist()}, " \
                          f"got {wg[tuple(bad[0])]} want {wr[tuple(bad[0])]}"
    say(f"    {what}: coarse max |d| {c.max():.3g}, window max rel {err.max():.3g}")


def test_features_learned_workload(dev):
    w = synth.make_workload("learned_100k", n_obj=48)
    ref = features_ref.features(w.offsets, w.t, w.y, w.f_min, w.f_max)
    got = gpu_features(dev, w.offsets, w.t, w.y, w.f_min, w.f_max)
    assert_features_close(got, ref, "learned_100k[:48]")
    # the coarse part carries the signal: its pooled argmax sits near the true
    # frequency for most objects
    df = (w.f_max - w.f_min) / lsp.FEAT_COARSE
    q_true = np.floor((w.true_freq - w.f_min) / df)
    hit = np.abs(np.argmax(got[:, :lsp.FEAT_COARSE], axis=1) - q_true) <= 1
    say(f"    coarse argmax within one pooled bin of the truth: {hit.mean():.2f}")


def test_features_edge_objects_and_options(dev):
    rng = np.random.default_rng(4)
    t_ok, y_ok, _ = synth.sine_object(120, 9)
    one_season = np.sort(rng.uniform(0, 50, 40))
    series = [
        (t_ok, y_ok),
        (np.zeros(0), np.zeros(0)),                                # empty
        (np.array([3.0]), np.array([1.0])),                        # N_t = 1
        (t_ok, np.full(len(t_ok), 0.7)),                           # no variance
        (t_ok, np.where(np.arange(len(t_ok)) == 7, np.nan, y_ok)),  # NaN
        (one_season, np.sin(2 * np.pi * 3.3 * one_season)),        # one season
        (np.concatenate([one_season, 400 + one_season[:5]]),       # + a short season
         np.sin(2 * np.pi * 3.3 * np.concatenate([one_season, 400 + one_season[:5]]))),
        (np.array([0.0, 100.0, 200.0, 300.0, 400.0]), rng.normal(size=5)),  # no qualifying season
    ]
    off, t, y = synth.pack(series)
    for gap, min_obs in ((60.0, 8), (10.0, 3), (1e9, 8)):
        ref = features_ref.features(off, t, y, 1.0, 12.0, gap=gap, min_obs=min_obs)
        got = gpu_features(dev, off, t, y, 1.0, 12.0, season_gap=gap, min_season_obs=min_obs)
        assert_features_close(got, ref, f"edge objects gap={gap} min_obs={min_obs}")
        assert np.all(got[1:5] == 0.0)


def test_features_small_groups(dev):
    """Groups of 3 and 4 observations, whose shifted denominators often come
    close to 0, on the learned_100k population: the FP64 recompute of
    unresolvable bins keeps every coarse value within 1e-3."""
    w = synth.make_workload("learned_100k", n_obj=24)
    for min_obs in (3, 4):
        ref = features_ref.features(w.offsets, w.t, w.y, w.f_min, w.f_max, gap=10.0,
                                    min_obs=min_obs)
        got = gpu_features(dev, w.offsets, w.t, w.y, w.f_min, w.f_max, season_gap=10.0,
                           min_season_obs=min_obs)
        assert_features_close(got, ref, f"learned_100k[:24] gap=10 min_obs={min_obs}")


def test_features_angular_unit(dev):
    w = synth.make_workload("learned_100k", n_obj=12)
    f_min, f_max = 2 * np.pi * w.f_min, 2 * np.pi * w.f_max
    ref = features_ref.features(w.offsets, w.t, w.y, f_min, f_max, unit=1)
    got = gpu_features(dev, w.offsets, w.t, w.y, f_min, f_max, unit=lsp.ANGULAR)
    assert_features_close(got, ref, "angular")


def test_features_long_series(dev):
    # more than one staging tile per object, seasons spanning tile boundaries
    w = synth.make_workload("single_4096")
    off = np.array([0, 700, 2300, w.n_obs], dtype=np.int64)
    ref = features_ref.features(off, w.t, w.y, w.f_min, w.f_max)
    got = gpu_features(dev, off, w.t, w.y, w.f_min, w.f_max)
    assert_features_close(got, ref, "long series")


def test_features_season_boundaries_at_word_and_tile_edges(dev):
    """Season starts on the edges of the kernel's bookkeeping: a staged tile
    holds 256 observations and its new-season flags are kept as 64-bit words,
    so starts at observations 63, 64, 65 (word edge, one-point seasons), 128,
    256 and 257 (tile edge), 511, 512 and the last observation alone, plus the
    second observation, must group exactly as the reference does."""
    rng = np.random.default_rng(21)
    n = 600
    starts = [1, 63, 64, 65, 127, 128, 256, 257, 300, 511, 512, n - 1]
    dt = rng.uniform(0.2, 0.6, size=n - 1)
    dt[np.array(starts) - 1] += 100.0
    t = np.concatenate([[0.0], np.cumsum(dt)])
    y = np.sin(2 * np.pi * 1.7 * t) + 0.1 * rng.standard_normal(n)
    off = np.array([0, n], dtype=np.int64)
    for min_obs in (2, 8, 70):
        ref = features_ref.features(off, t, y, 1.0, 12.0, gap=60.0, min_obs=min_obs)
        got = gpu_features(dev, off, t, y, 1.0, 12.0, season_gap=60.0, min_season_obs=min_obs)
        assert_features_close(got, ref, f"boundaries min_obs={min_obs}")
