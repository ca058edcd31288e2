"""Plain FP64 reference of the band-proposal features (test infrastructure only).

TEST INFRASTRUCTURE ONLY; shares no code with the GPU path.

The paper evaluates every trial frequency of every object.  The learned path
instead proposes a few frequency bands per object from cheap features and
evaluates only those.  The features of one object are 1,088 numbers:

Coarse part (1,024 values).  The series is cut into seasons: a new season
starts at every observation that follows the previous one by more than
``gap`` time units (observations are taken in the order given, which is time
order for sorted input).  Consecutive seasons are grouped: a group ends at the
first season boundary reached once it holds at least ``min_obs``
observations, so sparse seasons merge with their neighbours; a trailing group
with fewer observations is dropped.  Each group gets its own Lomb-Scargle
periodogram -- exactly the normalised power of Section 2 (Eq. 1 for tau, Eq. 2
for the power) of the object's centred magnitudes y - ybar (ybar the mean
over the whole object; the group's own mean is not removed again) -- on the
half-open grid of 8,192 bins over [f_min, f_max).  Bins are max-pooled in runs of 8, giving 1,024 values,
and the pooled values are averaged over the groups (all zero if there is
none).  A group spans far less time than the whole baseline, so its peaks are
wide enough to be resolved by 8,192 bins, and averaging over groups
reinforces a period that persists.

Window part (64 values).  Sampling and magnitude statistics of the whole
series: w0 = log10 N_t; w1 = log10 max(T, 1e-3) with T the time span; w2 =
number of seasons; w3 = number of seasons with >= min_obs observations; w4 =
log10 max(mean spacing, 1e-6) over consecutive observations within a season;
w5 = standard deviation of log10 max(spacing, 1e-6) over the same pairs; w6 =
fraction of observations in qualifying seasons; w7 = log10 of the standard
deviation sigma of y; w8 = skewness, w9 = excess kurtosis, w10 = max |y - ybar|
/ sigma; w11..w63 = spectral window |sum_j exp(2 pi i f_p t_j)|^2 / N_t^2 at
the 53 probe frequencies f_p = 10^(-3 + p (log10 30 + 3) / 52), in cycles per
time unit whatever the grid's unit.  Spacing features are 0 when there is no
within-season pair; moments w8..w10 are 0 when sigma is 0.

An object whose periodogram status is not OK (fewer than two observations,
no variance, non-finite data, bad CSR range) has all 1,088 features 0.
"""
from __future__ import annotations

import numpy as np

import oracle

COARSE = 1024
POOL = 8
COARSE_BINS = COARSE * POOL
WINDOW = 64
DIM = COARSE + WINDOW
N_PROBES = 53
SEASON_GAP = 60.0
MIN_SEASON_OBS = 8
PROBE_FREQS = 10.0 ** (-3.0 + np.arange(N_PROBES) * (np.log10(30.0) + 3.0) / (N_PROBES - 1))


def seasons(t, gap=SEASON_GAP):
    """[(start, end)) index ranges of the seasons of one series."""
    t = np.asarray(t, dtype=np.float64)
    if len(t) == 0:
        return []
    cut = np.nonzero(np.diff(t) > gap)[0] + 1
    starts = np.concatenate([[0], cut])
    ends = np.concatenate([cut, [len(t)]])
    return list(zip(starts.tolist(), ends.tolist()))


def season_groups(t, gap=SEASON_GAP, min_obs=MIN_SEASON_OBS):
    """[(start, end)) ranges of the season groups that get a periodogram."""
    out = []
    start = None
    for a, b in seasons(t, gap):
        if start is None:
            start = a
        if b - start >= min_obs:
            out.append((start, b))
            start = None
    return out


def coarse(t, y, f_min, f_max, unit=oracle.CYCLES, gap=SEASON_GAP, min_obs=MIN_SEASON_OBS):
    """Group-averaged, max-pooled coarse periodogram (1,024 values)."""
    acc = np.zeros(COARSE)
    count = 0
    yc = np.asarray(y, dtype=np.float64) - np.mean(y)
    for a, b in season_groups(t, gap, min_obs):
        pg, _ = oracle.single(t[a:b], yc[a:b], f_min, f_max, COARSE_BINS, unit=unit,
                              subtract_mean=False)
        acc += pg.reshape(COARSE, POOL).max(axis=1)
        count += 1
    return acc / count if count else acc


def window(t, y, gap=SEASON_GAP, min_obs=MIN_SEASON_OBS):
    """The 64 sampling and magnitude features."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(t)
    w = np.zeros(WINDOW)
    if n == 0:
        return w
    w[0] = np.log10(n)
    w[1] = np.log10(max(t.max() - t.min(), 1e-3))
    seg = seasons(t, gap)
    w[2] = len(seg)
    good = [(a, b) for a, b in seg if b - a >= min_obs]
    w[3] = len(good)
    d = np.diff(t)
    within = d[d <= gap]
    if len(within):
        w[4] = np.log10(max(within.mean(), 1e-6))
        w[5] = np.log10(np.maximum(within, 1e-6)).std()
    w[6] = sum(b - a for a, b in good) / n
    yc = y - y.mean()
    sigma = np.sqrt(np.mean(yc * yc))
    if sigma > 0:
        w[7] = np.log10(sigma)
        w[8] = np.mean(yc ** 3) / sigma ** 3
        w[9] = np.mean(yc ** 4) / sigma ** 4 - 3.0
        w[10] = np.abs(yc).max() / sigma
    else:
        w[7] = np.log10(1e-30)
    for p, f in enumerate(PROBE_FREQS):
        ph = 2.0 * np.pi * f * t
        w[11 + p] = (np.cos(ph).sum() ** 2 + np.sin(ph).sum() ** 2) / (n * n)
    return w


def features(offsets, t, y, f_min, f_max, unit=oracle.CYCLES, gap=SEASON_GAP,
             min_obs=MIN_SEASON_OBS):
    """[n_obj, 1088] features of a CSR batch."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n_obj = len(offsets) - 1
    out = np.zeros((n_obj, DIM))
    for o in range(n_obj):
        a, b = int(offsets[o]), int(offsets[o + 1])
        if a < 0 or b < a or b > len(t):
            continue
        to, yo = t[a:b], y[a:b]
        if not (np.all(np.isfinite(to)) and np.all(np.isfinite(yo))):
            continue
        _, pk = oracle.single(to, yo, f_min, f_max, 1, unit=unit)
        if pk["status"] != oracle.OK:
            continue
        out[o, :COARSE] = coarse(to, yo, f_min, f_max, unit, gap, min_obs)
        out[o, COARSE:] = window(to, yo, gap, min_obs)
    return out
