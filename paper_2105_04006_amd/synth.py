"""Seeded synthetic light curves shaped like the paper's workloads.

This module only draws inputs; it holds none of the periodogram's arithmetic,
so both the GPU path's tests and the CPU oracle's tests can use it.

The paper's own datasets (a 3,554-point synthetic object and ~1,000 ZTF-like
synthetic asteroids, Section 4.2) are not available, so these stand in for
them: times uniform over a 10-year baseline with a seasonal gap every year,
sinusoidal light curves with asteroid-like periods (0.1-1 d) plus Gaussian
noise, and CSR-packed batches with a spread of series lengths.

Sampling: "t uniform in [0, 3650) d, dropping t mod 365 in [120, 240]" is drawn
exactly, without rejection, by drawing u uniform over the 2,450 allowed days and
mapping it onto the allowed intervals of its year; this has the same
distribution as rejection sampling and yields exactly N_t points.

Streams: per-object parameters, times, noise and mixture labels come from
separate PCG64 streams, each consumed in object order, so the first k objects
of a workload are identical whether k or all objects are generated.

Photometric errors (``errors=True``, for the generalized periodogram of
Section 4.11, whose ZTF-like records carry per-point errors): dy is drawn
log-normally around the noise level, sigma * 10^(0.25 z) clipped to
[0.01, 0.3] mag, from a fifth stream, and the noise of each point is then
drawn with its own dy (the same standard-normal draws scaled by dy instead of
sigma), so the errors describe the scatter they come with.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2105040060
SPAN_DAYS = 3650.0
YEAR_DAYS = 365.0
GAP = (120.0, 240.0)
AMP = 0.3
NOISE_SIGMA = 0.05
PERIOD_RANGE = (0.1, 1.0)

# name -> (n_obj, (N_t min, N_t max), (f_min, f_max) cycles/day, N_f, mixture, seed id)
WORKLOADS = {
    "single_256": (1, (256, 256), (1.0, 12.0), 10_000, "sine", 1),
    "single_4096": (1, (4096, 4096), (0.5, 24.0), 500_000, "sine", 2),
    "batch_10k": (10_000, (50, 1000), (1.0, 12.0), 100_000, "sine", 3),
    "learned_100k": (100_000, (50, 500), (1.0, 12.0), 200_000, "sine", 4),
    "lsst_200k": (200_000, (20, 500), (0.5, 24.0), 250_000, "lsst", 5),
    # grid in rad/day (the paper's batch range), see make_asteroids
    "asteroids_1k": (1_000, (10, 1500), (1.005, 150.796), 200_000, "asteroid", 6),
    "asteroids_100k": (100_000, (10, 1500), (1.005, 150.796), 200_000, "asteroid", 7),
}

KIND_SINE, KIND_TWO_HARMONIC, KIND_NOISE = 0, 1, 2


@dataclass
class Workload:
    name: str
    offsets: np.ndarray  # int64 [n_obj + 1]
    t: np.ndarray  # float64 [n_obs], days, ascending within each object
    y: np.ndarray  # float64 [n_obs], magnitudes
    f_min: float
    f_max: float
    n_f: int
    unit: int = 0  # 0: cycles per day
    true_freq: np.ndarray = field(default=None)  # cycles/day, NaN for pure noise
    kind: np.ndarray = field(default=None)  # KIND_* per object
    seed: int = 0
    dy: np.ndarray = field(default=None)  # float64 [n_obs] photometric errors, or None

    @property
    def n_obj(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_obs(self) -> int:
        return len(self.t)

    @property
    def n_t(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def evals(self) -> int:
        return int(self.n_obs) * int(self.n_f)

    def obj(self, o):
        a, b = self.offsets[o], self.offsets[o + 1]
        return self.t[a:b], self.y[a:b]

    def subset(self, k: int) -> "Workload":
        """The first k objects (identical to generating only k)."""
        off = self.offsets[: k + 1].copy()
        n = off[-1]
        return Workload(self.name, off, self.t[:n].copy(), self.y[:n].copy(), self.f_min,
                        self.f_max, self.n_f, self.unit, self.true_freq[:k].copy(),
                        self.kind[:k].copy(), self.seed,
                        None if self.dy is None else self.dy[:n].copy())


def seasonal_times(u: np.ndarray) -> np.ndarray:
    """Map u in [0, 2450) onto [0, 3650) minus the yearly gap [120, 240]."""
    keep = YEAR_DAYS - (GAP[1] - GAP[0])  # 245 allowed days per year
    yr = np.floor(u / keep)
    r = u - yr * keep
    t = np.where(r < GAP[0], yr * YEAR_DAYS + r, yr * YEAR_DAYS + GAP[1] + (r - GAP[0]))
    return t


def in_gap(t: np.ndarray) -> np.ndarray:
    m = np.mod(t, YEAR_DAYS)
    return (m >= GAP[0]) & (m <= GAP[1])


def _draw_times(rng: np.random.Generator, n: int) -> np.ndarray:
    keep_total = (SPAN_DAYS / YEAR_DAYS) * (YEAR_DAYS - (GAP[1] - GAP[0]))
    t = seasonal_times(rng.random(n) * keep_total)
    bad = in_gap(t) | (t >= SPAN_DAYS)
    while bad.any():  # only boundary round-off can land here; redraw those points
        t[bad] = seasonal_times(rng.random(int(bad.sum())) * keep_total)
        bad = in_gap(t) | (t >= SPAN_DAYS)
    return t


def _sort_segments(t: np.ndarray, offsets: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """Sort t ascending within each CSR segment (exact; padded 2-D sorts per chunk)."""
    out = np.empty_like(t)
    n_obj = len(offsets) - 1
    for c0 in range(0, n_obj, chunk):
        c1 = min(n_obj, c0 + chunk)
        lens = np.diff(offsets[c0:c1 + 1])
        width = int(lens.max()) if len(lens) else 0
        if width == 0:
            continue
        col = np.arange(width)
        mask = col[None, :] < lens[:, None]
        pad = np.full((c1 - c0, width), np.inf)
        pad[mask] = t[offsets[c0]:offsets[c1]]
        pad.sort(axis=1)
        out[offsets[c0]:offsets[c1]] = pad[mask]
    return out


def make_workload(name: str, n_obj: int | None = None, seed: int | None = None,
                  errors: bool = False) -> Workload:
    """Generate a named workload (optionally only its first n_obj objects).

    ``errors=True`` adds per-point photometric errors ``dy`` and draws each
    point's noise with its own error."""
    full_obj, (nt_lo, nt_hi), (f_min, f_max), n_f, mix, sid = WORKLOADS[name]
    if mix == "asteroid":
        return make_asteroids(name, n_obj, seed)
    seed = SEED_BASE + sid if seed is None else int(seed)
    k = full_obj if n_obj is None else int(n_obj)
    ss = np.random.SeedSequence(seed)
    # spawn(5) gives the same first four children as spawn(4)
    r_len, r_par, r_t, r_noise, r_err = (np.random.Generator(np.random.PCG64(s))
                                         for s in ss.spawn(5))

    n_t = r_len.integers(nt_lo, nt_hi + 1, size=full_obj)[:k].astype(np.int64)
    # per-object parameters, drawn for the full population so prefixes agree
    logp = r_par.uniform(np.log10(PERIOD_RANGE[0]), np.log10(PERIOD_RANGE[1]), size=full_obj)
    phi = r_par.uniform(0.0, 2.0 * np.pi, size=full_obj)
    u_kind = r_par.random(full_obj)
    ratio = r_par.uniform(0.1, 0.5, size=full_obj)
    phi2 = r_par.uniform(0.0, 2.0 * np.pi, size=full_obj)
    period = (10.0 ** logp)[:k]
    phi, u_kind, ratio, phi2 = phi[:k], u_kind[:k], ratio[:k], phi2[:k]
    if mix == "lsst":
        kind = np.where(u_kind < 0.6, KIND_SINE,
                        np.where(u_kind < 0.9, KIND_TWO_HARMONIC, KIND_NOISE)).astype(np.int32)
    else:
        kind = np.full(k, KIND_SINE, dtype=np.int32)

    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(n_t, out=offsets[1:])
    n_obs = int(offsets[-1])
    owner = np.repeat(np.arange(k, dtype=np.int64), n_t)
    t = _sort_segments(_draw_times(r_t, n_obs), offsets)

    P = period[owner]
    y = AMP * np.sin(2.0 * np.pi * t / P + phi[owner])
    two = kind[owner] == KIND_TWO_HARMONIC
    y = y + np.where(two, ratio[owner] * AMP * np.sin(4.0 * np.pi * t / P + phi2[owner]), 0.0)
    y = np.where(kind[owner] == KIND_NOISE, 0.0, y)
    dy = None
    if errors:
        dy = np.clip(NOISE_SIGMA * 10.0 ** (0.25 * r_err.standard_normal(n_obs)), 0.01, 0.3)
        y = y + dy * r_noise.standard_normal(n_obs)
    else:
        y = y + r_noise.normal(0.0, NOISE_SIGMA, size=n_obs)

    true_freq = np.where(kind == KIND_NOISE, np.nan, 1.0 / period)
    return Workload(name, offsets, t, y, float(f_min), float(f_max), int(n_f), 0, true_freq, kind,
                    seed, dy)


# Asteroid-like population (Section 4.2's batch dataset: ~1,000 synthetic
# asteroids with ZTF-like cadences and photometric errors, a log-normal number
# of observations, rotation periods of a few hours to a few hundred hours).
AST_SPAN_DAYS = 1095.0        # three observing years
AST_NT_MEDIAN = 110.0         # log-normal N_t: median and log-sigma, clipped
AST_NT_LOG_SIGMA = 0.9
AST_PROT_MEDIAN_H = 8.0       # rotation periods: log-normal body (median, log-sigma) ...
AST_PROT_LOG_SIGMA = 0.9
AST_PROT_MIN_H = 2.0
AST_SLOW = (0.03, 100.0, 400.0)  # ... and a slow-rotator tail: fraction, log-uniform range (h)
AST_AMP = (0.1, 0.6)          # peak-to-peak light-curve amplitude, mag, log-uniform
AST_ERR = (0.02, 0.15)        # per-object photometric error level, mag, log-uniform


def make_asteroids(name: str, n_obj: int | None = None, seed: int | None = None) -> Workload:
    """The asteroid-like population, errors included.

    Cadence: each object is observed on nights drawn from the seasonal
    calendar (the yearly 120-day gap) over three years, at an evening time
    0.15-0.35 d into the night; half of the visits get a second exposure 30
    minutes later, as in survey pair cadences.  Light curve: an elongated body
    shows two maxima per rotation, so the dominant term is the second harmonic
    of the rotation frequency (the light-curve period is half the rotation
    period, which the periodogram finds), plus a weaker first harmonic; each
    point gets Gaussian noise with its own error dy.  Rotation periods are
    log-normal around 8 h (main-belt-like) with a 3% tail of slow rotators
    (100-400 h, a few beyond the grid's 300 h).  true_freq is the light-curve
    frequency in rad/day (the grid's unit).
    """
    full_obj, (nt_lo, nt_hi), (f_min, f_max), n_f, _, sid = WORKLOADS[name]
    seed = SEED_BASE + sid if seed is None else int(seed)
    k = full_obj if n_obj is None else int(n_obj)
    ss = np.random.SeedSequence(seed)
    r_len, r_par, r_t, r_noise, r_err = (np.random.Generator(np.random.PCG64(s))
                                         for s in ss.spawn(5))
    n_t = np.clip(np.round(AST_NT_MEDIAN * np.exp(AST_NT_LOG_SIGMA *
                                                  r_len.standard_normal(full_obj))),
                  nt_lo, nt_hi).astype(np.int64)[:k]
    body = AST_PROT_MEDIAN_H * np.exp(AST_PROT_LOG_SIGMA * r_par.standard_normal(full_obj))
    body = np.maximum(body, AST_PROT_MIN_H)
    slow = np.exp(r_par.uniform(np.log(AST_SLOW[1]), np.log(AST_SLOW[2]), size=full_obj))
    p_rot_h = np.where(r_par.random(full_obj) < AST_SLOW[0], slow, body)[:k]
    amp = np.exp(r_par.uniform(np.log(AST_AMP[0]), np.log(AST_AMP[1]), size=full_obj))[:k]
    phi1 = r_par.uniform(0.0, 2.0 * np.pi, size=full_obj)[:k]
    phi2 = r_par.uniform(0.0, 2.0 * np.pi, size=full_obj)[:k]
    asym = r_par.uniform(0.05, 0.3, size=full_obj)[:k]
    err = np.exp(r_par.uniform(np.log(AST_ERR[0]), np.log(AST_ERR[1]), size=full_obj))[:k]

    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(n_t, out=offsets[1:])
    n_obs = int(offsets[-1])
    owner = np.repeat(np.arange(k, dtype=np.int64), n_t)
    # nights from the seasonal calendar, evening times, optional pair exposures
    keep_total = (AST_SPAN_DAYS / YEAR_DAYS) * (YEAR_DAYS - (GAP[1] - GAP[0]))
    u = r_t.random((n_obs, 3))  # one row per observation keeps prefixes identical
    night = np.floor(seasonal_times(u[:, 0] * keep_total))
    t = night + 0.15 + 0.2 * u[:, 1]
    pair = u[:, 2] < 0.5
    # a pair's second exposure follows the point before it in the same object
    idx = np.arange(n_obs)
    first = np.zeros(n_obs, dtype=bool)
    first[offsets[:-1][n_t > 0]] = True
    take = pair & ~first
    t[take] = t[idx[take] - 1] + 30.0 / 1440.0
    t = _sort_segments(t, offsets)

    w_rot = 2.0 * np.pi * 24.0 / p_rot_h  # rad/day
    y = (0.5 * amp[owner] * np.cos(2.0 * w_rot[owner] * t + phi2[owner])
         + 0.5 * amp[owner] * asym[owner] * np.cos(w_rot[owner] * t + phi1[owner]))
    dy = np.clip(err[owner] * 10.0 ** (0.15 * r_err.standard_normal(n_obs)), 0.005, 0.5)
    y = y + dy * r_noise.standard_normal(n_obs)
    w = Workload(name, offsets, t, y, float(f_min), float(f_max), int(n_f), 1, 2.0 * w_rot,
                 np.zeros(k, dtype=np.int32), seed, dy)
    w.p_rot_hours = p_rot_h
    return w


def pack(series) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """CSR-pack a list of (t, y) pairs into (offsets, t, y)."""
    n_t = np.array([len(s[0]) for s in series], dtype=np.int64)
    offsets = np.zeros(len(series) + 1, dtype=np.int64)
    np.cumsum(n_t, out=offsets[1:])
    t = np.concatenate([np.asarray(s[0], np.float64) for s in series]) if len(series) else np.zeros(0)
    y = np.concatenate([np.asarray(s[1], np.float64) for s in series]) if len(series) else np.zeros(0)
    return offsets, t, y


def sine_object(n_t: int, seed: int, period: float | None = None, sigma: float = NOISE_SIGMA,
                amp: float = AMP):
    """One seasonal-cadence sinusoid; returns (t, y, true frequency in cycles/day)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if period is None:
        period = 10.0 ** rng.uniform(-1.0, 0.0)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    t = np.sort(_draw_times(rng, n_t))
    y = amp * np.sin(2.0 * np.pi * t / period + phi)
    if sigma > 0:
        y = y + rng.normal(0.0, sigma, size=n_t)
    return t, y, 1.0 / period
