"""Pins of the oracle's generalized periodogram (Section 4.11) to facts that do
not come from the oracle itself.

Each pin takes an ``oracle.Oracle`` and raises AssertionError on a mismatch, so
that the same pins check the real oracle (test_gen_oracle.py) and planted
mistakes in copies of it (test_oracle_mutants.py).

The generalized periodogram fits y = a cos wt + b sin wt + c by weighted least
squares with weights 1 / dy^2; its normalised power is the fraction of the
weighted variance about the weighted mean that the fit explains, and its
unnormalised power is half the reduction in chi^2.  The pins:
  - brute force: numpy's least-squares solver on the design [1, cos wt, sin wt]
    gives chi^2 of the fit directly, for small random objects and errors;
  - reduction: with unit errors on evenly spaced times at the Fourier
    frequencies k / N, sum cos wt = sum sin wt = 0, so the floating mean
    changes nothing and the power equals the standard periodogram's;
  - an exact sinusoid plus offset has power 1 at its own frequency, whatever
    the errors;
  - invariances: common scaling of the errors (normalised power unchanged,
    unnormalised scaled by 1/alpha^2), affine maps of y, shifts of t;
  - an observation listed twice weighs as one with error dy / sqrt(2);
  - equal errors give the unit-error power (unnormalised: scaled by 1/dy^2);
  - three observations are fitted exactly by three parameters (power 1);
  - w = 0 leaves only the constant: power 0;
  - object statuses for short, constant and invalid input.
"""
from __future__ import annotations

import numpy as np

import oracle


def _obj(seed, n, span=60.0):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, span, n))
    y = 3.0 + rng.normal(0.0, 1.0, n) + 0.8 * np.sin(2 * np.pi * 0.37 * t)
    dy = rng.uniform(0.1, 2.0, n)
    return t, y, dy


def _wls_chi2(t, y, dy, om):
    """(chi^2 about the weighted mean, chi^2 of the 3-parameter fit) by lstsq."""
    sw = 1.0 / dy
    a = np.stack([np.ones_like(t), np.cos(om * t), np.sin(om * t)], axis=1) * sw[:, None]
    b = y * sw
    x, *_ = np.linalg.lstsq(a, b, rcond=None)
    r = b - a @ x
    a0 = sw[:, None]
    x0, *_ = np.linalg.lstsq(a0, b, rcond=None)
    r0 = b - a0 @ x0
    return float(r0 @ r0), float(r @ r)


def pin_gen_brute_force_wls(ora):
    for seed, n, unit in ((1, 5, oracle.CYCLES), (2, 12, oracle.CYCLES), (3, 40, oracle.ANGULAR),
                          (4, 97, oracle.CYCLES)):
        t, y, dy = _obj(seed, n)
        f_min, f_max, n_f = (0.05, 1.3, 23) if unit == oracle.CYCLES else (0.3, 8.0, 23)
        pn, _ = ora.gen_single(t, y, dy, f_min, f_max, n_f, unit=unit, normalize=True)
        pu, _ = ora.gen_single(t, y, dy, f_min, f_max, n_f, unit=unit, normalize=False)
        for i in range(n_f):
            f = f_min + (f_max - f_min) / n_f * i
            om = f if unit == oracle.ANGULAR else 2 * np.pi * f
            c0, c1 = _wls_chi2(t, y, dy, om)
            assert abs(pn[i] - (c0 - c1) / c0) <= 1e-9, (seed, i, pn[i], (c0 - c1) / c0)
            assert abs(pu[i] - 0.5 * (c0 - c1)) <= 1e-9 * c0, (seed, i, pu[i], 0.5 * (c0 - c1))


def pin_gen_unit_errors_fourier_grid_is_standard(ora):
    n = 32
    t = np.arange(n, dtype=np.float64)
    rng = np.random.default_rng(7)
    y = rng.normal(size=n) + np.cos(2 * np.pi * 5 / n * t)
    # f_i = (1 + i) / n, i = 0..14: the Fourier frequencies below Nyquist
    g, _ = ora.gen_single(t, y, None, 1.0 / n, 16.0 / n, 15)
    s, _ = ora.single(t, y, 1.0 / n, 16.0 / n, 15)
    assert np.allclose(g, s, rtol=1e-10, atol=1e-12), np.abs(g - s).max()
    # and the floating mean does matter off that grid
    g2, _ = ora.gen_single(t, y, None, 0.013, 0.4, 17)
    s2, _ = ora.single(t, y, 0.013, 0.4, 17)
    assert np.abs(g2 - s2).max() > 1e-4


def pin_gen_sinusoid_with_offset(ora):
    rng = np.random.default_rng(11)
    t = np.sort(rng.uniform(0.0, 40.0, 60))
    f_min, df, k = 0.1, 0.01, 27
    f0 = f_min + df * k
    y = 5.0 + 1.5 * np.sin(2 * np.pi * f0 * t + 0.4)
    dy = rng.uniform(0.05, 1.0, 60)
    pg, pk = ora.gen_single(t, y, dy, f_min, f_min + df * 50, 50)
    assert abs(pg[k] - 1.0) <= 1e-10, pg[k]
    assert pk["index"] == k
    assert np.all(pg[np.arange(50) != k] < 1.0 - 1e-6)


def pin_gen_invariances(ora):
    t, y, dy = _obj(21, 50)
    args = (0.02, 1.5, 31)
    pn, _ = ora.gen_single(t, y, dy, *args)
    pu, _ = ora.gen_single(t, y, dy, *args, normalize=False)
    a = 3.7
    pn2, _ = ora.gen_single(t, y, a * dy, *args)
    pu2, _ = ora.gen_single(t, y, a * dy, *args, normalize=False)
    assert np.allclose(pn2, pn, rtol=1e-10, atol=1e-13)
    assert np.allclose(pu2 * a * a, pu, rtol=1e-10, atol=1e-13)
    pn3, _ = ora.gen_single(t, 2.5 * y - 7.0, dy, *args)
    assert np.allclose(pn3, pn, rtol=1e-10, atol=1e-13)
    pn4, _ = ora.gen_single(t + 123.4, y, dy, *args)
    assert np.allclose(pn4, pn, rtol=1e-8, atol=1e-11)


def pin_gen_equal_errors_are_unit_errors(ora):
    # equal errors give equal weights: the normalised power is that of unit
    # errors, and the unnormalised one scales by 1/dy^2
    t, y, _ = _obj(61, 33)
    a, _ = ora.gen_single(t, y, None, 0.02, 1.4, 27)
    b, _ = ora.gen_single(t, y, np.full(33, 0.37), 0.02, 1.4, 27)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14), np.abs(a - b).max()
    au, _ = ora.gen_single(t, y, None, 0.02, 1.4, 27, normalize=False)
    bu, _ = ora.gen_single(t, y, np.full(33, 0.37), 0.02, 1.4, 27, normalize=False)
    assert np.allclose(bu * 0.37 ** 2, au, rtol=1e-12, atol=1e-14)


def pin_gen_duplicate_is_weight(ora):
    t, y, dy = _obj(31, 25)
    j = 9
    t2 = np.insert(t, j, t[j])
    y2 = np.insert(y, j, y[j])
    dy2 = np.insert(dy, j, dy[j])
    dy1 = dy.copy()
    dy1[j] = dy[j] / np.sqrt(2.0)
    for norm in (True, False):
        a, _ = ora.gen_single(t2, y2, dy2, 0.03, 1.2, 29, normalize=norm)
        b, _ = ora.gen_single(t, y, dy1, 0.03, 1.2, 29, normalize=norm)
        assert np.allclose(a, b, rtol=1e-10, atol=1e-13), (norm, np.abs(a - b).max())


def pin_gen_three_points_exact(ora):
    t = np.array([0.0, 1.3, 4.1])
    y = np.array([1.0, -0.4, 2.2])
    dy = np.array([0.5, 1.0, 2.0])
    pg, _ = ora.gen_single(t, y, dy, 0.05, 0.3, 10)
    assert np.allclose(pg, 1.0, atol=1e-9), pg


def pin_gen_zero_frequency(ora):
    t, y, dy = _obj(41, 30)
    pg, _ = ora.gen_single(t, y, dy, 0.0, 1.0, 20)
    assert pg[0] == 0.0, pg[0]
    assert np.all(pg[1:] > 0.0)


def pin_gen_statuses(ora):
    t, y, dy = _obj(51, 12)
    cases = [
        (t[:1], y[:1], dy[:1], oracle.DEGENERATE),
        (t, np.full(12, 2.5), dy, oracle.DEGENERATE),
        (t, y, np.where(np.arange(12) == 3, 0.0, dy), oracle.NONFINITE),
        (t, y, np.where(np.arange(12) == 3, -1.0, dy), oracle.NONFINITE),
        (t, y, np.where(np.arange(12) == 3, np.inf, dy), oracle.NONFINITE),
        (t, y, np.where(np.arange(12) == 3, np.nan, dy), oracle.NONFINITE),
        (t, np.where(np.arange(12) == 5, np.nan, y), dy, oracle.NONFINITE),
        (t, y, dy, oracle.OK),
        (t, y, None, oracle.OK),
    ]
    for k, (tt, yy, dd, want) in enumerate(cases):
        pg, pk = ora.gen_single(tt, yy, dd, 0.1, 1.0, 8)
        assert pk["status"] == want, (k, pk["status"], want)
        if want == oracle.DEGENERATE:
            assert np.all(pg == 0.0) and pk["index"] == -1
        elif want == oracle.NONFINITE:
            assert np.all(np.isnan(pg)) and pk["index"] == -1


GEN_PINS = [
    pin_gen_brute_force_wls,
    pin_gen_unit_errors_fourier_grid_is_standard,
    pin_gen_sinusoid_with_offset,
    pin_gen_invariances,
    pin_gen_duplicate_is_weight,
    pin_gen_equal_errors_are_unit_errors,
    pin_gen_three_points_exact,
    pin_gen_zero_frequency,
    pin_gen_statuses,
]
