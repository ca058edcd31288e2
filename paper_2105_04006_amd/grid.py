"""Frequency-grid selection rule (Section 4.3, Table 2).

For an observing window T_max = |t_1 - t_N| (for a batch, the largest window
of any object) the paper takes an angular spacing df = 0.2 pi / T_max, i.e.
ten-fold oversampling of the 1/T_max resolution in cycles, and
N_f = (f_max - f_min) / df trial frequencies, rounded to the nearest integer.
This is host-side parameter selection, not part of the periodogram itself.
"""
from __future__ import annotations

import math

CYCLES, ANGULAR = 0, 1


def spacing_from_window(t_max_span: float, unit: int = ANGULAR) -> float:
    """Grid spacing for an observing window: 0.2 pi / T (angular) = 0.1 / T (cycles)."""
    if not (t_max_span > 0.0) or not math.isfinite(t_max_span):
        raise ValueError("observing window must be positive and finite")
    return (0.2 * math.pi if unit == ANGULAR else 0.1) / t_max_span


def n_freq(f_min: float, f_max: float, df: float) -> int:
    """Number of trial frequencies covering [f_min, f_max) at spacing df."""
    if not (f_max > f_min) or not (df > 0.0):
        raise ValueError("need f_max > f_min and df > 0")
    return int(round((f_max - f_min) / df))


def grid_from_window(t_max_span: float, f_min: float, f_max: float, unit: int = ANGULAR):
    """(f_min, f_max, N_f) following the paper's rule for a given observing window."""
    return f_min, f_max, n_freq(f_min, f_max, spacing_from_window(t_max_span, unit))
