"""Plain FP64 CPU oracle for the Lomb-Scargle periodogram (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product library never does.  It
shares no code with the GPU path.  The arithmetic lives in ``lsp_oracle.c``
(Section 2 of Gowanlock et al., arXiv 2105.04006: Eq. 1 for tau, Eq. 2 for the
power, the uniform half-open frequency grid; Section 3.3 for the argmax and
the period; Section 4.11 for the generalized periodogram with errors and a
floating mean, ``gen_*``).  This file only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsp_oracle.c")
_LIB = os.path.join(_HERE, "liblsp_oracle.so")

OK, DEGENERATE, BADRANGE, NONFINITE = 0, 1, 2, 3
CYCLES, ANGULAR = 0, 1

PEAK_DTYPE = np.dtype(
    [("index", "<i8"), ("freq", "<f8"), ("period", "<f8"), ("power", "<f8"),
     ("status", "<i4"), ("pad", "<i4")]
)


def compile_source(src: str, out: str) -> str:
    """gcc build of an oracle source file (no fast-math, no FP contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-Wall", "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library next to its source."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


def _bind(path):
    L = ctypes.CDLL(path)
    d, i32, i64, p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.ora_grid_freq.restype = d
    L.ora_grid_freq.argtypes = [d, d, i64, i64]
    L.ora_omega.restype = d
    L.ora_omega.argtypes = [d, i32]
    L.ora_period.restype = d
    L.ora_period.argtypes = [d, i32]
    L.ora_prep.restype = i32
    L.ora_prep.argtypes = [p, p, i64, i32, p, p]
    L.ora_tau.restype = d
    L.ora_tau.argtypes = [p, i64, d]
    L.ora_pls.restype = d
    L.ora_pls.argtypes = [p, p, i64, d, d, p]
    L.ora_argmax.restype = i64
    L.ora_argmax.argtypes = [p, i64]
    L.ora_single.restype = i32
    L.ora_single.argtypes = [p, p, i64, d, d, i64, i32, i32, i32, p, p, p, i32]
    L.ora_batch.restype = i32
    L.ora_batch.argtypes = [p, i64, i64, p, p, d, d, i64, i32, i32, i32, p, p, i32]
    L.ora_eval_bins.restype = i32
    L.ora_eval_bins.argtypes = [p, i64, i64, p, p, d, d, i64, i32, i32, i32, p, p, i64, p, i32]
    L.ora_gen_prep.restype = i32
    L.ora_gen_prep.argtypes = [p, p, p, i64, p, p, p, p]
    L.ora_gen_tau.restype = d
    L.ora_gen_tau.argtypes = [p, p, i64, d, d]
    L.ora_gen_pls.restype = d
    L.ora_gen_pls.argtypes = [p, p, p, i64, d, d, d, p]
    L.ora_gen_single.restype = i32
    L.ora_gen_single.argtypes = [p, p, p, i64, d, d, i64, i32, i32, p, p, p, p, i32]
    L.ora_gen_batch.restype = i32
    L.ora_gen_batch.argtypes = [p, i64, i64, p, p, p, d, d, i64, i32, i32, p, p, i32]
    L.ora_gen_eval_bins.restype = i32
    L.ora_gen_eval_bins.argtypes = [p, i64, i64, p, p, p, d, d, i64, i32, i32, p, p, i64, p, i32]
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Oracle:
    """One loaded build of the oracle (the default one, or a test's own build)."""

    def __init__(self, path=None):
        if path is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            path = _LIB
        self.path = path
        self.L = _bind(path)

    def grid_freq(self, f_min, f_max, n_f, i):
        """Section 2: f_i = f_min + i * (f_max - f_min) / N_f."""
        return self.L.ora_grid_freq(float(f_min), float(f_max), int(n_f), int(i))

    def omega(self, f, unit=CYCLES):
        return self.L.ora_omega(float(f), int(unit))

    def period(self, f, unit=CYCLES):
        """Section 3.3: p = 2 pi / w."""
        return self.L.ora_period(float(f), int(unit))

    def prep(self, t, y, subtract_mean=True):
        """Zero-mean magnitudes and S_yy; returns (status, yp, syy)."""
        t, y = _f64(t), _f64(y)
        yp = np.zeros(max(len(t), 1))
        syy = np.zeros(1)
        st = self.L.ora_prep(_ptr(t), _ptr(y), len(t), int(bool(subtract_mean)), _ptr(yp),
                             _ptr(syy))
        return st, yp[: len(t)], float(syy[0])

    def tau(self, t, w):
        """Eq. 1 at angular frequency w."""
        t = _f64(t)
        return self.L.ora_tau(_ptr(t), len(t), float(w))

    def pls_at(self, t, yp, w, tau_value):
        """Eq. 2 at angular frequency w and a given tau; returns (P_LS, [YC, YS, CC, SS])."""
        t, yp = _f64(t), _f64(yp)
        sums = np.zeros(4)
        v = self.L.ora_pls(_ptr(t), _ptr(yp), len(t), float(w), float(tau_value), _ptr(sums))
        return v, sums

    def argmax(self, p):
        p = _f64(p)
        return self.L.ora_argmax(_ptr(p), len(p))

    def single(self, t, y, f_min, f_max, n_f, unit=CYCLES, normalize=True, subtract_mean=True,
               threads=0):
        """Whole periodogram of one object; returns (pgram[n_f], peak record)."""
        t, y = _f64(t), _f64(y)
        yp = np.zeros(max(len(t), 1))
        pg = np.empty(int(n_f))
        pk = np.zeros(1, dtype=PEAK_DTYPE)
        self.L.ora_single(_ptr(t), _ptr(y), len(t), float(f_min), float(f_max), int(n_f),
                          int(unit), int(bool(normalize)), int(bool(subtract_mean)), _ptr(yp),
                          _ptr(pg), _ptr(pk), int(threads))
        return pg, pk[0]

    def batch(self, offsets, t, y, f_min, f_max, n_f, unit=CYCLES, normalize=True,
              subtract_mean=True, want_pgram=True, threads=0):
        """Batch mode over CSR objects; returns (pgram[n_obj, n_f] or None, peaks[n_obj])."""
        offsets, t, y = _i64(offsets), _f64(t), _f64(y)
        n_obj = len(offsets) - 1
        n_f = int(n_f)
        pk = np.zeros(n_obj, dtype=PEAK_DTYPE)
        pg = np.empty((n_obj, n_f)) if want_pgram else None
        rc = self.L.ora_batch(_ptr(offsets), n_obj, len(t), _ptr(t), _ptr(y), float(f_min),
                              float(f_max), n_f, int(unit), int(bool(normalize)),
                              int(bool(subtract_mean)), _ptr(pg), _ptr(pk), int(threads))
        if rc != 0:
            raise MemoryError("oracle batch could not allocate scratch")
        return pg, pk

    def eval_bins(self, offsets, t, y, f_min, f_max, n_f, obj, bins, unit=CYCLES,
                  normalize=True, subtract_mean=True, threads=0):
        """Power at chosen (object, grid index) pairs."""
        offsets, t, y = _i64(offsets), _f64(t), _f64(y)
        obj, bins = _i64(obj), _i64(bins)
        out = np.empty(len(obj))
        rc = self.L.ora_eval_bins(_ptr(offsets), len(offsets) - 1, len(t), _ptr(t), _ptr(y),
                                  float(f_min), float(f_max), int(n_f), int(unit),
                                  int(bool(normalize)), int(bool(subtract_mean)), _ptr(obj),
                                  _ptr(bins), len(obj), _ptr(out), int(threads))
        if rc != 0:
            raise MemoryError("oracle eval_bins could not allocate scratch")
        return out

    # -- generalized periodogram (Section 4.11): errors dy (None: unit errors)
    # and a floating mean.

    def gen_prep(self, t, y, dy=None):
        """Weights, weighted-mean-centred magnitudes, YY and W; returns (status, w, yw, yy, W)."""
        t, y = _f64(t), _f64(y)
        dy = None if dy is None else _f64(dy)
        n = len(t)
        w, yw = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        yy, ws = np.zeros(1), np.zeros(1)
        st = self.L.ora_gen_prep(_ptr(t), _ptr(y), _ptr(dy), n, _ptr(w), _ptr(yw), _ptr(yy),
                                 _ptr(ws))
        return st, w[:n], yw[:n], float(yy[0]), float(ws[0])

    def gen_tau(self, t, w, wsum, om):
        t, w = _f64(t), _f64(w)
        return self.L.ora_gen_tau(_ptr(t), _ptr(w), len(t), float(wsum), float(om))

    def gen_pls(self, t, yw, w, wsum, om, tau_value):
        """Half the chi^2 reduction at om and tau; returns (P, [YC, YS, CC, SS])."""
        t, yw, w = _f64(t), _f64(yw), _f64(w)
        sums = np.zeros(4)
        v = self.L.ora_gen_pls(_ptr(t), _ptr(yw), _ptr(w), len(t), float(wsum), float(om),
                               float(tau_value), _ptr(sums))
        return v, sums

    def gen_single(self, t, y, dy, f_min, f_max, n_f, unit=CYCLES, normalize=True, threads=0):
        """Whole generalized periodogram of one object; returns (pgram[n_f], peak record)."""
        t, y = _f64(t), _f64(y)
        dy = None if dy is None else _f64(dy)
        n = len(t)
        w, yw = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        pg = np.empty(int(n_f))
        pk = np.zeros(1, dtype=PEAK_DTYPE)
        self.L.ora_gen_single(_ptr(t), _ptr(y), _ptr(dy), n, float(f_min), float(f_max),
                              int(n_f), int(unit), int(bool(normalize)), _ptr(w), _ptr(yw),
                              _ptr(pg), _ptr(pk), int(threads))
        return pg, pk[0]

    def gen_batch(self, offsets, t, y, dy, f_min, f_max, n_f, unit=CYCLES, normalize=True,
                  want_pgram=True, threads=0):
        """Generalized batch over CSR objects; returns (pgram or None, peaks)."""
        offsets, t, y = _i64(offsets), _f64(t), _f64(y)
        dy = None if dy is None else _f64(dy)
        n_obj = len(offsets) - 1
        n_f = int(n_f)
        pk = np.zeros(n_obj, dtype=PEAK_DTYPE)
        pg = np.empty((n_obj, n_f)) if want_pgram else None
        rc = self.L.ora_gen_batch(_ptr(offsets), n_obj, len(t), _ptr(t), _ptr(y), _ptr(dy),
                                  float(f_min), float(f_max), n_f, int(unit),
                                  int(bool(normalize)), _ptr(pg), _ptr(pk), int(threads))
        if rc != 0:
            raise MemoryError("oracle gen_batch could not allocate scratch")
        return pg, pk

    def gen_eval_bins(self, offsets, t, y, dy, f_min, f_max, n_f, obj, bins, unit=CYCLES,
                      normalize=True, threads=0):
        """Generalized power at chosen (object, grid index) pairs."""
        offsets, t, y = _i64(offsets), _f64(t), _f64(y)
        dy = None if dy is None else _f64(dy)
        obj, bins = _i64(obj), _i64(bins)
        out = np.empty(len(obj))
        rc = self.L.ora_gen_eval_bins(_ptr(offsets), len(offsets) - 1, len(t), _ptr(t), _ptr(y),
                                      _ptr(dy), float(f_min), float(f_max), int(n_f), int(unit),
                                      int(bool(normalize)), _ptr(obj), _ptr(bins), len(obj),
                                      _ptr(out), int(threads))
        if rc != 0:
            raise MemoryError("oracle gen_eval_bins could not allocate scratch")
        return out


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def __getattr__(name):
    # module-level shortcuts: oracle.single(...), oracle.batch(...), ...
    if name in ("grid_freq", "omega", "period", "prep", "tau", "pls_at", "argmax", "single",
                "batch", "eval_bins", "gen_prep", "gen_tau", "gen_pls", "gen_single", "gen_batch",
                "gen_eval_bins"):
        return getattr(default(), name)
    raise AttributeError(name)
