"""Thin Python binding of liblsp.so (include/lsp.h): argument marshalling only.

Every step of the periodogram runs in the library's HIP kernels; this module
allocates the outputs and the workspace with PyTorch on the caller's device,
passes raw device pointers and the current HIP stream, and raises on any
non-OK status.  There is no CPU path: a missing library or a CPU tensor is an
error.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lsp.h")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ESCRATCH = 0, 1, 2, 3, 4, 5
STATIC_SCRATCH_BYTES = 64 << 20  # LSP_STATIC_SCRATCH_BYTES
OBJ_OK, OBJ_DEGENERATE, OBJ_BADRANGE, OBJ_NONFINITE = 0, 1, 2, 3
FORM_FP64, FORM_FP32P = 0, 1
CYCLES, ANGULAR = 0, 1
PGRAM_F32, PGRAM_F64 = 0, 1
SCHED_AUTO, SCHED_GRID, SCHED_PERSISTENT = 0, 1, 2
REC_AUTO, REC_ROTATION, REC_CHEBYSHEV = 0, 1, 2
WSPLIT_AUTO, WSPLIT_OFF, WSPLIT_ON = 0, 1, 2
OBS_AUTO, OBS_LDS, OBS_DIRECT = 0, 1, 2
TRIG_AUTO, TRIG_HW, TRIG_LIB, TRIG_POLY = 0, 1, 2, 3
ORDER_AUTO, ORDER_INPUT, ORDER_LPT = 0, 1, 2

PEAK_DTYPE = np.dtype(
    [("index", "<i8"), ("freq", "<f8"), ("period", "<f8"), ("power", "<f8"),
     ("status", "<i4"), ("reserved", "<i4")]
)
PEAK_BYTES = 40


class Grid(ctypes.Structure):
    _fields_ = [("f_min", ctypes.c_double), ("f_max", ctypes.c_double), ("n_f", ctypes.c_int64),
                ("unit", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("subtract_mean", ctypes.c_int32), ("pgram_dtype", ctypes.c_int32),
                ("k_per_lane", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32),
                ("t_split", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("recurrence", ctypes.c_int32), ("wave_split", ctypes.c_int32),
                ("obs_read", ctypes.c_int32), ("seed_trig", ctypes.c_int32),
                ("order", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FeatureOptions(ctypes.Structure):
    _fields_ = [("season_gap", ctypes.c_double), ("min_season_obs", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Mlp(ctypes.Structure):
    """lsp_mlp: layer widths and device pointers to the FP32 weights, biases
    and BF16 weight copies."""
    _fields_ = [("dims", ctypes.c_int32 * 4), ("w", ctypes.c_void_p * 3),
                ("b", ctypes.c_void_p * 3), ("w_bf16", ctypes.c_void_p * 3)]


class MlpGrads(ctypes.Structure):
    """lsp_mlp_grads: device pointers shaped like lsp_mlp's w and b."""
    _fields_ = [("w", ctypes.c_void_p * 3), ("b", ctypes.c_void_p * 3)]


FEAT_COARSE, FEAT_POOL, FEAT_WINDOW = 1024, 8, 64
FEAT_DIM = FEAT_COARSE + FEAT_WINDOW


class LspError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2105_04006_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, sz, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int32
        L.lsp_default_options.restype = Options
        L.lsp_default_options.argtypes = []
        L.lsp_workspace_bytes.restype = sz
        L.lsp_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Grid), ctypes.POINTER(Options)]
        L.lsp_single.restype = ctypes.c_int
        L.lsp_single.argtypes = [vp, vp, i64, ctypes.POINTER(Grid), ctypes.POINTER(Options), vp, vp,
                                 vp, sz, vp]
        L.lsp_batch.restype = ctypes.c_int
        L.lsp_batch.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                ctypes.POINTER(Options), vp, vp, vp, sz, vp]
        L.lsp_batch_static.restype = ctypes.c_int
        L.lsp_batch_static.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                       ctypes.POINTER(Options), vp, vp, vp]
        L.lsp_gen_workspace_bytes.restype = sz
        L.lsp_gen_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Grid),
                                              ctypes.POINTER(Options)]
        L.lsp_gen_single.restype = ctypes.c_int
        L.lsp_gen_single.argtypes = [vp, vp, vp, i64, ctypes.POINTER(Grid),
                                     ctypes.POINTER(Options), vp, vp, vp, sz, vp]
        L.lsp_gen_batch.restype = ctypes.c_int
        L.lsp_gen_batch.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(Grid),
                                    ctypes.POINTER(Options), vp, vp, vp, sz, vp]
        L.lsp_pipe_create.restype = ctypes.c_int
        L.lsp_pipe_create.argtypes = [i32, sz, sz, i32, ctypes.POINTER(vp)]
        L.lsp_pipe_destroy.restype = None
        L.lsp_pipe_destroy.argtypes = [vp]
        L.lsp_batch_to_host.restype = ctypes.c_int
        L.lsp_batch_to_host.argtypes = [vp, vp, i64, i64, vp, vp, vp, i32, ctypes.POINTER(Grid),
                                        ctypes.POINTER(Options), vp, vp, vp]
        L.lsp_gen_rows_workspace_bytes.restype = sz
        L.lsp_gen_rows_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Grid),
                                                   ctypes.POINTER(Options), i64, i64,
                                                   ctypes.c_int32]
        L.lsp_gen_batch_rows.restype = ctypes.c_int
        L.lsp_gen_batch_rows.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(Grid),
                                         ctypes.POINTER(Options), vp, vp, i64, i64,
                                         ctypes.c_int32, vp, vp, vp, sz, vp]
        L.lsp_gen_plan_create.restype = ctypes.c_int
        L.lsp_gen_plan_create.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(Grid),
                                          ctypes.POINTER(Options), vp, vp, vp, sz,
                                          ctypes.POINTER(vp)]
        L.lsp_rows_workspace_bytes.restype = sz
        L.lsp_rows_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Grid),
                                               ctypes.POINTER(Options), i64, i64, ctypes.c_int32]
        L.lsp_batch_rows.restype = ctypes.c_int
        L.lsp_batch_rows.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                     ctypes.POINTER(Options), vp, vp, i64, i64, ctypes.c_int32,
                                     vp, vp, vp, sz, vp]
        L.lsp_status_string.restype = ctypes.c_char_p
        L.lsp_status_string.argtypes = [ctypes.c_int]
        L.lsp_plan_create.restype = ctypes.c_int
        L.lsp_plan_create.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                      ctypes.POINTER(Options), vp, vp, vp, sz,
                                      ctypes.POINTER(vp)]
        L.lsp_plan_launch.restype = ctypes.c_int
        L.lsp_plan_launch.argtypes = [vp, vp]
        L.lsp_plan_destroy.restype = None
        L.lsp_plan_destroy.argtypes = [vp]
        L.lsp_autotune_workspace_bytes.restype = sz
        L.lsp_autotune_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Grid),
                                                   ctypes.POINTER(Options)]
        L.lsp_autotune.restype = ctypes.c_int
        L.lsp_autotune.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                   ctypes.POINTER(Options), ctypes.POINTER(Options), vp, vp, sz,
                                   ctypes.c_char_p, ctypes.c_int32, vp]
        i32, f32 = ctypes.c_int32, ctypes.c_float
        L.lsp_gemm_bf16.restype = ctypes.c_int
        L.lsp_gemm_bf16.argtypes = [i64, i64, i64, vp, i64, i64, vp, i64, i64, vp, vp, i32, vp,
                                    vp, i64, vp]
        L.lsp_softmax_xent.restype = ctypes.c_int
        L.lsp_softmax_xent.argtypes = [vp, vp, i64, i32, f32, vp, vp, vp, vp]
        L.lsp_col_sums.restype = ctypes.c_int
        L.lsp_col_sums.argtypes = [vp, i64, i32, vp, vp]
        L.lsp_col_stats.restype = ctypes.c_int
        L.lsp_col_stats.argtypes = [vp, i64, i32, vp, vp, vp]
        L.lsp_standardize_bf16.restype = ctypes.c_int
        L.lsp_standardize_bf16.argtypes = [vp, i64, i32, vp, vp, vp, vp]
        L.lsp_cast_bf16.restype = ctypes.c_int
        L.lsp_cast_bf16.argtypes = [vp, i64, vp, vp]
        L.lsp_adam.restype = ctypes.c_int
        L.lsp_adam.argtypes = [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp, vp]
        pm, pg = ctypes.POINTER(Mlp), ctypes.POINTER(MlpGrads)
        L.lsp_mlp_forward.restype = ctypes.c_int
        L.lsp_mlp_forward.argtypes = [pm, vp, i64, vp, vp, vp, vp]
        L.lsp_mlp_workspace_bytes.restype = sz
        L.lsp_mlp_workspace_bytes.argtypes = [pm, i64]
        L.lsp_mlp_backward.restype = ctypes.c_int
        L.lsp_mlp_backward.argtypes = [pm, vp, vp, i64, vp, vp, vp, f32, pg, vp, vp, sz, vp]
        L.lsp_mlp_adam.restype = ctypes.c_int
        L.lsp_mlp_adam.argtypes = [pm, pg, pg, pg, i32, f32, f32, f32, f32, vp]
        L.lsp_top_k.restype = ctypes.c_int
        L.lsp_top_k.argtypes = [vp, i64, i32, i32, vp, vp, vp]
        L.lsp_band_max.restype = ctypes.c_int
        L.lsp_band_max.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp]
        L.lsp_trim_bands.restype = ctypes.c_int
        L.lsp_trim_bands.argtypes = [vp, i64, i32, i32, vp, vp, i32, f32, f32, vp, vp, vp]
        L.lsp_merge_bands.restype = ctypes.c_int
        L.lsp_merge_bands.argtypes = [vp, i32, vp, i32, i64, i32, vp, vp]
        L.lsp_row_normalize.restype = ctypes.c_int
        L.lsp_row_normalize.argtypes = [vp, i64, i32, i32, i32, vp]
        L.lsp_pool_stats.restype = ctypes.c_int
        L.lsp_pool_stats.argtypes = [vp, vp, i32, i32, vp]
        L.lsp_shift_bands.restype = ctypes.c_int
        L.lsp_shift_bands.argtypes = [vp, vp, vp, i64, i32, i32, i32, i32, f32, vp, vp, vp]
        L.lsp_peak_bands.restype = ctypes.c_int
        L.lsp_peak_bands.argtypes = [vp, i64, i64, i32, vp, vp]
        L.lsp_select_fallback.restype = ctypes.c_int
        L.lsp_select_fallback.argtypes = [vp, vp, i64, f32, f32, vp, vp, vp]
        L.lsp_default_feature_options.restype = FeatureOptions
        L.lsp_default_feature_options.argtypes = []
        L.lsp_features_workspace_bytes.restype = sz
        L.lsp_features_workspace_bytes.argtypes = [i64]
        L.lsp_features.restype = ctypes.c_int
        L.lsp_features.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(Grid),
                                   ctypes.POINTER(FeatureOptions), vp, vp, sz, vp]
        L.lsp_describe_launch.restype = ctypes.c_int
        L.lsp_describe_launch.argtypes = [i64, i64, ctypes.POINTER(Grid), ctypes.POINTER(Options),
                                          i32, ctypes.POINTER(Options),
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.lsp_row_order_workspace_bytes.restype = sz
        L.lsp_row_order_workspace_bytes.argtypes = []
        L.lsp_row_order.restype = ctypes.c_int
        L.lsp_row_order.argtypes = [vp, i64, vp, vp, i64, i32, vp, vp, sz, vp]
        L.lsp_set_stage_events.restype = ctypes.c_int
        L.lsp_set_stage_events.argtypes = [vp, vp]
        L.lsp_version.restype = ctypes.c_int32
        L.lsp_version.argtypes = []
        _lib = L
    return _lib


def declared_functions():
    """Names of the functions include/lsp.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsp_[a-z_0-9]+)\s*\(", text)))


def set_stage_events(begin, end):
    """Record caller-owned hipEvent_t handles around the main kernel of later
    calls from this thread (None, None to stop)."""
    st = lib().lsp_set_stage_events(begin, end)
    if st != OK:
        raise LspError(st, "lsp_set_stage_events")


def describe_launch(n_obj, n_obs, grid, opt, generalized=False):
    """The launch shape a whole-grid call resolves (lsp_describe_launch):
    a dict with the resolved k_per_lane, waves_per_wg, t_split, schedule,
    recurrence, wave_split, obs_read, seed_trig, tile_freqs, tiles_per_item and
    n_items."""
    out = Options()
    tf, tpi, ni = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    st = lib().lsp_describe_launch(int(n_obj), int(n_obs), ctypes.byref(grid), ctypes.byref(opt),
                                   int(bool(generalized)), ctypes.byref(out), ctypes.byref(tf),
                                   ctypes.byref(tpi), ctypes.byref(ni))
    if st != OK:
        raise LspError(st, "lsp_describe_launch")
    d = {name: int(getattr(out, name)) for name, _ in Options._fields_}
    d["tile_freqs"], d["tiles_per_item"], d["n_items"] = int(tf.value), int(tpi.value), \
        int(ni.value)
    return d


def row_order(offsets, row_obj=None, row_band=None, rows_per_group=1, n_rows=None,
              stream=None):
    """lsp_row_order: the longest-first rank -> row permutation (int32 device
    tensor) of the rows of a batch, as the batch calls use it with
    ORDER_LPT."""
    _check(offsets, torch.int64, "offsets")
    n_obj = int(offsets.numel()) - 1
    if row_obj is not None:
        _check(row_obj, torch.int32, "row_obj")
        n_rows = int(row_obj.numel())
    elif n_rows is None:
        n_rows = n_obj * int(rows_per_group)
    if row_band is not None:
        _check(row_band, torch.int32, "row_band")
    perm = torch.empty(int(n_rows), dtype=torch.int32, device=offsets.device)
    nb = int(lib().lsp_row_order_workspace_bytes())
    ws = torch.empty(nb, dtype=torch.uint8, device=offsets.device)
    st = lib().lsp_row_order(_dev_ptr(offsets), n_obj, _dev_ptr(row_obj), _dev_ptr(row_band),
                             int(n_rows), int(rows_per_group), _dev_ptr(perm), _dev_ptr(ws), nb,
                             _stream_handle(stream))
    if st != OK:
        raise LspError(st, "lsp_row_order")
    return perm


def status_string(status):
    return lib().lsp_status_string(int(status)).decode()


def default_options():
    return lib().lsp_default_options()


def make_grid(f_min, f_max, n_f, unit=CYCLES):
    return Grid(float(f_min), float(f_max), int(n_f), int(unit), 0)


def make_options(form=FORM_FP64, normalize=True, subtract_mean=True, pgram_dtype=PGRAM_F32, k=0,
                 waves=0, t_split=0, schedule=SCHED_AUTO, recurrence=REC_AUTO,
                 wave_split=WSPLIT_AUTO, obs_read=0, seed_trig=0, order=ORDER_AUTO):
    o = Options()
    o.form, o.normalize, o.subtract_mean, o.pgram_dtype = (int(form), int(bool(normalize)),
                                                           int(bool(subtract_mean)),
                                                           int(pgram_dtype))
    o.k_per_lane, o.waves_per_wg, o.t_split, o.schedule = int(k), int(waves), int(t_split), int(
        schedule)
    o.recurrence = int(recurrence)
    o.wave_split = int(wave_split)
    o.obs_read = int(obs_read)
    o.seed_trig = int(seed_trig)
    o.order = int(order)
    return o


def workspace_bytes(n_obj, n_obs, grid, opt):
    return int(lib().lsp_workspace_bytes(int(n_obj), int(n_obs), ctypes.byref(grid),
                                         ctypes.byref(opt)))


def gen_workspace_bytes(n_obj, n_obs, grid, opt):
    return int(lib().lsp_gen_workspace_bytes(int(n_obj), int(n_obs), ctypes.byref(grid),
                                             ctypes.byref(opt)))


def _dev_ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _check(x, dtype, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor (the library has no CPU path)")
    if x.dtype != dtype or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Periodogram:
    """A periodogram call with its outputs and workspace allocated once.

    Calling the object enqueues the library's kernels on the stream and
    allocates nothing, so it can be timed in a loop or captured in a graph.
    ``offsets=None`` selects single-periodogram mode (lsp_single).
    ``method="generalized"`` selects the generalized periodogram with errors
    ``dy`` (None: unit errors) and a floating mean (lsp_gen_single /
    lsp_gen_batch).
    """

    def __init__(self, t, y, f_min, f_max, n_f, offsets=None, unit=CYCLES, form=FORM_FP64,
                 normalize=True, subtract_mean=True, pgram=True, pgram_dtype=PGRAM_F32,
                 peaks=True, k=0, waves=0, t_split=0, schedule=SCHED_AUTO,
                 recurrence=REC_AUTO, wave_split=WSPLIT_AUTO, method="standard", dy=None,
                 obs_read=0, seed_trig=0, order=ORDER_AUTO):
        _check(t, torch.float64, "t")
        _check(y, torch.float64, "y")
        if t.numel() != y.numel():
            raise ValueError("t and y differ in length")
        if offsets is not None:
            _check(offsets, torch.int64, "offsets")
        if method not in ("standard", "generalized"):
            raise ValueError(f"unknown method {method!r}")
        self.gen = method == "generalized"
        if dy is not None:
            if not self.gen:
                raise ValueError("errors dy are used by the generalized method only")
            _check(dy, torch.float64, "dy")
            if dy.numel() != t.numel():
                raise ValueError("dy and t differ in length")
        self.dy = dy
        self.t, self.y, self.offsets = t, y, offsets
        self.n_obs = int(t.numel())
        self.n_obj = 1 if offsets is None else int(offsets.numel()) - 1
        self.grid = make_grid(f_min, f_max, n_f, unit)
        self.opt = make_options(form, normalize, subtract_mean, pgram_dtype, k, waves, t_split,
                                schedule, recurrence, wave_split, obs_read, seed_trig, order)
        dev = t.device
        nb = (gen_workspace_bytes if self.gen else workspace_bytes)(self.n_obj, self.n_obs,
                                                                   self.grid, self.opt)
        if nb == 0:
            raise LspError(EINVAL, "lsp_gen_workspace_bytes" if self.gen
                           else "lsp_workspace_bytes")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
        pdt = torch.float64 if pgram_dtype == PGRAM_F64 else torch.float32
        self.pgram = (torch.empty((self.n_obj, int(n_f)), dtype=pdt, device=dev)
                      if pgram else None)
        self.peaks_raw = (torch.empty(self.n_obj * PEAK_BYTES, dtype=torch.uint8, device=dev)
                          if peaks else None)

    def __call__(self, stream=None):
        L = lib()
        s = _stream_handle(stream)
        ws = self.workspace
        if self.gen and self.offsets is None:
            st = L.lsp_gen_single(_dev_ptr(self.t), _dev_ptr(self.y), _dev_ptr(self.dy),
                                  self.n_obs, ctypes.byref(self.grid), ctypes.byref(self.opt),
                                  _dev_ptr(self.pgram), _dev_ptr(self.peaks_raw), _dev_ptr(ws),
                                  ws.numel(), s)
            what = "lsp_gen_single"
        elif self.gen:
            st = L.lsp_gen_batch(_dev_ptr(self.offsets), self.n_obj, self.n_obs,
                                 _dev_ptr(self.t), _dev_ptr(self.y), _dev_ptr(self.dy),
                                 ctypes.byref(self.grid), ctypes.byref(self.opt),
                                 _dev_ptr(self.pgram), _dev_ptr(self.peaks_raw), _dev_ptr(ws),
                                 ws.numel(), s)
            what = "lsp_gen_batch"
        elif self.offsets is None:
            st = L.lsp_single(_dev_ptr(self.t), _dev_ptr(self.y), self.n_obs,
                              ctypes.byref(self.grid), ctypes.byref(self.opt),
                              _dev_ptr(self.pgram), _dev_ptr(self.peaks_raw), _dev_ptr(ws),
                              ws.numel(), s)
            what = "lsp_single"
        else:
            st = L.lsp_batch(_dev_ptr(self.offsets), self.n_obj, self.n_obs, _dev_ptr(self.t),
                             _dev_ptr(self.y), ctypes.byref(self.grid), ctypes.byref(self.opt),
                             _dev_ptr(self.pgram), _dev_ptr(self.peaks_raw), _dev_ptr(ws),
                             ws.numel(), s)
            what = "lsp_batch"
        if st != OK:
            raise LspError(st, what)
        return self

    def launch(self):
        """The launch shape this call resolves (see describe_launch)."""
        return describe_launch(self.n_obj, self.n_obs, self.grid, self.opt, self.gen)

    def capture(self):
        """Record this call into a HIP graph (lsp_plan_create or
        lsp_gen_plan_create); returns a Plan."""
        return Plan(self)

    def peaks(self):
        """Peak records copied to the host as a numpy structured array."""
        if self.peaks_raw is None:
            return None
        return self.peaks_raw.cpu().numpy().view(PEAK_DTYPE).copy()


class HostPipe:
    """Streams, pinned staging buffers and copy threads for returning batch
    periodograms to host memory (lsp_pipe_create / lsp_batch_to_host).

    Zero arguments take the library's defaults (1 lane, 16 MiB staging per
    lane, 128 MiB chunks, 12 copy threads)."""

    def __init__(self, n_streams=0, staging_bytes=0, chunk_bytes=0, copy_threads=0):
        h = ctypes.c_void_p()
        st = lib().lsp_pipe_create(int(n_streams), int(staging_bytes), int(chunk_bytes),
                                   int(copy_threads), ctypes.byref(h))
        if st != OK:
            raise LspError(st, "lsp_pipe_create")
        self.handle = h

    def batch_to_host(self, offsets, t, y, f_min, f_max, n_f, dy=None, method="standard",
                      unit=CYCLES, pgram=True, peaks=True, stream=None, out=None, **opts):
        """Batch periodograms (and peaks) into host memory.  Returns
        (pgram numpy [n_obj, n_f] or None, peak records or None); ``out`` may
        supply the host array."""
        _check(offsets, torch.int64, "offsets")
        _check(t, torch.float64, "t")
        _check(y, torch.float64, "y")
        gen = method == "generalized"
        if dy is not None:
            _check(dy, torch.float64, "dy")
        n_obj = int(offsets.numel()) - 1
        grid = make_grid(f_min, f_max, n_f, unit)
        opt = make_options(**opts)
        dt = np.float64 if opt.pgram_dtype == PGRAM_F64 else np.float32
        if pgram and out is None:
            out = np.empty((n_obj, int(n_f)), dtype=dt)
        if pgram and (out.dtype != dt or out.shape != (n_obj, int(n_f))
                      or not out.flags["C_CONTIGUOUS"]):
            raise ValueError("out must be a C-contiguous host array of the periodogram's shape")
        pk = np.zeros(n_obj, dtype=PEAK_DTYPE) if peaks else None
        st = lib().lsp_batch_to_host(self.handle, _dev_ptr(offsets), n_obj, int(t.numel()),
                                     _dev_ptr(t), _dev_ptr(y), _dev_ptr(dy), int(gen),
                                     ctypes.byref(grid), ctypes.byref(opt),
                                     out.ctypes.data_as(ctypes.c_void_p) if pgram else None,
                                     pk.ctypes.data_as(ctypes.c_void_p) if peaks else None,
                                     _stream_handle(stream))
        if st != OK:
            raise LspError(st, "lsp_batch_to_host")
        return (out if pgram else None), pk

    def close(self):
        if getattr(self, "handle", None):
            lib().lsp_pipe_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A captured call (lsp_plan_*): launching it replays all of the call's
    kernels as one HIP graph on the given stream."""

    def __init__(self, call):
        self.call = call
        h = ctypes.c_void_p()
        if getattr(call, "gen", False):
            st = lib().lsp_gen_plan_create(_dev_ptr(call.offsets), call.n_obj, call.n_obs,
                                           _dev_ptr(call.t), _dev_ptr(call.y), _dev_ptr(call.dy),
                                           ctypes.byref(call.grid), ctypes.byref(call.opt),
                                           _dev_ptr(call.pgram), _dev_ptr(call.peaks_raw),
                                           _dev_ptr(call.workspace), call.workspace.numel(),
                                           ctypes.byref(h))
        else:
            st = lib().lsp_plan_create(_dev_ptr(call.offsets), call.n_obj, call.n_obs,
                                       _dev_ptr(call.t), _dev_ptr(call.y), ctypes.byref(call.grid),
                                       ctypes.byref(call.opt), _dev_ptr(call.pgram),
                                       _dev_ptr(call.peaks_raw), _dev_ptr(call.workspace),
                                       call.workspace.numel(), ctypes.byref(h))
        if st != OK:
            raise LspError(st, "lsp_plan_create")
        self.handle = h

    def __call__(self, stream=None):
        st = lib().lsp_plan_launch(self.handle, _stream_handle(stream))
        if st != OK:
            raise LspError(st, "lsp_plan_launch")
        return self.call

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            lib().lsp_plan_destroy(h)
            self.handle = None


class Rows:
    """A row-mode call (lsp_batch_rows) with its workspace allocated once.

    ``row_obj`` (int32 device tensor) names the object of each row;
    ``row_band`` (int32 device tensor or None) its band of ``band_bins`` bins.
    Groups of ``rows_per_group`` consecutive rows share one peak record, written
    at the group's object in ``peaks`` (an n_obj-record tensor the caller may
    pass in so that several calls fill one array).  ``pgram`` likewise may be
    passed in; only the rows' bins are written.
    """

    def __init__(self, offsets, t, y, f_min, f_max, n_f, row_obj, row_band=None, band_bins=0,
                 rows_per_group=1, unit=CYCLES, form=FORM_FP32P, normalize=True,
                 subtract_mean=True, pgram=None, pgram_dtype=PGRAM_F32, peaks=None, k=0,
                 waves=0, schedule=SCHED_AUTO, recurrence=REC_AUTO, max_rows=None,
                 method="standard", dy=None, order=ORDER_AUTO):
        for x, dt, nm in ((t, torch.float64, "t"), (y, torch.float64, "y"),
                          (offsets, torch.int64, "offsets")):
            _check(x, dt, nm)
        if row_obj is not None:
            _check(row_obj, torch.int32, "row_obj")
        if row_band is not None:
            _check(row_band, torch.int32, "row_band")
        if row_obj is None and row_band is None:
            raise ValueError("row mode needs row_obj, row_band or both")
        if method not in ("standard", "generalized"):
            raise ValueError(f"unknown method {method!r}")
        self.gen = method == "generalized"
        if dy is not None:
            if not self.gen:
                raise ValueError("errors dy are used by the generalized method only")
            _check(dy, torch.float64, "dy")
        self.dy = dy
        self.t, self.y, self.offsets = t, y, offsets
        self.n_obs = int(t.numel())
        self.n_obj = int(offsets.numel()) - 1
        self.grid = make_grid(f_min, f_max, n_f, unit)
        self.opt = make_options(form, normalize, subtract_mean, pgram_dtype, k, waves, 0,
                                schedule, recurrence, order=order)
        self.band_bins = int(band_bins) if row_band is not None else 0
        self.rows_per_group = int(rows_per_group)
        named = row_obj if row_obj is not None else row_band
        cap = int(max_rows if max_rows is not None else named.numel())
        size_fn = lib().lsp_gen_rows_workspace_bytes if self.gen else lib().lsp_rows_workspace_bytes
        nb = int(size_fn(self.n_obj, self.n_obs, ctypes.byref(self.grid), ctypes.byref(self.opt),
                         max(cap, 1), self.band_bins, self.rows_per_group))
        if nb == 0:
            raise LspError(EINVAL, "lsp_rows_workspace_bytes")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=t.device)
        self.pgram = pgram
        self.peaks_raw = (torch.empty(self.n_obj * PEAK_BYTES, dtype=torch.uint8,
                                      device=t.device) if peaks is None else peaks)
        self.set_rows(row_obj, row_band)

    def set_rows(self, row_obj, row_band=None):
        """Point the call at new row arrays (no more rows than the sized maximum).
        With row_obj None, row r belongs to object r // rows_per_group."""
        if row_obj is not None and row_band is not None and row_band.numel() != row_obj.numel():
            raise ValueError("row_obj and row_band differ in length")
        self.row_obj, self.row_band = row_obj, row_band
        self.n_rows = int((row_obj if row_obj is not None else row_band).numel())
        return self

    def __call__(self, stream=None):
        if self.n_rows == 0:
            return self
        if self.gen:
            st = lib().lsp_gen_batch_rows(_dev_ptr(self.offsets), self.n_obj, self.n_obs,
                                          _dev_ptr(self.t), _dev_ptr(self.y), _dev_ptr(self.dy),
                                          ctypes.byref(self.grid), ctypes.byref(self.opt),
                                          _dev_ptr(self.row_obj), _dev_ptr(self.row_band),
                                          self.n_rows, self.band_bins, self.rows_per_group,
                                          _dev_ptr(self.pgram), _dev_ptr(self.peaks_raw),
                                          _dev_ptr(self.workspace), self.workspace.numel(),
                                          _stream_handle(stream))
        else:
            st = lib().lsp_batch_rows(_dev_ptr(self.offsets), self.n_obj, self.n_obs,
                                      _dev_ptr(self.t), _dev_ptr(self.y), ctypes.byref(self.grid),
                                      ctypes.byref(self.opt), _dev_ptr(self.row_obj),
                                      _dev_ptr(self.row_band), self.n_rows, self.band_bins,
                                      self.rows_per_group, _dev_ptr(self.pgram),
                                      _dev_ptr(self.peaks_raw), _dev_ptr(self.workspace),
                                      self.workspace.numel(), _stream_handle(stream))
        if st != OK:
            raise LspError(st, "lsp_gen_batch_rows" if self.gen else "lsp_batch_rows")
        return self

    def peaks(self):
        return self.peaks_raw.cpu().numpy().view(PEAK_DTYPE).copy()


class Features:
    """Band-proposal features (lsp_features) with the workspace allocated once:
    calling it fills ``out`` ([n_obj, FEAT_DIM] float32) for the CSR batch."""

    def __init__(self, offsets, t, y, f_min, f_max, unit=CYCLES, season_gap=60.0,
                 min_season_obs=8, out=None):
        for x, dt, nm in ((t, torch.float64, "t"), (y, torch.float64, "y"),
                          (offsets, torch.int64, "offsets")):
            _check(x, dt, nm)
        self.offsets, self.t, self.y = offsets, t, y
        self.n_obj = int(offsets.numel()) - 1
        self.n_obs = int(t.numel())
        self.grid = make_grid(f_min, f_max, 1, unit)
        self.fopt = FeatureOptions()
        self.fopt.season_gap = float(season_gap)
        self.fopt.min_season_obs = int(min_season_obs)
        nb = int(lib().lsp_features_workspace_bytes(self.n_obj))
        if nb == 0:
            raise LspError(EINVAL, "lsp_features_workspace_bytes")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=t.device)
        if out is None:
            out = torch.empty((self.n_obj, FEAT_DIM), dtype=torch.float32, device=t.device)
        _check(out, torch.float32, "out")
        if out.numel() != self.n_obj * FEAT_DIM:
            raise ValueError("out must hold n_obj * FEAT_DIM floats")
        self.out = out

    def __call__(self, stream=None):
        st = lib().lsp_features(_dev_ptr(self.offsets), self.n_obj, self.n_obs, _dev_ptr(self.t),
                                _dev_ptr(self.y), ctypes.byref(self.grid),
                                ctypes.byref(self.fopt), _dev_ptr(self.out),
                                _dev_ptr(self.workspace), self.workspace.numel(),
                                _stream_handle(stream))
        if st != OK:
            raise LspError(st, "lsp_features")
        return self.out


def autotune(t, y, f_min, f_max, n_f, offsets=None, unit=CYCLES, normalize=True,
             subtract_mean=True, cache_path=None, repeats=3, stream=None):
    """Run lsp_autotune on device data; returns the tuned keyword options
    (k, waves, recurrence, schedule, t_split, wave_split) for Periodogram(form=FORM_FP32P)."""
    _check(t, torch.float64, "t")
    _check(y, torch.float64, "y")
    if offsets is not None:
        _check(offsets, torch.int64, "offsets")
    n_obj = 1 if offsets is None else int(offsets.numel()) - 1
    grid = make_grid(f_min, f_max, n_f, unit)
    base = make_options(FORM_FP32P, normalize, subtract_mean)
    nb = int(lib().lsp_autotune_workspace_bytes(n_obj, int(t.numel()), ctypes.byref(grid),
                                                ctypes.byref(base)))
    if nb == 0:
        raise LspError(EINVAL, "lsp_autotune_workspace_bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device=t.device)
    scratch = torch.empty(n_obj * PEAK_BYTES, dtype=torch.uint8, device=t.device)
    tuned = Options()
    st = lib().lsp_autotune(_dev_ptr(offsets), n_obj, int(t.numel()), _dev_ptr(t), _dev_ptr(y),
                            ctypes.byref(grid), ctypes.byref(base), ctypes.byref(tuned),
                            _dev_ptr(scratch), _dev_ptr(ws), nb,
                            cache_path.encode() if cache_path else None, int(repeats),
                            _stream_handle(stream))
    if st != OK:
        raise LspError(st, "lsp_autotune")
    return dict(k=tuned.k_per_lane, waves=tuned.waves_per_wg, recurrence=tuned.recurrence,
                schedule=tuned.schedule, t_split=tuned.t_split, wave_split=tuned.wave_split)


def batch_static(offsets, t, y, f_min, f_max, n_f, pgram=None, peaks=None, unit=CYCLES,
                 stream=None, **opts):
    """lsp_batch_static: lsp_batch with the library's static scratch instead of
    a workspace (nothing is allocated by the call).  pgram / peaks are caller
    tensors (a [n_obj, n_f] periodogram of the options' dtype, n_obj * 40
    bytes of peak records); returns the status (raises on anything but OK)."""
    _check(t, torch.float64, "t")
    _check(y, torch.float64, "y")
    _check(offsets, torch.int64, "offsets")
    grid = make_grid(f_min, f_max, n_f, unit)
    opt = make_options(**opts)
    st = lib().lsp_batch_static(_dev_ptr(offsets), int(offsets.numel()) - 1, int(t.numel()),
                                _dev_ptr(t), _dev_ptr(y), ctypes.byref(grid), ctypes.byref(opt),
                                _dev_ptr(pgram), _dev_ptr(peaks), _stream_handle(stream))
    if st != OK:
        raise LspError(st, "lsp_batch_static")
    return st


def single(t, y, f_min, f_max, n_f, **kw):
    """One series (Section 3.3); returns (pgram[n_f] tensor or None, peak record)."""
    p = Periodogram(t, y, f_min, f_max, n_f, offsets=None, **kw)()
    pk = p.peaks()
    return (p.pgram[0] if p.pgram is not None else None), (pk[0] if pk is not None else None)


def batch(offsets, t, y, f_min, f_max, n_f, **kw):
    """CSR batch (Section 3.4); returns (pgram[n_obj, n_f] tensor or None, peaks array)."""
    p = Periodogram(t, y, f_min, f_max, n_f, offsets=offsets, **kw)()
    return p.pgram, p.peaks()


def gen_single(t, y, dy, f_min, f_max, n_f, **kw):
    """Generalized periodogram of one series (Section 4.11); dy may be None."""
    p = Periodogram(t, y, f_min, f_max, n_f, offsets=None, method="generalized", dy=dy, **kw)()
    pk = p.peaks()
    return (p.pgram[0] if p.pgram is not None else None), (pk[0] if pk is not None else None)


def gen_batch(offsets, t, y, dy, f_min, f_max, n_f, **kw):
    """Generalized periodogram of a CSR batch (Section 4.11); dy may be None."""
    p = Periodogram(t, y, f_min, f_max, n_f, offsets=offsets, method="generalized", dy=dy, **kw)()
    return p.pgram, p.peaks()
