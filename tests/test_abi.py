"""The C ABI library loads, exports what include/lsp.h declares, and rejects bad
arguments on the host before touching a device (no GPU needed)."""
import ctypes

import pytest

from paper_2105_04006_amd import lsp


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


# Several tests pass a fake device address that every call must reject during
# host-side validation; a mistake in such a test would launch a kernel on it.
# They run only where no GPU is visible.
cpu_only = pytest.mark.skipif(_gpu_visible(), reason="fake device pointers: CPU-only check")


@pytest.fixture(scope="module")
def L():
    return lsp.lib()


def test_exports_every_declared_function(L):
    names = lsp.declared_functions()
    assert {"lsp_single", "lsp_batch", "lsp_workspace_bytes", "lsp_status_string",
            "lsp_default_options", "lsp_version"} <= set(names)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/lsp.h but not exported"


def test_struct_sizes_match_header(tmp_path):
    assert ctypes.sizeof(lsp.Grid) == 32
    assert ctypes.sizeof(lsp.Options) == 56
    assert lsp.PEAK_DTYPE.itemsize == lsp.PEAK_BYTES == 40
    assert ctypes.sizeof(lsp.FeatureOptions) == 16
    # the ctypes mirrors against the header itself, field by field
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields = [name for name, _ in lsp.Options._fields_]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lsp.h"\nint main(void) {\n'
                   '  printf("%zu %zu %zu %zu\\n", sizeof(lsp_grid), sizeof(lsp_options), '
                   'sizeof(lsp_peak), sizeof(lsp_feature_options));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(lsp_options, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c11", "-I", str(lsp.HEADER.rsplit("/", 1)[0]), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert [int(v) for v in out[:4]] == [ctypes.sizeof(lsp.Grid), ctypes.sizeof(lsp.Options),
                                         lsp.PEAK_BYTES, ctypes.sizeof(lsp.FeatureOptions)]
    assert [int(v) for v in out[4:]] == [getattr(lsp.Options, f).offset for f in fields]


def test_feature_constants_match_header():
    import re
    text = open(lsp.HEADER).read()
    for name, val in (("LSP_FEAT_COARSE", lsp.FEAT_COARSE), ("LSP_FEAT_POOL", lsp.FEAT_POOL),
                      ("LSP_FEAT_WINDOW", lsp.FEAT_WINDOW)):
        assert int(re.search(rf"#define {name} (\d+)", text).group(1)) == val
    from oracle import features_ref
    assert (features_ref.COARSE, features_ref.POOL, features_ref.WINDOW) == (
        lsp.FEAT_COARSE, lsp.FEAT_POOL, lsp.FEAT_WINDOW)


@cpu_only
def test_feature_argument_errors(L):
    g = lsp.make_grid(1.0, 12.0, 1)
    fo = L.lsp_default_feature_options()
    assert (fo.season_gap, fo.min_season_obs) == (60.0, 8)
    nb = L.lsp_features_workspace_bytes(10)
    assert nb >= 10 * 64 and nb % 256 == 0
    assert L.lsp_features_workspace_bytes(0) == 0

    def call(offsets=FAKE, n_obj=10, grid=g, fopt=fo, out=FAKE, ws=FAKE, ws_bytes=nb):
        return L.lsp_features(offsets, n_obj, 100, FAKE, FAKE, ctypes.byref(grid),
                              ctypes.byref(fopt), out, ws, ws_bytes, None)

    assert call(offsets=None) == lsp.EINVAL
    assert call(out=None) == lsp.EINVAL
    assert call(ws=None) == lsp.EINVAL
    assert call(n_obj=0) == lsp.EINVAL
    assert call(grid=lsp.make_grid(2.0, 1.0, 1)) == lsp.EINVAL
    assert call(ws=ctypes.c_void_p((1 << 20) + 8)) == lsp.EINVAL
    assert call(ws_bytes=nb - 1) == lsp.ENOMEM
    bad = lsp.FeatureOptions()
    bad.season_gap, bad.min_season_obs = -1.0, 8
    assert call(fopt=bad) == lsp.EINVAL
    bad.season_gap, bad.min_season_obs = 60.0, 0
    assert call(fopt=bad) == lsp.EINVAL
    bad.min_season_obs = 1          # a one-point group has no periodogram
    assert call(fopt=bad) == lsp.EINVAL
    bad.season_gap = float("nan")
    bad.min_season_obs = 8
    assert call(fopt=bad) == lsp.EINVAL


def test_default_options(L):
    o = lsp.default_options()
    assert (o.form, o.normalize, o.subtract_mean, o.pgram_dtype) == (lsp.FORM_FP64, 1, 1, 0)
    assert L.lsp_version() == 100


def test_status_strings():
    assert lsp.status_string(lsp.OK) == "ok"
    assert "workspace" in lsp.status_string(lsp.ENOMEM)
    assert lsp.status_string(99) == "unknown status"


def test_workspace_bytes():
    g = lsp.make_grid(1.0, 12.0, 10_000)
    for form in (lsp.FORM_FP64, lsp.FORM_FP32P):
        o = lsp.make_options(form=form)
        nb = lsp.workspace_bytes(1, 256, g, o)
        assert nb > 0 and nb % 256 == 0
        assert lsp.workspace_bytes(100, 50_000, g, o) > nb
    assert lsp.workspace_bytes(0, 10, g, lsp.make_options()) == 0
    assert lsp.workspace_bytes(1, 10, lsp.make_grid(2.0, 1.0, 10), lsp.make_options()) == 0
    assert lsp.workspace_bytes(1, 10, g, lsp.make_options(form=7)) == 0


FAKE = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: every call below fails validation


def _single(L, t=FAKE, y=FAKE, n=16, grid=None, opt=None, pgram=FAKE, peak=FAKE, ws=FAKE,
            nbytes=1 << 30):
    grid = grid or lsp.make_grid(1.0, 2.0, 100)
    opt = opt or lsp.make_options()
    return L.lsp_single(t, y, n, ctypes.byref(grid), ctypes.byref(opt), pgram, peak, ws, nbytes,
                        None)


@cpu_only
def test_argument_errors_are_reported_before_any_launch(L):
    assert _single(L, t=None) == lsp.EINVAL
    assert _single(L, ws=None) == lsp.EINVAL
    assert _single(L, n=-1) == lsp.EINVAL
    assert _single(L, pgram=None, peak=None) == lsp.EINVAL
    assert _single(L, ws=ctypes.c_void_p((1 << 20) + 8)) == lsp.EINVAL  # misaligned
    assert _single(L, nbytes=1) == lsp.ENOMEM
    for g in (lsp.make_grid(2.0, 1.0, 10), lsp.make_grid(1.0, 2.0, 0),
              lsp.make_grid(float("nan"), 2.0, 10), lsp.make_grid(1.0, float("inf"), 10),
              lsp.make_grid(1.0, 2.0, 10, unit=5)):
        assert _single(L, grid=g) == lsp.EINVAL
    bad_norm = lsp.make_options()
    bad_norm.normalize = 2
    bad_mean = lsp.make_options()
    bad_mean.subtract_mean = -1
    for o in (lsp.make_options(form=3), lsp.make_options(pgram_dtype=2), bad_norm, bad_mean,
              lsp.make_options(k=3), lsp.make_options(form=lsp.FORM_FP32P, k=2),
              lsp.make_options(waves=3), lsp.make_options(t_split=65),
              lsp.make_options(schedule=9), lsp.make_options(order=3),
              lsp.make_options(order=-1)):
        assert _single(L, opt=o) == lsp.EINVAL
    assert _single(L, opt=lsp.make_options(t_split=2)) == lsp.EUNSUPPORTED
    assert _single(L, opt=lsp.make_options(schedule=lsp.SCHED_PERSISTENT)) == lsp.EUNSUPPORTED
    g = lsp.make_grid(1.0, 2.0, 100)
    o = lsp.make_options(form=lsp.FORM_FP32P, t_split=2)
    assert L.lsp_batch(FAKE, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE, FAKE, FAKE,
                       1 << 30, None) == lsp.EUNSUPPORTED
    o = lsp.make_options()
    assert L.lsp_batch(None, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE, FAKE, FAKE,
                       1 << 30, None) == lsp.EINVAL
    assert L.lsp_batch(FAKE, 0, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE, FAKE, FAKE,
                       1 << 30, None) == lsp.EINVAL


@cpu_only
def test_plan_and_autotune_argument_errors(L):
    g = lsp.make_grid(1.0, 2.0, 100)
    o = lsp.make_options()
    h = ctypes.c_void_p()
    assert L.lsp_plan_create(FAKE, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                             FAKE, FAKE, 1 << 30, None) == lsp.EINVAL  # no plan pointer
    assert L.lsp_plan_create(None, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                             FAKE, FAKE, 1 << 30, ctypes.byref(h)) == lsp.EINVAL  # batch w/o CSR
    assert L.lsp_plan_create(FAKE, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                             FAKE, FAKE, 1, ctypes.byref(h)) == lsp.ENOMEM
    assert not h.value
    assert L.lsp_plan_launch(None, None) == lsp.EINVAL
    L.lsp_plan_destroy(None)
    tuned = lsp.Options()
    assert L.lsp_autotune(FAKE, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), None, FAKE,
                          FAKE, 1 << 30, None, 1, None) == lsp.EINVAL
    assert L.lsp_autotune(FAKE, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o),
                          ctypes.byref(tuned), FAKE, FAKE, 1 << 30, None, 0, None) == lsp.EINVAL
    assert lsp.lib().lsp_autotune_workspace_bytes(3, 30, ctypes.byref(g), ctypes.byref(o)) > 0


@cpu_only
def test_rows_argument_errors(L):
    g = lsp.make_grid(1.0, 2.0, 100)
    o = lsp.make_options(form=lsp.FORM_FP32P)

    def call(offsets=FAKE, row_obj=FAKE, row_band=FAKE, n_rows=8, band_bins=10, rpg=4, opt=o,
             ws_bytes=1 << 30):
        return L.lsp_batch_rows(offsets, 3, 30, FAKE, FAKE, ctypes.byref(g), ctypes.byref(opt),
                                row_obj, row_band, n_rows, band_bins, rpg, FAKE, FAKE, FAKE,
                                ws_bytes, None)

    assert call(offsets=None) == lsp.EINVAL
    assert call(row_obj=None) == lsp.EINVAL           # 8 rows != 3 objects * 4
    assert call(row_obj=None, n_rows=12, ws_bytes=1) == lsp.ENOMEM  # 12 == 3 * 4: accepted
    assert call(n_rows=0) == lsp.EINVAL
    assert call(rpg=0) == lsp.EINVAL
    assert call(rpg=3) == lsp.EINVAL        # 3 does not divide 8 rows
    assert call(band_bins=0) == lsp.EINVAL
    assert call(band_bins=101) == lsp.EINVAL
    assert call(ws_bytes=1) == lsp.ENOMEM
    assert call(opt=lsp.make_options(form=lsp.FORM_FP32P, t_split=2)) == lsp.EUNSUPPORTED
    ws = L.lsp_rows_workspace_bytes
    assert ws(3, 30, ctypes.byref(g), ctypes.byref(o), 8, 10, 4) > 0
    assert ws(3, 30, ctypes.byref(g), ctypes.byref(o), 8, 0, 1) > 0       # whole-grid rows
    assert ws(3, 30, ctypes.byref(g), ctypes.byref(o), 8, 10, 3) == 0
    assert ws(3, 30, ctypes.byref(g), ctypes.byref(o), 0, 10, 1) == 0
    # records grow with rows, not with objects
    assert (ws(3, 30, ctypes.byref(g), ctypes.byref(o), 800, 10, 4) >
            ws(3, 30, ctypes.byref(g), ctypes.byref(o), 8, 10, 4))


def test_binding_refuses_cpu_tensors():
    import torch

    t = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(TypeError):
        lsp.Periodogram(t, t, 1.0, 2.0, 10)


@cpu_only
def test_network_helper_argument_errors(L):
    f32 = ctypes.c_float
    assert L.lsp_band_max(FAKE, 4, 1088, 0, 64, 18, FAKE, None) == lsp.EINVAL   # past d
    assert L.lsp_band_max(None, 4, 1088, 0, 64, 16, FAKE, None) == lsp.EINVAL
    assert L.lsp_band_max(FAKE, 0, 1088, 0, 64, 16, None, None) == lsp.OK       # nothing to do
    assert L.lsp_merge_bands(FAKE, 4, FAKE, 8, 10, 0, FAKE, None) == lsp.EINVAL
    assert L.lsp_merge_bands(FAKE, 4, FAKE, 8, 10, 129, FAKE, None) == lsp.EINVAL
    assert L.lsp_merge_bands(None, 4, FAKE, 8, 10, 8, FAKE, None) == lsp.EINVAL
    assert L.lsp_row_normalize(FAKE, 4, 1088, 100, 1000, None) == lsp.EINVAL    # past d
    assert L.lsp_row_normalize(FAKE, 4, 1088, 0, 0, None) == lsp.EINVAL
    assert L.lsp_pool_stats(None, FAKE, 0, 16, None) == lsp.EINVAL
    assert L.lsp_pool_stats(FAKE, FAKE, 0, 0, None) == lsp.EINVAL
    # group * n_bands must equal n_coarse
    assert L.lsp_shift_bands(FAKE, FAKE, FAKE, 8, 1088, 1024, 15, 64, f32(0), FAKE, FAKE,
                             None) == lsp.EINVAL
    assert L.lsp_shift_bands(FAKE, FAKE, FAKE, 8, 1000, 1024, 16, 64, f32(0), FAKE, FAKE,
                             None) == lsp.EINVAL
    assert L.lsp_peak_bands(FAKE, 8, 0, 64, FAKE, None) == lsp.EINVAL
    assert L.lsp_select_fallback(FAKE, None, 8, f32(0), f32(0), FAKE, None, None) == lsp.EINVAL
    assert L.lsp_select_fallback(FAKE, None, 1 << 40, f32(0), f32(0), FAKE, FAKE,
                                 None) == lsp.EINVAL
    assert L.lsp_top_k(FAKE, 8, 129, 8, FAKE, None, None) == lsp.EINVAL
    assert L.lsp_top_k(FAKE, 8, 64, 65, FAKE, None, None) == lsp.EINVAL
    assert L.lsp_gemm_bf16(-1, 4, 4, FAKE, 4, 1, FAKE, 4, 1, None, None, 0, FAKE, None, 4,
                           None) == lsp.EINVAL


def test_gen_workspace_bytes():
    g = lsp.make_grid(0.5, 24.0, 500_000)
    o32 = lsp.make_options(form=lsp.FORM_FP32P)
    # one object on a long grid splits observations: 6 partial sums per bin
    # and split for the generalized form against 4 for the standard one
    assert lsp.gen_workspace_bytes(1, 4096, g, o32) > lsp.workspace_bytes(1, 4096, g, o32)
    for form in (lsp.FORM_FP64, lsp.FORM_FP32P):
        nb = lsp.gen_workspace_bytes(100, 50_000, g, lsp.make_options(form=form))
        assert nb > 0 and nb % 256 == 0
    assert lsp.gen_workspace_bytes(0, 10, g, o32) == 0
    assert lsp.gen_workspace_bytes(1, 10, lsp.make_grid(2.0, 1.0, 10), o32) == 0
    for o in (lsp.make_options(form=lsp.FORM_FP32P, recurrence=lsp.REC_ROTATION),
              lsp.make_options(form=lsp.FORM_FP32P, k=10),
              lsp.make_options(form=lsp.FORM_FP32P, k=32),
              lsp.make_options(form=lsp.FORM_FP32P, waves=4, wave_split=lsp.WSPLIT_ON)):
        assert lsp.gen_workspace_bytes(1, 4096, g, o) == 0
        assert lsp.workspace_bytes(1, 4096, g, o) > 0


@cpu_only
def test_gen_argument_errors(L):
    g = lsp.make_grid(1.0, 2.0, 100)

    def single(dy=FAKE, t=FAKE, n=16, opt=None, ws=FAKE, nbytes=1 << 30, pgram=FAKE, peak=FAKE):
        opt = opt or lsp.make_options()
        return L.lsp_gen_single(t, FAKE, dy, n, ctypes.byref(g), ctypes.byref(opt), pgram, peak,
                                ws, nbytes, None)

    assert single(t=None) == lsp.EINVAL
    assert single(ws=None) == lsp.EINVAL
    assert single(n=-1) == lsp.EINVAL
    assert single(pgram=None, peak=None) == lsp.EINVAL
    assert single(nbytes=1) == lsp.ENOMEM
    assert single(opt=lsp.make_options(form=9)) == lsp.EINVAL
    assert single(opt=lsp.make_options(t_split=2)) == lsp.EUNSUPPORTED  # FP64 form
    for o in (lsp.make_options(form=lsp.FORM_FP32P, recurrence=lsp.REC_ROTATION),
              lsp.make_options(form=lsp.FORM_FP32P, k=10),
              lsp.make_options(form=lsp.FORM_FP32P, waves=2, wave_split=lsp.WSPLIT_ON)):
        assert single(opt=o) == lsp.EUNSUPPORTED
        assert single(dy=None, opt=o) == lsp.EUNSUPPORTED
    o = lsp.make_options(form=lsp.FORM_FP32P)
    assert L.lsp_gen_batch(None, 3, 30, FAKE, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                           FAKE, FAKE, 1 << 30, None) == lsp.EINVAL
    assert L.lsp_gen_batch(FAKE, 0, 30, FAKE, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                           FAKE, FAKE, 1 << 30, None) == lsp.EINVAL
    assert L.lsp_gen_batch(FAKE, 3, 30, FAKE, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o), FAKE,
                           FAKE, FAKE, 1, None) == lsp.ENOMEM


@cpu_only
def test_pipe_argument_errors(L):
    h = ctypes.c_void_p()
    assert L.lsp_pipe_create(3, 0, 0, 0, None) == lsp.EINVAL
    for args in ((9, 0, 0, 0), (-1, 0, 0, 0), (3, 1000, 0, 0), (3, 5000, 0, 0),
                 (3, 0, 0, 65), (3, 0, 0, -2)):
        assert L.lsp_pipe_create(*args, ctypes.byref(h)) == lsp.EINVAL
        assert not h.value
    g = lsp.make_grid(1.0, 2.0, 100)
    o = lsp.make_options()
    assert L.lsp_batch_to_host(None, FAKE, 3, 30, FAKE, FAKE, None, 0, ctypes.byref(g),
                               ctypes.byref(o), FAKE, None, None) == lsp.EINVAL


def test_variant_options():
    g = lsp.make_grid(1.0, 12.0, 100_000)
    ok = lsp.make_options(form=lsp.FORM_FP32P, obs_read=lsp.OBS_DIRECT, seed_trig=lsp.TRIG_POLY)
    base = lsp.workspace_bytes(10, 5000, g, lsp.make_options(form=lsp.FORM_FP32P))
    # the direct read path adds the staged values: 24 bytes per observation
    assert lsp.workspace_bytes(10, 5000, g, ok) >= base + 24 * 5000
    for kw in (dict(form=lsp.FORM_FP64, obs_read=lsp.OBS_DIRECT),
               dict(form=lsp.FORM_FP64, seed_trig=lsp.TRIG_LIB),
               dict(form=lsp.FORM_FP32P, seed_trig=lsp.TRIG_LIB, recurrence=lsp.REC_ROTATION),
               dict(form=lsp.FORM_FP32P, obs_read=lsp.OBS_DIRECT, k=12),
               dict(form=lsp.FORM_FP32P, obs_read=lsp.OBS_DIRECT, waves=2),
               dict(form=lsp.FORM_FP32P, seed_trig=lsp.TRIG_POLY, waves=4,
                    wave_split=lsp.WSPLIT_ON)):
        assert lsp.workspace_bytes(10, 5000, g, lsp.make_options(**kw)) == 0, kw
    assert lsp.gen_workspace_bytes(10, 5000, g, ok) == 0
    for kw in (dict(obs_read=3), dict(obs_read=-1), dict(seed_trig=4)):
        assert lsp.workspace_bytes(10, 5000, g, lsp.make_options(form=lsp.FORM_FP32P, **kw)) == 0


@cpu_only
def test_gen_rows_and_plan_argument_errors(L):
    g = lsp.make_grid(1.0, 2.0, 100)
    o = lsp.make_options(form=lsp.FORM_FP32P)
    assert L.lsp_gen_batch_rows(None, 3, 30, FAKE, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o),
                                FAKE, FAKE, 8, 10, 4, FAKE, FAKE, FAKE, 1 << 30, None) == lsp.EINVAL
    assert L.lsp_gen_batch_rows(FAKE, 3, 30, FAKE, FAKE, FAKE, ctypes.byref(g), ctypes.byref(o),
                                FAKE, FAKE, 8, 10, 3, FAKE, FAKE, FAKE, 1 << 30, None) == lsp.EINVAL
    rot = lsp.make_options(form=lsp.FORM_FP32P, recurrence=lsp.REC_ROTATION)
    assert L.lsp_gen_batch_rows(FAKE, 3, 30, FAKE, FAKE, None, ctypes.byref(g),
                                ctypes.byref(rot), FAKE, FAKE, 8, 10, 4, FAKE, FAKE, FAKE,
                                1 << 30, None) == lsp.EUNSUPPORTED
    assert L.lsp_gen_rows_workspace_bytes(3, 30, ctypes.byref(g), ctypes.byref(o), 8, 10, 4) > 0
    assert L.lsp_gen_rows_workspace_bytes(3, 30, ctypes.byref(g), ctypes.byref(rot), 8, 10, 4) == 0
    h = ctypes.c_void_p()
    assert L.lsp_gen_plan_create(FAKE, 3, 30, FAKE, FAKE, None, ctypes.byref(g), ctypes.byref(o),
                                 FAKE, FAKE, FAKE, 1 << 30, None) == lsp.EINVAL
    assert L.lsp_gen_plan_create(FAKE, 3, 30, FAKE, FAKE, None, ctypes.byref(g), ctypes.byref(o),
                                 FAKE, FAKE, FAKE, 1, ctypes.byref(h)) == lsp.ENOMEM


def test_describe_launch_resolves_the_shape():
    """lsp_describe_launch reports the configuration the call would use: the
    cost model's K for the FP32 form, the single object's in-workgroup split
    (eight waves sharing each tile's bins) where it fills the chip and its
    observation split across workgroups where it does not, the persistent
    schedule for batches, and the caller's explicit choices."""
    g = lsp.make_grid(0.5, 24.0, 500_000)
    one = lsp.describe_launch(1, 4096, g, lsp.make_options(form=lsp.FORM_FP32P))
    assert one["k_per_lane"] in (8, 10, 12, 16) and one["schedule"] == lsp.SCHED_GRID
    assert (one["waves_per_wg"], one["wave_split"], one["t_split"]) == (8, lsp.WSPLIT_ON, 1)
    assert one["recurrence"] == lsp.REC_CHEBYSHEV
    assert one["tile_freqs"] == 64 * one["k_per_lane"]
    tiles = -(-500_000 // one["tile_freqs"])
    assert one["n_items"] == tiles and tiles * 8 >= 3584
    # too few tiles for eight waves each, too few observations, or the wave
    # split turned off: four waves and the observation split across workgroups
    for n_f, n_obs, ws in ((300_000, 4096, lsp.WSPLIT_AUTO), (500_000, 1000, lsp.WSPLIT_AUTO),
                           (500_000, 4096, lsp.WSPLIT_OFF)):
        sp = lsp.describe_launch(1, n_obs, lsp.make_grid(0.5, 24.0, n_f),
                                 lsp.make_options(form=lsp.FORM_FP32P, wave_split=ws))
        assert (sp["waves_per_wg"], sp["wave_split"]) == (4, lsp.WSPLIT_OFF)
        assert sp["t_split"] > 1 and sp["tile_freqs"] == 64 * sp["k_per_lane"] * 4
        assert sp["n_items"] == -(-n_f // sp["tile_freqs"]) * sp["t_split"]
    gb = lsp.make_grid(0.5, 24.0, 250_000)
    many = lsp.describe_launch(200_000, 52_000_000, gb, lsp.make_options(form=lsp.FORM_FP32P))
    assert many["schedule"] == lsp.SCHED_PERSISTENT and many["t_split"] == 1
    assert many["waves_per_wg"] == 1
    tiles_row = -(-250_000 // many["tile_freqs"])
    assert many["tiles_per_item"] == 16  # 49 M tiles: up to 16 consecutive tiles per item
    assert many["n_items"] == 200_000 * -(-tiles_row // 16)
    assert one["tiles_per_item"] == 1 and sp["tiles_per_item"] == 1  # few tiles, split objects
    few = lsp.describe_launch(10, 5000, gb, lsp.make_options(form=lsp.FORM_FP32P))
    assert few["tiles_per_item"] == 1 and few["n_items"] == 10 * -(-250_000 // few["tile_freqs"])
    fixed = lsp.describe_launch(10, 5000, gb, lsp.make_options(
        form=lsp.FORM_FP32P, k=12, recurrence=lsp.REC_ROTATION, schedule=lsp.SCHED_GRID))
    assert (fixed["k_per_lane"], fixed["recurrence"], fixed["schedule"]) == \
        (12, lsp.REC_ROTATION, lsp.SCHED_GRID)
    f64 = lsp.describe_launch(10, 5000, gb, lsp.make_options(form=lsp.FORM_FP64))
    assert f64["k_per_lane"] in (1, 2, 4) and f64["schedule"] == lsp.SCHED_GRID
    gen = lsp.describe_launch(10, 5000, gb, lsp.make_options(form=lsp.FORM_FP32P), True)
    assert gen["k_per_lane"] in (8, 12, 16)
    assert f64["tiles_per_item"] == 1
    # row order: longest first by default for large batches (>= 1e10 terms),
    # as given for small ones and for a single object, and on request
    assert many["order"] == lsp.ORDER_LPT and few["order"] == lsp.ORDER_INPUT
    assert one["order"] == lsp.ORDER_INPUT
    for od in (lsp.ORDER_INPUT, lsp.ORDER_LPT):
        assert lsp.describe_launch(10, 5000, gb, lsp.make_options(order=od))["order"] == od
        assert lsp.describe_launch(200_000, 52_000_000, gb, lsp.make_options(
            form=lsp.FORM_FP32P, order=od))["order"] == od
    assert lsp.describe_launch(1, 4096, g, lsp.make_options(
        form=lsp.FORM_FP32P, order=lsp.ORDER_LPT))["order"] == lsp.ORDER_INPUT
    # eight waves per workgroup: FP32 form with the wave split only
    ws8 = lsp.describe_launch(1, 4096, g, lsp.make_options(
        form=lsp.FORM_FP32P, waves=8, k=16, wave_split=lsp.WSPLIT_ON))
    assert (ws8["waves_per_wg"], ws8["wave_split"], ws8["t_split"]) == (8, lsp.WSPLIT_ON, 1)
    assert ws8["tile_freqs"] == 64 * 16 and ws8["n_items"] == -(-500_000 // 1024)
    for o in (lsp.make_options(form=lsp.FORM_FP32P, waves=8),
              lsp.make_options(form=lsp.FORM_FP64, waves=8),
              lsp.make_options(form=lsp.FORM_FP32P, waves=8, wave_split=lsp.WSPLIT_ON,
                               seed_trig=lsp.TRIG_LIB)):
        with pytest.raises(lsp.LspError):
            lsp.describe_launch(1, 4096, g, o)
    with pytest.raises(lsp.LspError):
        lsp.describe_launch(1, 4096, g, lsp.make_options(
            form=lsp.FORM_FP32P, waves=8, wave_split=lsp.WSPLIT_ON), generalized=True)
    with pytest.raises(lsp.LspError):
        lsp.describe_launch(0, 10, gb, lsp.make_options())
    with pytest.raises(lsp.LspError):
        lsp.describe_launch(2, 10, gb, lsp.make_options(form=lsp.FORM_FP32P, t_split=4))
    with pytest.raises(lsp.LspError):
        lsp.describe_launch(2, 10, gb, lsp.make_options(form=lsp.FORM_FP32P,
                                                        recurrence=lsp.REC_ROTATION), True)


@cpu_only
def test_batch_static_argument_errors(L):
    """lsp_batch_static rejects bad arguments and calls too large for its
    static scratch on the host, before looking up any device memory."""
    g = lsp.make_grid(0.5, 24.0, 250_000)
    o = lsp.make_options(form=lsp.FORM_FP32P)

    def call(off=FAKE, n_obj=4, n_obs=100, grid=g, opt=o, pgram=None, peaks=FAKE):
        return L.lsp_batch_static(off, n_obj, n_obs, FAKE, FAKE,
                                  ctypes.byref(grid) if grid is not None else None,
                                  ctypes.byref(opt), pgram, peaks, None)

    assert call(off=None) == lsp.EINVAL
    assert call(grid=None) == lsp.EINVAL
    assert call(n_obj=0) == lsp.EINVAL
    assert call(grid=lsp.make_grid(2.0, 1.0, 10)) == lsp.EINVAL
    assert call(opt=lsp.make_options(form=9)) == lsp.EINVAL
    assert call(opt=lsp.make_options(form=lsp.FORM_FP32P, t_split=4)) == lsp.EUNSUPPORTED
    # the FP32 form of the 200,000-object LSST-like batch fits (per-object peak
    # keys); the FP64 form's per-tile records do not
    assert lsp.workspace_bytes(200_000, 52_000_000, g, o) <= lsp.STATIC_SCRATCH_BYTES
    o64 = lsp.make_options(form=lsp.FORM_FP64)
    assert lsp.workspace_bytes(200_000, 52_000_000, g, o64) > lsp.STATIC_SCRATCH_BYTES
    assert call(n_obj=200_000, n_obs=52_000_000, opt=o64) == lsp.ESCRATCH
    assert lsp.status_string(lsp.ESCRATCH) != lsp.status_string(lsp.ENOMEM)


def test_static_scratch_size_matches_header():
    text = open(lsp.HEADER).read()
    assert "#define LSP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)" in text
    assert lsp.STATIC_SCRATCH_BYTES == 64 << 20


@cpu_only
def test_row_order_argument_errors(L):
    nb = L.lsp_row_order_workspace_bytes()
    assert nb >= 4416 * 4 and nb % 256 == 0

    def call(offsets=FAKE, n_obj=10, row_obj=None, row_band=None, n_rows=10, rpg=1, perm=FAKE,
             ws=FAKE, ws_bytes=nb):
        return L.lsp_row_order(offsets, n_obj, row_obj, row_band, n_rows, rpg, perm, ws,
                               ws_bytes, None)

    assert call(offsets=None) == lsp.EINVAL
    assert call(perm=None) == lsp.EINVAL
    assert call(ws=None) == lsp.EINVAL
    assert call(n_obj=0) == lsp.EINVAL
    assert call(n_rows=0) == lsp.EINVAL
    assert call(rpg=0) == lsp.EINVAL
    assert call(n_rows=11) == lsp.EINVAL              # row r is object r / rows_per_group
    assert call(n_rows=20, rpg=2, ws=ctypes.c_void_p((1 << 20) + 8)) == lsp.EINVAL
    assert call(row_obj=FAKE, n_rows=1 << 31) == lsp.EINVAL
    assert call(ws_bytes=nb - 1) == lsp.ENOMEM


def test_single_object_in_workgroup_split_keeps_no_partial_sums():
    """The single-object default on a wide grid adds its waves' sums on chip:
    its workspace holds no observation-split partial sums (16 B per bin and
    split), which the split across workgroups needs."""
    g = lsp.make_grid(0.5, 24.0, 500_000)
    ws8 = lsp.workspace_bytes(1, 4096, g, lsp.make_options(form=lsp.FORM_FP32P))
    opt_off = lsp.make_options(form=lsp.FORM_FP32P, wave_split=lsp.WSPLIT_OFF)
    off = lsp.workspace_bytes(1, 4096, g, opt_off)
    split = lsp.describe_launch(1, 4096, g, opt_off)["t_split"]
    assert split > 1 and off - ws8 >= 16 * 500_000 * split
    assert ws8 < 4096  # metadata, one peak key, flags and queue counters only


def test_mlp_structs_match_header(tmp_path):
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "mlp.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lsp.h"\nint main(void) {\n'
                   '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lsp_mlp), '
                   'offsetof(lsp_mlp, w), offsetof(lsp_mlp, b), offsetof(lsp_mlp, w_bf16), '
                   'sizeof(lsp_mlp_grads), offsetof(lsp_mlp_grads, w), '
                   'offsetof(lsp_mlp_grads, b));\n  return 0;\n}\n')
    exe = tmp_path / "mlp"
    subprocess.run(["gcc", "-std=c11", "-I", str(lsp.HEADER.rsplit("/", 1)[0]), str(src), "-o",
                    str(exe)], check=True)
    out = [int(v) for v in
           subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out == [ctypes.sizeof(lsp.Mlp), lsp.Mlp.w.offset, lsp.Mlp.b.offset,
                   lsp.Mlp.w_bf16.offset, ctypes.sizeof(lsp.MlpGrads), lsp.MlpGrads.w.offset,
                   lsp.MlpGrads.b.offset]


def _fake_mlp(dims=(1088, 512, 256, 64)):
    net = lsp.Mlp()
    net.dims[:] = list(dims)
    for l in range(3):
        net.w[l] = net.b[l] = net.w_bf16[l] = FAKE.value
    g = lsp.MlpGrads()
    for l in range(3):
        g.w[l] = g.b[l] = FAKE.value
    return net, g


@cpu_only
def test_mlp_argument_errors(L):
    f32, byref = ctypes.c_float, ctypes.byref
    net, g = _fake_mlp()
    fwd = L.lsp_mlp_forward
    assert fwd(None, FAKE, 4, FAKE, FAKE, FAKE, None) == lsp.EINVAL
    assert fwd(byref(net), FAKE, -1, FAKE, FAKE, FAKE, None) == lsp.EINVAL
    assert fwd(byref(net), None, 4, FAKE, FAKE, FAKE, None) == lsp.EINVAL
    assert fwd(byref(net), FAKE, 0, None, None, None, None) == lsp.OK  # nothing to do
    bad, _ = _fake_mlp((1088, 0, 256, 64))
    assert fwd(byref(bad), FAKE, 4, FAKE, FAKE, FAKE, None) == lsp.EINVAL
    bad, _ = _fake_mlp()
    bad.b[1] = None
    assert fwd(byref(bad), FAKE, 4, FAKE, FAKE, FAKE, None) == lsp.EINVAL
    # scratch: dlogits, dz2 and dz1 in FP32 and BF16, each 256-byte aligned
    assert L.lsp_mlp_workspace_bytes(None, 4) == 0
    assert L.lsp_mlp_workspace_bytes(byref(net), 0) == 0
    want = sum(-(-4 * c * b // 256) * 256 for c in (64, 256, 512) for b in (4, 2))
    nb = L.lsp_mlp_workspace_bytes(byref(net), 4)
    assert nb == want
    bwd = L.lsp_mlp_backward
    args = (FAKE, FAKE, 4, FAKE, FAKE, FAKE, f32(0.25))
    assert bwd(byref(net), FAKE, FAKE, 0, FAKE, FAKE, FAKE, f32(1), byref(g), None, FAKE, nb,
               None) == lsp.EINVAL
    assert bwd(byref(net), *args, None, None, FAKE, nb, None) == lsp.EINVAL
    assert bwd(byref(net), *args, byref(g), None, FAKE, nb - 1, None) == lsp.ENOMEM
    assert bwd(byref(net), *args, byref(g), None, None, nb, None) == lsp.EINVAL
    adam = L.lsp_mlp_adam
    hp = (f32(1e-3), f32(0.9), f32(0.999), f32(1e-8), None)
    assert adam(byref(net), byref(g), byref(g), byref(g), 0, *hp) == lsp.EINVAL
    assert adam(byref(net), byref(g), None, byref(g), 1, *hp) == lsp.EINVAL
    bad_g = lsp.MlpGrads()
    assert adam(byref(net), byref(bad_g), byref(g), byref(g), 1, *hp) == lsp.EINVAL


def test_single_object_launch_rule_thresholds():
    """The eight-wave in-workgroup split is chosen exactly when its 1,024-bin
    tiles (K = 16) give at least 3,584 waves and the object has at least
    2,048 observations."""
    opt = lsp.make_options(form=lsp.FORM_FP32P)
    cases = [(448 * 1024, 4096, True), (447 * 1024, 4096, False),
             (500_000, 2048, True), (500_000, 2047, False)]
    for n_f, n_obs, ws8 in cases:
        d = lsp.describe_launch(1, n_obs, lsp.make_grid(0.5, 24.0, n_f), opt)
        assert d["k_per_lane"] == 16
        got = (d["waves_per_wg"], d["wave_split"]) == (8, lsp.WSPLIT_ON) and d["t_split"] == 1
        assert got == ws8, (n_f, n_obs, d)
        if not ws8:
            assert d["waves_per_wg"] == 4 and d["wave_split"] == lsp.WSPLIT_OFF
    # batches, row mode and explicit shapes never get it by default
    many = lsp.describe_launch(2, 8192, lsp.make_grid(0.5, 24.0, 500_000), opt)
    assert many["wave_split"] == lsp.WSPLIT_OFF
    fixed = lsp.describe_launch(1, 4096, lsp.make_grid(0.5, 24.0, 500_000),
                                lsp.make_options(form=lsp.FORM_FP32P, waves=4))
    assert fixed["waves_per_wg"] == 4 and fixed["wave_split"] == lsp.WSPLIT_OFF


def test_generalized_single_object_split_fills_resident_slots():
    """The generalized kernel holds three waves per SIMD from K = 12 and four
    below: a single object's observation split fills those 3,072 or 4,096
    resident wave slots once."""
    g = lsp.make_grid(0.5, 24.0, 500_000)
    d = lsp.describe_launch(1, 4096, g, lsp.make_options(form=lsp.FORM_FP32P), generalized=True)
    waves = -(-500_000 // d["tile_freqs"]) * d["waves_per_wg"]
    assert d["k_per_lane"] == 16 and d["t_split"] == 3072 // waves == 6
    d8 = lsp.describe_launch(1, 4096, g, lsp.make_options(form=lsp.FORM_FP32P, k=8),
                             generalized=True)
    waves8 = -(-500_000 // d8["tile_freqs"]) * d8["waves_per_wg"]
    assert d8["t_split"] == 4096 // waves8 == 4
