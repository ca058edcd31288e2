// lsp_api.hip -- host side of the C ABI declared in include/lsp.h.
//
// Validates arguments on the host (nothing is enqueued on error), resolves the
// launch configuration from the options and the problem shape, carves the
// caller's workspace, and enqueues prep -> main kernel -> (combine) -> peaks on
// the caller's stream.  No device memory is allocated and the device is never
// synchronised, so a call can be captured into a HIP graph.
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <new>

#include "lsp_common.h"

namespace lsp {
namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxGrid = ((int64_t)1 << 31) - 1;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Which periodogram: the standard one (Section 2) or the generalized one
// with errors and a floating mean (Section 4.11).
struct Method {
    bool gen = false;
    const double* dy = nullptr;  // errors of the generalized form; NULL: unit errors
};

struct Config {
    int gen;
    int obs;   // LSP_OBS_LDS or LSP_OBS_DIRECT (FP32 form)
    int trig;  // LSP_TRIG_HW, _LIB or _POLY (FP32 form)
    int form;
    int rec;
    int k;
    int waves;
    int split;
    int persistent;
    int ws;
    int64_t tile_freqs;
    int64_t tiles_per_row;
    int64_t tiles_per_item;  // consecutive frequency tiles per work item
    int64_t chunks_per_row;
    int64_t n_items;
    int64_t rec_per_group;  // records per group (tile records or combine blocks)
    int64_t n_obs;
    bool keys;              // FP32 form, unsplit: per-group peak keys + tile flag bits
    bool lpt;               // rows handed out longest first (lsp_order.hip)
};

// Rows of work.  The whole-grid entry points use one row per object covering
// every bin; lsp_batch_rows names (object, band) rows and groups of rows that
// share a peak record.
struct Rows {
    const int32_t* row_obj;   // NULL: row r is object r
    const int32_t* row_band;  // NULL: every row covers the whole grid
    int64_t n_rows;
    int64_t band_bins;        // bins per band (n_f when row_band is NULL)
    int32_t rows_per_group;
    bool whole;               // lsp_single / lsp_batch: one whole-grid row per object
};

Rows whole_grid(int64_t n_obj, const lsp_grid* g) {
    return Rows{nullptr, nullptr, n_obj, g ? g->n_f : 0, 1, true};
}

struct Layout {
    size_t meta, rec, keys, bits, queue, part, stage_t, stage_o, perm, hist, total;
    size_t zero_words;  // u32 words cleared before the main kernel, from `keys` (key mode)
};

bool valid_grid(const lsp_grid* g) {
    return g && isfinite(g->f_min) && isfinite(g->f_max) && g->f_max > g->f_min && g->n_f >= 1 &&
           (g->unit == LSP_UNIT_CYCLES || g->unit == LSP_UNIT_ANGULAR) &&
           isfinite((g->f_max - g->f_min) / (double)g->n_f);
}

bool is_bool(int32_t v) { return v == 0 || v == 1; }

lsp_status valid_options(const lsp_options* o) {
    if (!(o->form == LSP_FORM_FP64 || o->form == LSP_FORM_FP32P)) return LSP_EINVAL;
    if (!is_bool(o->normalize) || !is_bool(o->subtract_mean)) return LSP_EINVAL;
    if (!(o->pgram_dtype == LSP_PGRAM_F32 || o->pgram_dtype == LSP_PGRAM_F64)) return LSP_EINVAL;
    if (!(o->waves_per_wg == 0 || o->waves_per_wg == 1 || o->waves_per_wg == 2 ||
          o->waves_per_wg == 4 || o->waves_per_wg == 8))
        return LSP_EINVAL;
    if (o->form == LSP_FORM_FP64) {
        if (!(o->k_per_lane == 0 || o->k_per_lane == 1 || o->k_per_lane == 2 ||
              o->k_per_lane == 4))
            return LSP_EINVAL;
    } else if (!(o->k_per_lane == 0 || o->k_per_lane == 4 || o->k_per_lane == 8 ||
                 o->k_per_lane == 10 || o->k_per_lane == 12 || o->k_per_lane == 16 ||
                 o->k_per_lane == 32)) {
        return LSP_EINVAL;
    }
    if (o->t_split < 0 || o->t_split > 64) return LSP_EINVAL;
    if (o->schedule < LSP_SCHED_AUTO || o->schedule > LSP_SCHED_PERSISTENT) return LSP_EINVAL;
    if (o->recurrence < LSP_REC_AUTO || o->recurrence > LSP_REC_CHEBYSHEV) return LSP_EINVAL;
    if (o->wave_split < LSP_WSPLIT_AUTO || o->wave_split > LSP_WSPLIT_ON) return LSP_EINVAL;
    if (o->obs_read < LSP_OBS_AUTO || o->obs_read > LSP_OBS_DIRECT) return LSP_EINVAL;
    if (o->seed_trig < LSP_TRIG_AUTO || o->seed_trig > LSP_TRIG_POLY) return LSP_EINVAL;
    if (o->order < LSP_ORDER_AUTO || o->order > LSP_ORDER_LPT) return LSP_EINVAL;
    return LSP_OK;
}

// Launch configuration: a pure function of the shape and the options, so that
// lsp_workspace_bytes and the call agree.
lsp_status resolve(int64_t n_obj, int64_t n_obs, const lsp_grid* g, const lsp_options* o,
                   const Rows& rows, Config* c, const Method& method = Method{}) {
    // Launch shapes are sized for the bins of one row.
    const int64_t n_f = rows.row_band ? (rows.band_bins < g->n_f ? rows.band_bins : g->n_f) : g->n_f;
    const bool whole = rows.whole;
    c->gen = method.gen;
    c->obs = o->obs_read == LSP_OBS_DIRECT ? LSP_OBS_DIRECT : LSP_OBS_LDS;
    c->trig = o->seed_trig == LSP_TRIG_AUTO ? LSP_TRIG_HW : o->seed_trig;
    // The read-path and seed-trig variants exist for the standard FP32 form
    // with the three-term recurrence, no wave split, K in {8, 16} and 1 or 4
    // waves per workgroup.
    const bool variant = c->obs != LSP_OBS_LDS || c->trig != LSP_TRIG_HW;
    if (variant) {
        if (o->form != LSP_FORM_FP32P || method.gen) return LSP_EUNSUPPORTED;
        if (o->recurrence == LSP_REC_ROTATION || o->wave_split == LSP_WSPLIT_ON)
            return LSP_EUNSUPPORTED;
        if (!(o->k_per_lane == 0 || o->k_per_lane == 8 || o->k_per_lane == 16))
            return LSP_EUNSUPPORTED;
        if (o->waves_per_wg == 2 || o->waves_per_wg == 8) return LSP_EUNSUPPORTED;
    }
    c->form = o->form;
    // The three-term recurrence needs fewer operations per bin and measured as
    // accurate as the rotation, so it is the default.
    c->rec = o->recurrence == LSP_REC_ROTATION ? LSP_REC_ROTATION : LSP_REC_CHEBYSHEV;
    c->persistent = 0;
    c->split = 1;
    c->ws = 0;
    if (o->form == LSP_FORM_FP64) {
        c->k = o->k_per_lane ? o->k_per_lane : 2;
        c->waves = o->waves_per_wg ? o->waves_per_wg : 4;
        if (!o->waves_per_wg)
            while ((int64_t)kWave * c->k * c->waves > n_f && c->waves > 1) c->waves /= 2;
        if (!o->k_per_lane)
            while ((int64_t)kWave * c->k * c->waves > n_f && c->k > 1) c->k /= 2;
        if (o->t_split > 1) return LSP_EUNSUPPORTED;
        if (o->schedule == LSP_SCHED_PERSISTENT || o->waves_per_wg == 8) return LSP_EUNSUPPORTED;
    } else {
        // Measured defaults: one object on the whole grid runs best with four
        // waves per workgroup sharing its staged observations; many rows run
        // best as single-wave workgroups fed from the per-XCD queues.
        const bool one_row = whole && n_obj == 1;
        c->waves = o->waves_per_wg ? o->waves_per_wg : (one_row ? 4 : 1);
        if (method.gen) {
            // The generalized kernel has the three-term recurrence only, no
            // in-workgroup wave split, and K in {4, 8, 12, 16}.
            if (o->recurrence == LSP_REC_ROTATION || o->wave_split == LSP_WSPLIT_ON)
                return LSP_EUNSUPPORTED;
            if (o->k_per_lane == 10 || o->k_per_lane == 32 || o->waves_per_wg == 8)
                return LSP_EUNSUPPORTED;
        }
        if (o->k_per_lane) {
            c->k = o->k_per_lane;
        } else if (variant) {
            c->k = 16;
        } else if (method.gen) {
            // 8 instructions per (bin, observation) plus about 12.6 per
            // observation and lane for the scaled seed, shared by the K bins.
            const int ks[] = {8, 12, 16};
            double best = 1e300;
            c->k = 16;
            for (int k : ks) {
                const int64_t tile = (int64_t)kWave * k * c->waves;
                const double cost = (double)((n_f + tile - 1) / tile * tile) * (8.0 + 12.6 / k);
                if (cost < best * (1.0 - 1e-9)) {
                    best = cost;
                    c->k = k;
                }
            }
        } else {
            // Frequencies per lane: the fewest instructions for the row,
            // counting the bins of the last, partly used tile.  Per (bin,
            // observation) the loop issues 6 instructions plus about 10.6 per
            // observation and lane for the seed, shared by the K bins.
            const int ks[] = {8, 10, 12, 16};
            double best = 1e300;
            c->k = 16;
            for (int k : ks) {
                const int64_t tile = (int64_t)kWave * k * c->waves;
                const double cost = (double)((n_f + tile - 1) / tile * tile) * (6.0 + 10.6 / k);
                if (cost < best * (1.0 - 1e-9)) {
                    best = cost;
                    c->k = k;
                }
            }
        }
        if (!o->waves_per_wg)
            while ((int64_t)kWave * c->k * c->waves > n_f && c->waves > 1) c->waves /= 2;
        if (!o->k_per_lane)
            while ((int64_t)kWave * c->k * c->waves > n_f && c->k > 4) c->k = c->k > 8 ? 8 : 4;
        if (variant) {
            if (c->waves == 2) c->waves = 1;
            if (c->k < 8) c->k = 8;
        }
        c->persistent = o->schedule == LSP_SCHED_PERSISTENT ||
                        (o->schedule == LSP_SCHED_AUTO && !one_row);
        c->ws = c->waves > 1 && o->wave_split == LSP_WSPLIT_ON;
        // One object on the whole grid: eight waves that share each tile's
        // bins and split its observations inside the workgroup (sums added in
        // LDS, no partial sums in HBM, no combine launch) when that alone
        // gives about 3.5 waves per SIMD and every wave at least a staging
        // tile of observations to add before the sums meet.  Measured against
        // four waves with the cross-workgroup observation split: on a
        // 4,096-point object 3-7% faster from N_f = 5e5 (3,912 waves) to 4e6
        // and 12-32% slower at 3e5-4e5 (2,344-3,128 waves), where the split
        // below stays; on 2,048-65,536-point objects within 2.5% either way
        // at 5e5 and 0-5% faster at 1e6.  It writes no partial sums.
        if (one_row && !method.gen && !variant && o->wave_split == LSP_WSPLIT_AUTO &&
            !o->waves_per_wg && o->t_split == 0 && n_obs >= 8 * (int64_t)kTile) {
            const int64_t tw = (int64_t)kWave * c->k;
            if ((n_f + tw - 1) / tw * 8 >= 3584) {
                c->waves = 8;
                c->ws = 1;
            }
        }
        // eight waves per workgroup exist only with the wave split
        if (c->waves == 8 && !c->ws) return LSP_EUNSUPPORTED;
        if (o->t_split > 1) {
            if (n_obj != 1 || !whole) return LSP_EUNSUPPORTED;
            c->split = o->t_split;
        } else if (o->t_split == 0 && n_obj == 1 && whole) {
            // Too few frequency tiles to occupy 1024 SIMDs with a few waves
            // each: split the observation axis as well, into as many parts as
            // fill the chip's resident wave slots once (four waves per SIMD;
            // three for the generalized kernel from K = 12, whose registers
            // allow no more).  Measured on one 4,096-point object with errors
            // (N_f = 5e5, K = 16): splits 6 / 8 / 12 (0.96 / 1.28 / 1.92
            // rounds of its 3,072 slots) ran the main kernel in 0.383 / 0.389
            // / 0.367 ms and a split of 7 (1.12 rounds) in 0.436 ms.
            const int64_t tpw = (int64_t)kWave * c->k * (c->ws ? 1 : c->waves);
            const int64_t waves_total = ((n_f + tpw - 1) / tpw) * c->waves;
            const int64_t slots = (int64_t)1024 * (method.gen && c->k > 8 ? 3 : 4);
            int64_t want = slots / (waves_total > 0 ? waves_total : 1);
            int64_t cap = n_obs / kTile;
            if (cap > 64) cap = 64;
            if (want > cap) want = cap;
            c->split = want > 1 ? (int)want : 1;
        }
    }
    c->tile_freqs = (int64_t)kWave * c->k * (c->ws ? 1 : c->waves);
    c->tiles_per_row = (n_f + c->tile_freqs - 1) / c->tile_freqs;
    if (c->tiles_per_row * rows.rows_per_group > kMaxGrid / rows.n_rows / c->split)
        return LSP_EUNSUPPORTED;
    // The FP32 forms give each work item up to 16 consecutive
    // frequency tiles of one row -- one queue pop and one peak-key merge per
    // item, and an object that fits in one staging pass is staged once --
    // while items stay small against one wave's share of the launch: about
    // 200 items per resident wave (4,096 on the chip), so that the last items
    // do not leave the chip idle.  Measured: lsst_200k (49 M tiles, 16 per
    // item) 0.5% faster; batch_10k (1 M tiles) 6% slower at 14 per item,
    // where this rule keeps 1.
    c->tiles_per_item = 1;
    if (o->form == LSP_FORM_FP32P && c->split == 1) {
        int64_t tpi = rows.n_rows * c->tiles_per_row / (200 * 4096);
        if (tpi > 16) tpi = 16;
        if (tpi > c->tiles_per_row) tpi = c->tiles_per_row;
        c->tiles_per_item = tpi > 1 ? tpi : 1;
    }
    c->chunks_per_row = (c->tiles_per_row + c->tiles_per_item - 1) / c->tiles_per_item;
    c->n_items = rows.n_rows * c->chunks_per_row * c->split;
    c->n_obs = n_obs;
    c->rec_per_group = c->split > 1 ? (n_f + kCombineThreads - 1) / kCombineThreads
                                    : c->tiles_per_row * rows.rows_per_group;
    // The FP32 forms merge each group's peak into one 64-bit key whose index
    // field holds 32 bits (peak_key).
    c->keys = c->form == LSP_FORM_FP32P && c->split == 1;
    if (c->keys && g->n_f > (int64_t)0xFFFFFFFE) return LSP_EUNSUPPORTED;
    // Longest-first order needs rows of different objects to order.  By
    // default it is used for calls of at least 1e10 (observation, bin) terms,
    // where its four small launches cost under 1%.  Measured: a heavy-tailed
    // population (asteroids_100k, N_t 10..1500) 1.3% faster; batch_10k and
    // lsst_200k (uniform N_t) unchanged.
    const bool orderable =
        rows.n_rows > 1 && rows.n_rows <= (int64_t)INT32_MAX && n_obj > 1 && c->split == 1;
    const double terms = (double)n_obs * (double)n_f * ((double)rows.n_rows / (double)n_obj);
    c->lpt = orderable && (o->order == LSP_ORDER_LPT || (o->order == LSP_ORDER_AUTO && terms >= 1e10));
    return LSP_OK;
}

Layout layout(int64_t n_obj, const lsp_grid* g, const Rows& rows, const Config& c) {
    Layout L;
    size_t off = 0;
    const size_t n_groups = (size_t)(rows.n_rows / rows.rows_per_group);
    L.meta = off;
    off += align_up((size_t)n_obj * sizeof(ObjMeta));
    L.rec = off;
    off += c.keys ? 0 : align_up(n_groups * (size_t)c.rec_per_group * sizeof(PeakRec));
    // key mode: group keys, tile flag bits and the queue counters back to back,
    // so that one fill clears them
    const size_t n_words = c.keys ? ((size_t)rows.n_rows * (size_t)c.tiles_per_row + 31) / 32 : 0;
    L.keys = off;
    off += c.keys ? n_groups * sizeof(unsigned long long) : 0;
    L.bits = off;
    off += n_words * 4;
    L.queue = off;
    off += kXcds * 4;
    L.zero_words = c.keys ? (off - L.keys) / 4 : 0;
    off = align_up(off);
    L.part = off;
    off += c.split > 1
               ? align_up((size_t)c.split * (c.gen ? 6 : 4) * (size_t)g->n_f * sizeof(float))
               : 0;
    // LSP_OBS_DIRECT: per-observation staged values (indexed like t)
    const size_t n_obs = c.obs == LSP_OBS_DIRECT ? (size_t)c.n_obs : 0;
    L.stage_t = off;
    off += align_up(n_obs * sizeof(double));
    L.stage_o = off;
    off += align_up(n_obs * 16);
    // longest-first order: the rank -> row permutation and the sort's buckets
    L.perm = off;
    off += c.lpt ? align_up((size_t)rows.n_rows * sizeof(int32_t)) : 0;
    L.hist = off;
    off += c.lpt ? align_up((size_t)(kOrderBlocks + 1) * kOrderBuckets * sizeof(unsigned int))
                 : 0;
    L.total = off;
    return L;
}

thread_local hipEvent_t t_main_begin = nullptr;
thread_local hipEvent_t t_main_end = nullptr;

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Host-side argument checks shared by every entry point; nothing is enqueued.
lsp_status valid_rows(const Rows& r, const lsp_grid* grid) {
    if (r.n_rows < 1 || r.rows_per_group < 1 || r.n_rows % r.rows_per_group) return LSP_EINVAL;
    if (r.row_band && (r.band_bins < 1 || r.band_bins > grid->n_f)) return LSP_EINVAL;
    return LSP_OK;
}

lsp_status validate(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                    const double* y, const lsp_grid* grid, const lsp_options* opt_in,
                    const void* pgram, const lsp_peak* peaks, const void* ws, size_t ws_bytes,
                    const Rows& rows, const Method& method = Method{}) {
    (void)offsets;
    if (!grid || !ws) return LSP_EINVAL;
    if (n_obj < 1 || n_obs < 0) return LSP_EINVAL;
    if (n_obs > 0 && (!t || !y)) return LSP_EINVAL;
    if (!valid_grid(grid)) return LSP_EINVAL;
    if (!pgram && !peaks) return LSP_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return LSP_EINVAL;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    lsp_status st = valid_options(&opt);
    if (st != LSP_OK) return st;
    st = valid_rows(rows, grid);
    if (st != LSP_OK) return st;
    Config c;
    st = resolve(n_obj, n_obs, grid, &opt, rows, &c, method);
    if (st != LSP_OK) return st;
    if (ws_bytes < layout(n_obj, grid, rows, c).total) return LSP_ENOMEM;
    return LSP_OK;
}

lsp_status run(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
               const double* y, const lsp_grid* grid, const lsp_options* opt_in, void* pgram,
               lsp_peak* peaks, void* ws, size_t ws_bytes, void* stream, const Rows& rows,
               const Method& method = Method{}) {
    lsp_status st = validate(offsets, n_obj, n_obs, t, y, grid, opt_in, pgram, peaks, ws,
                             ws_bytes, rows, method);
    if (st != LSP_OK) return st;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    Config c;
    resolve(n_obj, n_obs, grid, &opt, rows, &c, method);
    const Layout L = layout(n_obj, grid, rows, c);
    const int64_t n_groups = rows.n_rows / rows.rows_per_group;

    hipStream_t s = static_cast<hipStream_t>(stream);
    const double df = (grid->f_max - grid->f_min) / (double)grid->n_f;
    const double to_cyc = grid->unit == LSP_UNIT_CYCLES ? 1.0 : kInvTwoPi;
    const bool f32 = c.form == LSP_FORM_FP32P;

    PrepParams pp;
    pp.offsets = offsets;
    pp.t = t;
    pp.y = y;
    pp.n_obj = n_obj;
    pp.n_obs = n_obs;
    pp.subtract_mean = opt.subtract_mean;
    pp.normalize = opt.normalize;
    pp.meta = at<ObjMeta>(ws, L.meta);
    pp.dy = method.dy;
    pp.gen = method.gen;
    if (launch_prep(pp, s) != hipSuccess) return LSP_EHIP;

    MainParams mp;
    mp.meta = pp.meta;
    mp.t = t;
    mp.y = y;
    mp.step_cyc = (double)kWave * df * to_cyc;
    mp.f_min = grid->f_min;
    mp.df = df;
    mp.to_cyc = to_cyc;
    mp.n_f = grid->n_f;
    mp.n_obj = n_obj;
    mp.row_obj = rows.row_obj;
    mp.row_band = rows.row_band;
    mp.band_bins = rows.row_band ? rows.band_bins : grid->n_f;
    mp.rows_per_group = rows.rows_per_group;
    mp.pad_rows = 0;
    mp.tiles_per_row = c.tiles_per_row;
    mp.tiles_per_item = c.tiles_per_item;
    mp.chunks_per_row = c.chunks_per_row;
    mp.n_items = c.n_items;
    mp.n_split = c.split;
    mp.pgram_f64 = opt.pgram_dtype == LSP_PGRAM_F64;
    mp.pgram = pgram;
    mp.rec = c.keys ? nullptr : at<PeakRec>(ws, L.rec);
    mp.keys = c.keys ? at<unsigned long long>(ws, L.keys) : nullptr;
    mp.ill_bits = c.keys ? at<uint32_t>(ws, L.bits) : nullptr;
    mp.part = c.split > 1 ? at<float>(ws, L.part) : nullptr;
    mp.queue = at<unsigned int>(ws, L.queue);
    mp.persistent = c.persistent;
    mp.wave_split = c.ws;
    mp.dy = method.dy;
    mp.gen = method.gen;
    if (c.obs == LSP_OBS_DIRECT) {
        mp.stage_t = at<double>(ws, L.stage_t);
        mp.stage_o = at<float4>(ws, L.stage_o);
        if (launch_stage(mp.meta, t, y, n_obj, mp.step_cyc, c.trig, at<double>(ws, L.stage_t),
                         at<float4>(ws, L.stage_o), s) != hipSuccess)
            return LSP_EHIP;
    }

    // key mode: clear keys, flag bits and queue counters in one fill kernel
    // (a kernel, not a memset node, so that captured graphs replay it safely)
    if (c.keys) {
        if (launch_fill_u32(at<unsigned int>(ws, L.keys), (int64_t)L.zero_words, 0u, s) !=
            hipSuccess)
            return LSP_EHIP;
    } else if (f32 && c.persistent && launch_fill_u32(mp.queue, kXcds, 0u, s) != hipSuccess) {
        return LSP_EHIP;
    }
    if (c.lpt) {
        OrderParams op;
        op.offsets = offsets;
        op.n_obj = n_obj;
        op.row_obj = rows.row_obj;
        op.row_band = rows.row_band;
        op.n_rows = rows.n_rows;
        op.rows_per_group = rows.rows_per_group;
        op.pad = 0;
        op.hist = at<unsigned int>(ws, L.hist);
        op.total = op.hist + (size_t)kOrderBlocks * kOrderBuckets;
        op.perm = at<int32_t>(ws, L.perm);
        if (launch_row_order(op, s) != hipSuccess) return LSP_EHIP;
        mp.row_perm = op.perm;
        mp.n_work = op.total + (kOrderBuckets - 1);
    }
    if (t_main_begin && hipEventRecord(t_main_begin, s) != hipSuccess) return LSP_EHIP;
    if (method.gen) {
        if ((f32 ? launch_gen_fp32p(mp, c.k, c.waves, s) : launch_gen_fp64(mp, c.k, c.waves, s)) !=
            hipSuccess)
            return LSP_EHIP;
    } else if (f32) {
        if (launch_fp32p(mp, c.k, c.waves, c.rec, s, c.obs, c.trig) != hipSuccess)
            return LSP_EHIP;
    } else {
        if (launch_fp64(mp, c.k, c.waves, s) != hipSuccess) return LSP_EHIP;
    }
    if (t_main_end && hipEventRecord(t_main_end, s) != hipSuccess) return LSP_EHIP;
    if (f32) {
        if (c.split == 1) {
            FixupParams fp;
            fp.meta = mp.meta;
            fp.t = t;
            fp.y = y;
            fp.ill_bits = mp.ill_bits;
            fp.keys = mp.keys;
            fp.f_min = mp.f_min;
            fp.df = df;
            fp.to_cyc = to_cyc;
            fp.n_f = mp.n_f;
            fp.n_obj = n_obj;
            fp.row_obj = mp.row_obj;
            fp.row_band = mp.row_band;
            fp.band_bins = mp.band_bins;
            fp.rows_per_group = mp.rows_per_group;
            fp.pad_rows = 0;
            fp.tiles_per_row = c.tiles_per_row;
            fp.n_tiles = rows.n_rows * c.tiles_per_row;
            fp.tile_freqs = c.tile_freqs;
            fp.pgram_f64 = mp.pgram_f64;
            fp.pad = 0;
            fp.pgram = pgram;
            fp.rec = mp.rec;
            fp.dy = method.dy;
            fp.gen = method.gen;
            if (launch_fixup(fp, s) != hipSuccess) return LSP_EHIP;
        } else {
            CombineParams cp;
            cp.meta = mp.meta;
            cp.t = t;
            cp.y = y;
            cp.part = mp.part;
            cp.n_split = c.split;
            cp.pgram_f64 = mp.pgram_f64;
            cp.f_min = mp.f_min;
            cp.df = df;
            cp.to_cyc = to_cyc;
            cp.n_f = mp.n_f;
            cp.pgram = pgram;
            cp.rec = mp.rec;
            cp.dy = method.dy;
            cp.gen = method.gen;
            if (launch_combine(cp, s) != hipSuccess) return LSP_EHIP;
        }
    }

    if (peaks) {
        PeakParams kp;
        kp.meta = mp.meta;
        kp.rec = mp.rec;
        kp.keys = mp.keys;
        kp.n_obj = n_obj;
        kp.n_groups = n_groups;
        kp.row_obj = rows.row_obj;
        kp.rows_per_group = rows.rows_per_group;
        kp.pad2 = 0;
        kp.rec_per_obj = c.rec_per_group;
        kp.f_min = grid->f_min;
        kp.df = df;
        kp.unit = grid->unit;
        kp.pad = 0;
        kp.peaks = peaks;
        if (launch_peaks(kp, s) != hipSuccess) return LSP_EHIP;
    }
    return LSP_OK;
}

}  // namespace

// Whole-grid batch call and its workspace size, for the host-return pipeline.
// `one_batch` false runs a part of a larger batch: the launch configuration
// is then the multi-object one even for a single object, so that every part
// computes exactly what the whole batch would.
Rows batch_rows(int64_t n_obj, const lsp_grid* grid, bool one_batch) {
    Rows r = whole_grid(n_obj, grid);
    r.whole = one_batch;
    return r;
}

size_t batch_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                             const lsp_options* opt_in, bool gen, bool one_batch) {
    if (n_obj < 1 || n_obs < 0 || !valid_grid(grid)) return 0;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    if (valid_options(&opt) != LSP_OK) return 0;
    const Rows rows = batch_rows(n_obj, grid, one_batch);
    Method method;
    method.gen = gen;
    Config c;
    if (resolve(n_obj, n_obs, grid, &opt, rows, &c, method) != LSP_OK) return 0;
    return layout(n_obj, grid, rows, c).total;
}

lsp_status batch_call(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                      const double* y, const double* dy, bool gen, const lsp_grid* grid,
                      const lsp_options* opt, void* pgram, lsp_peak* peaks, void* ws,
                      size_t ws_bytes, void* stream, bool one_batch) {
    Method method;
    method.gen = gen;
    method.dy = dy;
    return run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, ws, ws_bytes, stream,
               batch_rows(n_obj, grid, one_batch), method);
}

}  // namespace lsp

struct lsp_plan_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

// Scratch of lsp_batch_static: one copy of this array lives on every device
// the library's code object is loaded on.  In host code `scratch` is only a
// stand-in symbol, never a device address: the address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[LSP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// The calling thread's current device and its copy of `scratch` (nullptr on
// failure).  The lookup runs once per device, with that device current.
void* device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::call_once(g_scratch_once[dev], [dev] {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    });
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

lsp_options lsp_default_options(void) {
    lsp_options o = {};
    o.form = LSP_FORM_FP64;
    o.normalize = 1;
    o.subtract_mean = 1;
    o.pgram_dtype = LSP_PGRAM_F32;
    return o;
}

size_t lsp_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                           const lsp_options* opt_in) {
    if (n_obj < 1 || n_obs < 0 || !lsp::valid_grid(grid)) return 0;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    if (lsp::valid_options(&opt) != LSP_OK) return 0;
    const lsp::Rows rows = lsp::whole_grid(n_obj, grid);
    lsp::Config c;
    if (lsp::resolve(n_obj, n_obs, grid, &opt, rows, &c) != LSP_OK) return 0;
    return lsp::layout(n_obj, grid, rows, c).total;
}

static size_t rows_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                                   const lsp_options* opt_in, int64_t n_rows, int64_t band_bins,
                                   int32_t rows_per_group, const lsp::Method& method) {
    if (n_obj < 1 || n_obs < 0 || !lsp::valid_grid(grid)) return 0;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    if (lsp::valid_options(&opt) != LSP_OK) return 0;
    // Any non-null band pointer stands for "banded" when sizing.
    static const int32_t kBanded = 0;
    const lsp::Rows rows{nullptr, band_bins > 0 ? &kBanded : nullptr, n_rows, band_bins,
                         rows_per_group, false};
    if (lsp::valid_rows(rows, grid) != LSP_OK) return 0;
    lsp::Config c;
    if (lsp::resolve(n_obj, n_obs, grid, &opt, rows, &c, method) != LSP_OK) return 0;
    return lsp::layout(n_obj, grid, rows, c).total;
}

size_t lsp_rows_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                                const lsp_options* opt, int64_t n_rows, int64_t band_bins,
                                int32_t rows_per_group) {
    return rows_workspace_bytes(n_obj, n_obs, grid, opt, n_rows, band_bins, rows_per_group,
                                lsp::Method{});
}

size_t lsp_gen_rows_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                                    const lsp_options* opt, int64_t n_rows, int64_t band_bins,
                                    int32_t rows_per_group) {
    lsp::Method method;
    method.gen = true;
    return rows_workspace_bytes(n_obj, n_obs, grid, opt, n_rows, band_bins, rows_per_group,
                                method);
}

lsp_status lsp_single(const double* t, const double* y, int64_t n_t, const lsp_grid* grid,
                      const lsp_options* opt, void* pgram, lsp_peak* peak, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (n_t < 0) return LSP_EINVAL;
    return lsp::run(nullptr, 1, n_t, t, y, grid, opt, pgram, peak, workspace, workspace_bytes,
                    stream, lsp::whole_grid(1, grid));
}

lsp_status lsp_batch(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                     const double* y, const lsp_grid* grid, const lsp_options* opt, void* pgram,
                     lsp_peak* peaks, void* workspace, size_t workspace_bytes, void* stream) {
    if (!offsets) return LSP_EINVAL;
    return lsp::run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                    workspace_bytes, stream, lsp::whole_grid(n_obj, grid));
}

lsp_status lsp_batch_static(const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                            const double* t, const double* y, const lsp_grid* grid,
                            const lsp_options* opt, void* pgram, lsp_peak* peaks, void* stream) {
    if (!offsets || !grid) return LSP_EINVAL;
    const size_t need = lsp_workspace_bytes(n_obj, n_obs, grid, opt);
    if (need == 0) {
        // invalid arguments: let the common validation name the error (the
        // stand-in workspace is never dereferenced)
        alignas(256) static const unsigned char kStandIn[1] = {0};
        const lsp_status st = lsp::validate(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks,
                                            kStandIn, 0, lsp::whole_grid(n_obj, grid));
        return st == LSP_OK || st == LSP_ENOMEM ? LSP_EINVAL : st;
    }
    if (need > LSP_STATIC_SCRATCH_BYTES) return LSP_ESCRATCH;
    void* ws = device_scratch();
    if (!ws) return LSP_EHIP;
    return lsp::run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, ws,
                    LSP_STATIC_SCRATCH_BYTES, stream, lsp::whole_grid(n_obj, grid));
}

size_t lsp_gen_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                               const lsp_options* opt_in) {
    if (n_obj < 1 || n_obs < 0 || !lsp::valid_grid(grid)) return 0;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    if (lsp::valid_options(&opt) != LSP_OK) return 0;
    const lsp::Rows rows = lsp::whole_grid(n_obj, grid);
    lsp::Method method;
    method.gen = true;
    lsp::Config c;
    if (lsp::resolve(n_obj, n_obs, grid, &opt, rows, &c, method) != LSP_OK) return 0;
    return lsp::layout(n_obj, grid, rows, c).total;
}

lsp_status lsp_gen_single(const double* t, const double* y, const double* dy, int64_t n_t,
                          const lsp_grid* grid, const lsp_options* opt, void* pgram,
                          lsp_peak* peak, void* workspace, size_t workspace_bytes, void* stream) {
    if (n_t < 0) return LSP_EINVAL;
    lsp::Method method;
    method.gen = true;
    method.dy = dy;
    return lsp::run(nullptr, 1, n_t, t, y, grid, opt, pgram, peak, workspace, workspace_bytes,
                    stream, lsp::whole_grid(1, grid), method);
}

lsp_status lsp_gen_batch(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                         const double* y, const double* dy, const lsp_grid* grid,
                         const lsp_options* opt, void* pgram, lsp_peak* peaks, void* workspace,
                         size_t workspace_bytes, void* stream) {
    if (!offsets) return LSP_EINVAL;
    lsp::Method method;
    method.gen = true;
    method.dy = dy;
    return lsp::run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                    workspace_bytes, stream, lsp::whole_grid(n_obj, grid), method);
}

static lsp_status batch_rows(const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                             const double* t, const double* y, const lsp_grid* grid,
                             const lsp_options* opt, const int32_t* row_obj,
                             const int32_t* row_band, int64_t n_rows, int64_t band_bins,
                             int32_t rows_per_group, void* pgram, lsp_peak* peaks,
                             void* workspace, size_t workspace_bytes, void* stream,
                             const lsp::Method& method) {
    if (!offsets) return LSP_EINVAL;
    if (!row_obj && n_rows != n_obj * (int64_t)rows_per_group) return LSP_EINVAL;
    if (!row_band) band_bins = grid ? grid->n_f : 0;
    const lsp::Rows rows{row_obj, row_band, n_rows, band_bins, rows_per_group, false};
    return lsp::run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                    workspace_bytes, stream, rows, method);
}

lsp_status lsp_batch_rows(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                          const double* y, const lsp_grid* grid, const lsp_options* opt,
                          const int32_t* row_obj, const int32_t* row_band, int64_t n_rows,
                          int64_t band_bins, int32_t rows_per_group, void* pgram,
                          lsp_peak* peaks, void* workspace, size_t workspace_bytes,
                          void* stream) {
    return batch_rows(offsets, n_obj, n_obs, t, y, grid, opt, row_obj, row_band, n_rows,
                      band_bins, rows_per_group, pgram, peaks, workspace, workspace_bytes,
                      stream, lsp::Method{});
}

lsp_status lsp_gen_batch_rows(const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                              const double* t, const double* y, const double* dy,
                              const lsp_grid* grid, const lsp_options* opt,
                              const int32_t* row_obj, const int32_t* row_band, int64_t n_rows,
                              int64_t band_bins, int32_t rows_per_group, void* pgram,
                              lsp_peak* peaks, void* workspace, size_t workspace_bytes,
                              void* stream) {
    lsp::Method method;
    method.gen = true;
    method.dy = dy;
    return batch_rows(offsets, n_obj, n_obs, t, y, grid, opt, row_obj, row_band, n_rows,
                      band_bins, rows_per_group, pgram, peaks, workspace, workspace_bytes,
                      stream, method);
}

static lsp_status plan_create(const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                              const double* t, const double* y, const lsp_grid* grid,
                              const lsp_options* opt, void* pgram, lsp_peak* peaks,
                              void* workspace, size_t workspace_bytes, lsp_plan* plan,
                              const lsp::Method& method) {
    if (!plan) return LSP_EINVAL;
    *plan = nullptr;
    if (!offsets && n_obj != 1) return LSP_EINVAL;
    // Validate first, on the host, so that an argument error never leaves a
    // half-open capture behind.
    {
        lsp_status st = lsp::validate(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks,
                                      workspace, workspace_bytes, lsp::whole_grid(n_obj, grid),
                                      method);
        if (st != LSP_OK) return st;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LSP_EHIP;
    hipGraph_t graph = nullptr;
    lsp_status st = LSP_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = LSP_EHIP;
    } else {
        st = lsp::run(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                      workspace_bytes, cs, lsp::whole_grid(n_obj, grid), method);
        if (hipStreamEndCapture(cs, &graph) != hipSuccess && st == LSP_OK) st = LSP_EHIP;
    }
    (void)hipStreamDestroy(cs);
    if (st != LSP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return LSP_EHIP;
    }
    lsp_plan p = new (std::nothrow) lsp_plan_s{graph, exec};
    if (!p) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return LSP_EHIP;
    }
    *plan = p;
    return LSP_OK;
}

lsp_status lsp_plan_create(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                           const double* y, const lsp_grid* grid, const lsp_options* opt,
                           void* pgram, lsp_peak* peaks, void* workspace, size_t workspace_bytes,
                           lsp_plan* plan) {
    return plan_create(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                       workspace_bytes, plan, lsp::Method{});
}

lsp_status lsp_gen_plan_create(const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                               const double* t, const double* y, const double* dy,
                               const lsp_grid* grid, const lsp_options* opt, void* pgram,
                               lsp_peak* peaks, void* workspace, size_t workspace_bytes,
                               lsp_plan* plan) {
    lsp::Method method;
    method.gen = true;
    method.dy = dy;
    return plan_create(offsets, n_obj, n_obs, t, y, grid, opt, pgram, peaks, workspace,
                       workspace_bytes, plan, method);
}

lsp_status lsp_plan_launch(lsp_plan plan, void* stream) {
    if (!plan) return LSP_EINVAL;
    return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? LSP_OK
                                                                                       : LSP_EHIP;
}

void lsp_plan_destroy(lsp_plan plan) {
    if (!plan) return;
    (void)hipGraphExecDestroy(plan->exec);
    (void)hipGraphDestroy(plan->graph);
    delete plan;
}

lsp_status lsp_describe_launch(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                               const lsp_options* opt_in, int32_t generalized,
                               lsp_options* resolved, int64_t* tile_freqs,
                               int64_t* tiles_per_item, int64_t* n_items) {
    if (!grid || !resolved || n_obj < 1 || n_obs < 0 || !lsp::is_bool(generalized))
        return LSP_EINVAL;
    if (!lsp::valid_grid(grid)) return LSP_EINVAL;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    lsp_status st = lsp::valid_options(&opt);
    if (st != LSP_OK) return st;
    lsp::Method method;
    method.gen = generalized != 0;
    lsp::Config c;
    st = lsp::resolve(n_obj, n_obs, grid, &opt, lsp::whole_grid(n_obj, grid), &c, method);
    if (st != LSP_OK) return st;
    lsp_options r = opt;
    r.k_per_lane = c.k;
    r.waves_per_wg = c.waves;
    r.t_split = c.split;
    r.schedule = c.persistent ? LSP_SCHED_PERSISTENT : LSP_SCHED_GRID;
    r.order = c.lpt ? LSP_ORDER_LPT : LSP_ORDER_INPUT;
    if (c.form == LSP_FORM_FP32P) {
        r.recurrence = c.rec;
        r.wave_split = c.ws ? LSP_WSPLIT_ON : LSP_WSPLIT_OFF;
        r.obs_read = c.obs;
        r.seed_trig = c.trig;
    }
    *resolved = r;
    if (tile_freqs) *tile_freqs = c.tile_freqs;
    if (tiles_per_item) *tiles_per_item = c.tiles_per_item;
    if (n_items) *n_items = c.n_items;
    return LSP_OK;
}

size_t lsp_row_order_workspace_bytes(void) {
    return ((size_t)(lsp::kOrderBlocks + 1) * lsp::kOrderBuckets * sizeof(unsigned int) + 255) /
           256 * 256;
}

lsp_status lsp_row_order(const int64_t* offsets, int64_t n_obj, const int32_t* row_obj,
                         const int32_t* row_band, int64_t n_rows, int32_t rows_per_group,
                         int32_t* perm, void* workspace, size_t workspace_bytes, void* stream) {
    if (!offsets || !perm || !workspace || n_obj < 1 || n_rows < 1 || rows_per_group < 1)
        return LSP_EINVAL;
    if (n_rows > (int64_t)INT32_MAX) return LSP_EINVAL;
    if (!row_obj && n_rows != n_obj * (int64_t)rows_per_group) return LSP_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % lsp::kAlign) return LSP_EINVAL;
    if (workspace_bytes < lsp_row_order_workspace_bytes()) return LSP_ENOMEM;
    lsp::OrderParams op;
    op.offsets = offsets;
    op.n_obj = n_obj;
    op.row_obj = row_obj;
    op.row_band = row_band;
    op.n_rows = n_rows;
    op.rows_per_group = rows_per_group;
    op.pad = 0;
    op.hist = static_cast<unsigned int*>(workspace);
    op.total = op.hist + (size_t)lsp::kOrderBlocks * lsp::kOrderBuckets;
    op.perm = perm;
    return lsp::launch_row_order(op, static_cast<hipStream_t>(stream)) == hipSuccess ? LSP_OK
                                                                                      : LSP_EHIP;
}

lsp_status lsp_set_stage_events(void* main_begin, void* main_end) {
    if ((main_begin == nullptr) != (main_end == nullptr)) return LSP_EINVAL;
    lsp::t_main_begin = static_cast<hipEvent_t>(main_begin);
    lsp::t_main_end = static_cast<hipEvent_t>(main_end);
    return LSP_OK;
}

const char* lsp_status_string(lsp_status status) {
    switch (status) {
        case LSP_OK: return "ok";
        case LSP_EINVAL: return "invalid argument";
        case LSP_ENOMEM: return "workspace too small";
        case LSP_EHIP: return "HIP launch failed";
        case LSP_EUNSUPPORTED: return "unsupported option combination";
        case LSP_ESCRATCH: return "call exceeds the static scratch of lsp_batch_static";
        default: return "unknown status";
    }
}

int32_t lsp_version(void) { return 100; }

}  // extern "C"
