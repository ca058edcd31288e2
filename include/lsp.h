/*
 * lsp.h -- C ABI of the MI355X (gfx950) Lomb-Scargle periodogram library.
 *
 * The library computes, for every (object, trial frequency) pair, the
 * Lomb-Scargle power of Gowanlock et al., arXiv 2105.04006:
 *   - the time offset tau of Eq. 1, tan(2 w tau) = sum sin 2wt / sum cos 2wt;
 *   - the shifted sums of Eq. 2, sum y cos w(t - tau), sum y sin w(t - tau),
 *     sum cos^2 w(t - tau), sum sin^2 w(t - tau), and from them the power;
 *   - the argmax over the grid and the best period p = 2 pi / w (Section 3.3).
 * It follows the paper's two modes: one series (Section 3.3, lsp_single) and a
 * batch of series sharing one frequency grid (Section 3.4, lsp_batch), with the
 * periodogram returned or left out and per-object peaks returned.
 *
 * Conventions common to every call
 *   - Array arguments are DEVICE pointers owned by the caller; the library never
 *     allocates, frees or retains them.  Struct arguments (grid, options) are
 *     HOST pointers read during the call only.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream) and enqueue only kernels, so they may be captured into a HIP
 *     graph.  They never synchronise the device.
 *   - Argument errors are detected on the host before anything is enqueued and
 *     returned as LSP_EINVAL / LSP_ENOMEM; nothing is written in that case.
 *   - Problems with one object's data are reported in that object's peak
 *     `status` (LSP_OBJ_*), never as a call failure.
 *   - No exceptions cross this interface; all functions are thread-safe.
 */
#ifndef LSP_H
#define LSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Call status. */
typedef enum {
    LSP_OK = 0,
    LSP_EINVAL = 1,       /* bad argument (NULL pointer, empty grid, bad enum ...) */
    LSP_ENOMEM = 2,       /* workspace smaller than lsp_workspace_bytes()          */
    LSP_EHIP = 3,         /* the HIP runtime refused a launch                      */
    LSP_EUNSUPPORTED = 4  /* valid but unsupported combination of options          */
} lsp_status;

/* Per-object status carried in lsp_peak.status. */
enum {
    LSP_OBJ_OK = 0,
    LSP_OBJ_DEGENERATE = 1, /* N_t < 2, or the centred magnitudes have no variance:
                               power 0 everywhere, peak index -1                   */
    LSP_OBJ_BADRANGE = 2,   /* CSR range negative, reversed or past n_obs:
                               power NaN everywhere, peak index -1                 */
    LSP_OBJ_NONFINITE = 3   /* a time or magnitude is Inf/NaN: power NaN, index -1 */
};

/* Arithmetic form of the hot loop. */
enum {
    LSP_FORM_FP64 = 0,  /* reference form: FP64 phases, FP64 library sin/cos per
                           term, FP64 sums (the method exactly as Section 2 states it) */
    LSP_FORM_FP32P = 1  /* FP32 sums and trig, phases reduced in FP64; sin/cos seeded
                           by the hardware per observation and advanced across a lane's
                           frequencies by angle addition; ill-conditioned bins
                           recomputed in FP64                                         */
};

/* Frequency unit of the grid. */
enum {
    LSP_UNIT_CYCLES = 0, /* f in cycles per time unit, w = 2 pi f, period = 1/f */
    LSP_UNIT_ANGULAR = 1 /* f is w itself (the paper's code), period = 2 pi / w  */
};

/* Element type of the periodogram output. */
enum { LSP_PGRAM_F32 = 0, LSP_PGRAM_F64 = 1 };

/* Work scheduling of the batch path. */
enum {
    LSP_SCHED_AUTO = 0,
    LSP_SCHED_GRID = 1,      /* one workgroup per (object, frequency tile)          */
    LSP_SCHED_PERSISTENT = 2 /* resident workgroups pop (object, tile) items from
                                per-XCD atomic queues                                */
};

/*
 * Uniform half-open grid of Section 2: df = (f_max - f_min) / n_f and
 * f_i = f_min + i * df for i = 0 .. n_f - 1 (f_max itself is excluded).
 */
typedef struct {
    double f_min;
    double f_max;
    int64_t n_f;
    int32_t unit; /* LSP_UNIT_* */
    int32_t reserved;
} lsp_grid;

/*
 * Options.  A zero-initialised struct means: FP64 form, unnormalised P_LS, y
 * used as given, FP32 periodogram, library-chosen tuning; callers normally
 * start from lsp_default_options().  Tuning fields left at 0 are chosen by the
 * library (built-in heuristics for the shape).
 */
typedef struct {
    int32_t form;          /* LSP_FORM_*                                               */
    int32_t normalize;     /* 1: P = 2 P_LS / sum (y - ybar)^2, in [0, 1];  0: P_LS     */
    int32_t subtract_mean; /* 1: remove each object's mean (FP64) before the sums;
                              0: use y as given (the paper assumes it is zero-mean)     */
    int32_t pgram_dtype;   /* LSP_PGRAM_F32 or LSP_PGRAM_F64                            */
    int32_t k_per_lane;    /* frequencies per lane: FP32P 4/8/16/32, FP64 1/2/4         */
    int32_t waves_per_wg;  /* wavefronts per workgroup: 1, 2 or 4                       */
    int32_t t_split;       /* single object: split of the observation axis, 1..64       */
    int32_t schedule;      /* LSP_SCHED_*                                               */
    int32_t reserved[4];
} lsp_options;

/* One object's peak (40 bytes). */
typedef struct {
    int64_t index;  /* argmax grid index, lowest on ties; -1 if status != OK         */
    double freq;    /* f_index in the grid's unit (NaN if index < 0)                 */
    double period;  /* 1/f (cycles) or 2 pi / f (angular); NaN if index < 0          */
    double power;   /* power at index (0 for DEGENERATE, NaN for BADRANGE/NONFINITE) */
    int32_t status; /* LSP_OBJ_*                                                     */
    int32_t reserved;
} lsp_peak;

/* Defaults: FP64 form, normalised power, mean removed, FP32 periodogram, auto tuning. */
lsp_options lsp_default_options(void);

/*
 * Device workspace (bytes, 256-aligned) that lsp_batch / lsp_single need for
 * n_obj objects holding n_obs observations in total on `grid` with `opt`.
 * Returns 0 if the arguments are invalid.  The workspace holds per-object
 * statistics (mean, S_yy, time origin, status), per-tile peak records and
 * flags, queue counters and (single object with t_split > 1) partial sums; its
 * contents are scratch.  t and y are only read, so objects whose CSR ranges
 * overlap are each computed from their own range.
 */
size_t lsp_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                           const lsp_options *opt);

/*
 * Single-periodogram mode (Section 3.3): one series of n_t observations.
 *   t, y      : device, n_t doubles each (time, magnitude), any order.
 *   pgram     : device, n_f elements of opt->pgram_dtype, or NULL (not written).
 *   peak      : device, one lsp_peak, or NULL.  At least one of pgram/peak must be
 *               non-NULL.
 *   workspace : device, >= lsp_workspace_bytes(1, n_t, grid, opt) bytes, 256-aligned.
 * Errors: LSP_EINVAL for NULL t/y/workspace, n_t < 0, n_f < 1, non-finite or
 * empty grid (f_max <= f_min), unknown enum values; LSP_ENOMEM for a short
 * workspace; LSP_EHIP if a launch fails.
 */
lsp_status lsp_single(const double *t, const double *y, int64_t n_t, const lsp_grid *grid,
                      const lsp_options *opt, void *pgram, lsp_peak *peak, void *workspace,
                      size_t workspace_bytes, void *stream);

/*
 * Batch mode (Section 3.4): n_obj series packed as CSR, object o owning
 * observations [offsets[o], offsets[o+1]) of t and y; all objects share `grid`.
 *   offsets   : device, n_obj + 1 int64 values.
 *   t, y      : device, n_obs doubles each.
 *   pgram     : device, n_obj * n_f elements (row-major, object-major) of
 *               opt->pgram_dtype, or NULL to keep only the peaks (Section 3.4's
 *               peaks-only variant).
 *   peaks     : device, n_obj lsp_peak records, or NULL.
 *   workspace : device, >= lsp_workspace_bytes(n_obj, n_obs, grid, opt) bytes.
 * Errors as lsp_single, plus LSP_EINVAL for NULL offsets or n_obj < 1, and
 * LSP_EUNSUPPORTED for t_split > 1 with n_obj > 1.
 */
lsp_status lsp_batch(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                     const double *y, const lsp_grid *grid, const lsp_options *opt, void *pgram,
                     lsp_peak *peaks, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Optional instrumentation for profiling.  After a call with non-NULL
 * handles, every later lsp_single / lsp_batch call made by the same host
 * thread records `main_begin` on its stream just before the main periodogram
 * kernel and `main_end` just after it, so hipEventElapsedTime gives that
 * kernel's own device time.  Both handles are hipEvent_t values owned by the caller; pass
 * NULL, NULL to stop.  Returns LSP_EINVAL if exactly one handle is NULL.
 */
lsp_status lsp_set_stage_events(void *main_begin, void *main_end);

/* Static, human-readable text for a status code. */
const char *lsp_status_string(lsp_status status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t lsp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LSP_H */
