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
    LSP_EUNSUPPORTED = 4, /* valid but unsupported combination of options          */
    LSP_ESCRATCH = 5      /* lsp_batch_static: the call needs more scratch than the
                             library's static device array holds                    */
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

/* Frequency-to-frequency recurrence of the FP32 form (within one lane). */
enum {
    LSP_REC_AUTO = 0,      /* the library's choice (currently LSP_REC_CHEBYSHEV)    */
    LSP_REC_ROTATION = 1,  /* (c, s) <- (c C - s S, s C + c S): 4 ops per step        */
    LSP_REC_CHEBYSHEV = 2  /* x_{k+1} = 2C x_k - x_{k-1} for x = cos, sin: 2 ops/step */
};

/* How the waves of a workgroup share a frequency tile (FP32 form). */
enum {
    LSP_WSPLIT_AUTO = 0, /* the library's choice: on, with 8 waves and no t_split, for
                            one object of >= 2,048 points on the whole grid when the
                            64 K-bin tiles give >= 3,584 waves (standard FP32 form
                            with waves_per_wg and t_split left at 0); else off     */
    LSP_WSPLIT_OFF = 1,  /* each wave owns 64 K of the tile's bins                   */
    LSP_WSPLIT_ON = 2    /* all waves cover the same 64 K bins and split the
                            observations; sums are added in LDS in wave order        */
};

/* How the FP32 form's workgroups read the observations (Sections 3.6 and 4.9
 * compare shared-memory staging with reading global memory directly). */
enum {
    LSP_OBS_AUTO = 0,   /* the library's choice (currently LSP_OBS_LDS)                */
    LSP_OBS_LDS = 1,    /* each workgroup stages tiles of (t - t0, y - ybar, step
                           rotation) in LDS; waves read them as broadcasts           */
    LSP_OBS_DIRECT = 2  /* a staging pass writes those per-observation values once to
                           the workspace; waves read them from global memory (wave-
                           uniform loads), no LDS and no barriers in the loop.  The
                           objects' CSR ranges must not overlap.                      */
};

/* How the FP32 form takes sin and cos of its FP64-reduced seed phases and of
 * the per-observation step rotation (Section 4.12 weighs the fast hardware
 * sine against the library function). */
enum {
    LSP_TRIG_AUTO = 0, /* the library's choice (currently LSP_TRIG_HW)                  */
    LSP_TRIG_HW = 1,   /* hardware v_sin_f32 / v_cos_f32 on the phase in revolutions   */
    LSP_TRIG_LIB = 2,  /* the HIP math library's sincospif                              */
    LSP_TRIG_POLY = 3  /* quarter-turn reduction and Taylor polynomials (degree 9 for
                          sin, 8 for cos) in FP32 FMAs                                */
};

/* Order in which a batch's rows (objects, or (object, band) rows of
 * lsp_batch_rows) are handed to the workgroups.  No result depends on it:
 * every bin and every peak is computed the same way in any order. */
enum {
    LSP_ORDER_AUTO = 0,  /* the library's choice: LPT for calls of >= 1e10 terms     */
    LSP_ORDER_INPUT = 1, /* rows in the order given                                  */
    LSP_ORDER_LPT = 2    /* longest processing time first: rows by descending N_t,
                            dealt round-robin over the 8 XCDs (lsp_row_order)      */
};

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
 * The FP32 forms merge each object's peak into a 64-bit key whose index field
 * holds 32 bits, so unless a single object's observations are split across
 * workgroups (t_split > 1) they accept n_f <= 2^32 - 2 and return
 * LSP_EUNSUPPORTED beyond; the FP64 form takes any n_f.
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
    int32_t k_per_lane;    /* frequencies per lane: FP32P 4/8/10/12/16/32, FP64 1/2/4   */
    int32_t waves_per_wg;  /* wavefronts per workgroup: 1, 2 or 4; 8 with wave_split on  */
    int32_t t_split;       /* single object: split of the observation axis, 1..64       */
    int32_t schedule;      /* LSP_SCHED_*                                               */
    int32_t recurrence;    /* LSP_REC_* (FP32 form only)                                */
    int32_t wave_split;    /* LSP_WSPLIT_* (FP32 form only)                             */
    int32_t obs_read;      /* LSP_OBS_* (FP32 form only)                                */
    int32_t seed_trig;     /* LSP_TRIG_* (FP32 form only)                               */
    int32_t order;         /* LSP_ORDER_* (batches and row mode)                        */
    int32_t reserved;      /* 0                                                         */
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
 * lsp_batch without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The scratch lsp_batch takes from `workspace` comes
 * instead from a static device array of LSP_STATIC_SCRATCH_BYTES that every
 * GPU the library runs on holds from the library's first use on it until the
 * process ends.  The call allocates nothing and, like lsp_batch, enqueues only
 * kernels on `stream`; its results equal lsp_batch's bit for bit (same
 * kernels, same launch configuration).
 *   All arguments: as lsp_batch.
 * The array's contents persist from call to call (each call re-initialises
 * what it reads), and all calls on one GPU share it: calls that overlap on
 * one GPU -- concurrent streams, host threads, or graph launches that may run
 * at the same time -- race and must be serialised by the caller.
 * Errors: as lsp_batch; LSP_ESCRATCH (nothing enqueued) when
 * lsp_workspace_bytes(n_obj, n_obs, grid, opt) exceeds
 * LSP_STATIC_SCRATCH_BYTES; LSP_EHIP if the array's device address cannot
 * be obtained.
 */
#define LSP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
lsp_status lsp_batch_static(const int64_t *offsets, int64_t n_obj, int64_t n_obs,
                            const double *t, const double *y, const lsp_grid *grid,
                            const lsp_options *opt, void *pgram, lsp_peak *peaks, void *stream);

/*
 * Generalized periodogram (Section 4.11): each observation carries an error
 * dy_j, and at every trial frequency the model y = a cos wt + b sin wt + c is
 * fitted by weighted least squares with weights 1 / dy_j^2 (the generalized
 * Lomb-Scargle method that the paper takes from Astropy, Zechmeister &
 * Kuerster 2009).  With normalize = 1 the power is the fraction of the
 * weighted variance about the weighted mean that the two trigonometric terms
 * explain, in [0, 1]; with normalize = 0 it is half the reduction in chi^2.
 * The mean is always fitted: subtract_mean has no effect.
 *   t, y, n_t, offsets, n_obj, n_obs, grid, pgram, peak(s), stream : as
 *               lsp_single / lsp_batch.
 *   dy        : device, errors in the layout of y (n_t or n_obs doubles), or
 *               NULL for unit errors (the floating-mean periodogram).  An object
 *               with an error that is not finite or not > 0 gets status
 *               LSP_OBJ_NONFINITE (power NaN, index -1).
 *   opt       : as lsp_single; form FP64 or FP32P.  The FP32P form has the
 *               three-term recurrence only and k_per_lane in {0, 4, 8, 12, 16}.
 *   workspace : >= lsp_gen_workspace_bytes(n_obj, n_obs, grid, opt) bytes
 *               (n_obj = 1 for lsp_gen_single), 256-byte aligned, owned by the
 *               caller.
 * Per-bin terms whose denominator is <= 1e-12 * sum(1/dy^2) are dropped; bins
 * the FP32P form cannot resolve are recomputed in FP64, as for lsp_single.
 * Errors as lsp_single / lsp_batch, plus LSP_EUNSUPPORTED for recurrence =
 * LSP_REC_ROTATION, wave_split = LSP_WSPLIT_ON, or k_per_lane 10 or 32 with
 * the FP32P form.  lsp_gen_workspace_bytes returns 0 for invalid arguments.
 */
size_t lsp_gen_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                               const lsp_options *opt);
lsp_status lsp_gen_single(const double *t, const double *y, const double *dy, int64_t n_t,
                          const lsp_grid *grid, const lsp_options *opt, void *pgram,
                          lsp_peak *peak, void *workspace, size_t workspace_bytes, void *stream);
lsp_status lsp_gen_batch(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                         const double *y, const double *dy, const lsp_grid *grid,
                         const lsp_options *opt, void *pgram, lsp_peak *peaks, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * Row mode and plan capture of the generalized periodogram: lsp_batch_rows,
 * lsp_rows_workspace_bytes and lsp_plan_create with errors dy (device, layout
 * of y, or NULL for unit errors) after y, and the generalized method's
 * option rules (see lsp_gen_batch).  Arguments, layouts and errors are
 * otherwise those of the standard calls; plans are launched and destroyed
 * with lsp_plan_launch / lsp_plan_destroy.
 */
size_t lsp_gen_rows_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                                    const lsp_options *opt, int64_t n_rows, int64_t band_bins,
                                    int32_t rows_per_group);
lsp_status lsp_gen_batch_rows(const int64_t *offsets, int64_t n_obj, int64_t n_obs,
                              const double *t, const double *y, const double *dy,
                              const lsp_grid *grid, const lsp_options *opt,
                              const int32_t *row_obj, const int32_t *row_band, int64_t n_rows,
                              int64_t band_bins, int32_t rows_per_group, void *pgram,
                              lsp_peak *peaks, void *workspace, size_t workspace_bytes,
                              void *stream);

/*
 * Returning whole periodograms to host memory (Section 3.5).  A pipe owns
 * n_streams lanes, each with a kernel and a copy HIP stream (default
 * priority), a pinned host staging buffer of staging_bytes and device buffers
 * for two chunks of objects (allocated on first use, grown when a later call
 * needs more), plus copy_threads host threads shared by the lanes;
 * lsp_pipe_destroy releases everything.  Zero arguments select the defaults:
 * 1 lane, 16 MiB staging, 128 MiB chunks, 12 copy threads.
 *   n_streams    : lanes, 1..8
 *   staging_bytes: >= 2 KiB, a multiple of 512; each half is one DMA piece
 *   chunk_bytes  : periodogram bytes per chunk of objects (at least one object)
 *   copy_threads : 1..64 host threads moving staged pieces to the caller's array
 * Returns LSP_EINVAL for out-of-range arguments or a NULL pipe pointer and
 * LSP_EHIP if a stream, event or pinned buffer cannot be had (*pipe is NULL).
 *
 * lsp_batch_to_host computes the batch (lsp_batch, or lsp_gen_batch when
 * generalized = 1) chunk by chunk on the pipe's streams and copies the
 * periodograms and/or peak records into HOST memory, overlapping one chunk's
 * kernels with another's device-to-host copy and a third's host copy; the
 * [n_obj x n_f] periodogram is never resident on the device.  It returns when
 * every byte has arrived.
 *   offsets, n_obj, n_obs, t, y, grid, opt : as lsp_batch (device inputs);
 *               t_split must be 0 or 1.
 *   dy        : device errors for the generalized periodogram, or NULL (must be
 *               NULL when generalized = 0).
 *   host_pgram: host (pageable or pinned) array of n_obj * n_f values of
 *               opt->pgram_dtype, row-major, or NULL.
 *   host_peaks: host array of n_obj lsp_peak records, or NULL; at least one of
 *               host_pgram / host_peaks must be given.
 *   stream    : the caller's stream; the pipe's streams wait until it reaches
 *               the call before reading the inputs.
 * The results equal lsp_batch's bit for bit.  Calls on one pipe must not
 * overlap.  Errors: LSP_EINVAL for NULL pipe, offsets or grid, n_obj < 1,
 * both outputs NULL, dy with generalized = 0, or options / grid that
 * lsp_batch (lsp_gen_batch) would reject; LSP_EUNSUPPORTED for t_split > 1;
 * LSP_EHIP if a device buffer cannot be allocated or a launch or copy fails.
 */
typedef struct lsp_pipe_s *lsp_pipe;
lsp_status lsp_pipe_create(int32_t n_streams, size_t staging_bytes, size_t chunk_bytes,
                           int32_t copy_threads, lsp_pipe *pipe);
void lsp_pipe_destroy(lsp_pipe pipe);
lsp_status lsp_batch_to_host(lsp_pipe pipe, const int64_t *offsets, int64_t n_obj, int64_t n_obs,
                             const double *t, const double *y, const double *dy,
                             int32_t generalized, const lsp_grid *grid, const lsp_options *opt,
                             void *host_pgram, lsp_peak *host_peaks, void *stream);

/*
 * Row mode: the batch kernels of Section 3.4 applied to chosen parts of the
 * grid, for refining proposed frequency bands or re-running chosen objects
 * (the paper evaluates whole grids only; this is the same per-bin arithmetic
 * on fewer bins).  A row is one object and either its whole grid (row_band ==
 * NULL) or band b, the bins [b * band_bins, min((b + 1) * band_bins, n_f)).
 * Consecutive runs of rows_per_group rows form a group whose peak is reduced
 * together and written to peaks[row_obj[first row of the group]]; every row
 * of a group must name that same object and no object may head two groups.
 *   offsets, t, y, grid, opt : as lsp_batch (per-object statistics are taken
 *               over the whole CSR range, whatever the rows).
 *   row_obj   : device, n_rows int32 object indices in [0, n_obj), or NULL
 *               when n_rows == n_obj * rows_per_group and row r belongs to object
 *               r / rows_per_group.  Rows naming an index outside [0, n_obj), or
 *               a negative band, evaluate nothing.
 *   row_band  : device, n_rows int32 band indices, or NULL.
 *   band_bins : bins per band, 1..n_f (ignored when row_band is NULL).
 *   pgram     : as lsp_batch, but only the bins of the rows are written.
 *   peaks     : device, n_obj records of which only group heads are written;
 *               the peak is the best bin over the group's rows (index -1 and
 *               power NaN if they hold no bin).
 *   workspace : >= lsp_rows_workspace_bytes(n_obj, n_obs, grid, opt, n_rows,
 *               band_bins (0 when row_band is NULL), rows_per_group) bytes.
 * Errors as lsp_batch, plus LSP_EINVAL for NULL row_obj with n_rows other than
 * n_obj * rows_per_group, n_rows < 1,
 * rows_per_group < 1 or not dividing n_rows, band_bins outside 1..n_f, and
 * LSP_EUNSUPPORTED for t_split > 1.
 */
size_t lsp_rows_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                                const lsp_options *opt, int64_t n_rows, int64_t band_bins,
                                int32_t rows_per_group);
lsp_status lsp_batch_rows(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                          const double *y, const lsp_grid *grid, const lsp_options *opt,
                          const int32_t *row_obj, const int32_t *row_band, int64_t n_rows,
                          int64_t band_bins, int32_t rows_per_group, void *pgram,
                          lsp_peak *peaks, void *workspace, size_t workspace_bytes,
                          void *stream);

/*
 * Captured calls (HIP graphs).  A plan records one lsp_single (offsets ==
 * NULL, n_obj == 1) or lsp_batch call with fixed arguments and buffers into a
 * HIP graph; launching the plan replays every kernel of the call with one
 * hipGraphLaunch, removing the per-kernel launch overhead of repeated calls on
 * the same buffers (Section 3.4 notes that many small launches cost time).
 * The buffers must stay allocated, unmoved and unaliased by other work for the
 * plan's lifetime; their contents may change between launches.  The plan owns
 * only host-side graph objects.  Argument errors are those of lsp_single /
 * lsp_batch; LSP_EHIP if capture or instantiation fails.  Launches of one plan
 * must not overlap each other (they share the workspace).
 */
typedef struct lsp_plan_s *lsp_plan;

lsp_status lsp_plan_create(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                           const double *y, const lsp_grid *grid, const lsp_options *opt,
                           void *pgram, lsp_peak *peaks, void *workspace, size_t workspace_bytes,
                           lsp_plan *plan);
lsp_status lsp_gen_plan_create(const int64_t *offsets, int64_t n_obj, int64_t n_obs,
                               const double *t, const double *y, const double *dy,
                               const lsp_grid *grid, const lsp_options *opt, void *pgram,
                               lsp_peak *peaks, void *workspace, size_t workspace_bytes,
                               lsp_plan *plan);
lsp_status lsp_plan_launch(lsp_plan plan, void *stream);
void lsp_plan_destroy(lsp_plan plan);

/*
 * Launch-shape autotuner for the FP32 form.  Times candidate shapes (K
 * frequencies per lane, wavefronts per workgroup, recurrence, schedule and,
 * for one object, the observation split) on the caller's data -- for a batch,
 * on a prefix of its objects holding about 1e11 evaluations -- and writes the
 * fastest candidate whose peaks agree with the FP64 form on those objects
 * (within one bin on >= 99.9% of them, |dP| <= 1e-3 at the peaks) to *tuned
 * (base's other fields are kept).  offsets == NULL tunes single-object mode.
 *   peak_scratch : device, >= n_obj lsp_peak records (overwritten).
 *   workspace    : device, >= lsp_autotune_workspace_bytes(...) bytes; smaller
 *                  workspaces skip the candidates that do not fit.
 *   cache_path   : host string or NULL.  When given, a JSON-lines file keyed by
 *                  device architecture and the log2 classes of n_obj, mean N_t
 *                  and n_f: a cached entry is returned without timing, and new
 *                  results are appended.
 *   repeats      : timed launches per candidate (>= 1).
 * Synchronous (it reads results back to the host); allocates no device
 * memory.  Errors as lsp_batch, LSP_EUNSUPPORTED if no candidate passes.
 */
size_t lsp_autotune_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                                    const lsp_options *base);
lsp_status lsp_autotune(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                        const double *y, const lsp_grid *grid, const lsp_options *base,
                        lsp_options *tuned, lsp_peak *peak_scratch, void *workspace,
                        size_t workspace_bytes, const char *cache_path, int32_t repeats,
                        void *stream);

/*
 * Band-proposal features.  The paper evaluates every bin; the learned path
 * evaluates only bands proposed from these per-object features (1,088 FP32
 * values per object, row-major [n_obj][LSP_FEAT_DIM]):
 *   [0, 1024)    coarse spectrum: the series is cut into seasons (a new season
 *                at every gap longer than season_gap) and consecutive seasons
 *                are grouped until a group holds min_season_obs observations (a
 *                trailing group with fewer is dropped); each group gets the
 *                normalised power of Section 2 (Eq. 1-2) of the object's
 *                centred magnitudes y - ybar (the group mean is not removed
 *                again) on 8,192 bins over [grid->f_min, grid->f_max) in the
 *                grid's unit;
 *                bins are max-pooled in runs of 8 and averaged over the groups
 *                (0 if none).  FP32 arithmetic as in LSP_FORM_FP32P, no FP64 fix-up;
 *                each value is clamped to [0, 1].
 *   [1024, 1088) sampling and magnitude statistics (FP64; the spectral window
 *                below takes FP64-reduced phases into FP32 sin/cos): log10 N_t,
 *                log10 max(span, 1e-3), number of seasons, number with >=
 *                min_season_obs points, log10 max(mean within-season spacing,
 *                1e-6), standard deviation of log10 max(spacing, 1e-6), fraction
 *                of points in qualifying seasons, log10 sigma_y, skewness,
 *                excess kurtosis, max |y - ybar| / sigma_y, then the spectral
 *                window |sum_j exp(2 pi i f_p t_j)|^2 / N_t^2 at the 53
 *                frequencies f_p = 10^(-3 + p (log10 30 + 3) / 52), p = 0..52,
 *                in cycles per time unit.
 * Observations are taken in the order given (time order for sorted input).
 * Objects whose status would not be LSP_OBJ_OK get an all-zero row.
 *   grid      : f_min, f_max and unit are used; n_f is ignored.
 *   features  : device, n_obj * LSP_FEAT_DIM floats.
 *   workspace : device, >= lsp_features_workspace_bytes(n_obj) bytes, 256-aligned.
 * Errors: LSP_EINVAL for NULL offsets/features/workspace/grid, n_obj < 1, a
 * bad grid range or unit, season_gap negative or non-finite, min_season_obs < 2;
 * LSP_ENOMEM for a short workspace.
 */
#define LSP_FEAT_COARSE 1024
#define LSP_FEAT_POOL 8
#define LSP_FEAT_WINDOW 64
#define LSP_FEAT_DIM (LSP_FEAT_COARSE + LSP_FEAT_WINDOW)

typedef struct {
    double season_gap;      /* time units; default 60                         */
    int32_t min_season_obs; /* default 8, at least 2                          */
    int32_t reserved;
} lsp_feature_options;

lsp_feature_options lsp_default_feature_options(void);
size_t lsp_features_workspace_bytes(int64_t n_obj);
lsp_status lsp_features(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                        const double *y, const lsp_grid *grid, const lsp_feature_options *fopt,
                        float *features, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Learned band proposal: building blocks of the small network that proposes
 * which frequency bands to refine.  BF16 arrays are passed as raw 16-bit words
 * (upper half of an IEEE single, round-to-nearest-even); all pointers are
 * device pointers; all calls are asynchronous on `stream`.
 *
 * lsp_gemm_bf16: C = op(A) op(B) (+ bias) (ReLU) (masked), M x N, FP32
 *   accumulation on the matrix cores.  A(m, k) is A[m*sam + k*sak] and B(k, n)
 *   is B[k*sbk + n*sbn] (BF16), so X.W, dY.W^T and X^T.dY are all expressible.
 *   bias: FP32 [N] or NULL.  relu: 0/1.  mask: BF16 [M x ldc] or NULL; where
 *   mask <= 0 the result is set to 0 (ReLU backward).  Results go to C (FP32)
 *   and/or C_bf16 (BF16), leading dimension ldc >= N; at least one non-NULL.
 *   Errors: LSP_EINVAL for negative sizes, NULL operands, ldc < N;
 *   LSP_EUNSUPPORTED if M or N exceeds 65535 tiles of 64.
 */
lsp_status lsp_gemm_bf16(int64_t M, int64_t N, int64_t K, const void *A, int64_t sam,
                         int64_t sak, const void *B, int64_t sbk, int64_t sbn, const float *bias,
                         const void *mask, int32_t relu, float *C, void *C_bf16, int64_t ldc,
                         void *stream);

/* Row-wise softmax cross-entropy of logits [n x c] against labels [n]:
 * loss_rows[i] = log sum_j exp z_ij - z_i,label, gradient (softmax - onehot) *
 * scale into dlogits (FP32) and/or dlogits_bf16.  A row whose label lies
 * outside [0, c) is ignored: zero loss and zero gradient.  Output pointers may
 * be NULL. */
lsp_status lsp_softmax_xent(const float *logits, const int32_t *labels, int64_t n, int32_t c,
                            float scale, float *dlogits, void *dlogits_bf16, float *loss_rows,
                            void *stream);

/* out[j] = sum_i x[i*c + j] (FP32, fixed order): bias gradients. */
lsp_status lsp_col_sums(const float *x, int64_t n, int32_t c, float *out, void *stream);

/* Column mean and 1/standard deviation of x [n x d] (0 where a column is
 * constant, so that it standardises to 0), for standardising network inputs. */
lsp_status lsp_col_stats(const float *x, int64_t n, int32_t d, float *mean, float *inv_std,
                         void *stream);

/* out = BF16((x - mean) * inv_std) column-wise, x [n x d] FP32. */
lsp_status lsp_standardize_bf16(const float *x, int64_t n, int32_t d, const float *mean,
                                const float *inv_std, void *out, void *stream);

/* out[i] = BF16(x[i]). */
lsp_status lsp_cast_bf16(const float *x, int64_t count, void *out, void *stream);

/* One Adam step (bias-corrected, step >= 1) on FP32 parameters param[count]
 * with moments m, v; refreshes param_bf16 (BF16 copy) when non-NULL. */
lsp_status lsp_adam(float *param, const float *grad, float *m, float *v, int64_t count,
                    int32_t step, float lr, float beta1, float beta2, float eps,
                    void *param_bf16, void *stream);

/*
 * The proposal network as a whole (not in the paper: it picks the bands on
 * which Section 2's power is evaluated; the layer order lives here, behind
 * the ABI): input
 * x [n x dims[0]] BF16 -> ReLU(x W_0 + b_0) -> ReLU(. W_1 + b_1) -> . W_2 + b_2
 * = logits [n x dims[3]] FP32.  W_l is [dims[l] x dims[l+1]] row-major; the
 * GEMMs read its BF16 copy w_bf16[l], the optimiser updates the FP32 master
 * w[l] and refreshes the copy.  Every pointer is a caller-owned device
 * pointer; nothing is allocated or freed.
 */
typedef struct {
    int32_t dims[4]; /* input, first hidden, second hidden, output widths (each >= 1) */
    float *w[3];     /* FP32 master weights W_l                                        */
    float *b[3];     /* FP32 biases b_l [dims[l+1]]                                   */
    void *w_bf16[3]; /* BF16 copies of W_l (the GEMM operands)                        */
} lsp_mlp;

/* Per-parameter arrays shaped like lsp_mlp's w and b: gradients, or Adam's
 * first and second moments. */
typedef struct {
    float *w[3];
    float *b[3];
} lsp_mlp_grads;

/* Forward pass of n rows: the two hidden activations go to h1 [n x dims[1]]
 * and h2 [n x dims[2]] (BF16, kept for lsp_mlp_backward) and the logits to
 * logits [n x dims[3]] (FP32).  Errors: LSP_EINVAL for a NULL or malformed
 * net (a width < 1 or a NULL parameter), n < 0, NULL arrays with n > 0. */
lsp_status lsp_mlp_forward(const lsp_mlp *net, const void *x_bf16, int64_t n, void *h1_bf16,
                           void *h2_bf16, float *logits, void *stream);

/* Device scratch lsp_mlp_backward needs for n rows (0 for a malformed net or
 * n < 1).  Its layout, for callers that inspect the intermediate gradients:
 * dlogits FP32 [n x dims[3]], dlogits BF16, dz2 FP32 [n x dims[2]], dz2 BF16,
 * dz1 FP32 [n x dims[1]], dz1 BF16, in that order, each section starting on
 * a 256-byte boundary (dz_l: the gradient at hidden layer l's
 * pre-activation). */
size_t lsp_mlp_workspace_bytes(const lsp_mlp *net, int64_t n);

/* Gradients of sum_i scale * loss_i, with loss_i the softmax cross-entropy of
 * row i's logits against labels[i] (a label outside [0, dims[3]) contributes
 * nothing), from the activations and logits of lsp_mlp_forward on the same
 * x: dW_l, db_l into grads (overwritten), and each row's loss into loss_rows
 * [n] (may be NULL).  The hidden-layer gradients pass through BF16 as the
 * GEMM operands do.  Errors: LSP_EINVAL for a malformed net or grads, n < 1,
 * NULL inputs; LSP_ENOMEM if workspace_bytes < lsp_mlp_workspace_bytes. */
lsp_status lsp_mlp_backward(const lsp_mlp *net, const void *x_bf16, const int32_t *labels,
                            int64_t n, const void *h1_bf16, const void *h2_bf16,
                            const float *logits, float scale, const lsp_mlp_grads *grads,
                            float *loss_rows, void *workspace, size_t workspace_bytes,
                            void *stream);

/* One Adam step (lsp_adam) on every parameter of net, W_0, b_0, W_1, b_1, W_2,
 * b_2 in that order, with moments m and v, refreshing the BF16 weight copies.
 * Errors: LSP_EINVAL for a malformed net, grads or moments, step < 1. */
lsp_status lsp_mlp_adam(const lsp_mlp *net, const lsp_mlp_grads *grads, const lsp_mlp_grads *m,
                        const lsp_mlp_grads *v, int32_t step, float lr, float beta1, float beta2,
                        float eps, void *stream);

/* Per row of logits [n x c] (c <= 128): the k largest entries' indices in
 * decreasing order (lowest index on ties) into idx [n x k], and the softmax
 * probability mass of those k entries into mass [n] (may be NULL). */
lsp_status lsp_top_k(const float *logits, int64_t n, int32_t c, int32_t k, int32_t *idx,
                     float *mass, void *stream);

/* Band strength from the coarse spectrum: out[i][b] = max of row i's columns
 * [start + b*group, start + (b+1)*group), b < n_bands (FP32 in, FP32 out
 * [n x n_bands]).  With lsp_top_k it gives the bands whose coarse power peaks
 * highest, proposals that need no training. */
lsp_status lsp_band_max(const float *x, int64_t n, int32_t d, int32_t start, int32_t n_bands,
                        int32_t group, float *out, void *stream);

/* Adaptive band count.  Row i's `top` proposed bands idx [n x top] -- the
 * first n_net from the network in decreasing probability, the rest by
 * decreasing coarse power (as lsp_top_k and lsp_merge_bands leave them) --
 * are copied to out [n x top] or replaced by -1 (a row lsp_batch_rows skips):
 * a network slot is kept while the softmax mass of the kept network slots
 * before it is below tau (the first is always kept; tau > 1 keeps all); a
 * coarse slot is kept if score[i][band] >= alpha * max_b score[i][b] (alpha
 * <= 0 keeps all; the first slot of a row with n_net = 0 is always kept).
 * logits, score: [n x c] FP32 (c <= 128 bands), logits required when
 * n_net > 0, score may be NULL (coarse slots then kept).  kept_mass [n] (may
 * be NULL) receives the softmax mass of the kept network slots.  Errors:
 * LSP_EINVAL for bad sizes, NaN thresholds or missing arrays; LSP_EHIP. */
lsp_status lsp_trim_bands(const int32_t *idx, int64_t n, int32_t top, int32_t n_net,
                          const float *logits, const float *score, int32_t c, float tau,
                          float alpha, int32_t *out, float *kept_mass, void *stream);

/* Per row, merge two band lists: the entries of a [n x ka] in order, then
 * those of b [n x kb] not already taken, until k_out (<= 128) distinct
 * non-negative bands are in out [n x k_out]; -1 fills the rest (a row with
 * band -1 evaluates nothing in lsp_batch_rows). */
lsp_status lsp_merge_bands(const int32_t *a, int32_t ka, const int32_t *b, int32_t kb, int64_t n,
                           int32_t k_out, int32_t *out, void *stream);

/* In place, for each row of x [n x d] (FP32): columns [start, start + count)
 * become (x - row mean) / row standard deviation over those columns (0 for a
 * constant row).  Applied to the coarse spectrum so that the network sees its
 * shape rather than its level. */
lsp_status lsp_row_normalize(float *x, int64_t n, int32_t d, int32_t start, int32_t count,
                             void *stream);

/* Pool the statistics of columns [start, start + count) (as produced by
 * lsp_col_stats) into one mean and 1/std for the whole block, so that columns
 * that are shifted copies of each other share one scale. */
lsp_status lsp_pool_stats(float *mean, float *inv_std, int32_t start, int32_t count,
                          void *stream);

/* Training-time shift augmentation of BF16 rows x [n x d]: the first n_coarse
 * = group * n_bands columns move by shifts[i] groups of `group` columns
 * (vacated columns get `fill`), other columns are copied, and labels[i] moves
 * by shifts[i] (-1 if it leaves [0, n_bands) or was -1).  Shifts are supplied
 * by the caller (its random draws). */
lsp_status lsp_shift_bands(const void *x_bf16, const int32_t *labels, const int32_t *shifts,
                           int64_t n, int32_t d, int32_t n_coarse, int32_t group, int32_t n_bands,
                           float fill, void *out_bf16, int32_t *out_labels, void *stream);

/* Training labels for the proposal: labels[i] = peaks[i].index / band_bins for
 * an object with status OK and a peak in bands [0, n_bands), else -1 (ignored
 * by lsp_softmax_xent). */
lsp_status lsp_peak_bands(const lsp_peak *peaks, int64_t n, int64_t band_bins, int32_t n_bands,
                          int32_t *labels, void *stream);

/* Fallback selection after refining proposed bands: writes to objects[] the
 * indices, in increasing order, of the objects with status OK whose refined
 * peak is missing, has power below power_min (or NaN), or whose proposal mass
 * (mass[i], the softmax mass of the refined bands; mass may be NULL) is below
 * mass_min, and their number to *count (device int32).  objects must hold n
 * entries.  One workgroup; n <= INT32_MAX. */
lsp_status lsp_select_fallback(const lsp_peak *peaks, const float *mass, int64_t n,
                               float mass_min, float power_min, int32_t *objects, int32_t *count,
                               void *stream);

/*
 * The launch shape a whole-grid call (lsp_single when n_obj == 1, else
 * lsp_batch; lsp_gen_* when generalized == 1) resolves for this shape and
 * these options: the tuning fields of `opt` left at 0 filled with the
 * library's choices, the bins one frequency tile covers, the consecutive
 * tiles one work item takes and the number of work items.  It is what the
 * call would enqueue; nothing is launched.  Used to state the K, recurrence
 * and schedule behind a measurement (the work per bin of Section 2 depends
 * on them).
 *   resolved : host, receives the options with every AUTO / 0 field resolved
 *              (form, normalize, subtract_mean and pgram_dtype as given).
 *   tile_freqs, tiles_per_item, n_items : host, may be NULL.
 * Errors: LSP_EINVAL / LSP_EUNSUPPORTED as the call itself would return them
 * (NULL grid or resolved, n_obj < 1, n_obs < 0, bad grid or options).
 */
lsp_status lsp_describe_launch(int64_t n_obj, int64_t n_obs, const lsp_grid *grid,
                               const lsp_options *opt, int32_t generalized,
                               lsp_options *resolved, int64_t *tile_freqs,
                               int64_t *tiles_per_item, int64_t *n_items);

/*
 * The longest-first row order the batch calls use with LSP_ORDER_LPT
 * (Graham's longest-processing-time-first rule for independent jobs).  The
 * paper gives each object its own thread block (Section 3.4) and leaves the
 * order to the hardware; here a row's cost is the observation count of its
 * object, offsets[o+1] - offsets[o] (0 for a negative count), compared exactly
 * below 1,024 and to 1/64 of an octave above; rows with no work at all (an
 * object index outside 0..n_obj-1 or a negative band) come after every other
 * row.  Position s of the descending order is dealt to XCD
 * s % 8: perm lists XCD 0's rows, then XCD 1's, ..., each run in descending
 * cost; the runs are contiguous and balanced (the first n_rows % 8 runs hold
 * one row more).  Rows of equal cost appear in no particular order.
 *   offsets        : device, n_obj + 1 int64 (CSR offsets as lsp_batch).
 *   row_obj        : device int32[n_rows], or NULL: row r is object
 *                    r / rows_per_group (then n_rows = n_obj * rows_per_group).
 *   row_band       : device int32[n_rows], or NULL; as lsp_batch_rows.
 *   perm           : device int32[n_rows], written: a permutation of 0..n_rows-1.
 *   workspace      : device, >= lsp_row_order_workspace_bytes() bytes,
 *                    256-aligned, scratch.
 * Errors: LSP_EINVAL for NULL offsets/perm/workspace, n_obj < 1, n_rows < 1 or
 * above 2^31 - 1, rows_per_group < 1, a row count that does not match, or a
 * misaligned workspace; LSP_ENOMEM for a short workspace; LSP_EHIP if a launch
 * fails.  Asynchronous on `stream`; enqueues kernels only (no memset, no
 * allocation).
 */
size_t lsp_row_order_workspace_bytes(void);
lsp_status lsp_row_order(const int64_t *offsets, int64_t n_obj, const int32_t *row_obj,
                         const int32_t *row_band, int64_t n_rows, int32_t rows_per_group,
                         int32_t *perm, void *workspace, size_t workspace_bytes, void *stream);

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
