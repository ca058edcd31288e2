/*
 * lsp_oracle.c -- plain, slow, FP64 CPU oracle for the Lomb-Scargle periodogram.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU-baseline
 * leg of the benchmark have an independent statement of what the method
 * computes.  It shares no code, header, constant or table with the GPU path.
 *
 * What it computes (Gowanlock et al., arXiv 2105.04006, Section 2):
 *   - the magnitudes are made zero-mean first (Section 2, first paragraph);
 *   - tau from Eq. 1:  tan(2 w tau) = sum_j sin(2 w t_j) / sum_j cos(2 w t_j);
 *   - the power from Eq. 2, literally, as a second pass over the series:
 *       P_LS = 1/2 [ (sum X_j cos w(t_j-tau))^2 / sum cos^2 w(t_j-tau)
 *                  + (sum X_j sin w(t_j-tau))^2 / sum sin^2 w(t_j-tau) ];
 *   - the uniform half-open grid of Section 2: df = (f_max - f_min)/N_f,
 *     f_i = f_min + i*df, i = 0..N_f-1;
 *   - the best period from the argmax of the periodogram, first index on ties,
 *     p = 2 pi / w (Section 3.3; equivalently 1/f when f is in cycles).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - normalised power P_norm = 2 P_LS / sum_j (y_j - ybar)^2, which lies in [0,1];
 *   - a term of Eq. 2 whose denominator is <= 1e-12 * N_t is dropped (this is the
 *     projection onto the non-vanishing regressor; it makes w = 0 give P = 0);
 *   - w = 0 gives tau = 0 (Eq. 1 is 0/0 there);
 *   - an object with N_t < 2, or whose centred magnitudes have no variance
 *     (S_yy <= 1e-20 * sum y^2), is DEGENERATE: power 0, peak index -1;
 *   - an object with a non-finite time or magnitude is NONFINITE and a CSR range
 *     that is negative, reversed or past the end is BADRANGE: power NaN, index -1.
 *
 * Sums use Neumaier's compensated summation and every angle w (t - tau) is
 * formed and reduced modulo 2 pi in long double before the double sin and cos,
 * so that the oracle is the more accurate side of every comparison.  Compile with -ffp-contract=off and no
 * fast-math: every operation is the one written.
 *
 * Parallelism follows the paper's CPU port (Section 4.5): a static split over
 * frequencies for one object, dynamic scheduling over objects for a batch.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_DEGENERATE 1
#define ORA_BADRANGE 2
#define ORA_NONFINITE 3

#define ORA_UNIT_CYCLES 0
#define ORA_UNIT_ANGULAR 1

static const double ORA_TWO_PI = 6.283185307179586476925286766559;
static const long double ORA_TWO_PI_L = 6.283185307179586476925286766559L;

typedef struct {
    int64_t index;
    double freq;
    double period;
    double power;
    int32_t status;
    int32_t pad;
} ora_peak;

/* Neumaier compensated accumulator. */
typedef struct {
    double s;
    double c;
} ora_sum;

static void ora_sum_add(ora_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double ora_sum_get(const ora_sum *a) { return a->s + a->c; }

/* Section 2: df = (f_max - f_min) / N_f and f_i = f_min + i * df. */
double ora_grid_freq(double f_min, double f_max, int64_t n_f, int64_t i)
{
    double df = (f_max - f_min) / (double)n_f;
    return f_min + df * (double)i;
}

/* Section 2: w = 2 pi f.  The paper's code takes w directly (angular unit). */
double ora_omega(double f, int32_t unit)
{
    if (unit == ORA_UNIT_ANGULAR)
        return f;
    return ORA_TWO_PI * f;
}

/* Section 3.3: period from the peak frequency, p = 2 pi / w. */
double ora_period(double f, int32_t unit)
{
    return ORA_TWO_PI / ora_omega(f, unit);
}

/* Angular frequency in long double (exact for the angular unit). */
static long double ora_omega_l(double f, int32_t unit)
{
    if (unit == ORA_UNIT_ANGULAR)
        return (long double)f;
    return ORA_TWO_PI_L * (long double)f;
}

/*
 * sin and cos of the angle w (t - shift).  On the workloads the angle reaches
 * ~5e5 rad (24 cycles/day over 3,650 days), where forming it in double would
 * round it by up to ~1e-10 rad -- more than the GPU forms' phases, which are
 * taken on re-centred times -- so it is formed and reduced modulo 2 pi in long
 * double (64-bit significand; the reduced angle is off by ~1e-13 rad at most),
 * and only the reduced angle goes to the double-precision sin and cos.
 */
static void ora_sincos(long double w, double t, long double shift, double *s, double *c)
{
    long double a = w * ((long double)t - shift);
    long double k = rintl(a / ORA_TWO_PI_L);
    double r = (double)(a - k * ORA_TWO_PI_L);
    *s = sin(r);
    *c = cos(r);
}

/*
 * Mean removal (Section 2 assumes zero-mean magnitudes).  Writes the centred
 * magnitudes to yp[n] and their sum of squares to *syy; returns the object's
 * status.
 */
int32_t ora_prep(const double *t, const double *y, int64_t n, int32_t subtract_mean,
                 double *yp, double *syy)
{
    int64_t j;
    ora_sum sy = {0.0, 0.0}, sq = {0.0, 0.0}, sraw = {0.0, 0.0};
    double ybar = 0.0;
    *syy = 0.0;
    for (j = 0; j < n; j++)
        if (!isfinite(t[j]) || !isfinite(y[j]))
            return ORA_NONFINITE;
    if (n < 2) {
        for (j = 0; j < n; j++)
            yp[j] = 0.0;
        return ORA_DEGENERATE;
    }
    if (subtract_mean) {
        for (j = 0; j < n; j++)
            ora_sum_add(&sy, y[j]);
        ybar = ora_sum_get(&sy) / (double)n;
    }
    for (j = 0; j < n; j++) {
        yp[j] = y[j] - ybar;
        ora_sum_add(&sq, yp[j] * yp[j]);
        ora_sum_add(&sraw, y[j] * y[j]);
    }
    *syy = ora_sum_get(&sq);
    if (*syy <= 1e-20 * ora_sum_get(&sraw) || *syy == 0.0)
        return ORA_DEGENERATE;
    return ORA_OK;
}

/* Eq. 1: tau = atan2(sum sin 2wt, sum cos 2wt) / (2w); tau = 0 at w = 0. */
static long double ora_tau_l(const double *t, int64_t n, long double w)
{
    int64_t j;
    ora_sum ss = {0.0, 0.0}, sc = {0.0, 0.0};
    if (w == 0.0L)
        return 0.0L;
    for (j = 0; j < n; j++) {
        double s2, c2;
        ora_sincos(2.0L * w, t[j], 0.0L, &s2, &c2);
        ora_sum_add(&ss, s2);
        ora_sum_add(&sc, c2);
    }
    return (long double)atan2(ora_sum_get(&ss), ora_sum_get(&sc)) / (2.0L * w);
}

double ora_tau(const double *t, int64_t n, double w)
{
    return (double)ora_tau_l(t, n, (long double)w);
}

/*
 * Eq. 2 at a given tau: the second pass over the series.  Returns P_LS and,
 * when sums != NULL, stores {YC, YS, CC, SS} = {sum y cos, sum y sin,
 * sum cos^2, sum sin^2} of the shifted phase w (t_j - tau).
 */
static double ora_pls_l(const double *t, const double *yp, int64_t n, long double w,
                        long double tau, double *sums)
{
    int64_t j;
    ora_sum yc = {0.0, 0.0}, ys = {0.0, 0.0}, cc = {0.0, 0.0}, ss = {0.0, 0.0};
    double YC, YS, CC, SS, p;
    for (j = 0; j < n; j++) {
        double c, s;
        ora_sincos(w, t[j], tau, &s, &c);
        ora_sum_add(&yc, yp[j] * c);
        ora_sum_add(&ys, yp[j] * s);
        ora_sum_add(&cc, c * c);
        ora_sum_add(&ss, s * s);
    }
    YC = ora_sum_get(&yc);
    YS = ora_sum_get(&ys);
    CC = ora_sum_get(&cc);
    SS = ora_sum_get(&ss);
    if (sums) {
        sums[0] = YC;
        sums[1] = YS;
        sums[2] = CC;
        sums[3] = SS;
    }
    p = 0.0;
    if (CC > 1e-12 * (double)n)
        p += YC * YC / CC;
    if (SS > 1e-12 * (double)n)
        p += YS * YS / SS;
    return 0.5 * p;
}

double ora_pls(const double *t, const double *yp, int64_t n, double w, double tau, double *sums)
{
    return ora_pls_l(t, yp, n, (long double)w, (long double)tau, sums);
}

/* Power of one object at one frequency (centred magnitudes, known S_yy). */
static double ora_power_one(const double *t, const double *yp, int64_t n, double syy, double f,
                            int32_t unit, int32_t normalize)
{
    long double w = ora_omega_l(f, unit);
    long double tau = ora_tau_l(t, n, w);
    double pls = ora_pls_l(t, yp, n, w, tau, NULL);
    if (normalize)
        return 2.0 * pls / syy;
    return pls;
}

/* Section 3.3: argmax of the periodogram, first (lowest) index on ties. */
int64_t ora_argmax(const double *p, int64_t n)
{
    int64_t i, best = -1;
    double bp = 0.0;
    for (i = 0; i < n; i++) {
        if (isnan(p[i]))
            continue;
        if (best < 0 || p[i] > bp) {
            best = i;
            bp = p[i];
        }
    }
    return best;
}

static void ora_fill_peak(ora_peak *pk, int32_t status, const double *pgram, int64_t n_f,
                          double f_min, double f_max, int32_t unit)
{
    pk->status = status;
    pk->pad = 0;
    pk->index = -1;
    pk->freq = NAN;
    pk->period = NAN;
    pk->power = (status == ORA_DEGENERATE) ? 0.0 : NAN;
    if (status != ORA_OK)
        return;
    pk->index = ora_argmax(pgram, n_f);
    if (pk->index < 0)
        return;
    pk->freq = ora_grid_freq(f_min, f_max, n_f, pk->index);
    pk->period = ora_period(pk->freq, unit);
    pk->power = pgram[pk->index];
}

static void ora_fill_row(double *row, int64_t n_f, int32_t status)
{
    int64_t i;
    double v = (status == ORA_DEGENERATE) ? 0.0 : NAN;
    for (i = 0; i < n_f; i++)
        row[i] = v;
}

static int ora_threads(int32_t nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * Single-object mode (Section 3.3): the whole periodogram of one series.
 * yp is caller scratch of n doubles.  The frequency loop is split statically
 * over threads as in the paper's CPU port.  pgram[n_f] must be non-NULL.
 */
int32_t ora_single(const double *t, const double *y, int64_t n, double f_min, double f_max,
                   int64_t n_f, int32_t unit, int32_t normalize, int32_t subtract_mean,
                   double *yp, double *pgram, ora_peak *peak, int32_t nthreads)
{
    double syy = 0.0;
    int64_t i;
    int32_t st = ora_prep(t, y, n, subtract_mean, yp, &syy);
    if (st != ORA_OK) {
        ora_fill_row(pgram, n_f, st);
    } else {
#pragma omp parallel for schedule(static) num_threads(ora_threads(nthreads))
        for (i = 0; i < n_f; i++)
            pgram[i] = ora_power_one(t, yp, n, syy, ora_grid_freq(f_min, f_max, n_f, i), unit,
                                     normalize);
    }
    if (peak)
        ora_fill_peak(peak, st, pgram, n_f, f_min, f_max, unit);
    return st;
}

static int32_t ora_range_status(const int64_t *offsets, int64_t o, int64_t n_obs)
{
    int64_t a = offsets[o], b = offsets[o + 1];
    if (a < 0 || b < a || b > n_obs)
        return ORA_BADRANGE;
    return ORA_OK;
}

/*
 * Batch mode (Section 3.4): object o owns observations [offsets[o], offsets[o+1]).
 * pgram is [n_obj * n_f] row-major, or NULL for peaks only.  Each object gets
 * private scratch, so objects whose ranges overlap do not interfere.
 * Objects are scheduled dynamically over threads as in the paper's CPU port.
 * Returns -1 if scratch memory cannot be had.
 */
int32_t ora_batch(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                  const double *y, double f_min, double f_max, int64_t n_f, int32_t unit,
                  int32_t normalize, int32_t subtract_mean, double *pgram, ora_peak *peaks,
                  int32_t nthreads)
{
    int64_t o;
    int32_t failed = 0;
#pragma omp parallel for schedule(dynamic) num_threads(ora_threads(nthreads))
    for (o = 0; o < n_obj; o++) {
        double *row = pgram ? pgram + o * n_f : (double *)malloc(sizeof(double) * (size_t)n_f);
        double *yp = NULL;
        int32_t st = ora_range_status(offsets, o, n_obs);
        int64_t i;
        if (!row) {
#pragma omp atomic write
            failed = 1;
            continue;
        }
        if (st == ORA_OK) {
            int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
            double syy = 0.0;
            yp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            if (!yp) {
#pragma omp atomic write
                failed = 1;
                if (!pgram)
                    free(row);
                continue;
            }
            st = ora_prep(t + a, y + a, n, subtract_mean, yp, &syy);
            if (st == ORA_OK)
                for (i = 0; i < n_f; i++)
                    row[i] = ora_power_one(t + a, yp, n, syy, ora_grid_freq(f_min, f_max, n_f, i),
                                           unit, normalize);
            free(yp);
        }
        if (st != ORA_OK)
            ora_fill_row(row, n_f, st);
        if (peaks)
            ora_fill_peak(&peaks[o], st, row, n_f, f_min, f_max, unit);
        if (!pgram)
            free(row);
    }
    return failed ? -1 : ORA_OK;
}

/*
 * Power at selected (object, bin) pairs, for spot checks at sizes where the
 * whole periodogram is too slow to compute here.  out[k] is the power of
 * object obj[k] at grid index bin[k] (0 for DEGENERATE objects, NaN for
 * BADRANGE/NONFINITE ones).  Returns -1 if scratch memory cannot be had.
 */
int32_t ora_eval_bins(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                      const double *y, double f_min, double f_max, int64_t n_f, int32_t unit,
                      int32_t normalize, int32_t subtract_mean, const int64_t *obj,
                      const int64_t *bin, int64_t n_req, double *out, int32_t nthreads)
{
    int64_t k;
    int32_t failed = 0;
    (void)n_obj;
#pragma omp parallel for schedule(dynamic) num_threads(ora_threads(nthreads))
    for (k = 0; k < n_req; k++) {
        int64_t o = obj[k];
        int32_t st = ora_range_status(offsets, o, n_obs);
        double v = NAN;
        if (st == ORA_OK) {
            int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
            double syy = 0.0;
            double *yp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            if (!yp) {
#pragma omp atomic write
                failed = 1;
            } else {
                st = ora_prep(t + a, y + a, n, subtract_mean, yp, &syy);
                if (st == ORA_OK)
                    v = ora_power_one(t + a, yp, n, syy, ora_grid_freq(f_min, f_max, n_f, bin[k]),
                                      unit, normalize);
                else if (st == ORA_DEGENERATE)
                    v = 0.0;
                free(yp);
            }
        }
        out[k] = v;
    }
    return failed ? -1 : ORA_OK;
}

/* ------------------------------------------------------------------------
 * Generalized periodogram with photometric errors and a floating mean
 * (Section 4.11 of the paper, which follows the generalized Lomb-Scargle
 * method of Zechmeister & Kuerster 2009 as implemented in Astropy).
 *
 * Each observation carries an error dy_j and the weight w_j = 1 / dy_j^2.  At
 * angular frequency w the model y = a cos wt + b sin wt + c is fitted by
 * weighted least squares; the power is the fraction of the weighted variance
 * about the weighted mean that the two trigonometric terms explain.  The
 * steps are those of the published method, in its order:
 *   - weighted mean ybar_w = sum w y / W (W = sum w), centred yw = y - ybar_w,
 *     YY = sum w yw^2;
 *   - tau from the weighted, mean-removed second moments of cos wt and sin wt:
 *     tan(2 w tau) = 2 CS / (CC - SS) with CC = sum w (cos wt - C/W)^2,
 *     SS = sum w (sin wt - S/W)^2, CS = sum w (cos wt - C/W)(sin wt - S/W),
 *     C = sum w cos wt, S = sum w sin wt;
 *   - at the shifted phase th_j = w (t_j - tau), with the weighted means of
 *     cos th and sin th removed again, YC = sum w yw cos~, YS = sum w yw sin~,
 *     CC = sum w cos~^2, SS = sum w sin~^2;
 *   - half the reduction in chi^2, P = 1/2 (YC^2 / CC + YS^2 / SS); the
 *     normalised power is 2 P / YY, which lies in [0, 1].
 * Every mean-removed quantity is formed from explicitly centred terms (one
 * more pass over the series) rather than by subtracting C^2 / W.
 *
 * Readings (listed with the other readings in the design notes):
 *   - dy == NULL means unit errors (floating-mean periodogram without errors);
 *   - an error that is not finite or not > 0 makes the object NONFINITE;
 *   - a term whose denominator is <= 1e-12 * W is dropped, as for Eq. 2
 *     (with unit errors W = N_t, the same rule);
 *   - N_t < 2, or YY <= 1e-20 * sum w y^2 (or 0), is DEGENERATE.
 * ------------------------------------------------------------------------ */

/*
 * Weights, weighted mean and YY.  Writes w[n] and the centred magnitudes
 * yw[n]; returns the object's status.
 */
int32_t ora_gen_prep(const double *t, const double *y, const double *dy, int64_t n, double *w,
                     double *yw, double *yy, double *wsum)
{
    int64_t j;
    ora_sum sw = {0.0, 0.0}, swy = {0.0, 0.0}, sq = {0.0, 0.0}, sraw = {0.0, 0.0};
    double ybar;
    *yy = 0.0;
    *wsum = 0.0;
    for (j = 0; j < n; j++) {
        if (!isfinite(t[j]) || !isfinite(y[j]))
            return ORA_NONFINITE;
        if (dy && !(isfinite(dy[j]) && dy[j] > 0.0))
            return ORA_NONFINITE;
    }
    for (j = 0; j < n; j++) {
        w[j] = dy ? 1.0 / (dy[j] * dy[j]) : 1.0;
        yw[j] = 0.0;
    }
    if (n < 2)
        return ORA_DEGENERATE;
    for (j = 0; j < n; j++) {
        ora_sum_add(&sw, w[j]);
        ora_sum_add(&swy, w[j] * y[j]);
    }
    *wsum = ora_sum_get(&sw);
    ybar = ora_sum_get(&swy) / *wsum;
    for (j = 0; j < n; j++) {
        yw[j] = y[j] - ybar;
        ora_sum_add(&sq, w[j] * yw[j] * yw[j]);
        ora_sum_add(&sraw, w[j] * y[j] * y[j]);
    }
    *yy = ora_sum_get(&sq);
    if (*yy <= 1e-20 * ora_sum_get(&sraw) || *yy == 0.0)
        return ORA_DEGENERATE;
    return ORA_OK;
}

/* Weighted means of cos(w (t - shift)) and sin(w (t - shift)). */
static void ora_gen_means(const double *t, const double *w, int64_t n, double wsum,
                          long double om, long double shift, double *mc, double *ms)
{
    int64_t j;
    ora_sum c = {0.0, 0.0}, s = {0.0, 0.0};
    for (j = 0; j < n; j++) {
        double sj, cj;
        ora_sincos(om, t[j], shift, &sj, &cj);
        ora_sum_add(&c, w[j] * cj);
        ora_sum_add(&s, w[j] * sj);
    }
    *mc = ora_sum_get(&c) / wsum;
    *ms = ora_sum_get(&s) / wsum;
}

/* tau of the generalized method: tan(2 w tau) = 2 CS / (CC - SS); 0 at w = 0. */
static long double ora_gen_tau_l(const double *t, const double *w, int64_t n, double wsum,
                                 long double om)
{
    int64_t j;
    double mc, ms;
    ora_sum cc = {0.0, 0.0}, ss = {0.0, 0.0}, cs = {0.0, 0.0};
    if (om == 0.0L)
        return 0.0L;
    ora_gen_means(t, w, n, wsum, om, 0.0L, &mc, &ms);
    for (j = 0; j < n; j++) {
        double sj, cj, dc, ds;
        ora_sincos(om, t[j], 0.0L, &sj, &cj);
        dc = cj - mc;
        ds = sj - ms;
        ora_sum_add(&cc, w[j] * dc * dc);
        ora_sum_add(&ss, w[j] * ds * ds);
        ora_sum_add(&cs, w[j] * dc * ds);
    }
    return (long double)atan2(2.0 * ora_sum_get(&cs), ora_sum_get(&cc) - ora_sum_get(&ss)) /
           (2.0L * om);
}

double ora_gen_tau(const double *t, const double *w, int64_t n, double wsum, double om)
{
    return (double)ora_gen_tau_l(t, w, n, wsum, (long double)om);
}

/*
 * Half the chi^2 reduction at angular frequency om and a given tau.  When
 * sums != NULL, stores {YC, YS, CC, SS} of the shifted, mean-removed terms.
 */
static double ora_gen_pls_l(const double *t, const double *yw, const double *w, int64_t n,
                            double wsum, long double om, long double tau, double *sums)
{
    int64_t j;
    double mc, ms, gc, gs, gcc, gss, p;
    ora_sum yc = {0.0, 0.0}, ys = {0.0, 0.0}, cc = {0.0, 0.0}, ss = {0.0, 0.0};
    ora_gen_means(t, w, n, wsum, om, tau, &mc, &ms);
    for (j = 0; j < n; j++) {
        double sj, cj, dc, ds;
        ora_sincos(om, t[j], tau, &sj, &cj);
        dc = cj - mc;
        ds = sj - ms;
        ora_sum_add(&yc, w[j] * yw[j] * dc);
        ora_sum_add(&ys, w[j] * yw[j] * ds);
        ora_sum_add(&cc, w[j] * dc * dc);
        ora_sum_add(&ss, w[j] * ds * ds);
    }
    gc = ora_sum_get(&yc);
    gs = ora_sum_get(&ys);
    gcc = ora_sum_get(&cc);
    gss = ora_sum_get(&ss);
    if (sums) {
        sums[0] = gc;
        sums[1] = gs;
        sums[2] = gcc;
        sums[3] = gss;
    }
    p = 0.0;
    if (gcc > 1e-12 * wsum)
        p += gc * gc / gcc;
    if (gss > 1e-12 * wsum)
        p += gs * gs / gss;
    return 0.5 * p;
}

double ora_gen_pls(const double *t, const double *yw, const double *w, int64_t n, double wsum,
                   double om, double tau, double *sums)
{
    return ora_gen_pls_l(t, yw, w, n, wsum, (long double)om, (long double)tau, sums);
}

static double ora_gen_power_one(const double *t, const double *yw, const double *w, int64_t n,
                                double wsum, double yy, double f, int32_t unit, int32_t normalize)
{
    long double om = ora_omega_l(f, unit);
    long double tau = ora_gen_tau_l(t, w, n, wsum, om);
    double pls = ora_gen_pls_l(t, yw, w, n, wsum, om, tau, NULL);
    if (normalize)
        return 2.0 * pls / yy;
    return pls;
}

/* Generalized single-object mode.  w and yw are caller scratch of n doubles. */
int32_t ora_gen_single(const double *t, const double *y, const double *dy, int64_t n,
                       double f_min, double f_max, int64_t n_f, int32_t unit, int32_t normalize,
                       double *w, double *yw, double *pgram, ora_peak *peak, int32_t nthreads)
{
    double yy = 0.0, wsum = 0.0;
    int64_t i;
    int32_t st = ora_gen_prep(t, y, dy, n, w, yw, &yy, &wsum);
    if (st != ORA_OK) {
        ora_fill_row(pgram, n_f, st);
    } else {
#pragma omp parallel for schedule(static) num_threads(ora_threads(nthreads))
        for (i = 0; i < n_f; i++)
            pgram[i] = ora_gen_power_one(t, yw, w, n, wsum, yy,
                                         ora_grid_freq(f_min, f_max, n_f, i), unit, normalize);
    }
    if (peak)
        ora_fill_peak(peak, st, pgram, n_f, f_min, f_max, unit);
    return st;
}

/*
 * Generalized batch mode over CSR objects (dy may be NULL).  pgram is
 * [n_obj * n_f] or NULL.  Returns -1 if scratch memory cannot be had.
 */
int32_t ora_gen_batch(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                      const double *y, const double *dy, double f_min, double f_max, int64_t n_f,
                      int32_t unit, int32_t normalize, double *pgram, ora_peak *peaks,
                      int32_t nthreads)
{
    int64_t o;
    int32_t failed = 0;
#pragma omp parallel for schedule(dynamic) num_threads(ora_threads(nthreads))
    for (o = 0; o < n_obj; o++) {
        double *row = pgram ? pgram + o * n_f : (double *)malloc(sizeof(double) * (size_t)n_f);
        int32_t st = ora_range_status(offsets, o, n_obs);
        int64_t i;
        if (!row) {
#pragma omp atomic write
            failed = 1;
            continue;
        }
        if (st == ORA_OK) {
            int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
            double yy = 0.0, wsum = 0.0;
            double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            double *yw = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            if (!w || !yw) {
#pragma omp atomic write
                failed = 1;
                free(w);
                free(yw);
                if (!pgram)
                    free(row);
                continue;
            }
            st = ora_gen_prep(t + a, y + a, dy ? dy + a : NULL, n, w, yw, &yy, &wsum);
            if (st == ORA_OK)
                for (i = 0; i < n_f; i++)
                    row[i] = ora_gen_power_one(t + a, yw, w, n, wsum, yy,
                                               ora_grid_freq(f_min, f_max, n_f, i), unit,
                                               normalize);
            free(w);
            free(yw);
        }
        if (st != ORA_OK)
            ora_fill_row(row, n_f, st);
        if (peaks)
            ora_fill_peak(&peaks[o], st, row, n_f, f_min, f_max, unit);
        if (!pgram)
            free(row);
    }
    return failed ? -1 : ORA_OK;
}

/* Generalized power at selected (object, bin) pairs; as ora_eval_bins. */
int32_t ora_gen_eval_bins(const int64_t *offsets, int64_t n_obj, int64_t n_obs, const double *t,
                          const double *y, const double *dy, double f_min, double f_max,
                          int64_t n_f, int32_t unit, int32_t normalize, const int64_t *obj,
                          const int64_t *bin, int64_t n_req, double *out, int32_t nthreads)
{
    int64_t k;
    int32_t failed = 0;
    (void)n_obj;
#pragma omp parallel for schedule(dynamic) num_threads(ora_threads(nthreads))
    for (k = 0; k < n_req; k++) {
        int64_t o = obj[k];
        int32_t st = ora_range_status(offsets, o, n_obs);
        double v = NAN;
        if (st == ORA_OK) {
            int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
            double yy = 0.0, wsum = 0.0;
            double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            double *yw = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            if (!w || !yw) {
#pragma omp atomic write
                failed = 1;
            } else {
                st = ora_gen_prep(t + a, y + a, dy ? dy + a : NULL, n, w, yw, &yy, &wsum);
                if (st == ORA_OK)
                    v = ora_gen_power_one(t + a, yw, w, n, wsum, yy,
                                          ora_grid_freq(f_min, f_max, n_f, bin[k]), unit,
                                          normalize);
                else if (st == ORA_DEGENERATE)
                    v = 0.0;
            }
            free(w);
            free(yw);
        }
        out[k] = v;
    }
    return failed ? -1 : ORA_OK;
}
