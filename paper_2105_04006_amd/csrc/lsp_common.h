// lsp_common.h -- definitions shared by the library's HIP sources (device side
// and host launchers).  Not part of the public interface (see include/lsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lsp.h"

namespace lsp {

constexpr int kWave = 64;
// Observations staged in LDS per pass of a workgroup over its object.
constexpr int kTile = 256;
constexpr int kPrepThreads = 256;
constexpr int kCombineThreads = 256;
constexpr int kXcds = 8;

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
// A term of Eq. 2 whose denominator is at most kDenEps * N_t is dropped: the
// corresponding regressor vanishes on the data (w = 0, or every 2wt equal).
constexpr double kDenEps = 1e-12;
// An object whose centred magnitudes have sum of squares <= kVarEps * sum y^2
// (or exactly 0) has no variance to explain.
constexpr double kVarEps = 1e-20;
// FP32 form: a bin whose smaller shifted denominator, N - |sum e^{2iwt}|, is
// below this fraction of N is ill-conditioned in FP32 and is recomputed in FP64.
constexpr float kIllTheta = 1.0f / 32.0f;

// Per-object statistics written by the prep kernel.  For the generalized
// periodogram the weights are rescaled to w'_j = wnorm / dy_j^2 with
// wnorm = N / sum(1/dy^2), so that they sum to N as unit weights do: ybar is
// then the weighted mean, syy = sum w' (y - ybar)^2, and scale takes half the
// chi^2 reduction in w' units to the reported power.
struct ObjMeta {
    int64_t j0;      // first observation of the object in the packed arrays
    int64_t n;       // number of observations
    double ybar;     // mean removed from y (0 when the caller's y is used as is)
    double syy;      // (weighted) sum of squared centred magnitudes
    double t0;       // time origin: mid-point of the object's time span
    double scale;    // factor from P_LS to the reported power
    int32_t status;  // LSP_OBJ_*
    int32_t pad;
    double wnorm;    // generalized form: N / sum(1/dy^2) (1 for unit errors)
};
static_assert(sizeof(ObjMeta) == 64, "ObjMeta layout");

// Best (power, index) of one frequency tile; index -1 means none.
struct PeakRec {
    double p;
    int64_t i;
};

// Frequency of grid index i, rounded exactly as f_min + df * i written out in
// IEEE double: the product and the sum each rounded, never fused, so every
// path (and the oracle) evaluates the same frequencies.  HIP's __dmul_rn and
// __dadd_rn are plain operators that the compiler may still fuse; the pragma
// is what forbids it.
__device__ __forceinline__ double grid_freq(double f_min, double df, int64_t i) {
#pragma clang fp contract(off)
    return f_min + df * (double)i;
}

// (p, i) ordering of the argmax: larger power wins, lower index on ties; NaN
// never wins.
__device__ __forceinline__ bool better(double p, int64_t i, double bp, int64_t bi) {
    if (!(p == p)) return false;
    if (bi < 0) return true;
    return p > bp || (p == bp && i < bi);
}

// The FP32 forms reduce each group's peak with one 64-bit atomic maximum:
// the key holds the power's FP32 bit pattern above the complement of the bin
// index, so that unsigned order is the argmax order of `better` -- larger
// power first, then the lower index (powers are >= 0, whose bit patterns
// order like their values; -0 is mapped to +0).  Key 0 means no bin.  Bin
// indices must stay below 2^32 - 1.
__device__ __forceinline__ unsigned long long peak_key(double p, int64_t i) {
    const float pf = (float)p;
    const uint32_t pb = __float_as_uint(pf > 0.0f ? pf : 0.0f);
    return ((unsigned long long)pb << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}

// Largest key of the wavefront, in every lane.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)k, off, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(k >> 32), off, kWave);
        k = umax64(k, ((unsigned long long)hi << 32) | lo);
    }
    return k;
}

__device__ __forceinline__ PeakRec key_peak(unsigned long long k) {
    if (k == 0ull) return PeakRec{0.0, -1};
    return PeakRec{(double)__uint_as_float((uint32_t)(k >> 32)),
                   (int64_t)(0xFFFFFFFFu - (uint32_t)k)};
}

__device__ __forceinline__ PeakRec wave_best(PeakRec r) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        PeakRec o;
        o.p = __shfl_xor(r.p, off, kWave);
        o.i = __shfl_xor(r.i, off, kWave);
        if (better(o.p, o.i, r.p, r.i)) r = o;
    }
    return r;
}

// A time re-centred on the object's origin, t - t0, as the unevaluated sum
// hi + lo of its rounded value and the rounding error (Knuth's two-sum, exact
// for any two doubles).
__device__ __forceinline__ void recentre64(double t, double t0, double* hi, double* lo) {
#pragma clang fp contract(off)
    const double s = t - t0;
    const double bb = s - t;
    *hi = s;
    *lo = (t - (s - bb)) - (t0 + bb);
}

// sin and cos of 2 pi f (hi + lo) for a re-centred time hi + lo (recentre64):
// the product f hi is split exactly into p + e with a fused multiply-add, the
// whole cycles of p are removed exactly, and e + f lo is added back, so the
// phase handed to the library is off by its final rounding only (~6e-17
// cycles), whatever the frequency and time span.  Contraction is off: fusing
// p - rint(p) into fma(f, hi, -rint(p)) would count e twice.
__device__ __forceinline__ void sincos_cycles64(double f_cyc, double hi, double lo, double* s,
                                                double* c) {
#pragma clang fp contract(off)
    const double p = f_cyc * hi;
    const double e = fma(f_cyc, hi, -p);
    const double r = (p - rint(p)) + fma(f_cyc, lo, e);
    sincospi(2.0 * r, s, c);
}

struct Sums64 {
    double xc, xs, cc, ss, cs;  // sum y cos, y sin, cos^2, sin^2, cos sin at angle wt
};

__device__ __forceinline__ void sums64_add(Sums64& a, double yj, double s, double c) {
    a.xc = fma(yj, c, a.xc);
    a.xs = fma(yj, s, a.xs);
    a.cc = fma(c, c, a.cc);
    a.ss = fma(s, s, a.ss);
    a.cs = fma(c, s, a.cs);
}

// Power from the single-pass sums in FP64.  Eq. 1 fixes the shift angle
// a = w tau through the sums at angle 2wt, which are (cc - ss, 2 cs); Eq. 2's
// shifted sums then follow from the angle-difference identities.  P_LS is
// multiplied by `scale`.
__device__ __forceinline__ double power64(const Sums64& s, double n, double scale) {
    const double c2 = s.cc - s.ss;
    const double s2 = 2.0 * s.cs;
    const double two_a = atan2(s2, c2);
    double sa, ca;
    sincos(0.5 * two_a, &sa, &ca);
    const double ycs = ca * s.xc + sa * s.xs;                 // sum y cos w(t - tau)
    const double ysn = ca * s.xs - sa * s.xc;                 // sum y sin w(t - tau)
    const double rot = c2 * (ca * ca - sa * sa) + s2 * (2.0 * sa * ca);  // sum cos 2w(t - tau)
    const double tot = s.cc + s.ss;
    const double dcos = 0.5 * (tot + rot);                    // sum cos^2 w(t - tau)
    const double dsin = 0.5 * (tot - rot);                    // sum sin^2 w(t - tau)
    double p = 0.0;
    if (dcos > kDenEps * n) p += ycs * ycs / dcos;
    if (dsin > kDenEps * n) p += ysn * ysn / dsin;
    return 0.5 * p * scale;
}

// Power from FP32 sums (cc = sum cos^2, cs = sum cos sin; sum sin^2 = N - cc).
// The shift needs no angle: with C2 + i S2 = sum e^{2iwt} and R = |C2 + i S2|,
// the shifted denominators are (N + R)/2 and (N - R)/2, and with A = xc^2 + xs^2
// and B R = (xc^2 - xs^2) C2 + 2 xc xs S2 (the numerators' sum and difference,
// rotated by the half angle) Eq. 2 becomes
//   P_LS = (A + B)/(2 (N + R)) + (A - B)/(2 (N - R)) = (A N - B R) / (N^2 - R^2):
// one reciprocal, no square root and no angle.  `ill` reports a bin whose
// N - R is at most N/32 (R^2 >= (31/32)^2 N^2), where FP32 sums cannot
// resolve the sine term; such bins are recomputed in FP64.
__device__ __forceinline__ float power32(float xc, float xs, float cc, float cs, float n,
                                         float scale, bool& ill) {
    const float c2 = fmaf(2.0f, cc, -n);
    const float s2 = 2.0f * cs;
    const float r2 = fmaf(c2, c2, s2 * s2);
    const float n2 = n * n;
    ill = !(r2 < (1.0f - kIllTheta) * (1.0f - kIllTheta) * n2);
    const float a = fmaf(xc, xc, xs * xs);
    const float br = fmaf(fmaf(xc, xc, -(xs * xs)), c2, 2.0f * xc * xs * s2);
    // A N - B R >= 0 exactly; rounding must not report a negative power
    return fmaxf(fmaf(a, n, -br), 0.0f) * __builtin_amdgcn_rcpf(n2 - r2) * scale;
}

// FP64 power of one (object, frequency) pair straight from the caller's
// series, re-centred on the fly; used to recompute FP32 bins flagged
// ill-conditioned (never from the FP32 hot kernel itself).
__device__ __forceinline__ double power64_bin(const ObjMeta& m, const double* __restrict__ t,
                                              const double* __restrict__ y, double f_cyc) {
    Sums64 a = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = m.j0; j < m.j0 + m.n; ++j) {
        double s, c, hi, lo;
        recentre64(t[j], m.t0, &hi, &lo);
        sincos_cycles64(f_cyc, hi, lo, &s, &c);
        sums64_add(a, y[j] - m.ybar, s, c);
    }
    return power64(a, (double)m.n, m.scale);
}

// ---------------------------------------------------------------------------
// Generalized periodogram (errors and a floating mean).  With weights w' and
// weighted-mean-centred magnitudes yw, the sums at angle wt are
//   c1 = sum w' cos, s1 = sum w' sin, yc = sum w' yw cos, ys = sum w' yw sin,
//   wcc = sum w' cos^2, wcs = sum w' cos sin (and wss = sum w' sin^2 = N - wcc).
// Removing the weighted means of cos and sin gives the 2 x 2 moment matrix
//   M = [[wcc - c1^2/N, wcs - c1 s1/N], [wcs - c1 s1/N, wss - s1^2/N]]
// and half the chi^2 reduction of the fit is 1/2 g' M^-1 g with g = (yc, ys)
// (yw has weighted mean 0, so g needs no correction).  The shift tau of the
// published method rotates onto M's eigenvectors; without forming it, with
// trace T, R = lambda_+ - lambda_- and Q = |g|^2, the projections of g on the
// eigenvectors are (Q +- Delta) / 2 and the denominators (T +- R) / 2.

struct SumsGen64 {
    double c1, s1, yc, ys, wcc, wss, wcs;
};

__device__ __forceinline__ void sumsgen64_add(SumsGen64& a, double w, double wy, double s,
                                              double c) {
    const double wc = w * c, ws = w * s;
    a.c1 += wc;
    a.s1 += ws;
    a.yc = fma(wy, c, a.yc);
    a.ys = fma(wy, s, a.ys);
    a.wcc = fma(wc, c, a.wcc);
    a.wss = fma(ws, s, a.wss);
    a.wcs = fma(wc, s, a.wcs);
}

// FP64 power of the generalized form; a term whose denominator is at most
// kDenEps * N is dropped, as for Eq. 2.
__device__ __forceinline__ double power64_gen(const SumsGen64& a, double n, double scale) {
    const double in = 1.0 / n;
    const double cc = a.wcc - a.c1 * a.c1 * in;
    const double ss = a.wss - a.s1 * a.s1 * in;
    const double cs = a.wcs - a.c1 * a.s1 * in;
    const double tr = cc + ss;
    const double df = cc - ss;
    const double r = sqrt(df * df + 4.0 * cs * cs);
    const double q = a.yc * a.yc + a.ys * a.ys;
    const double dl = r > 0.0 ? ((a.yc * a.yc - a.ys * a.ys) * df + 4.0 * cs * a.yc * a.ys) / r
                              : 0.0;
    double p = 0.0;
    if (0.5 * (tr + r) > kDenEps * n) p += (q + dl) / (tr + r);
    if (0.5 * (tr - r) > kDenEps * n) p += (q - dl) / (tr - r);
    return 0.5 * p * scale;
}

// The same from FP32 sums, flagging bins whose smaller denominator T - R is
// too small for FP32 to resolve (they are recomputed in FP64).
__device__ __forceinline__ float power32_gen(float c1, float s1, float yc, float ys, float wcc,
                                             float wcs, float n, float scale, bool& ill) {
    const float in = __builtin_amdgcn_rcpf(n);
    const float cc = fmaf(-c1 * in, c1, wcc);
    const float ss = fmaf(-s1 * in, s1, n - wcc);
    const float cs = fmaf(-c1 * in, s1, wcs);
    const float tr = cc + ss;
    const float df = cc - ss;
    const float r = __builtin_amdgcn_sqrtf(fmaf(df, df, 4.0f * cs * cs));
    const float dp = tr + r;
    const float dm = tr - r;
    ill = !(dm > kIllTheta * n);
    const float q = fmaf(yc, yc, ys * ys);
    float dl = 0.0f;
    if (r > 0.0f)
        dl = fmaf(fmaf(yc, yc, -(ys * ys)), df, 4.0f * cs * yc * ys) * __builtin_amdgcn_rcpf(r);
    float p = (q + dl) * __builtin_amdgcn_rcpf(dp);
    if (dm > 0.0f) p = fmaf(q - dl, __builtin_amdgcn_rcpf(dm), p);
    return 0.5f * p * scale;
}

// Weight w' of observation j (1 for unit errors).
__device__ __forceinline__ double gen_weight(const double* __restrict__ dy, int64_t j,
                                             double wnorm) {
    if (!dy) return 1.0;
    const double e = dy[j];
    return wnorm / (e * e);
}

// FP64 generalized power of one (object, frequency) pair from the caller's
// series (FP64 fix-up of the FP32 form).
__device__ __forceinline__ double power64_gen_bin(const ObjMeta& m, const double* __restrict__ t,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ dy, double f_cyc) {
    SumsGen64 a = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = m.j0; j < m.j0 + m.n; ++j) {
        double s, c, hi, lo;
        recentre64(t[j], m.t0, &hi, &lo);
        sincos_cycles64(f_cyc, hi, lo, &s, &c);
        const double w = gen_weight(dy, j, m.wnorm);
        sumsgen64_add(a, w, w * (y[j] - m.ybar), s, c);
    }
    return power64_gen(a, (double)m.n, m.scale);
}

// sin and cos of 2 pi r for a reduced phase |r| <= 1/2 revolution, three ways
// (LSP_TRIG_*): the hardware's v_sin / v_cos, which take revolutions; the math
// library's sincospif; or a quarter-turn reduction followed by the Taylor
// series of sin (to a^9) and cos (to a^8) at |a| <= pi/4, whose truncation
// errors (a^11/11! < 2e-9, a^10/10! < 3e-8) are below FP32 rounding.
template <int TRIG>
__device__ __forceinline__ void seed_sincos(float r, float* s, float* c) {
    if (TRIG == LSP_TRIG_LIB) {
        sincospif(2.0f * r, s, c);
    } else if (TRIG == LSP_TRIG_POLY) {
        const float q = rintf(4.0f * r);
        const float a = fmaf(-0.25f, q, r) * 6.283185307179586f;
        const float a2 = a * a;
        float ps = fmaf(a2, 1.0f / 362880.0f, -1.0f / 5040.0f);
        ps = fmaf(a2, ps, 1.0f / 120.0f);
        ps = fmaf(a2, ps, -1.0f / 6.0f);
        const float sa = fmaf(a * a2, ps, a);
        float pc = fmaf(a2, 1.0f / 40320.0f, -1.0f / 720.0f);
        pc = fmaf(a2, pc, 1.0f / 24.0f);
        pc = fmaf(a2, pc, -0.5f);
        const float ca = fmaf(a2, pc, 1.0f);
        // rotate (cos a, sin a) by q quarter turns
        const int k = (int)q & 3;
        const float sx = (k & 1) ? ca : sa;
        const float cx = (k & 1) ? sa : ca;
        *s = (k & 2) ? -sx : sx;
        *c = ((k + 1) & 2) ? -cx : cx;
    } else {
        *s = __builtin_amdgcn_sinf(r);
        *c = __builtin_amdgcn_cosf(r);
    }
}

// One observation's contribution to a lane's K bins (the FP32 hot loop of the
// periodogram and of the coarse proposal features): seed (cos, sin) of the
// lane's first phase, then the recurrence across its bins.  o = (y - ybar,
// cos step, sin step, -), tq = t - t0.
template <int K, bool CHEB, int TRIG>
__device__ __forceinline__ void accumulate_obs(double fl, double tq, float4 o, float (&xc)[K],
                                               float (&xs)[K], float (&cc)[K], float (&cs)[K]) {
    double ph = fl * tq;
    ph -= rint(ph);
    const float r = (float)ph;
    float s, c;
    seed_sincos<TRIG>(r, &s, &c);
    if (!CHEB) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xc[k] = fmaf(o.x, c, xc[k]);
            xs[k] = fmaf(o.x, s, xs[k]);
            cc[k] = fmaf(c, c, cc[k]);
            cs[k] = fmaf(c, s, cs[k]);
            if (k + 1 < K) {
                const float cn = fmaf(c, o.y, -(s * o.z));
                s = fmaf(s, o.y, c * o.z);
                c = cn;
            }
        }
    } else {
        // One rotation to reach the second frequency, then the three-term
        // recurrence x_{k+1} = 2C x_k - x_{k-1}, which cos and sin of an
        // arithmetic progression of angles obey.
        const float two_c = o.y + o.y;
        float cp = c, sp = s;
        c = fmaf(cp, o.y, -(sp * o.z));
        s = fmaf(sp, o.y, cp * o.z);
        xc[0] = fmaf(o.x, cp, xc[0]);
        xs[0] = fmaf(o.x, sp, xs[0]);
        cc[0] = fmaf(cp, cp, cc[0]);
        cs[0] = fmaf(cp, sp, cs[0]);
#pragma unroll
        for (int k = 1; k < K; ++k) {
            xc[k] = fmaf(o.x, c, xc[k]);
            xs[k] = fmaf(o.x, s, xs[k]);
            cc[k] = fmaf(c, c, cc[k]);
            cs[k] = fmaf(c, s, cs[k]);
            if (k + 1 < K) {
                const float cn = fmaf(two_c, c, -cp);
                const float sn = fmaf(two_c, s, -sp);
                cp = c;
                sp = s;
                c = cn;
                s = sn;
            }
        }
    }
}

// Value written for every bin of an object whose status is not OK.
__device__ __forceinline__ double fill_value(int32_t status) {
    return status == LSP_OBJ_DEGENERATE ? 0.0 : __builtin_nan("");
}

__device__ __forceinline__ void store_pgram(void* pgram, int32_t f64, int64_t idx, double v) {
    if (f64)
        static_cast<double*>(pgram)[idx] = v;
    else
        static_cast<float*>(pgram)[idx] = (float)v;
}

// Launch grids: the dispatch packet counts work-items in 32 bits per
// dimension, so large launches are folded into (x, y) with at most kGridX
// blocks along x; kernels recover the linear block index and drop the excess.
constexpr int64_t kGridX = 32768;

inline dim3 grid_for(int64_t blocks) {
    if (blocks <= kGridX) return dim3((unsigned)blocks, 1, 1);
    return dim3((unsigned)kGridX, (unsigned)((blocks + kGridX - 1) / kGridX), 1);
}

__device__ __forceinline__ int64_t linear_block() {
    return (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

// A value the whole workgroup read from LDS, marked wave-uniform.  Loops whose
// trip count or exit depends on an LDS broadcast must test a value the
// compiler can prove uniform: otherwise the exit is treated as per-lane, and
// the structurised control flow may let some lanes re-enter a barrier-bearing
// loop body without the lanes that were to update the broadcast.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int32_t uniform_i32(int32_t v) {
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

// One queue pop for the whole workgroup: thread 0 takes the next item number
// and every thread receives it as a wave-uniform value.  The leading barrier
// keeps thread 0 from overwriting the broadcast slot while other threads may
// still be reading the previous item's LDS data.
__device__ __forceinline__ int64_t pop_item(unsigned int* counter, int64_t lo, int64_t* s_item) {
    __syncthreads();
    if (threadIdx.x == 0) *s_item = lo + (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    return uniform_i64(*s_item);
}

// A row of work: one object's whole grid, or one band of it.
struct RowRange {
    int64_t obj;
    int64_t f_lo, f_hi;  // frequency indices [f_lo, f_hi); empty if the row is invalid
};

__device__ __forceinline__ RowRange decode_row(const int32_t* row_obj, const int32_t* row_band,
                                               int64_t band_bins, int32_t rows_per_group,
                                               int64_t n_obj, int64_t n_f, int64_t row) {
    RowRange r;
    r.obj = row_obj ? (int64_t)row_obj[row] : row / rows_per_group;
    r.f_lo = 0;
    r.f_hi = n_f;
    if (row_band) {
        const int64_t b = row_band[row];
        r.f_lo = b * band_bins;
        r.f_hi = r.f_lo + band_bins < n_f ? r.f_lo + band_bins : n_f;
        if (b < 0) r.f_lo = r.f_hi = 0;
    }
    if (r.obj < 0 || r.obj >= n_obj) {
        r.obj = -1;
        r.f_lo = r.f_hi = 0;
    }
    // The row index is wave-uniform, so these are too; say so to the compiler,
    // since they bound loops that hold barriers.
    r.obj = uniform_i64(r.obj);
    r.f_lo = uniform_i64(r.f_lo);
    r.f_hi = uniform_i64(r.f_hi);
    return r;
}


// The row a work item's rank stands for: the rank itself, or, under the
// longest-first order, the row the ordering kernels placed at that rank
// (wave-uniform, like the rank).
__device__ __forceinline__ int64_t item_row(const int32_t* perm, int64_t rank) {
    return perm ? uniform_i64((int64_t)perm[rank]) : rank;
}

// The first row rank of XCD x's share when n_rows ranks are dealt out in
// eight contiguous, balanced runs (the first n_rows % 8 runs one longer); the
// longest-first order places its rows the same way.
__device__ __forceinline__ int64_t xcd_first_rank(int x, int64_t n_rows) {
    const int64_t base = n_rows / kXcds, rem = n_rows % kXcds;
    return (int64_t)x * base + (x < rem ? (int64_t)x : rem);
}

// The end of XCD x's queue: the items of its run of ranks, cut, under the
// longest-first order, after the ranks that hold rows with work (position
// s of the sorted order sits in XCD s % 8's run, so XCD x holds the
// positions below n_work that are x mod 8).
__device__ __forceinline__ int64_t xcd_queue_end(int x, int64_t n_rows, int64_t per_row,
                                                 const unsigned int* n_work) {
    int64_t end = xcd_first_rank(x + 1, n_rows);
    if (n_work) {
        const int64_t nw = uniform_i64((int64_t)*n_work);
        const int64_t mine = nw > x ? (nw - x + kXcds - 1) / kXcds : 0;
        const int64_t cut = xcd_first_rank(x, n_rows) + mine;
        if (cut < end) end = cut;
    }
    return end * per_row;
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs,
// so block b runs on XCD b % 8.  Remap so that each XCD receives a contiguous
// run of items (and hence the same objects stay in one XCD's L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
    const int64_t full = (n / kXcds) * kXcds;
    if (b >= full) return b;
    return (b % kXcds) * (full / kXcds) + b / kXcds;
}

// ---------------------------------------------------------------------------
// Kernel parameter blocks and host launchers.

struct PrepParams {
    const int64_t* offsets;  // NULL: one object spanning [0, n_obs)
    const double* t;
    const double* y;
    int64_t n_obj;
    int64_t n_obs;
    int32_t subtract_mean;
    int32_t normalize;
    ObjMeta* meta;
    const double* dy = nullptr;  // generalized form: errors (NULL: unit errors)
    int32_t gen = 0;             // generalized form: weights and a floating mean
};

struct MainParams {
    const ObjMeta* meta;
    const double* t;  // caller's times and magnitudes (read-only)
    const double* y;
    double f_min, df, to_cyc;
    double step_cyc;  // FP32 form: lane-stride frequency step (kWave bins) in cycles
    int64_t n_f;
    int64_t n_obj;
    const int32_t* row_obj;   // object of each row, or NULL: row r is object r / rows_per_group
    const int32_t* row_band;  // band of each row ([b*band_bins, (b+1)*band_bins)), or NULL
    int64_t band_bins;
    int32_t rows_per_group;
    int32_t pad_rows;
    int64_t tiles_per_row;  // frequency tiles per row
    int64_t tiles_per_item; // consecutive frequency tiles per work item (FP32 form)
    int64_t chunks_per_row; // ceil(tiles_per_row / tiles_per_item)
    int64_t n_items;        // n_rows * chunks_per_row * n_split
    int32_t n_split;        // observation-axis split (single object only)
    int32_t pgram_f64;
    void* pgram;             // NULL: peaks only
    PeakRec* rec;            // FP64 form: [n_rows * tiles_per_row] tile records
    unsigned long long* keys;  // FP32 form, n_split == 1: [n_groups] peak keys (peak_key)
    uint32_t* ill_bits;      // FP32 form, n_split == 1: bit per tile, set when the tile
                             // needs the FP64 fix-up (its key then comes from the fix-up)
    float* part;             // [n_split][4][n_f] when n_split > 1
    unsigned int* queue;     // persistent schedule: kXcds counters
    const int32_t* row_perm = nullptr;  // rank -> row (longest first); NULL: rank = row
    // with row_perm: the number of rows with work (they hold the first ranks
    // of every XCD's run); the persistent schedule stops each queue there
    const unsigned int* n_work = nullptr;
    int32_t persistent;
    int32_t wave_split;      // the waves of a workgroup split observations, not bins
    const double* dy = nullptr;  // generalized form: errors (NULL: unit errors)
    int32_t gen = 0;             // generalized form (part holds 6 sums per split)
    // LSP_OBS_DIRECT: per-observation values written by the staging pass,
    // indexed like t (t - t0 of the object; (y - ybar, cos step, sin step, 0))
    const double* stage_t = nullptr;
    const float4* stage_o = nullptr;
};

struct CombineParams {
    const ObjMeta* meta;
    const double* t;
    const double* y;
    const float* part;
    int32_t n_split;
    int32_t pgram_f64;
    double f_min, df, to_cyc;
    int64_t n_f;
    void* pgram;
    PeakRec* rec;  // [ceil(n_f / kCombineThreads)]
    const double* dy = nullptr;
    int32_t gen = 0;
};

struct FixupParams {
    const ObjMeta* meta;
    const double* t;
    const double* y;
    const uint32_t* ill_bits;  // bit per tile (MainParams::ill_bits)
    unsigned long long* keys;  // group peak keys the recomputed tiles are merged into
    double f_min, df, to_cyc;
    int64_t n_f;
    int64_t n_obj;
    const int32_t* row_obj;
    const int32_t* row_band;
    int64_t band_bins;
    int32_t rows_per_group;
    int32_t pad_rows;
    int64_t tiles_per_row;
    int64_t n_tiles;
    int64_t tile_freqs;
    int32_t pgram_f64;
    int32_t pad;
    void* pgram;
    PeakRec* rec;
    const double* dy = nullptr;
    int32_t gen = 0;
};

struct PeakParams {
    const ObjMeta* meta;
    const PeakRec* rec;               // records, rec_per_obj per group (or NULL)
    const unsigned long long* keys;   // or one peak key per group (FP32 forms)
    int64_t n_obj;
    int64_t n_groups;        // groups of rows; group g covers rows [g R, (g+1) R)
    const int32_t* row_obj;  // object of each row, or NULL (group g is object g)
    int32_t rows_per_group;  // R
    int32_t pad2;
    int64_t rec_per_obj;     // records per group
    double f_min, df;
    int32_t unit;
    int32_t pad;
    lsp_peak* peaks;
};

hipError_t launch_prep(const PrepParams& p, hipStream_t s);
hipError_t launch_fp64(const MainParams& p, int kf, int waves, hipStream_t s);
hipError_t launch_fp32p(const MainParams& p, int k, int waves, int rec, hipStream_t s,
                        int obs_read = LSP_OBS_LDS, int trig = LSP_TRIG_HW);
// Per-observation staging values for LSP_OBS_DIRECT (one workgroup per object).
hipError_t launch_stage(const ObjMeta* meta, const double* t, const double* y, int64_t n_obj,
                        double step_cyc, int trig, double* stage_t, float4* stage_o,
                        hipStream_t s);
hipError_t launch_gen_fp32p(const MainParams& p, int k, int waves, hipStream_t s);
hipError_t launch_gen_fp64(const MainParams& p, int kf, int waves, hipStream_t s);
hipError_t launch_fixup(const FixupParams& p, hipStream_t s);
hipError_t launch_combine(const CombineParams& p, hipStream_t s);
hipError_t launch_peaks(const PeakParams& p, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* dst, int64_t n, unsigned int v, hipStream_t s);

// Longest-first row order (lsp_order.hip).
// N_t < 1024 exact, 64 per octave above, and one bucket for rows with no work
constexpr int kOrderBuckets = 1024 + 53 * 64 + 1;
constexpr int kOrderBlocks = 64;               // workgroups of the two-level sort
struct OrderParams {
    const int64_t* offsets;  // CSR offsets of the objects (n_obj + 1)
    int64_t n_obj;
    const int32_t* row_obj;   // object of each row, or NULL (row r is object r / rows_per_group)
    const int32_t* row_band;  // band of each row, or NULL; a negative band costs nothing
    int64_t n_rows;
    int32_t rows_per_group;
    int32_t pad;
    unsigned int* hist;   // [kOrderBlocks x kOrderBuckets] per-workgroup counts (scratch)
    unsigned int* total;  // [kOrderBuckets] bucket counts, then first positions (scratch)
    int32_t* perm;       // [n_rows]: rank -> row
};
hipError_t launch_row_order(const OrderParams& p, hipStream_t s);

// Host side (lsp_api.hip): the whole-grid batch call of lsp_batch /
// lsp_gen_batch and its workspace size.  one_batch = false treats the objects
// as a part of a larger batch (the multi-object launch configuration even for
// one object).
size_t batch_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                             const lsp_options* opt, bool gen, bool one_batch);
lsp_status batch_call(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                      const double* y, const double* dy, bool gen, const lsp_grid* grid,
                      const lsp_options* opt, void* pgram, lsp_peak* peaks, void* ws,
                      size_t ws_bytes, void* stream, bool one_batch);


}  // namespace lsp
