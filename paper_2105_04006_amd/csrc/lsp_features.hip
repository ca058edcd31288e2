// lsp_features.hip -- per-object features for the learned band proposal.
//
// The paper evaluates every bin of every object.  The learned path first
// computes, per object, 1,088 cheap features and lets a small network propose
// the few frequency bands worth evaluating.  Two kernels fill one feature row
// per object:
//
//   coarse_kernel : the object is cut into seasons (a new season at every gap
//     longer than `season_gap`), and consecutive seasons are grouped until a
//     group holds at least `min_season_obs` observations (a trailing group
//     with fewer is dropped).  For each group, the normalised Lomb-Scargle
//     power of Section 2 (Eq. 1-2 without tau, through the 2x2 moment
//     matrix of cos and sin) of the object's
//     centred magnitudes y - ybar is evaluated on 8,192 bins over
//     [f_min, f_max), max-pooled over runs of 8 bins and averaged over the
//     groups -> features [0, 1024).  The group's own mean is not removed
//     again: that only changes power near zero frequency, and it keeps the
//     loop the FP32 hot loop of the main kernel (accumulate_obs: FP64 phase
//     reduction, hardware sin/cos per observation, three-term recurrence
//     across a lane's frequencies, four sums), with the same FP64 recompute
//     of bins FP32 cannot resolve.
//   window_kernel : one wavefront per object computes sampling and magnitude
//     statistics in FP64 and the spectral window at 53 probe frequencies
//     (FP64 phases, hardware FP32 sin/cos, FP64 sums) -> features [1024, 1088).
//
// Objects whose status is not OK get an all-zero row.
#include <math.h>

#include <cmath>

#include "lsp_common.h"

namespace lsp {
namespace {

constexpr int kCoarseK = 16;     // frequencies per lane
constexpr int kCoarseW = 1;      // wavefronts per workgroup
constexpr int kCoarseTile = kWave * kCoarseK * kCoarseW;  // 1,024 bins
constexpr int kTilesPerObj = LSP_FEAT_COARSE * LSP_FEAT_POOL / kCoarseTile;
constexpr int kProbes = LSP_FEAT_WINDOW - 11;
constexpr int kWindowStage = 1024;  // objects up to this many points keep t - t0 in LDS

static_assert(LSP_FEAT_POOL == 8, "pooling uses three lane-exchange steps");
static_assert(kCoarseW == 1, "the coarse staging loop gives each lane one observation per round");
static_assert(kTilesPerObj * kCoarseTile == LSP_FEAT_COARSE * LSP_FEAT_POOL, "tile split");

struct FeatParams {
    const ObjMeta* meta;
    const double* t;
    const double* y;
    double f_min, df, to_cyc;  // coarse grid: df = (f_max - f_min) / 8192
    double step_cyc;           // phase advance over kWave coarse bins, in cycles
    double gap;
    int64_t n_obj;
    int32_t min_obs;
    int32_t pad;
    float* out;            // [n_obj][LSP_FEAT_DIM]
    unsigned int* queue;   // kXcds item counters (zeroed before the launch)
    double probe[kProbes];  // spectral-window probe frequencies, 10^-3 .. 30 log-spaced
};

// Normalised power of the observations [g0, g0 + n) of one object (magnitudes
// centred on the object's mean, normalised by the group's own sum of
// squares) at f_cyc cycles per time unit, in FP64 as the main kernel's FP64
// form computes it: exact re-centred phases, library sin/cos, Eq. 1-2 through
// power64 with its drop rule.  Not inlined: its FP64 registers stay out of
// the coarse kernel's hot loop.
__device__ __noinline__ double group_power64(const double* __restrict__ t, const double* __restrict__ y,
                                double t0, double ybar, int64_t g0, int64_t n, double f_cyc) {
    Sums64 a = {0.0, 0.0, 0.0, 0.0, 0.0};
    double syy = 0.0;
    for (int64_t j = g0; j < g0 + n; ++j) {
        double s, c, hi, lo;
        recentre64(t[j], t0, &hi, &lo);
        sincos_cycles64(f_cyc, hi, lo, &s, &c);
        const double yj = y[j] - ybar;
        sums64_add(a, yj, s, c);
        syy = fma(yj, yj, syy);
    }
    return syy > 0.0 ? power64(a, (double)n, 2.0 / syy) : 0.0;
}

// Maximum over each run of 8 lanes, in all 8 lanes, through DPP lane moves:
// swap neighbours (quad_perm 1,0,3,2), swap pairs (quad_perm 2,3,0,1), then
// mirror within each half-row of 8 lanes (lane i with lane 7 - i), which pairs
// each 4-lane maximum with the other's.  The values are non-negative floats,
// whose bit patterns order as the values do, so the maximum is taken on the
// integers (no NaN handling, and the lane move folds into the max).
template <int CTRL>
__device__ __forceinline__ int dpp_max_i32(int x) {
    return max(x, __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float pool8_max(float v) {
    int x = __float_as_int(v);
    x = dpp_max_i32<0xB1>(x);
    x = dpp_max_i32<0x4E>(x);
    x = dpp_max_i32<0x141>(x);
    return __int_as_float(x);
}

// One (object, 1,024-bin tile) item; called by every thread of the workgroup.
__device__ __forceinline__ void coarse_item(const FeatParams& P, int64_t item, double* s_tau,
                                            float4* s_obs, unsigned long long* s_starts) {
    constexpr int K = kCoarseK;
    const int64_t obj = item / kTilesPerObj;
    const int tile = (int)(item - obj * kTilesPerObj);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t i0 = (int64_t)tile * kCoarseTile + (int64_t)wave * kWave * K + lane;
    float* out = P.out + obj * LSP_FEAT_DIM;
    const ObjMeta m = P.meta[obj];

    float feat[K];
#pragma unroll
    for (int k = 0; k < K; ++k) feat[k] = 0.0f;
    int n_good = 0;

    if (m.status == LSP_OBJ_OK) {
        const double fl = grid_freq(P.f_min, P.df, i0) * P.to_cyc;
        float xc[K], xs[K], cc[K], cs[K];
#pragma unroll
        for (int k = 0; k < K; ++k) xc[k] = xs[k] = cc[k] = cs[k] = 0.0f;
        // group count, first observation and sum of squares of y - ybar
        // (wave-uniform)
        int ns = 0;
        int64_t g0 = m.j0;
        float syy = 0.0f;

        // Close the current group, the observations [g0, g0 + ns): add its
        // pooled power to the features if it has enough observations.  As in
        // the main kernel, a bin whose smaller shifted denominator N - R is at
        // most N/32 cannot be resolved in FP32 and is recomputed in FP64 from
        // the group's observations (group_power64); the others keep the FP32
        // value, with a hardware reciprocal (about 1 ulp).  The next group
        // starts at j_next.
        auto close_group = [&](int64_t j_next) {
            if (ns >= P.min_obs) {
                const float N = (float)ns;
                const float scale = syy > 0.0f ? 1.0f / syy : 0.0f;
                float p32[K];
                float det_min = INFINITY;  // smallest det M of this lane's bins
                // With g = (xc, xs) and the moment matrix M = [[cc, cs],
                // [cs, N - cc]] of (cos, sin), twice P_LS is g^T M^-1 g =
                // (xc^2 (N - cc) - 2 xc xs cs + xs^2 cc) / det M, the tau-free
                // form (A + B)/(N + R) + (A - B)/(N - R) of Eq. 1-2 written out
                // (N^2 - R^2 = 4 det M): one reciprocal and no square root per
                // bin.  N - R <= N/32 (the main kernel's rule) is
                // det M <= (1 - (31/32)^2) N^2 / 4.
                const float ill_det =
                    0.25f * (1.0f - (1.0f - kIllTheta) * (1.0f - kIllTheta)) * N * N;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float sn = N - cc[k];
                    const float det = fmaf(cc[k], sn, -(cs[k] * cs[k]));
                    const float num =
                        fmaf(xc[k] * sn, xc[k], xs[k] * fmaf(-2.0f, xc[k] * cs[k], xs[k] * cc[k]));
                    // (a negative value from rounding is clamped to zero with the
                    // others before pooling)
                    p32[k] = num * __builtin_amdgcn_rcpf(det) * scale;
                    det_min = fminf(det_min, det);
                }
                // FP64 recompute of the unresolvable bins, one bin at a time
                // (a rolled loop, so that the FP64 path stays out of the
                // unrolled code and its registers; the value goes to its bin by
                // a select over the lane's bins, so no LDS is set aside for
                // this rare path); which bins they are is worked out only here,
                // where some are
                if (__any(!(det_min > ill_det))) {
                    uint32_t ill = 0u;  // bins of this lane FP32 cannot resolve
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const float det = fmaf(cc[k], N - cc[k], -(cs[k] * cs[k]));
                        if (!(det > ill_det)) ill |= 1u << k;
                    }
#pragma unroll 1
                    for (int k = 0; k < K; ++k) {
                        if ((ill >> k) & 1u) {
                            const double f =
                                grid_freq(P.f_min, P.df, i0 + (int64_t)kWave * k) * P.to_cyc;
                            const float v = (float)group_power64(P.t, P.y, m.t0, m.ybar, g0, ns, f);
#pragma unroll
                            for (int u = 0; u < K; ++u) p32[u] = u == k ? v : p32[u];
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k)
                    feat[k] += pool8_max(fminf(fmaxf(p32[k], 0.0f), 1.0f));
                ++n_good;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) xc[k] = xs[k] = cc[k] = cs[k] = 0.0f;
            ns = 0;
            g0 = j_next;
            syy = 0.0f;
        };

        const int64_t j_end = m.j0 + m.n;
        for (int64_t jt = m.j0; jt < j_end; jt += kTile) {
            const int cnt = (int)((j_end - jt) < kTile ? (j_end - jt) : kTile);
            __syncthreads();
            // Stage the tile in rounds of 64 observations (one per lane); each
            // round's new-season flags go to LDS as one ballot word.
            for (int r = 0; r * kWave < cnt; ++r) {
                const int q = r * kWave + lane;
                bool starts = false;
                if (q < cnt) {
                    const int64_t j = jt + q;
                    const double tj = P.t[j];
                    const double tc = tj - m.t0;
                    s_tau[q] = tc;
                    double sp = P.step_cyc * tc;
                    sp -= rint(sp);
                    const float rs = (float)sp;
                    // (the previous time is loaded unconditionally, clamped to
                    // the object's first observation, so the two loads go out
                    // together)
                    const double tprev = P.t[j > m.j0 ? j - 1 : j];
                    starts = j > m.j0 && tj - tprev > P.gap;
                    s_obs[q] = make_float4((float)(P.y[j] - m.ybar), __builtin_amdgcn_cosf(rs),
                                           __builtin_amdgcn_sinf(rs), 0.0f);
                }
                const unsigned long long word = __ballot(starts);
                if (lane == 0) s_starts[r] = word;
            }
            __syncthreads();
            // Walk the tile from season boundary to season boundary.  A
            // boundary closes the current group once it holds min_obs
            // observations (sparser seasons merge with the next); between
            // boundaries the loop is the main kernel's hot loop alone.
            int q = 0;
            while (q < cnt) {
                const uint64_t here = (uint64_t)uniform_i64((int64_t)s_starts[q / kWave]);
                if (((here >> (q % kWave)) & 1ull) && ns >= P.min_obs) close_group(jt + q);
                // the next boundary after q, or the tile's end
                int b = cnt;
                for (int w = (q + 1) / kWave; w * kWave < cnt; ++w) {
                    uint64_t bits = (uint64_t)uniform_i64((int64_t)s_starts[w]);
                    if (w == (q + 1) / kWave) bits &= ~0ull << ((q + 1) % kWave);
                    if (bits) {
                        b = w * kWave + (int)__builtin_ctzll(bits);
                        break;
                    }
                }
                for (int j = q; j < b; ++j) {
                    const float4 o = s_obs[j];
                    const double tq = s_tau[j];  // both reads in flight together
                    // the main kernel's hot loop: FP64-reduced seed, hardware
                    // sin/cos, three-term recurrence across the lane's bins
                    accumulate_obs<K, true, LSP_TRIG_HW>(fl, tq, o, xc, xs, cc, cs);
                    syy = fmaf(o.x, o.x, syy);
                }
                ns += b - q;
                q = b;
            }
        }
        close_group(j_end);
    }

    const float inv = n_good > 0 ? 1.0f / (float)n_good : 0.0f;
    if ((lane & (LSP_FEAT_POOL - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t q = (i0 + (int64_t)kWave * k) / LSP_FEAT_POOL;
            out[q] = feat[k] * inv;
        }
    }
}

// Resident workgroups take (object, tile) items from eight per-XCD queues, as
// the batch periodogram does; a workgroup that drains its own XCD's queue
// moves on to the next one and exits once every queue is empty.
// Four waves per SIMD (at most 128 VGPRs), as the main kernel's K = 16 loop:
// the hot loop stays spill-free; the rare FP64 recompute and the staging loop
// keep a few values in scratch.
__global__ __launch_bounds__(kWave* kCoarseW)
    __attribute__((amdgpu_waves_per_eu(4))) void coarse_kernel(const FeatParams P) {
    __shared__ double s_tau[kTile];
    __shared__ float4 s_obs[kTile];  // (y - ybar, cos step, sin step, 0)
    __shared__ unsigned long long s_starts[kTile / kWave];  // new-season flags, one bit each
    __shared__ int64_t s_item;
    const int64_t n_items = P.n_obj * kTilesPerObj;
    const int64_t per = (n_items + kXcds - 1) / kXcds;
    const int x0 = (int)(blockIdx.x % kXcds);
    for (int d = 0; d < kXcds; ++d) {
        const int x = (x0 + d) % kXcds;
        const int64_t lo = (int64_t)x * per;
        const int64_t hi = lo + per < n_items ? lo + per : n_items;
        int64_t item = pop_item(&P.queue[x], lo, &s_item);
        while (item < hi) {
            coarse_item(P, item, s_tau, s_obs, s_starts);
            item = pop_item(&P.queue[x], lo, &s_item);
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// One wavefront per object.
__global__ __launch_bounds__(kWave) void window_kernel(const FeatParams P) {
    __shared__ double s_tc[kWindowStage];
    const int64_t obj = linear_block();
    if (obj >= P.n_obj) return;
    const int lane = threadIdx.x;
    float* out = P.out + obj * LSP_FEAT_DIM + LSP_FEAT_COARSE;
    const ObjMeta m = P.meta[obj];
    if (m.status != LSP_OBJ_OK) {
        out[lane] = 0.0f;
        return;
    }
    const int64_t j0 = m.j0, n = m.n, j1 = j0 + n;

    // Pass 1: time span, moments of y - ybar, within-season spacings.
    double tmin = __builtin_inf(), tmax = -__builtin_inf();
    double m3 = 0.0, m4 = 0.0, amax = 0.0;
    double dsum = 0.0, lsum = 0.0, lsq = 0.0, dcnt = 0.0;
    for (int64_t j = j0 + lane; j < j1; j += kWave) {
        const double tj = P.t[j];
        const double yc = P.y[j] - m.ybar;
        tmin = fmin(tmin, tj);
        tmax = fmax(tmax, tj);
        const double y2 = yc * yc;
        m3 += y2 * yc;
        m4 += y2 * y2;
        amax = fmax(amax, fabs(yc));
        if (j > j0) {
            const double d = tj - P.t[j - 1];
            if (d <= P.gap) {
                const double l = log10(fmax(d, 1e-6));
                dsum += d;
                lsum += l;
                lsq += l * l;
                dcnt += 1.0;
            }
        }
    }
    tmin = wave_min(tmin);
    tmax = wave_max(tmax);
    m3 = wave_sum(m3);
    m4 = wave_sum(m4);
    amax = wave_max(amax);
    dsum = wave_sum(dsum);
    lsum = wave_sum(lsum);
    lsq = wave_sum(lsq);
    dcnt = wave_sum(dcnt);

    // Pass 2: seasons, 64 observations per step.  The ballot of season starts
    // is wave-uniform, so the loop over its set bits is too.
    int64_t n_seasons = 0, n_good = 0, good_obs = 0, start = j0;
    for (int64_t jb = j0; jb < j1; jb += kWave) {
        const int64_t j = jb + lane;
        const bool st = j < j1 && j > j0 && P.t[j] - P.t[j - 1] > P.gap;
        uint64_t mask = __ballot(st);
        while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int64_t s = jb + b;
            ++n_seasons;
            if (s - start >= P.min_obs) {
                ++n_good;
                good_obs += s - start;
            }
            start = s;
        }
    }
    if (n > 0) {
        ++n_seasons;
        if (j1 - start >= P.min_obs) {
            ++n_good;
            good_obs += j1 - start;
        }
    }

    const double nd = (double)n;
    const double var = m.syy / nd;
    const double sigma = sqrt(var);
    double w = 0.0;
    switch (lane) {
        case 0: w = log10(nd); break;
        case 1: w = log10(fmax(tmax - tmin, 1e-3)); break;
        case 2: w = (double)n_seasons; break;
        case 3: w = (double)n_good; break;
        case 4: w = dcnt > 0.0 ? log10(fmax(dsum / dcnt, 1e-6)) : 0.0; break;
        case 5: {
            if (dcnt > 0.0) {
                const double mu = lsum / dcnt;
                w = sqrt(fmax(lsq / dcnt - mu * mu, 0.0));
            }
            break;
        }
        case 6: w = (double)good_obs / nd; break;
        case 7: w = sigma > 0.0 ? log10(sigma) : -30.0; break;
        case 8: w = sigma > 0.0 ? (m3 / nd) / (var * sigma) : 0.0; break;
        case 9: w = sigma > 0.0 ? (m4 / nd) / (var * var) - 3.0 : 0.0; break;
        case 10: w = sigma > 0.0 ? amax / sigma : 0.0; break;
        default: break;
    }

    // Pass 3: spectral window |sum_j exp(2 pi i f_p t_j)|^2 / N^2, phases
    // taken from the object's mid-span origin (the modulus does not depend on
    // it) and reduced to [-1/2, 1/2] cycles in FP64, then the hardware FP32
    // sin/cos (argument in revolutions) as in the periodogram kernels, summed
    // in FP64.  The probe frequencies come with the parameters; an object of
    // up to kWindowStage points reads its t - t0 from LDS for every probe.
    const bool staged = n <= kWindowStage;
    if (staged) {
        for (int64_t j = j0 + lane; j < j1; j += kWave) s_tc[j - j0] = P.t[j] - m.t0;
        __syncthreads();
    }
    for (int p = 0; p < kProbes; ++p) {
        const double f = P.probe[p];
        double sc = 0.0, ss = 0.0;
        for (int64_t j = j0 + lane; j < j1; j += kWave) {
            double ph = f * (staged ? s_tc[j - j0] : P.t[j] - m.t0);
            ph -= rint(ph);
            const float r = (float)ph;
            sc += (double)__builtin_amdgcn_cosf(r);
            ss += (double)__builtin_amdgcn_sinf(r);
        }
        sc = wave_sum(sc);
        ss = wave_sum(ss);
        if (lane == 11 + p) w = (sc * sc + ss * ss) / (nd * nd);
    }
    out[lane] = (float)w;
}

}  // namespace

static hipError_t launch_features(const ObjMeta* meta, unsigned int* queue, const double* t,
                                  const double* y, double f_min,
                           double f_max, int unit, double gap, int min_obs, int64_t n_obj,
                           float* out, hipStream_t s) {
    if (n_obj <= 0) return hipSuccess;
    FeatParams p;
    p.meta = meta;
    p.t = t;
    p.y = y;
    p.f_min = f_min;
    p.df = (f_max - f_min) / (double)(LSP_FEAT_COARSE * LSP_FEAT_POOL);
    p.to_cyc = unit == LSP_UNIT_CYCLES ? 1.0 : kInvTwoPi;
    p.step_cyc = (double)kWave * p.df * p.to_cyc;
    p.gap = gap;
    p.n_obj = n_obj;
    p.min_obs = min_obs;
    p.pad = 0;
    p.out = out;
    p.queue = queue;
    const double lstep = (log10(30.0) + 3.0) / (double)(kProbes - 1);
    for (int q = 0; q < kProbes; ++q) p.probe[q] = pow(10.0, -3.0 + (double)q * lstep);
    hipError_t e0 = launch_fill_u32(queue, kXcds, 0u, s);
    if (e0 != hipSuccess) return e0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, coarse_kernel, kWave * kCoarseW, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    hipLaunchKernelGGL(coarse_kernel, dim3((unsigned)(per_cu * cus)), dim3(kWave * kCoarseW), 0, s,
                       p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(window_kernel, grid_for(n_obj), dim3(kWave), 0, s, p);
    return hipGetLastError();
}

}  // namespace lsp

extern "C" {

lsp_feature_options lsp_default_feature_options(void) {
    lsp_feature_options o = {};
    o.season_gap = 60.0;
    o.min_season_obs = 8;
    return o;
}

size_t lsp_features_workspace_bytes(int64_t n_obj) {
    if (n_obj < 1) return 0;
    // per-object statistics, then 256 bytes of queue counters
    return ((size_t)n_obj * sizeof(lsp::ObjMeta) + 255) / 256 * 256 + 256;
}

lsp_status lsp_features(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                        const double* y, const lsp_grid* grid, const lsp_feature_options* fopt_in,
                        float* features, void* workspace, size_t workspace_bytes, void* stream) {
    if (!offsets || !grid || !features || !workspace) return LSP_EINVAL;
    if (n_obj < 1 || n_obs < 0 || (n_obs > 0 && (!t || !y))) return LSP_EINVAL;
    if (!(std::isfinite(grid->f_min) && std::isfinite(grid->f_max) && grid->f_max > grid->f_min) ||
        !(grid->unit == LSP_UNIT_CYCLES || grid->unit == LSP_UNIT_ANGULAR))
        return LSP_EINVAL;
    const lsp_feature_options fo = fopt_in ? *fopt_in : lsp_default_feature_options();
    if (!(std::isfinite(fo.season_gap) && fo.season_gap >= 0.0) || fo.min_season_obs < 2)
        return LSP_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return LSP_EINVAL;
    if (workspace_bytes < lsp_features_workspace_bytes(n_obj)) return LSP_ENOMEM;
    if (n_obj > (((int64_t)1 << 31) - 1) / lsp::kTilesPerObj) return LSP_EUNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    lsp::PrepParams pp;
    pp.offsets = offsets;
    pp.t = t;
    pp.y = y;
    pp.n_obj = n_obj;
    pp.n_obs = n_obs;
    pp.subtract_mean = 1;
    pp.normalize = 1;
    pp.meta = static_cast<lsp::ObjMeta*>(workspace);
    if (lsp::launch_prep(pp, s) != hipSuccess) return LSP_EHIP;
    unsigned int* queue = reinterpret_cast<unsigned int*>(
        static_cast<char*>(workspace) + lsp_features_workspace_bytes(n_obj) - 256);
    if (lsp::launch_features(pp.meta, queue, t, y, grid->f_min, grid->f_max, grid->unit,
                             fo.season_gap,
                             fo.min_season_obs, n_obj, features, s) != hipSuccess)
        return LSP_EHIP;
    return LSP_OK;
}

}  // extern "C"
