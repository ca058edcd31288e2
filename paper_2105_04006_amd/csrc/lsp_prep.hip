// lsp_prep.hip -- per-object statistics ahead of the periodogram kernels.
//
// Section 2 assumes zero-mean magnitudes; this kernel finds each object's mean
// ybar in FP64 and S_yy = sum (y - ybar)^2, which normalises the power, and the
// time origin t0 = mid-span of the object's times (the power does not depend
// on the time origin, and |t - t0| halves the phase magnitude the FP32 form
// must reduce).  The periodogram kernels re-centre t and y with these values
// as they stage observations, so nothing per observation is written here and
// objects whose CSR ranges overlap cannot interfere.  One workgroup per
// object; all reductions are in a fixed order (bitwise reproducible).
//
// Generalized form (Section 4.11): weights 1/dy^2 (unit weights without
// errors), the weighted mean, and the weighted S_yy; the mean is always
// removed (it is one of the fitted parameters).  An error that is not finite
// or not positive makes the object NONFINITE.
#include "lsp_common.h"

namespace lsp {
namespace {

struct Red {
    double sw, sy, syy_raw, tmin, tmax;
    int bad;
};

__device__ __forceinline__ Red combine(Red a, const Red& b) {
    a.sw += b.sw;
    a.sy += b.sy;
    a.syy_raw += b.syy_raw;
    a.tmin = fmin(a.tmin, b.tmin);
    a.tmax = fmax(a.tmax, b.tmax);
    a.bad |= b.bad;
    return a;
}

// Fixed-order reduction: butterfly within each wavefront, then the wave
// results in wave order (bitwise reproducible, one barrier pair).
__device__ Red block_reduce(Red r, Red* sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        Red b;
        b.sw = __shfl_xor(r.sw, o, kWave);
        b.sy = __shfl_xor(r.sy, o, kWave);
        b.syy_raw = __shfl_xor(r.syy_raw, o, kWave);
        b.tmin = __shfl_xor(r.tmin, o, kWave);
        b.tmax = __shfl_xor(r.tmax, o, kWave);
        b.bad = __shfl_xor(r.bad, o, kWave);
        r = combine(r, b);
    }
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) sh[wave] = r;
    __syncthreads();
    Red out = sh[0];
    for (int w = 1; w < kPrepThreads / kWave; ++w) out = combine(out, sh[w]);
    __syncthreads();
    return out;
}

__device__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) sh[wave] = v;
    __syncthreads();
    double out = sh[0];
    for (int w = 1; w < kPrepThreads / kWave; ++w) out += sh[w];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(kPrepThreads) void prep_kernel(const PrepParams P) {
    __shared__ Red sh_red[kPrepThreads / kWave];
    __shared__ double sh_sum[kPrepThreads / kWave];
    const int64_t o = linear_block();
    const int tid = threadIdx.x;
    if (o >= P.n_obj) return;

    int64_t j0 = 0, j1 = P.n_obs;
    if (P.offsets) {
        j0 = P.offsets[o];
        j1 = P.offsets[o + 1];
    }
    if (j0 < 0 || j1 < j0 || j1 > P.n_obs) {
        if (tid == 0) {
            ObjMeta m = {};
            m.j0 = 0;
            m.n = 0;
            m.status = LSP_OBJ_BADRANGE;
            P.meta[o] = m;
        }
        return;
    }
    const int64_t n = j1 - j0;

    Red r = {0.0, 0.0, 0.0, __builtin_inf(), -__builtin_inf(), 0};
    for (int64_t j = j0 + tid; j < j1; j += kPrepThreads) {
        const double tj = P.t[j], yj = P.y[j];
        if (!isfinite(tj) || !isfinite(yj)) r.bad = 1;
        double w = 1.0;
        if (P.gen && P.dy) {
            const double e = P.dy[j];
            if (!(isfinite(e) && e > 0.0)) r.bad = 1;
            w = 1.0 / (e * e);
        }
        r.sw += w;
        r.sy += w * yj;
        r.syy_raw += w * yj * yj;
        r.tmin = fmin(r.tmin, tj);
        r.tmax = fmax(r.tmax, tj);
    }
    r = block_reduce(r, sh_red);

    // Weights are rescaled to sum to N (wnorm / dy^2), which leaves the
    // normalised power unchanged and keeps the sums on the scale of unit weights.
    const bool ok_w = P.gen && !r.bad && n > 0 && r.sw > 0.0 && isfinite(r.sw);
    const double wnorm = ok_w && P.dy ? (double)n / r.sw : 1.0;
    const double ybar = P.gen ? (ok_w ? r.sy / r.sw : 0.0)
                              : ((P.subtract_mean && n > 0) ? r.sy / (double)n : 0.0);
    const double t0 = (n > 0 && !r.bad) ? 0.5 * (r.tmin + r.tmax) : 0.0;

    double sq = 0.0;
    for (int64_t j = j0 + tid; j < j1; j += kPrepThreads) {
        const double yc = P.y[j] - ybar;
        const double w = P.gen ? gen_weight(P.dy, j, wnorm) : 1.0;
        sq += w * yc * yc;
    }
    const double syy = block_sum(sq, sh_sum);

    if (tid == 0) {
        ObjMeta m = {};
        m.j0 = j0;
        m.n = n;
        m.ybar = ybar;
        m.syy = syy;
        m.t0 = t0;
        m.wnorm = wnorm;
        int32_t st = LSP_OBJ_OK;
        if (r.bad || (P.gen && n > 0 && !ok_w))
            st = LSP_OBJ_NONFINITE;
        else if (n < 2 || syy == 0.0 || syy <= kVarEps * r.syy_raw * wnorm)
            st = LSP_OBJ_DEGENERATE;
        m.status = st;
        // generalized, unnormalised: half the chi^2 reduction in the caller's
        // weights is 1 / wnorm times that in the rescaled weights
        m.scale = P.normalize ? (st == LSP_OBJ_OK ? 2.0 / syy : 0.0) : 1.0 / wnorm;
        P.meta[o] = m;
    }
}

// Staging pass of LSP_OBS_DIRECT: the per-observation values the main
// kernel would otherwise stage in LDS, written once per observation of each
// object (t - t0, and y - ybar with the step rotation of the FP32 form).
template <int TRIG>
__global__ __launch_bounds__(kPrepThreads) void stage_kernel(const ObjMeta* __restrict__ meta,
                                                             const double* __restrict__ t,
                                                             const double* __restrict__ y,
                                                             int64_t n_obj, double step_cyc,
                                                             double* stage_t, float4* stage_o) {
    const int64_t o = linear_block();
    if (o >= n_obj) return;
    const ObjMeta m = meta[o];
    if (m.status != LSP_OBJ_OK) return;
    for (int64_t j = m.j0 + threadIdx.x; j < m.j0 + m.n; j += kPrepThreads) {
        const double tc = t[j] - m.t0;
        double sp = step_cyc * tc;
        sp -= rint(sp);
        float ss, cs;
        seed_sincos<TRIG>((float)sp, &ss, &cs);
        stage_t[j] = tc;
        stage_o[j] = make_float4((float)(y[j] - m.ybar), cs, ss, 0.0f);
    }
}

}  // namespace

hipError_t launch_stage(const ObjMeta* meta, const double* t, const double* y, int64_t n_obj,
                        double step_cyc, int trig, double* stage_t, float4* stage_o,
                        hipStream_t s) {
    if (n_obj <= 0) return hipSuccess;
    const dim3 grid = grid_for(n_obj);
    switch (trig) {
        case LSP_TRIG_HW:
            hipLaunchKernelGGL(stage_kernel<LSP_TRIG_HW>, grid, dim3(kPrepThreads), 0, s, meta, t,
                               y, n_obj, step_cyc, stage_t, stage_o);
            break;
        case LSP_TRIG_LIB:
            hipLaunchKernelGGL(stage_kernel<LSP_TRIG_LIB>, grid, dim3(kPrepThreads), 0, s, meta,
                               t, y, n_obj, step_cyc, stage_t, stage_o);
            break;
        case LSP_TRIG_POLY:
            hipLaunchKernelGGL(stage_kernel<LSP_TRIG_POLY>, grid, dim3(kPrepThreads), 0, s, meta,
                               t, y, n_obj, step_cyc, stage_t, stage_o);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prep(const PrepParams& p, hipStream_t s) {
    if (p.n_obj <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, grid_for(p.n_obj), dim3(kPrepThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace lsp
