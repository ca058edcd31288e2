// lsp_reduce.hip -- per-object peak from the per-tile (power, index) records
// (FP64 form and split single objects) or from the per-group peak keys the
// FP32 forms merge atomically, and a small fill kernel for counters and flags.
//
// Section 3.3 takes the argmax of the periodogram (first maximal index) and
// converts it to a period, p = 2 pi / w; Section 3.4 keeps, per object, the best
// (power, index) found by each thread and reduces them.  Here every frequency
// tile has already reduced its bins to one record; one workgroup per object
// reduces the object's records with the same (power desc, index asc) order, so
// the result does not depend on execution order.
#include "lsp_common.h"

namespace lsp {
namespace {

constexpr int kPeakThreads = 256;

// The peak record of one object from its best (power, index).
__device__ __forceinline__ lsp_peak make_peak(const PeakParams& P, const ObjMeta& m, PeakRec b) {
    lsp_peak pk;
    pk.status = m.status;
    pk.reserved = 0;
    if (m.status == LSP_OBJ_OK && b.i >= 0) {
        const double f = grid_freq(P.f_min, P.df, b.i);
        pk.index = b.i;
        pk.freq = f;
        pk.period = P.unit == LSP_UNIT_ANGULAR ? kTwoPi / f : 1.0 / f;
        pk.power = b.p;
    } else {
        pk.index = -1;
        pk.freq = __builtin_nan("");
        pk.period = __builtin_nan("");
        pk.power = m.status == LSP_OBJ_OK ? __builtin_nan("") : fill_value(m.status);
    }
    return pk;
}

__global__ __launch_bounds__(kPeakThreads) void peaks_kernel(const PeakParams P) {
    __shared__ PeakRec s_red[kPeakThreads / kWave];
    const int64_t grp = linear_block();
    if (grp >= P.n_groups) return;
    const int64_t o =
        P.row_obj ? (int64_t)P.row_obj[grp * P.rows_per_group] : grp;  // uniform per group
    // (without row_obj, row r belongs to object r / rows_per_group, so group g is object g)
    if (o < 0 || o >= P.n_obj) return;
    const ObjMeta m = P.meta[o];
    PeakRec best{0.0, -1};
    if (m.status == LSP_OBJ_OK) {
        const PeakRec* r = P.rec + grp * P.rec_per_obj;
        for (int64_t q = threadIdx.x; q < P.rec_per_obj; q += kPeakThreads) {
            const PeakRec c = r[q];
            if (c.i >= 0 && better(c.p, c.i, best.p, best.i)) best = c;
        }
    }
    best = wave_best(best);
    if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        PeakRec b = s_red[0];
        for (int w = 1; w < kPeakThreads / kWave; ++w)
            if (better(s_red[w].p, s_red[w].i, b.p, b.i)) b = s_red[w];
        P.peaks[o] = make_peak(P, m, b);
    }
}

// The FP32 forms' groups: one thread per group decodes the group's peak key.
__global__ __launch_bounds__(kPeakThreads) void peaks_from_keys_kernel(const PeakParams P) {
    const int64_t grp = linear_block() * kPeakThreads + threadIdx.x;
    if (grp >= P.n_groups) return;
    const int64_t o = P.row_obj ? (int64_t)P.row_obj[grp * P.rows_per_group] : grp;
    if (o < 0 || o >= P.n_obj) return;
    const ObjMeta m = P.meta[o];
    const PeakRec b = m.status == LSP_OBJ_OK ? key_peak(P.keys[grp]) : PeakRec{0.0, -1};
    P.peaks[o] = make_peak(P, m, b);
}

__global__ void fill_u32_kernel(unsigned int* dst, int64_t n, unsigned int v) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

}  // namespace

hipError_t launch_peaks(const PeakParams& p, hipStream_t s) {
    if (p.n_groups <= 0) return hipSuccess;
    if (p.keys)
        hipLaunchKernelGGL(peaks_from_keys_kernel,
                           grid_for((p.n_groups + kPeakThreads - 1) / kPeakThreads),
                           dim3(kPeakThreads), 0, s, p);
    else
        hipLaunchKernelGGL(peaks_kernel, grid_for(p.n_groups), dim3(kPeakThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* dst, int64_t n, unsigned int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, grid_for((n + 255) / 256), dim3(256), 0, s, dst, n, v);
    return hipGetLastError();
}

}  // namespace lsp
