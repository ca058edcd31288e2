// lsp_fp64.hip -- the plain FP64 form of the periodogram (reference form).
//
// Every term of the sums gets its own FP64 sin/cos from the HIP math library,
// as in the paper's kernel (Section 3.7): one pass over the object's
// observations accumulates sum y cos wt, y sin wt, cos^2, sin^2 and cos sin,
// and Eq. 1 and Eq. 2 are then applied to those sums (power64).  The phase is
// formed in cycles from the re-centred time and its rounding error with an
// exact split of the frequency-time product (sincos_cycles64), and reduced
// exactly before the library call, which keeps the library on its
// short-argument path and the phase accurate to its last rounding.
//
// This file also holds the FP64 fix-up of the FP32 form (fixup_kernel), for
// the standard and the generalized periodogram.
//
// Work decomposition: a workgroup of W wavefronts owns one (object, frequency
// tile) item; the object is staged through LDS in chunks of kTile observations
// and every lane of a wavefront owns KF frequencies spaced 64 bins apart, so
// that each periodogram store of the wavefront is 64 consecutive bins.
#include "lsp_common.h"

namespace lsp {
namespace {

template <int KF, int W>
__global__ __launch_bounds__(kWave* W) void fp64_kernel(const MainParams P) {
    __shared__ double s_tau[kTile];
    __shared__ double s_tlo[kTile];
    __shared__ double s_y[kTile];
    __shared__ PeakRec s_red[W];

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t tile_freqs = (int64_t)kWave * KF * W;
    const int64_t b = linear_block();
    if (b >= P.n_items) return;
    const int64_t rank_item = xcd_remap(b, P.n_items);
    const int64_t rank = rank_item / P.tiles_per_row;
    const int64_t ftile = rank_item - rank * P.tiles_per_row;
    const int64_t row = item_row(P.row_perm, rank);
    const int64_t item = row * P.tiles_per_row + ftile;  // the tile's record
    const RowRange rr = decode_row(P.row_obj, P.row_band, P.band_bins, P.rows_per_group, P.n_obj, P.n_f, row);
    const int64_t obj = rr.obj;
    const int64_t i0 = rr.f_lo + ftile * tile_freqs + (int64_t)wave * kWave * KF + lane;
    const int64_t f_hi = rr.f_hi;
    if (obj < 0 || rr.f_lo + ftile * tile_freqs >= f_hi) {
        if (threadIdx.x == 0) P.rec[item] = PeakRec{0.0, -1};
        return;
    }
    const ObjMeta m = P.meta[obj];

    if (m.status != LSP_OBJ_OK) {
        if (P.pgram) {
            const double v = fill_value(m.status);
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                const int64_t i = i0 + (int64_t)kWave * k;
                if (i < f_hi) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, v);
            }
        }
        if (threadIdx.x == 0) P.rec[item] = PeakRec{0.0, -1};
        return;
    }

    double fc[KF];
    Sums64 acc[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        fc[k] = grid_freq(P.f_min, P.df, i0 + (int64_t)kWave * k) * P.to_cyc;
        acc[k] = Sums64{0.0, 0.0, 0.0, 0.0, 0.0};
    }

    const int64_t j_end = m.j0 + m.n;
    for (int64_t jt = m.j0; jt < j_end; jt += kTile) {
        const int cnt = (int)((j_end - jt) < kTile ? (j_end - jt) : kTile);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kWave * W) {
            recentre64(P.t[jt + q], m.t0, &s_tau[q], &s_tlo[q]);
            s_y[q] = P.y[jt + q] - m.ybar;
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double tq = s_tau[q];
            const double tl = s_tlo[q];
            const double yq = s_y[q];
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                double s, c;
                sincos_cycles64(fc[k], tq, tl, &s, &c);
                sums64_add(acc[k], yq, s, c);
            }
        }
    }

    PeakRec best{0.0, -1};
    const double n = (double)m.n;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        const int64_t i = i0 + (int64_t)kWave * k;
        if (i < f_hi) {
            const double p = power64(acc[k], n, m.scale);
            if (P.pgram) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, p);
            if (better(p, i, best.p, best.i)) best = PeakRec{p, i};
        }
    }
    best = wave_best(best);
    if (lane == 0) s_red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        PeakRec b = s_red[0];
#pragma unroll
        for (int w = 1; w < W; ++w)
            if (better(s_red[w].p, s_red[w].i, b.p, b.i)) b = s_red[w];
        P.rec[item] = b;
    }
}

// FP64 recompute of FP32-form tiles flagged ill-conditioned.  Workgroups stride
// over the tiles' flag bits 256 at a time, collect the flagged ones in LDS, and
// recompute every bin of each such tile from the FP64 series (rounding the
// power to FP32 so the argmax still compares FP32 values), then rewrite the
// tile's periodogram bins and merge its best bin into the group's peak key.
constexpr int kFixThreads = 256;

__global__ __launch_bounds__(kFixThreads) void fixup_kernel(const FixupParams P) {
    __shared__ int64_t s_list[kFixThreads];
    __shared__ int s_count;
    __shared__ PeakRec s_red[kFixThreads / kWave];
    for (int64_t base = (int64_t)blockIdx.x * kFixThreads; base < P.n_tiles;
         base += (int64_t)gridDim.x * kFixThreads) {
        if (threadIdx.x == 0) s_count = 0;
        __syncthreads();
        const int64_t mine = base + threadIdx.x;
        if (mine < P.n_tiles && ((P.ill_bits[mine >> 5] >> (mine & 31)) & 1u))
            s_list[atomicAdd(&s_count, 1)] = mine;
        __syncthreads();
        const int count = uniform_i32(s_count);
        for (int q = 0; q < count; ++q) {
            const int64_t tile = uniform_i64(s_list[q]);
            const int64_t row = tile / P.tiles_per_row;
            const RowRange rr =
                decode_row(P.row_obj, P.row_band, P.band_bins, P.rows_per_group, P.n_obj, P.n_f, row);
            const int64_t obj = rr.obj < 0 ? 0 : rr.obj;
            const int64_t f0 = rr.f_lo + (tile - row * P.tiles_per_row) * P.tile_freqs;
            const ObjMeta m = P.meta[obj];
            PeakRec best{0.0, -1};
            for (int64_t i = f0 + threadIdx.x; i < f0 + P.tile_freqs && i < rr.f_hi;
                 i += kFixThreads) {
                const double f = grid_freq(P.f_min, P.df, i) * P.to_cyc;
                const double p = (double)(float)(P.gen ? power64_gen_bin(m, P.t, P.y, P.dy, f)
                                                       : power64_bin(m, P.t, P.y, f));
                if (P.pgram) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, p);
                if (better(p, i, best.p, best.i)) best = PeakRec{p, i};
            }
            best = wave_best(best);
            if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = best;
            __syncthreads();
            if (threadIdx.x == 0) {
                PeakRec b = s_red[0];
                for (int w = 1; w < kFixThreads / kWave; ++w)
                    if (better(s_red[w].p, s_red[w].i, b.p, b.i)) b = s_red[w];
                if (rr.obj >= 0 && b.i >= 0)
                    atomicMax(&P.keys[row / P.rows_per_group], peak_key(b.p, b.i));
            }
            __syncthreads();
        }
        __syncthreads();
    }
}

template <int KF>
hipError_t launch_kf(const MainParams& p, int waves, hipStream_t s) {
    const dim3 grid = grid_for(p.n_items);
    switch (waves) {
        case 1: hipLaunchKernelGGL((fp64_kernel<KF, 1>), grid, dim3(kWave * 1), 0, s, p); break;
        case 2: hipLaunchKernelGGL((fp64_kernel<KF, 2>), grid, dim3(kWave * 2), 0, s, p); break;
        case 4: hipLaunchKernelGGL((fp64_kernel<KF, 4>), grid, dim3(kWave * 4), 0, s, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fixup(const FixupParams& p, hipStream_t s) {
    if (p.n_tiles <= 0) return hipSuccess;
    int64_t blocks = (p.n_tiles + kFixThreads - 1) / kFixThreads;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(fixup_kernel, dim3((unsigned)blocks), dim3(kFixThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fp64(const MainParams& p, int kf, int waves, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    switch (kf) {
        case 1: return launch_kf<1>(p, waves, s);
        case 2: return launch_kf<2>(p, waves, s);
        case 4: return launch_kf<4>(p, waves, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lsp
