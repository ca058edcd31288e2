// lsp_gen.hip -- the generalized periodogram (Section 4.11): photometric
// errors as weights 1/dy^2 and a floating mean, i.e. the weighted
// least-squares fit of a sinusoid plus offset at every trial frequency.
//
// Both forms accumulate, per (object, frequency), the sums of SumsGen64 in
// lsp_common.h over the object's observations and finalise them without
// forming tau (power64_gen / power32_gen).  The prep kernel has already
// rescaled the weights to w' = wnorm / dy^2 (summing to N) and found the
// weighted mean; both are applied while observations are staged into LDS.
//
// FP32 form.  As in lsp_fp32p.hip, each lane owns K frequencies 64 bins apart,
// seeds cos and sin of its first phase from an FP64-reduced argument with the
// hardware v_sin/v_cos, and walks the other K - 1 by the three-term
// recurrence.  The seeds are scaled by sqrt(w'): the recurrence is linear, so
// u = sqrt(w') cos and v = sqrt(w') sin follow it too, and the six sums are six
// FMAs per bin,
//   sum w' cos = sum sqrt(w') u,  sum w' sin = sum sqrt(w') v,
//   sum w' yw cos = sum (sqrt(w') yw) u,  sum w' yw sin = sum (sqrt(w') yw) v,
//   sum w' cos^2 = sum u u,  sum w' cos sin = sum u v,
// plus two for the recurrence: 8 instructions per evaluation against the
// standard form's 6.  Bins whose smaller denominator is below N/32 mark their
// tile for the FP64 fix-up, which recomputes it with power64_gen_bin.
//
// FP64 form: a library sincos per term, as the standard FP64 form.
#include "lsp_common.h"

namespace lsp {
namespace {

template <int K, int W>
__device__ __forceinline__ void gen_item(const MainParams& P, int64_t item, double* s_tau,
                                         float4* s_obs, PeakRec* s_red) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t tile_freqs = (int64_t)kWave * K * W;
    // item = (row, chunk of tiles_per_item consecutive frequency tiles,
    // observation split); a split object has one tile per chunk
    const int64_t chunk_id = item / P.n_split;
    const int split = (int)(item - chunk_id * P.n_split);
    const int64_t rank = chunk_id / P.chunks_per_row;
    const int64_t chunk = chunk_id - rank * P.chunks_per_row;
    const int64_t row = item_row(P.row_perm, rank);
    const RowRange rr =
        decode_row(P.row_obj, P.row_band, P.band_bins, P.rows_per_group, P.n_obj, P.n_f, row);
    const int64_t obj = rr.obj;
    const int64_t t_lo = chunk * P.tiles_per_item;
    const int64_t t_hi = t_lo + P.tiles_per_item < P.tiles_per_row ? t_lo + P.tiles_per_item
                                                                   : P.tiles_per_row;
    const int64_t lane_off = (int64_t)wave * kWave * K + lane;
    const int64_t f_hi = rr.f_hi;
    // invalid row or empty chunk: no bin, nothing to record
    if (obj < 0 || rr.f_lo + t_lo * tile_freqs >= f_hi) return;
    const ObjMeta m = P.meta[obj];

    if (m.status != LSP_OBJ_OK) {
        if (P.n_split == 1 && P.pgram) {
            const double v = fill_value(m.status);
            for (int64_t ft = t_lo; ft < t_hi; ++ft)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int64_t i = rr.f_lo + ft * tile_freqs + lane_off + (int64_t)kWave * k;
                    if (i < f_hi) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, v);
                }
        }
        return;
    }

    const int64_t span = (m.n + P.n_split - 1) / P.n_split;
    const int64_t lo = (int64_t)split * span < m.n ? (int64_t)split * span : m.n;
    const int64_t hi = lo + span < m.n ? lo + span : m.n;
    const int64_t js = m.j0 + lo, je = m.j0 + hi;
    const double swn = sqrt(m.wnorm);
    // an object that fits in one staging pass is staged once for all the
    // chunk's tiles
    const bool one_pass = je - js <= kTile;

    unsigned long long best = 0ull;  // this lane's best key over the chunk's resolvable tiles
    for (int64_t ft = t_lo; ft < t_hi; ++ft) {
        if (rr.f_lo + ft * tile_freqs >= f_hi) break;
        const int64_t i0 = rr.f_lo + ft * tile_freqs + lane_off;
        const double fl = grid_freq(P.f_min, P.df, i0) * P.to_cyc;

        float c1[K], s1[K], yc[K], ys[K], wcc[K], wcs[K];
#pragma unroll
        for (int k = 0; k < K; ++k) c1[k] = s1[k] = yc[k] = ys[k] = wcc[k] = wcs[k] = 0.0f;

        for (int64_t jt = js; jt < je; jt += kTile) {
            const int cnt = (int)((je - jt) < kTile ? (je - jt) : kTile);
            if (!one_pass || ft == t_lo) {
                __syncthreads();
                for (int q = threadIdx.x; q < cnt; q += kWave * W) {
                    const int64_t j = jt + q;
                    const double tc = P.t[j] - m.t0;
                    s_tau[q] = tc;
                    double sp = P.step_cyc * tc;
                    sp -= rint(sp);
                    const float rs = (float)sp;
                    const double sw = P.dy ? swn / P.dy[j] : 1.0;
                    s_obs[q] = make_float4((float)(sw * (P.y[j] - m.ybar)),
                                           __builtin_amdgcn_cosf(rs), __builtin_amdgcn_sinf(rs),
                                           (float)sw);
                }
                __syncthreads();
            }
            for (int q = 0; q < cnt; ++q) {
                const double tq = s_tau[q];
                const float4 o = s_obs[q];  // (sqrt(w') yw, cos step, sin step, sqrt(w'))
                double ph = fl * tq;
                ph -= rint(ph);
                const float r = (float)ph;
                const float two_c = o.y + o.y;
                float cp = __builtin_amdgcn_cosf(r) * o.w;
                float sp = __builtin_amdgcn_sinf(r) * o.w;
                float c = fmaf(cp, o.y, -(sp * o.z));
                float s = fmaf(sp, o.y, cp * o.z);
                c1[0] = fmaf(o.w, cp, c1[0]);
                s1[0] = fmaf(o.w, sp, s1[0]);
                yc[0] = fmaf(o.x, cp, yc[0]);
                ys[0] = fmaf(o.x, sp, ys[0]);
                wcc[0] = fmaf(cp, cp, wcc[0]);
                wcs[0] = fmaf(cp, sp, wcs[0]);
#pragma unroll
                for (int k = 1; k < K; ++k) {
                    c1[k] = fmaf(o.w, c, c1[k]);
                    s1[k] = fmaf(o.w, s, s1[k]);
                    yc[k] = fmaf(o.x, c, yc[k]);
                    ys[k] = fmaf(o.x, s, ys[k]);
                    wcc[k] = fmaf(c, c, wcc[k]);
                    wcs[k] = fmaf(c, s, wcs[k]);
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

        if (P.n_split > 1) {
            const int64_t nf = P.n_f;
            float* base = P.part + (int64_t)split * 6 * nf;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t i = i0 + (int64_t)kWave * k;
                if (i < f_hi) {
                    base[i] = c1[k];
                    base[nf + i] = s1[k];
                    base[2 * nf + i] = yc[k];
                    base[3 * nf + i] = ys[k];
                    base[4 * nf + i] = wcc[k];
                    base[5 * nf + i] = wcs[k];
                }
            }
            continue;
        }

        unsigned long long tb = 0ull;  // the tile's best key in this lane
        const float n = (float)m.n;
        const float scale = (float)m.scale;
        bool any_ill = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t i = i0 + (int64_t)kWave * k;
            if (i < f_hi) {
                bool ill;
                const float p =
                    power32_gen(c1[k], s1[k], yc[k], ys[k], wcc[k], wcs[k], n, scale, ill);
                any_ill |= ill;
                if (P.pgram) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, (double)p);
                if (p == p) tb = umax64(tb, peak_key(p, i));  // NaN never wins
            }
        }
        // A tile holding an ill-conditioned bin sets its bit for the fix-up
        // kernel, which recomputes the whole tile in FP64 and merges its best
        // into the group's key; the other tiles' bins join the running best.
        any_ill = __syncthreads_or(any_ill);
        if (any_ill) {
            if (threadIdx.x == 0) {
                const int64_t tile = row * P.tiles_per_row + ft;
                atomicOr(&P.ill_bits[tile >> 5], 1u << (tile & 31));
            }
        } else {
            best = umax64(best, tb);
        }
    }
    if (P.n_split > 1) return;

    // the chunk's best bin goes into its group's peak key (one atomic per item)
    best = wave_max_u64(best);
    unsigned long long* s_key = reinterpret_cast<unsigned long long*>(s_red);
    if (lane == 0) s_key[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = s_key[0];
#pragma unroll
        for (int w = 1; w < W; ++w) b = umax64(b, s_key[w]);
        if (b != 0ull) atomicMax(&P.keys[row / P.rows_per_group], b);
    }
}

// Six sums per bin: up to K = 12 the kernel keeps four waves per SIMD (at most
// 128 VGPRs, K = 8) or three (168, K = 12); K = 16 is held to three.
template <int K, int W>
__global__ __launch_bounds__(kWave* W)
    __attribute__((amdgpu_waves_per_eu(K <= 8 ? 4 : 3))) void gen_fp32p_kernel(const MainParams P) {
    __shared__ double s_tau[kTile];
    __shared__ float4 s_obs[kTile];
    __shared__ PeakRec s_red[W];
    __shared__ int64_t s_item;

    if (!P.persistent) {
        const int64_t b = linear_block();
        if (b < P.n_items) gen_item<K, W>(P, xcd_remap(b, P.n_items), s_tau, s_obs, s_red);
        return;
    }
    // each XCD's queue holds the items of one contiguous run of row ranks
    const int64_t per_row = P.chunks_per_row * P.n_split;
    const int64_t n_rows = P.n_items / per_row;
    const int x0 = (int)(blockIdx.x % kXcds);
    for (int d = 0; d < kXcds; ++d) {
        const int x = (x0 + d) % kXcds;
        const int64_t lo = xcd_first_rank(x, n_rows) * per_row;
        const int64_t hi = xcd_queue_end(x, n_rows, per_row, P.n_work);
        int64_t item = pop_item(&P.queue[x], lo, &s_item);
        while (item < hi) {
            gen_item<K, W>(P, item, s_tau, s_obs, s_red);
            item = pop_item(&P.queue[x], lo, &s_item);
        }
    }
}

template <int KF, int W>
__global__ __launch_bounds__(kWave* W) void gen_fp64_kernel(const MainParams P) {
    __shared__ double s_tau[kTile];
    __shared__ double s_tlo[kTile];
    __shared__ double s_w[kTile];
    __shared__ double s_wy[kTile];
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
    const RowRange rr =
        decode_row(P.row_obj, P.row_band, P.band_bins, P.rows_per_group, P.n_obj, P.n_f, row);
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
    SumsGen64 acc[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        fc[k] = grid_freq(P.f_min, P.df, i0 + (int64_t)kWave * k) * P.to_cyc;
        acc[k] = SumsGen64{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    }

    const int64_t j_end = m.j0 + m.n;
    for (int64_t jt = m.j0; jt < j_end; jt += kTile) {
        const int cnt = (int)((j_end - jt) < kTile ? (j_end - jt) : kTile);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kWave * W) {
            const int64_t j = jt + q;
            const double w = gen_weight(P.dy, j, m.wnorm);
            recentre64(P.t[j], m.t0, &s_tau[q], &s_tlo[q]);
            s_w[q] = w;
            s_wy[q] = w * (P.y[j] - m.ybar);
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double tq = s_tau[q];
            const double tl = s_tlo[q];
            const double wq = s_w[q];
            const double wyq = s_wy[q];
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                double s, c;
                sincos_cycles64(fc[k], tq, tl, &s, &c);
                sumsgen64_add(acc[k], wq, wyq, s, c);
            }
        }
    }

    PeakRec best{0.0, -1};
    const double n = (double)m.n;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        const int64_t i = i0 + (int64_t)kWave * k;
        if (i < f_hi) {
            const double p = power64_gen(acc[k], n, m.scale);
            if (P.pgram) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, p);
            if (better(p, i, best.p, best.i)) best = PeakRec{p, i};
        }
    }
    best = wave_best(best);
    if (lane == 0) s_red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        PeakRec b2 = s_red[0];
#pragma unroll
        for (int w = 1; w < W; ++w)
            if (better(s_red[w].p, s_red[w].i, b2.p, b2.i)) b2 = s_red[w];
        P.rec[item] = b2;
    }
}

template <int K, int W>
int gen_occupancy_blocks() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gen_fp32p_kernel<K, W>, kWave * W,
                                                     0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    return per_cu * cus;
}

template <int K, int W>
hipError_t launch_gkw(const MainParams& p, hipStream_t s) {
    const dim3 grid =
        p.persistent ? dim3((unsigned)gen_occupancy_blocks<K, W>()) : grid_for(p.n_items);
    hipLaunchKernelGGL((gen_fp32p_kernel<K, W>), grid, dim3(kWave * W), 0, s, p);
    return hipGetLastError();
}

template <int K>
hipError_t launch_gk(const MainParams& p, int waves, hipStream_t s) {
    switch (waves) {
        case 1: return launch_gkw<K, 1>(p, s);
        case 2: return launch_gkw<K, 2>(p, s);
        case 4: return launch_gkw<K, 4>(p, s);
        default: return hipErrorInvalidValue;
    }
}

template <int KF>
hipError_t launch_g64(const MainParams& p, int waves, hipStream_t s) {
    const dim3 grid = grid_for(p.n_items);
    switch (waves) {
        case 1: hipLaunchKernelGGL((gen_fp64_kernel<KF, 1>), grid, dim3(kWave * 1), 0, s, p); break;
        case 2: hipLaunchKernelGGL((gen_fp64_kernel<KF, 2>), grid, dim3(kWave * 2), 0, s, p); break;
        case 4: hipLaunchKernelGGL((gen_fp64_kernel<KF, 4>), grid, dim3(kWave * 4), 0, s, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gen_fp32p(const MainParams& p, int k, int waves, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    switch (k) {
        case 4: return launch_gk<4>(p, waves, s);
        case 8: return launch_gk<8>(p, waves, s);
        case 12: return launch_gk<12>(p, waves, s);
        case 16: return launch_gk<16>(p, waves, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gen_fp64(const MainParams& p, int kf, int waves, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    switch (kf) {
        case 1: return launch_g64<1>(p, waves, s);
        case 2: return launch_g64<2>(p, waves, s);
        case 4: return launch_g64<4>(p, waves, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lsp
