// lsp_fp32p.hip -- the FP32 form of the periodogram with FP64 phase reduction.
//
// The sums of the single-pass form (Section 2) are accumulated in FP32.  Each
// lane owns K frequencies spaced 64 bins apart, f_k = f_0 + 64 k df.  For every
// observation the lane
//   1. forms its first phase f_0 (t_j - t0) in cycles in FP64 and reduces it
//      exactly to [-1/2, 1/2] (the only FP64 work per observation),
//   2. seeds (cos, sin) of that phase with the hardware v_cos_f32 / v_sin_f32,
//      whose argument is in revolutions,
//   3. walks its other K-1 frequencies by angle addition with the
//      observation's step rotation (cos, sin)(2 pi 64 df (t_j - t0)), formed
//      the same way (FP64 reduction, hardware sin/cos) when the observation is
//      staged into LDS, and
//   4. accumulates sum y cos, sum y sin, sum cos^2 and sum cos sin per frequency.
// The recurrence restarts from an exact FP64-reduced seed at every
// observation, so its rounding error never grows beyond K - 1 steps.  This is
// the frequency-to-frequency recurrence Section 4.5 describes and sets aside
// for a sequential loop over the whole grid; here each lane runs it over only
// its own K frequencies, so every lane stays independent.
//
// Eq. 1 and Eq. 2 are applied to the FP32 sums without forming tau (power32).
// A bin whose smaller shifted denominator is too small for FP32 to resolve
// marks its tile, and the FP64 fix-up kernel (lsp_fp64.hip) recomputes that
// whole tile from the FP64 series; the hot kernel itself carries no FP64 trig.
//
// Items are (object, frequency tile[, observation split]).  A workgroup of W
// wavefronts covers 64 K W frequencies of one object, sharing the LDS-staged
// observations.  Items are either one per workgroup (grid schedule, with an
// XCD-aware order) or popped by resident workgroups from eight per-XCD atomic
// queues (persistent schedule); a workgroup that drains its own XCD's queue
// moves on to the next XCD's, and exits once every queue is empty.
#include "lsp_common.h"

namespace lsp {
namespace {

// Per-observation staged values: t - t0 (FP64) and (y - ybar, cos, sin of the
// step rotation 2 pi 64 df (t - t0), 0), the step phase reduced in FP64.
template <int TRIG>
__device__ __forceinline__ float4 stage_obs(double step_cyc, double tc, double yc) {
    double sp = step_cyc * tc;
    sp -= rint(sp);
    float ss, cs;
    seed_sincos<TRIG>((float)sp, &ss, &cs);
    return make_float4((float)yc, cs, ss, 0.0f);
}

// SRC: LSP_OBS_LDS stages tiles of observations in LDS; LSP_OBS_DIRECT reads
// the staging pass's values from global memory.  TRIG: LSP_TRIG_*.
// WS (wave split): the W waves of a workgroup share the same 64 K bins and
// each takes every W-th staged observation; their sums are added in LDS, as a
// fixed tree over the waves, before the finish.  This multiplies the waves working on one
// object without the per-split partial sums in HBM that the observation split
// across workgroups needs.

// Observations staged per pass: one per thread for the eight-wave split.
template <int W, bool WS>
constexpr int stage_tile() { return WS && W * kWave > kTile ? W * kWave : kTile; }

template <int K, int W, bool CHEB, bool WS, int SRC, int TRIG>
__device__ __forceinline__ void fp32p_item(const MainParams& P, int64_t item, double* s_tau,
                                           float4* s_obs, PeakRec* s_red, float* s_part) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    constexpr int WT = WS ? 1 : W;  // waves across the tile's frequencies
    const int64_t tile_freqs = (int64_t)kWave * K * WT;
    // item = (row, chunk of tiles_per_item consecutive frequency tiles,
    // observation split); a split object has one tile per chunk
    const int64_t chunk_id = item / P.n_split;
    const int split = (int)(item - chunk_id * P.n_split);
    const int64_t rank = chunk_id / P.chunks_per_row;
    const int64_t chunk = chunk_id - rank * P.chunks_per_row;
    const int64_t row = item_row(P.row_perm, rank);
    const RowRange rr = decode_row(P.row_obj, P.row_band, P.band_bins, P.rows_per_group, P.n_obj, P.n_f, row);
    const int64_t obj = rr.obj;
    const int64_t t_lo = chunk * P.tiles_per_item;
    const int64_t t_hi = t_lo + P.tiles_per_item < P.tiles_per_row ? t_lo + P.tiles_per_item
                                                                   : P.tiles_per_row;
    const int64_t lane_off = (WS ? 0 : (int64_t)wave * kWave * K) + lane;
    const int64_t f_hi = rr.f_hi;
    const bool owner = !WS || wave == 0;  // the wave that finishes the tile's bins
    // invalid row or empty chunk: no bin, nothing to record
    if (obj < 0 || rr.f_lo + t_lo * tile_freqs >= f_hi) return;
    const ObjMeta m = P.meta[obj];

    if (m.status != LSP_OBJ_OK) {
        if (P.n_split == 1 && P.pgram && owner) {
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
    // an object that fits in one staging pass is staged once for all the
    // chunk's tiles
    constexpr int ST = stage_tile<W, WS>();
    const bool one_pass = je - js <= ST;

    unsigned long long best = 0ull;  // this lane's best key over the chunk's resolvable tiles
    for (int64_t ft = t_lo; ft < t_hi; ++ft) {
        if (rr.f_lo + ft * tile_freqs >= f_hi) break;
        const int64_t i0 = rr.f_lo + ft * tile_freqs + lane_off;
        const double fl = grid_freq(P.f_min, P.df, i0) * P.to_cyc;

        float xc[K], xs[K], cc[K], cs[K];
#pragma unroll
        for (int k = 0; k < K; ++k) xc[k] = xs[k] = cc[k] = cs[k] = 0.0f;

        if (SRC == LSP_OBS_DIRECT) {
            // the staging pass's values, read straight from global memory; the
            // index is wave-uniform, so every lane loads the same address
            for (int64_t j = js; j < je; ++j)
                accumulate_obs<K, CHEB, TRIG>(fl, P.stage_t[j], P.stage_o[j], xc, xs, cc, cs);
        } else if (WS && W * kWave > kTile) {
            // Eight waves that share the bins see only an eighth of each
            // staging pass, too few observations to hide the staging loads:
            // a pass stages one observation per thread (512), and each
            // thread's t and y for the next pass are loaded before the current
            // pass's accumulation, so that the loads' latency hides behind it
            const int tid = (int)threadIdx.x;
            double nt = 0.0, ny = 0.0;
            if (tid < je - js) {
                nt = P.t[js + tid];
                ny = P.y[js + tid];
            }
            for (int64_t jt = js; jt < je; jt += ST) {
                const int cnt = (int)((je - jt) < ST ? (je - jt) : ST);
                if (!one_pass || ft == t_lo) {
                    __syncthreads();
                    if (tid < cnt) {
                        const double tc = nt - m.t0;
                        s_tau[tid] = tc;
                        s_obs[tid] = stage_obs<TRIG>(P.step_cyc, tc, ny - m.ybar);
                    }
                    __syncthreads();
                    const int64_t jn = jt + ST;
                    if (jn < je && tid < je - jn) {
                        nt = P.t[jn + tid];
                        ny = P.y[jn + tid];
                    }
                }
                for (int q = uniform_i32(wave); q < cnt; q += W)
                    accumulate_obs<K, CHEB, TRIG>(fl, s_tau[q], s_obs[q], xc, xs, cc, cs);
            }
        } else {
            for (int64_t jt = js; jt < je; jt += kTile) {
                const int cnt = (int)((je - jt) < kTile ? (je - jt) : kTile);
                if (!one_pass || ft == t_lo) {
                    __syncthreads();
                    for (int q = threadIdx.x; q < cnt; q += kWave * W) {
                        const double tc = P.t[jt + q] - m.t0;
                        s_tau[q] = tc;
                        // step rotation: the phase advance over kWave bins
                        s_obs[q] = stage_obs<TRIG>(P.step_cyc, tc, P.y[jt + q] - m.ybar);
                    }
                    __syncthreads();
                }
                // (the wave index is uniform across the wave; say so, so that the
                // staged reads stay scalar-addressed broadcasts)
                for (int q = WS ? uniform_i32(wave) : 0; q < cnt; q += WS ? W : 1)
                    accumulate_obs<K, CHEB, TRIG>(fl, s_tau[q], s_obs[q], xc, xs, cc, cs);
            }
        }

        if (WS) {
            // add the waves' sums into wave 0's, one array at a time, as a
            // tree: in each round the upper half of the remaining waves hands
            // its sums through LDS to the lower half (a fixed order)
            // (one base address per wave, the bins at fixed offsets from it)
            auto gather = [&](float(&v)[K]) {
#pragma unroll
                for (int half = W / 2; half >= 1; half /= 2) {
                    __syncthreads();
                    if (wave >= half && wave < 2 * half) {
                        float* dst = s_part + (wave - half) * (K * kWave) + lane;
#pragma unroll
                        for (int k = 0; k < K; ++k) dst[k * kWave] = v[k];
                    }
                    __syncthreads();
                    if (wave < half) {
                        const float* src = s_part + wave * (K * kWave) + lane;
#pragma unroll
                        for (int k = 0; k < K; ++k) v[k] += src[k * kWave];
                    }
                }
            };
            gather(xc);
            gather(xs);
            gather(cc);
            gather(cs);
        }

        if (P.n_split > 1) {
            const int64_t nf = P.n_f;
            float* base = P.part + (int64_t)split * 4 * nf;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t i = i0 + (int64_t)kWave * k;
                if (owner && i < f_hi) {
                    base[i] = xc[k];
                    base[nf + i] = xs[k];
                    base[2 * nf + i] = cc[k];
                    base[3 * nf + i] = cs[k];
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
            if (owner && i < f_hi) {
                bool ill;
                const float p = power32(xc[k], xs[k], cc[k], cs[k], n, scale, ill);
                any_ill |= ill;
                if (P.pgram) store_pgram(P.pgram, P.pgram_f64, obj * P.n_f + i, (double)p);
                if (p == p) tb = umax64(tb, peak_key(p, i));  // NaN never wins
            }
        }
        // A tile holding an ill-conditioned bin sets its bit for the fix-up
        // kernel, which recomputes the whole tile in FP64, rewrites its bins
        // and merges its best into the group's key; the other tiles' bins
        // join the running best.
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

// Up to K = 16 the kernel must keep four waves per SIMD (at most 128 VGPRs):
// with three, the VALU waits on latency more often.
template <int K, int W, bool CHEB, bool WS, int SRC = LSP_OBS_LDS, int TRIG = LSP_TRIG_HW>
__global__ __launch_bounds__(kWave* W)
    __attribute__((amdgpu_waves_per_eu(K <= 16 ? 4 : 1))) void fp32p_kernel(
        const MainParams P) {
    __shared__ double s_tau[stage_tile<W, WS>()];
    __shared__ float4 s_obs[stage_tile<W, WS>()];
    __shared__ PeakRec s_red[W];
    __shared__ int64_t s_item;
    __shared__ float s_part[WS ? (W / 2) * K * kWave : 1];

    if (!P.persistent) {
        const int64_t b = linear_block();
        if (b < P.n_items)
            fp32p_item<K, W, CHEB, WS, SRC, TRIG>(P, xcd_remap(b, P.n_items), s_tau, s_obs, s_red,
                                                  s_part);
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
            fp32p_item<K, W, CHEB, WS, SRC, TRIG>(P, item, s_tau, s_obs, s_red, s_part);
            item = pop_item(&P.queue[x], lo, &s_item);
        }
    }
}

// Sum the per-split partial sums of a single object in a fixed order, then
// finalise exactly as the unsplit path does (4 sums per bin for the standard
// periodogram, 6 for the generalized one).
__global__ __launch_bounds__(kCombineThreads) void combine_kernel(const CombineParams P) {
    __shared__ PeakRec s_red[kCombineThreads / kWave];
    const int64_t blk = linear_block();
    const int64_t i = blk * kCombineThreads + threadIdx.x;
    const ObjMeta m = P.meta[0];
    PeakRec best{0.0, -1};
    if (i < P.n_f) {
        if (m.status != LSP_OBJ_OK) {
            if (P.pgram) store_pgram(P.pgram, P.pgram_f64, i, fill_value(m.status));
        } else {
            const int64_t nf = P.n_f;
            bool ill;
            double p;
            if (!P.gen) {
                float xc = 0.0f, xs = 0.0f, cc = 0.0f, cs = 0.0f;
                for (int s = 0; s < P.n_split; ++s) {
                    const float* b = P.part + (int64_t)s * 4 * nf;
                    xc += b[i];
                    xs += b[nf + i];
                    cc += b[2 * nf + i];
                    cs += b[3 * nf + i];
                }
                p = (double)power32(xc, xs, cc, cs, (float)m.n, (float)m.scale, ill);
            } else {
                float v[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                for (int s = 0; s < P.n_split; ++s) {
                    const float* b = P.part + (int64_t)s * 6 * nf;
#pragma unroll
                    for (int q = 0; q < 6; ++q) v[q] += b[q * nf + i];
                }
                p = (double)power32_gen(v[0], v[1], v[2], v[3], v[4], v[5], (float)m.n,
                                        (float)m.scale, ill);
            }
            if (ill) {
                const double f = grid_freq(P.f_min, P.df, i) * P.to_cyc;
                p = (double)(float)(P.gen ? power64_gen_bin(m, P.t, P.y, P.dy, f)
                                          : power64_bin(m, P.t, P.y, f));
            }
            if (P.pgram) store_pgram(P.pgram, P.pgram_f64, i, p);
            best = PeakRec{p, i};
            if (!(p == p)) best = PeakRec{0.0, -1};
        }
    }
    best = wave_best(best);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) s_red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        PeakRec b = s_red[0];
        for (int w = 1; w < kCombineThreads / kWave; ++w)
            if (better(s_red[w].p, s_red[w].i, b.p, b.i)) b = s_red[w];
        P.rec[blk] = b;
    }
}

template <int K, int W, bool CHEB, bool WS, int SRC, int TRIG>
int occupancy_blocks() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, fp32p_kernel<K, W, CHEB, WS, SRC, TRIG>, kWave * W, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    return per_cu * cus;
}

template <int K, int W, bool CHEB, bool WS, int SRC = LSP_OBS_LDS, int TRIG = LSP_TRIG_HW>
hipError_t launch_kwc(const MainParams& p, hipStream_t s) {
    const dim3 grid = p.persistent
                          ? dim3((unsigned)occupancy_blocks<K, W, CHEB, WS, SRC, TRIG>())
                          : grid_for(p.n_items);
    hipLaunchKernelGGL((fp32p_kernel<K, W, CHEB, WS, SRC, TRIG>), grid, dim3(kWave * W), 0, s, p);
    return hipGetLastError();
}

// The read-path and seed-trig variants: three-term recurrence, no wave split,
// K in {8, 16}, 1 or 4 waves per workgroup.
template <int SRC, int TRIG>
hipError_t launch_variant(const MainParams& p, int k, int waves, hipStream_t s) {
    if (k == 8 && waves == 1) return launch_kwc<8, 1, true, false, SRC, TRIG>(p, s);
    if (k == 8 && waves == 4) return launch_kwc<8, 4, true, false, SRC, TRIG>(p, s);
    if (k == 16 && waves == 1) return launch_kwc<16, 1, true, false, SRC, TRIG>(p, s);
    if (k == 16 && waves == 4) return launch_kwc<16, 4, true, false, SRC, TRIG>(p, s);
    return hipErrorInvalidValue;
}

template <int K, bool CHEB>
hipError_t launch_kc(const MainParams& p, int waves, hipStream_t s) {
    const bool ws = p.wave_split != 0;
    switch (waves) {
        case 1: return launch_kwc<K, 1, CHEB, false>(p, s);
        case 2: return ws ? launch_kwc<K, 2, CHEB, true>(p, s) : launch_kwc<K, 2, CHEB, false>(p, s);
        case 4: return ws ? launch_kwc<K, 4, CHEB, true>(p, s) : launch_kwc<K, 4, CHEB, false>(p, s);
        case 8: return ws ? launch_kwc<K, 8, CHEB, true>(p, s) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <bool CHEB>
hipError_t launch_c(const MainParams& p, int k, int waves, hipStream_t s) {
    switch (k) {
        case 4: return launch_kc<4, CHEB>(p, waves, s);
        case 8: return launch_kc<8, CHEB>(p, waves, s);
        case 10: return launch_kc<10, CHEB>(p, waves, s);
        case 12: return launch_kc<12, CHEB>(p, waves, s);
        case 16: return launch_kc<16, CHEB>(p, waves, s);
        case 32: return launch_kc<32, CHEB>(p, waves, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fp32p(const MainParams& p, int k, int waves, int rec, hipStream_t s,
                        int obs_read, int trig) {
    if (p.n_items <= 0) return hipSuccess;
    if (obs_read == LSP_OBS_LDS && trig == LSP_TRIG_HW)
        return rec == LSP_REC_CHEBYSHEV ? launch_c<true>(p, k, waves, s)
                                        : launch_c<false>(p, k, waves, s);
    if (rec != LSP_REC_CHEBYSHEV || p.wave_split) return hipErrorInvalidValue;
    if (obs_read == LSP_OBS_LDS) {
        if (trig == LSP_TRIG_LIB) return launch_variant<LSP_OBS_LDS, LSP_TRIG_LIB>(p, k, waves, s);
        if (trig == LSP_TRIG_POLY) return launch_variant<LSP_OBS_LDS, LSP_TRIG_POLY>(p, k, waves, s);
    } else if (obs_read == LSP_OBS_DIRECT) {
        if (trig == LSP_TRIG_HW) return launch_variant<LSP_OBS_DIRECT, LSP_TRIG_HW>(p, k, waves, s);
        if (trig == LSP_TRIG_LIB) return launch_variant<LSP_OBS_DIRECT, LSP_TRIG_LIB>(p, k, waves, s);
        if (trig == LSP_TRIG_POLY)
            return launch_variant<LSP_OBS_DIRECT, LSP_TRIG_POLY>(p, k, waves, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_combine(const CombineParams& p, hipStream_t s) {
    if (p.n_f <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, grid_for((p.n_f + kCombineThreads - 1) / kCombineThreads),
                       dim3(kCombineThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace lsp
