// lsp_mlp.hip -- kernels of the learned band proposal: a BF16 matrix-core GEMM
// with FP32 accumulation (forward X.W, backward-data dY.W^T and
// backward-weight X^T.dY all use it through strides), and the small element
// kernels around it (softmax cross-entropy, column sums, Adam, feature
// standardisation, top-k bands, FP32 -> BF16).
//
// GEMM tiling: a 256-thread workgroup (4 wavefronts) owns a 64 x 64 tile of C
// and walks K in steps of 32.  Each step stages a 64 x 32 slice of A and a
// 32 x 64 slice of B into LDS with K contiguous (whatever the source strides),
// then each wavefront issues 2 x 2 v_mfma_f32_16x16x32_bf16 for its 32 x 32
// quarter.  A lane supplies row (lane % 16) of A and column (lane % 16) of B
// with eight consecutive k; both operands use the same k assignment, so the
// product does not depend on how the instruction orders k internally.  The
// 16 x 16 result is held as rows 4 (lane / 16) + r, column lane % 16.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "lsp_common.h"

namespace lsp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;
constexpr int kLdsK = kBK + 8;  // padded row: 80 bytes, keeps 16-byte fragment reads aligned
constexpr int kGemmThreads = 256;  // the 64 x 64 tile's four waves

__host__ __device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

struct GemmArgs {
    int64_t M, N, K;
    const uint16_t* A;
    int64_t sam, sak;
    const uint16_t* B;
    int64_t sbk, sbn;
    const float* bias;     // [N] or NULL
    const uint16_t* mask;  // BF16 [M x N], leading dimension ldc: keep C where mask > 0
    int32_t relu;
    int32_t pad;
    float* Cf;             // FP32 output or NULL
    uint16_t* Cb;          // BF16 output or NULL
    int64_t ldc;
    int32_t a_mode, b_mode;  // how each operand is staged: kLoad*
};

// How an operand tile is read from global memory: 8 consecutive k in one
// 16-byte load, 8 consecutive rows (m of A, n of B) in one 16-byte load that
// is transposed on its way into LDS, or element by element.
enum { kLoadK = 0, kLoadRows = 1, kLoadScalar = 2 };

// Stage rows [o0, o0 + BO) x k [k0, k0 + kBK) of an operand whose element
// (o, k) is X[o * so + k * sk] into Xs[o][k] (k contiguous, padded rows);
// outside the matrix the tile holds zeros.
template <int BO, int NT>
__device__ __forceinline__ void stage_operand(uint16_t* Xs, const uint16_t* X, int64_t so,
                                              int64_t sk, int64_t O, int64_t K, int64_t o0,
                                              int64_t k0, int mode, int tid) {
    constexpr int kChunks = BO * (kBK / 8);  // 8 elements each
#pragma unroll
    for (int c0 = 0; c0 < kChunks; c0 += NT) {
        const int c = c0 + tid;
        if (mode == kLoadRows) {
            // 8 consecutive rows at one k
            const int kk = c / (BO / 8), oc = (c % (BO / 8)) * 8;
            const int64_t o = o0 + oc, k = k0 + kk;
            uint16_t v[8];
            if (o + 8 <= O && k < K) {
                const uint4 q = *reinterpret_cast<const uint4*>(X + o + k * sk);
                memcpy(v, &q, sizeof q);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = (o + e < O && k < K) ? X[(o + e) + k * sk] : 0;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) Xs[(oc + e) * kLdsK + kk] = v[e];
        } else {
            // 8 consecutive k of one row
            const int oo = c / (kBK / 8), kc = (c % (kBK / 8)) * 8;
            const int64_t o = o0 + oo, k = k0 + kc;
            uint4 q;
            if (mode == kLoadK && o < O && k + 8 <= K) {
                q = *reinterpret_cast<const uint4*>(X + o * so + k);
            } else {
                uint16_t v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = (o < O && k + e < K) ? X[o * so + (k + e) * sk] : 0;
                memcpy(&q, v, sizeof q);
            }
            *reinterpret_cast<uint4*>(&Xs[oo * kLdsK + kc]) = q;
        }
    }
}

// C (BM x BN tile per workgroup) = A B on the matrix cores: WM x WN waves,
// each accumulating (BM / WM) x (BN / WN) from 16 x 16 x 32 BF16 products
// into FP32.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void gemm_bf16_kernel(const GemmArgs g) {
    constexpr int NT = 64 * WM * WN;
    constexpr int TI = BM / WM / 16, TJ = BN / WN / 16;  // 16 x 16 fragments per wave
    __shared__ __attribute__((aligned(16))) uint16_t As[BM * kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * kLdsK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
    const int wm = (wave / WN) * (BM / WM), wn = (wave % WN) * (BN / WN);

    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int64_t k0 = 0; k0 < g.K; k0 += kBK) {
        stage_operand<BM, NT>(As, g.A, g.sam, g.sak, g.M, g.K, m0, k0, g.a_mode, tid);
        stage_operand<BN, NT>(Bs, g.B, g.sbn, g.sbk, g.N, g.K, n0, k0, g.b_mode, tid);
        __syncthreads();
        bf16x8 a[TI], b[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + 16 * i + fr) * kLdsK + fk]);
#pragma unroll
        for (int j = 0; j < TJ; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + 16 * j + fr) * kLdsK + fk]);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int64_t n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (g.bias) v += g.bias[n];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.mask && !(bf16_bits_to_f32(g.mask[m * g.ldc + n]) > 0.f)) v = 0.f;
                if (g.Cf) g.Cf[m * g.ldc + n] = v;
                if (g.Cb) g.Cb[m * g.ldc + n] = f32_to_bf16_bits(v);
            }
}

// One wavefront per row: softmax of the row's logits, cross-entropy against
// the label, and the gradient (softmax - onehot) * scale.
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float* __restrict__ logits,
                                                           const int32_t* __restrict__ labels,
                                                           int64_t n, int32_t c, float scale,
                                                           float* dlogits, uint16_t* dlogits_bf16,
                                                           float* loss_rows) {
    const int64_t row = linear_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float* z = logits + row * c;
    float mx = -INFINITY;
    for (int j = lane; j < c; j += 64) mx = fmaxf(mx, z[j]);
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    float se = 0.f;
    for (int j = lane; j < c; j += 64) se += expf(z[j] - mx);
    for (int off = 32; off >= 1; off >>= 1) se += __shfl_xor(se, off, 64);
    const int32_t lab = labels[row];
    const bool keep = lab >= 0 && lab < c;  // other labels mark rows to ignore
    for (int j = lane; j < c; j += 64) {
        const float p = expf(z[j] - mx) / se;
        const float d = keep ? (p - (j == lab ? 1.f : 0.f)) * scale : 0.f;
        if (dlogits) dlogits[row * c + j] = d;
        if (dlogits_bf16) dlogits_bf16[row * c + j] = f32_to_bf16_bits(d);
    }
    if (lane == 0 && loss_rows)
        loss_rows[row] = keep ? (logf(se) + mx - z[lab]) : 0.f;
}

// Training labels from full-grid peaks: the band holding each peak, or -1 for
// an object without a peak.
__global__ void peak_bands_kernel(const lsp_peak* __restrict__ peaks, int64_t n,
                                  int64_t band_bins, int32_t n_bands, int32_t* labels) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const lsp_peak pk = peaks[i];
    int32_t b = -1;
    if (pk.status == LSP_OBJ_OK && pk.index >= 0) {
        const int64_t q = pk.index / band_bins;
        b = q < n_bands ? (int32_t)q : -1;
    }
    labels[i] = b;
}

// Objects whose refined peak must be confirmed on the whole grid, listed in
// increasing order: status OK and (proposal mass below mass_min, or refined
// power below power_min or not a number, or no peak found).  One workgroup
// walks the objects 1,024 at a time; each wave compacts its flags with a
// ballot and the waves' counts are prefix-summed in LDS.
constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void select_kernel(const lsp_peak* __restrict__ peaks,
                                                           const float* __restrict__ mass,
                                                           int64_t n, float mass_min,
                                                           float power_min, int32_t* out,
                                                           int32_t* count) {
    __shared__ int32_t s_cnt[kSelThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t done = 0;
    for (int64_t base = 0; base < n; base += kSelThreads) {
        const int64_t i = base + threadIdx.x;
        bool need = false;
        if (i < n) {
            const lsp_peak pk = peaks[i];
            if (pk.status == LSP_OBJ_OK)
                need = !(pk.index >= 0) || !(pk.power >= (double)power_min) ||
                       (mass && !(mass[i] >= mass_min));
        }
        const uint64_t m = __ballot(need);
        if (lane == 0) s_cnt[wave] = __popcll(m);
        __syncthreads();
        int64_t off = done;
        int32_t total = 0;
        for (int w = 0; w < kSelThreads / 64; ++w) {
            if (w < wave) off += s_cnt[w];
            total += s_cnt[w];
        }
        if (need) {
            const uint64_t below = lane ? (m & ((~0ull) >> (64 - lane))) : 0ull;
            out[off + __popcll(below)] = (int32_t)i;
        }
        done += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = (int32_t)done;
}

// Column sums of an n x c FP32 matrix.  A workgroup covers 64 columns with 16
// row phases (row i goes to phase i mod 16); each thread sums its phase in row
// order and the 16 phase sums are added in phase order, so the result does not
// depend on scheduling.
constexpr int kSumCols = 64, kSumPhases = 16;

__global__ __launch_bounds__(kSumCols* kSumPhases) void col_sums_kernel(
    const float* __restrict__ x, int64_t n, int32_t c, float* out) {
    __shared__ float s_part[kSumPhases][kSumCols];
    const int tx = threadIdx.x % kSumCols, ph = threadIdx.x / kSumCols;
    const int32_t j = blockIdx.x * kSumCols + tx;
    float s = 0.f;
    if (j < c)
        for (int64_t i = ph; i < n; i += kSumPhases) s += x[i * c + j];
    s_part[ph][tx] = s;
    __syncthreads();
    if (ph == 0 && j < c) {
        float t = s_part[0][tx];
        for (int q = 1; q < kSumPhases; ++q) t += s_part[q][tx];
        out[j] = t;
    }
}

// Column mean and 1/std (population) of an n x d FP32 matrix; a column with no
// spread gets 1/std = 1.  One thread per column, fixed order, FP64 sums.
__global__ void col_stats_kernel(const float* __restrict__ x, int64_t n, int32_t d, float* mean,
                                 float* inv_std) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (double)x[i * d + j];
    const double mu = n > 0 ? s / (double)n : 0.0;
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double e = (double)x[i * d + j] - mu;
        q += e * e;
    }
    const double sd = n > 0 ? sqrt(q / (double)n) : 0.0;
    mean[j] = (float)mu;
    inv_std[j] = sd > 1e-12 ? (float)(1.0 / sd) : 0.0f;  // a constant column carries nothing
}

// Replace the statistics of columns [start, start + count) by those of the
// pooled block (every entry of those columns taken together):
// mean = mean_j m_j, var = mean_j (var_j + m_j^2) - mean^2.  One workgroup,
// fixed-order sums.
__global__ __launch_bounds__(256) void pool_stats_kernel(float* mean, float* inv_std,
                                                         int32_t start, int32_t count) {
    __shared__ double s_m[256], s_q[256];
    double m = 0.0, q = 0.0;
    for (int32_t j = threadIdx.x; j < count; j += 256) {
        const double mj = mean[start + j];
        const double is = inv_std[start + j];
        m += mj;
        q += (is > 0.0 ? 1.0 / (is * is) : 0.0) + mj * mj;
    }
    s_m[threadIdx.x] = m;
    s_q[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_m[threadIdx.x] += s_m[threadIdx.x + w];
            s_q[threadIdx.x] += s_q[threadIdx.x + w];
        }
        __syncthreads();
    }
    const double mu = s_m[0] / (double)count;
    const double var = s_q[0] / (double)count - mu * mu;
    const float is = var > 1e-24 ? (float)(1.0 / sqrt(var)) : 0.0f;
    for (int32_t j = threadIdx.x; j < count; j += 256) {
        mean[start + j] = (float)mu;
        inv_std[start + j] = is;
    }
}

// Row standardisation of a column block: in each row of x [n x d], the
// columns [start, start + count) become (x - row mean) / row std over those
// columns (0 where the row is constant).  One wavefront per row, FP64 sums,
// fixed order.  Makes the coarse spectrum's shape, not its overall level,
// what the network sees: a short series has a much higher noise floor than a
// long one, while the band that holds the peak is a property of the shape.
__global__ __launch_bounds__(256) void row_norm_kernel(float* x, int64_t n, int32_t d,
                                                       int32_t start, int32_t count) {
    const int64_t row = linear_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    float* r = x + row * d + start;
    double s = 0.0, q = 0.0;
    for (int32_t j = lane; j < count; j += 64) {
        const double v = r[j];
        s += v;
        q += v * v;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    const double mu = s / (double)count;
    const double var = q / (double)count - mu * mu;
    const double inv = var > 1e-24 ? 1.0 / sqrt(var) : 0.0;
    for (int32_t j = lane; j < count; j += 64) r[j] = (float)(((double)r[j] - mu) * inv);
}

// Largest value of each band's columns: row i's columns [start + b*group,
// start + (b+1)*group) for b < n_bands.  One thread per (row, band).
__global__ void band_max_kernel(const float* __restrict__ x, int64_t n, int32_t d, int32_t start,
                                int32_t n_bands, int32_t group, float* __restrict__ out) {
    const int64_t e = linear_block() * blockDim.x + threadIdx.x;
    if (e >= n * n_bands) return;
    const int64_t i = e / n_bands;
    const int32_t b = (int32_t)(e - i * n_bands);
    const float* r = x + i * d + start + (int64_t)b * group;
    float m = r[0];
    for (int32_t j = 1; j < group; ++j) m = fmaxf(m, r[j]);
    out[e] = m;
}

// Per row: the entries of a (in order), then those of b not already taken,
// until k_out distinct non-negative bands; -1 fills what is left.
__global__ void merge_bands_kernel(const int32_t* __restrict__ a, int32_t ka,
                                   const int32_t* __restrict__ b, int32_t kb, int64_t n,
                                   int32_t k_out, int32_t* __restrict__ out) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t* o = out + i * k_out;
    int32_t m = 0;
    for (int32_t src = 0; src < 2; ++src) {
        const int32_t* v = src == 0 ? a + i * ka : b + i * kb;
        const int32_t kv = src == 0 ? ka : kb;
        for (int32_t j = 0; j < kv && m < k_out; ++j) {
            const int32_t band = v[j];
            if (band < 0) continue;
            bool seen = false;
            for (int32_t q = 0; q < m; ++q) seen |= o[q] == band;
            if (!seen) o[m++] = band;
        }
    }
    for (; m < k_out; ++m) o[m] = -1;
}

// Training-time shift augmentation.  Row i's first n_coarse columns hold
// n_bands groups of `group` columns, one group per frequency band; they move
// by shift[i] groups (vacated columns get `fill`), the other columns are
// copied, and the label moves with them (-1 if it leaves [0, n_bands) or was
// already -1).  A signal whose frequency moves by one band width moves its
// coarse spectrum by one group, so this multiplies the labelled examples.
__global__ void shift_bands_kernel(const uint16_t* __restrict__ x,
                                   const int32_t* __restrict__ labels,
                                   const int32_t* __restrict__ shifts, int64_t n, int32_t d,
                                   int32_t n_coarse, int32_t group, int32_t n_bands,
                                   uint16_t fill, uint16_t* __restrict__ out,
                                   int32_t* __restrict__ out_labels) {
    const int64_t e = linear_block() * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t i = e / d;
    const int32_t j = (int32_t)(e - i * d);
    const int32_t sh = shifts[i];
    uint16_t v;
    if (j < n_coarse) {
        const int64_t src = (int64_t)j - (int64_t)sh * group;
        v = (src >= 0 && src < n_coarse) ? x[i * d + src] : fill;
    } else {
        v = x[e];
    }
    out[e] = v;
    if (j == 0) {
        const int32_t lab = labels[i];
        const int32_t nl = lab + sh;
        out_labels[i] = (lab >= 0 && nl >= 0 && nl < n_bands) ? nl : -1;
    }
}

__global__ void standardize_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                   const float* __restrict__ mean,
                                   const float* __restrict__ inv_std, uint16_t* out) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i >= n * d) return;
    const int32_t j = (int32_t)(i % d);
    out[i] = f32_to_bf16_bits((x[i] - mean[j]) * inv_std[j]);
}

__global__ void cast_bf16_kernel(const float* __restrict__ x, int64_t count, uint16_t* out) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i < count) out[i] = f32_to_bf16_bits(x[i]);
}

// Adam with bias correction on FP32 master parameters; optionally refreshes
// the BF16 copy the GEMMs read.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ grad,
                            float* __restrict__ m, float* __restrict__ v, int64_t count,
                            float lr, float b1, float b2, float eps, float c1, float c2,
                            uint16_t* p_bf16) {
    const int64_t i = linear_block() * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (p_bf16) p_bf16[i] = f32_to_bf16_bits(pi);
}

// One wavefront per row: the k largest of c logits (lowest index on ties), in
// decreasing order, and the softmax probability mass they carry.
__global__ __launch_bounds__(256) void top_k_kernel(const float* __restrict__ logits, int64_t n,
                                                    int32_t c, int32_t k, int32_t* idx,
                                                    float* mass) {
    const int64_t row = linear_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float* z = logits + row * c;
    // each lane holds up to two logits (c <= 128)
    float v0 = lane < c ? z[lane] : -INFINITY;
    float v1 = lane + 64 < c ? z[lane + 64] : -INFINITY;
    float mx = fmaxf(v0, v1);
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    float se = (lane < c ? expf(v0 - mx) : 0.f) + (lane + 64 < c ? expf(v1 - mx) : 0.f);
    for (int off = 32; off >= 1; off >>= 1) se += __shfl_xor(se, off, 64);
    float taken = 0.f;
    for (int r = 0; r < k; ++r) {
        float bv = v0;
        int bi = lane < c ? lane : 1 << 30;
        if (v1 > bv || (v1 == bv && lane + 64 < c && lane + 64 < bi)) {
            bv = v1;
            bi = lane + 64 < c ? lane + 64 : 1 << 30;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const float ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) idx[row * k + r] = bi < c ? bi : -1;
        if (bi < c) taken += expf(bv - mx);
        if (bi == lane) v0 = -INFINITY;
        if (bi == lane + 64) v1 = -INFINITY;
    }
    if (lane == 0 && mass) mass[row] = taken / se;
}

// Adaptive band count, one wavefront per row.  Row i's `top` proposed bands
// idx[i][r] -- slots r < n_net from the network in decreasing probability,
// the rest in decreasing coarse power -- are copied to out[i][r] or replaced
// by -1:
//   a network slot is kept while the softmax mass of the kept network slots
//   before it is below tau (the first is always kept);
//   a coarse slot is kept if its band's score is at least alpha times the
//   row's largest band score (the first slot of a row without network slots
//   is always kept).
// kept_mass[i] (if not NULL) receives the softmax mass of the kept network
// slots, each probability exp(z_b - max z) / sum_j exp(z_j - max z) in FP32.
__global__ __launch_bounds__(256) void trim_bands_kernel(
    const int32_t* __restrict__ idx, int64_t n, int32_t top, int32_t n_net,
    const float* __restrict__ logits, const float* __restrict__ score, int32_t c, float tau,
    float alpha, int32_t* __restrict__ out, float* __restrict__ kept_mass) {
    const int64_t row = linear_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    // softmax normaliser of the logits and the largest band score (c <= 128)
    float mx = -INFINITY, se = 0.f, smax = -INFINITY;
    if (logits) {
        const float* z = logits + row * c;
        const float v0 = lane < c ? z[lane] : -INFINITY;
        const float v1 = lane + 64 < c ? z[lane + 64] : -INFINITY;
        mx = fmaxf(v0, v1);
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        se = (lane < c ? expf(v0 - mx) : 0.f) + (lane + 64 < c ? expf(v1 - mx) : 0.f);
        for (int off = 32; off >= 1; off >>= 1) se += __shfl_xor(se, off, 64);
    }
    if (score) {
        const float* q = score + row * c;
        smax = fmaxf(lane < c ? q[lane] : -INFINITY, lane + 64 < c ? q[lane + 64] : -INFINITY);
        for (int off = 32; off >= 1; off >>= 1) smax = fmaxf(smax, __shfl_xor(smax, off, 64));
    }
    if (lane != 0) return;
    const int32_t* in = idx + row * top;
    int32_t* o = out + row * top;
    float cum = 0.f;
    bool any_net = false;
    for (int32_t r = 0; r < top; ++r) {
        const int32_t b = in[r];
        bool keep = false;
        if (b >= 0 && b < c) {
            if (r < n_net) {
                keep = !any_net || cum < tau;
                if (keep) {
                    any_net = true;
                    if (logits) cum += expf(logits[row * c + b] - mx) / se;
                }
            } else {
                keep = (n_net == 0 && r == 0) || !score || score[row * c + b] >= alpha * smax;
            }
        }
        o[r] = keep ? b : -1;
    }
    if (kept_mass) kept_mass[row] = cum;
}

}  // namespace
}  // namespace lsp

extern "C" {

lsp_status lsp_gemm_bf16(int64_t M, int64_t N, int64_t K, const void* A, int64_t sam, int64_t sak,
                         const void* B, int64_t sbk, int64_t sbn, const float* bias,
                         const void* mask, int32_t relu, float* C, void* C_bf16, int64_t ldc,
                         void* stream) {
    if (M < 0 || N < 0 || K < 0 || (M > 0 && N > 0 && (!A || !B)) || (!C && !C_bf16) ||
        ldc < N || (relu != 0 && relu != 1))
        return LSP_EINVAL;
    if ((M + 63) / 64 > 65535 || (N + 63) / 64 > 65535) return LSP_EUNSUPPORTED;
    if (M == 0 || N == 0) return LSP_OK;
    lsp::GemmArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = static_cast<const uint16_t*>(A);
    g.sam = sam;
    g.sak = sak;
    g.B = static_cast<const uint16_t*>(B);
    g.sbk = sbk;
    g.sbn = sbn;
    g.bias = bias;
    g.mask = static_cast<const uint16_t*>(mask);
    g.relu = relu;
    g.pad = 0;
    g.Cf = C;
    g.Cb = static_cast<uint16_t*>(C_bf16);
    g.ldc = ldc;
    // 16-byte loads where an operand's k (or its rows) are contiguous and
    // every 8-element chunk the tiles read starts on a 16-byte boundary
    auto mode = [](const void* X, int64_t so, int64_t sk) {
        const bool aligned = (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
        if (aligned && sk == 1 && so % 8 == 0) return (int32_t)lsp::kLoadK;
        if (aligned && so == 1 && sk % 8 == 0) return (int32_t)lsp::kLoadRows;
        return (int32_t)lsp::kLoadScalar;
    };
    g.a_mode = mode(A, sam, sak);
    g.b_mode = mode(B, sbn, sbk);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // 128 x 128 tiles (eight waves of 64 x 32) where they still give a few
    // hundred workgroups, else 64 x 64 (four waves of 32 x 32)
    if (M >= 128 && N >= 128 && ((M + 127) / 128) * ((N + 127) / 128) >= 256) {
        const dim3 grid((unsigned)((N + 127) / 128), (unsigned)((M + 127) / 128));
        hipLaunchKernelGGL((lsp::gemm_bf16_kernel<128, 128, 2, 4>), grid, dim3(512), 0, s, g);
    } else {
        const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
        hipLaunchKernelGGL((lsp::gemm_bf16_kernel<64, 64, 2, 2>), grid, dim3(lsp::kGemmThreads), 0,
                           s, g);
    }
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_softmax_xent(const float* logits, const int32_t* labels, int64_t n, int32_t c,
                            float scale, float* dlogits, void* dlogits_bf16, float* loss_rows,
                            void* stream) {
    if (n < 0 || c < 1 || (n > 0 && (!logits || !labels))) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::softmax_xent_kernel, lsp::grid_for((n + 3) / 4), dim3(256), 0,
                       static_cast<hipStream_t>(stream), logits, labels, n, c, scale, dlogits,
                       static_cast<uint16_t*>(dlogits_bf16), loss_rows);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_col_sums(const float* x, int64_t n, int32_t c, float* out, void* stream) {
    if (n < 0 || c < 1 || !out || (n > 0 && !x)) return LSP_EINVAL;
    hipLaunchKernelGGL(lsp::col_sums_kernel, dim3((c + lsp::kSumCols - 1) / lsp::kSumCols),
                       dim3(lsp::kSumCols * lsp::kSumPhases), 0, static_cast<hipStream_t>(stream),
                       x, n, c, out);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_col_stats(const float* x, int64_t n, int32_t d, float* mean, float* inv_std,
                         void* stream) {
    if (n < 0 || d < 1 || !mean || !inv_std || (n > 0 && !x)) return LSP_EINVAL;
    hipLaunchKernelGGL(lsp::col_stats_kernel, dim3((d + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, n, d, mean, inv_std);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_standardize_bf16(const float* x, int64_t n, int32_t d, const float* mean,
                                const float* inv_std, void* out, void* stream) {
    if (n < 0 || d < 1 || !mean || !inv_std || (n > 0 && (!x || !out))) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::standardize_kernel, lsp::grid_for((n * d + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, n, d, mean, inv_std,
                       static_cast<uint16_t*>(out));
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_cast_bf16(const float* x, int64_t count, void* out, void* stream) {
    if (count < 0 || (count > 0 && (!x || !out))) return LSP_EINVAL;
    if (count == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::cast_bf16_kernel, lsp::grid_for((count + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, count, static_cast<uint16_t*>(out));
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_adam(float* param, const float* grad, float* m, float* v, int64_t count,
                    int32_t step, float lr, float beta1, float beta2, float eps, void* param_bf16,
                    void* stream) {
    if (count < 0 || step < 1 || (count > 0 && (!param || !grad || !m || !v))) return LSP_EINVAL;
    if (count == 0) return LSP_OK;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(lsp::adam_kernel, lsp::grid_for((count + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), param, grad, m, v, count, lr, beta1,
                       beta2, eps, c1, c2, static_cast<uint16_t*>(param_bf16));
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

// ---- the network as a whole: the layer order of lsp_mlp, from the primitives

static bool mlp_ok(const lsp_mlp* net) {
    if (!net) return false;
    for (int l = 0; l < 4; ++l)
        if (net->dims[l] < 1) return false;
    for (int l = 0; l < 3; ++l)
        if (!net->w[l] || !net->b[l] || !net->w_bf16[l]) return false;
    return true;
}

static bool grads_ok(const lsp_mlp_grads* g) {
    if (!g) return false;
    for (int l = 0; l < 3; ++l)
        if (!g->w[l] || !g->b[l]) return false;
    return true;
}

// Backward scratch: dlogits, dz2, dz1 in FP32 and in BF16, 256-byte aligned.
struct MlpScratch {
    size_t off[6];
    size_t total;
};

static MlpScratch mlp_scratch(const lsp_mlp* net, int64_t n) {
    const int64_t rows[3] = {net->dims[3], net->dims[2], net->dims[1]};
    MlpScratch s{};
    size_t at = 0;
    for (int q = 0; q < 3; ++q) {
        s.off[2 * q] = at;
        at += ((size_t)n * rows[q] * 4 + 255) / 256 * 256;
        s.off[2 * q + 1] = at;
        at += ((size_t)n * rows[q] * 2 + 255) / 256 * 256;
    }
    s.total = at;
    return s;
}

lsp_status lsp_mlp_forward(const lsp_mlp* net, const void* x_bf16, int64_t n, void* h1_bf16,
                           void* h2_bf16, float* logits, void* stream) {
    if (!mlp_ok(net) || n < 0 || (n > 0 && (!x_bf16 || !h1_bf16 || !h2_bf16 || !logits)))
        return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    const int64_t d0 = net->dims[0], d1 = net->dims[1], d2 = net->dims[2], d3 = net->dims[3];
    lsp_status st = lsp_gemm_bf16(n, d1, d0, x_bf16, d0, 1, net->w_bf16[0], d1, 1, net->b[0],
                                  nullptr, 1, nullptr, h1_bf16, d1, stream);
    if (st != LSP_OK) return st;
    st = lsp_gemm_bf16(n, d2, d1, h1_bf16, d1, 1, net->w_bf16[1], d2, 1, net->b[1], nullptr, 1,
                       nullptr, h2_bf16, d2, stream);
    if (st != LSP_OK) return st;
    return lsp_gemm_bf16(n, d3, d2, h2_bf16, d2, 1, net->w_bf16[2], d3, 1, net->b[2], nullptr, 0,
                         logits, nullptr, d3, stream);
}

size_t lsp_mlp_workspace_bytes(const lsp_mlp* net, int64_t n) {
    if (!net || n < 1) return 0;
    for (int l = 0; l < 4; ++l)
        if (net->dims[l] < 1) return 0;
    return mlp_scratch(net, n).total;
}

lsp_status lsp_mlp_backward(const lsp_mlp* net, const void* x_bf16, const int32_t* labels,
                            int64_t n, const void* h1_bf16, const void* h2_bf16,
                            const float* logits, float scale, const lsp_mlp_grads* grads,
                            float* loss_rows, void* workspace, size_t workspace_bytes,
                            void* stream) {
    if (!mlp_ok(net) || !grads_ok(grads) || n < 1 || !x_bf16 || !labels || !h1_bf16 ||
        !h2_bf16 || !logits || !workspace)
        return LSP_EINVAL;
    const MlpScratch sc = mlp_scratch(net, n);
    if (workspace_bytes < sc.total) return LSP_ENOMEM;
    const int64_t d0 = net->dims[0], d1 = net->dims[1], d2 = net->dims[2], d3 = net->dims[3];
    char* ws = static_cast<char*>(workspace);
    float* g3 = reinterpret_cast<float*>(ws + sc.off[0]);
    void* g3b = ws + sc.off[1];
    float* dz2 = reinterpret_cast<float*>(ws + sc.off[2]);
    void* dz2b = ws + sc.off[3];
    float* dz1 = reinterpret_cast<float*>(ws + sc.off[4]);
    void* dz1b = ws + sc.off[5];
    lsp_status st = lsp_softmax_xent(logits, labels, n, (int32_t)d3, scale, g3, g3b, loss_rows,
                                     stream);
    if (st != LSP_OK) return st;
    // layer 3: dW_2 = h2^T g3, db_2 = column sums of g3, dz2 = (g3 W_2^T) where h2 > 0
    if ((st = lsp_gemm_bf16(d2, d3, n, h2_bf16, 1, d2, g3b, d3, 1, nullptr, nullptr, 0,
                            grads->w[2], nullptr, d3, stream)) != LSP_OK)
        return st;
    if ((st = lsp_col_sums(g3, n, (int32_t)d3, grads->b[2], stream)) != LSP_OK) return st;
    if ((st = lsp_gemm_bf16(n, d2, d3, g3b, d3, 1, net->w_bf16[2], 1, d3, nullptr, h2_bf16, 0,
                            dz2, dz2b, d2, stream)) != LSP_OK)
        return st;
    // layer 2
    if ((st = lsp_gemm_bf16(d1, d2, n, h1_bf16, 1, d1, dz2b, d2, 1, nullptr, nullptr, 0,
                            grads->w[1], nullptr, d2, stream)) != LSP_OK)
        return st;
    if ((st = lsp_col_sums(dz2, n, (int32_t)d2, grads->b[1], stream)) != LSP_OK) return st;
    if ((st = lsp_gemm_bf16(n, d1, d2, dz2b, d2, 1, net->w_bf16[1], 1, d2, nullptr, h1_bf16, 0,
                            dz1, dz1b, d1, stream)) != LSP_OK)
        return st;
    // layer 1
    if ((st = lsp_gemm_bf16(d0, d1, n, x_bf16, 1, d0, dz1b, d1, 1, nullptr, nullptr, 0,
                            grads->w[0], nullptr, d1, stream)) != LSP_OK)
        return st;
    return lsp_col_sums(dz1, n, (int32_t)d1, grads->b[0], stream);
}

lsp_status lsp_mlp_adam(const lsp_mlp* net, const lsp_mlp_grads* grads, const lsp_mlp_grads* m,
                        const lsp_mlp_grads* v, int32_t step, float lr, float beta1, float beta2,
                        float eps, void* stream) {
    if (!mlp_ok(net) || !grads_ok(grads) || !grads_ok(m) || !grads_ok(v) || step < 1)
        return LSP_EINVAL;
    for (int l = 0; l < 3; ++l) {
        const int64_t nw = (int64_t)net->dims[l] * net->dims[l + 1];
        lsp_status st = lsp_adam(net->w[l], grads->w[l], m->w[l], v->w[l], nw, step, lr, beta1,
                                 beta2, eps, net->w_bf16[l], stream);
        if (st != LSP_OK) return st;
        st = lsp_adam(net->b[l], grads->b[l], m->b[l], v->b[l], net->dims[l + 1], step, lr,
                      beta1, beta2, eps, nullptr, stream);
        if (st != LSP_OK) return st;
    }
    return LSP_OK;
}

lsp_status lsp_top_k(const float* logits, int64_t n, int32_t c, int32_t k, int32_t* idx,
                     float* mass, void* stream) {
    if (n < 0 || c < 1 || c > 128 || k < 1 || k > c || (n > 0 && (!logits || !idx)))
        return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::top_k_kernel, lsp::grid_for((n + 3) / 4), dim3(256), 0,
                       static_cast<hipStream_t>(stream), logits, n, c, k, idx, mass);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_row_normalize(float* x, int64_t n, int32_t d, int32_t start, int32_t count,
                             void* stream) {
    if (n < 0 || d < 1 || start < 0 || count < 1 || (int64_t)start + count > d) return LSP_EINVAL;
    if (n > 0 && !x) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::row_norm_kernel, lsp::grid_for((n + 3) / 4), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, n, d, start, count);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_band_max(const float* x, int64_t n, int32_t d, int32_t start, int32_t n_bands,
                        int32_t group, float* out, void* stream) {
    if (n < 0 || d < 1 || start < 0 || n_bands < 1 || group < 1 ||
        (int64_t)start + (int64_t)n_bands * group > d)
        return LSP_EINVAL;
    if (n > 0 && (!x || !out)) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::band_max_kernel, lsp::grid_for((n * n_bands + 255) / 256), dim3(256),
                       0, static_cast<hipStream_t>(stream), x, n, d, start, n_bands, group, out);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_merge_bands(const int32_t* a, int32_t ka, const int32_t* b, int32_t kb, int64_t n,
                           int32_t k_out, int32_t* out, void* stream) {
    if (n < 0 || ka < 0 || kb < 0 || k_out < 1 || k_out > 128) return LSP_EINVAL;
    if (n > 0 && (!out || (ka > 0 && !a) || (kb > 0 && !b))) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::merge_bands_kernel, lsp::grid_for((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), a, ka, b, kb, n, k_out, out);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_trim_bands(const int32_t* idx, int64_t n, int32_t top, int32_t n_net,
                          const float* logits, const float* score, int32_t c, float tau,
                          float alpha, int32_t* out, float* kept_mass, void* stream) {
    if (n < 0 || top < 1 || top > 128 || n_net < 0 || n_net > top || c < 1 || c > 128)
        return LSP_EINVAL;
    if (!(tau == tau) || !(alpha == alpha)) return LSP_EINVAL;
    if (n > 0 && (!idx || !out || (n_net > 0 && !logits))) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::trim_bands_kernel, lsp::grid_for((n + 3) / 4), dim3(256), 0,
                       static_cast<hipStream_t>(stream), idx, n, top, n_net, logits, score, c, tau,
                       alpha, out, kept_mass);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_pool_stats(float* mean, float* inv_std, int32_t start, int32_t count,
                          void* stream) {
    if (!mean || !inv_std || start < 0 || count < 1) return LSP_EINVAL;
    hipLaunchKernelGGL(lsp::pool_stats_kernel, dim3(1), dim3(256), 0,
                       static_cast<hipStream_t>(stream), mean, inv_std, start, count);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_shift_bands(const void* x_bf16, const int32_t* labels, const int32_t* shifts,
                           int64_t n, int32_t d, int32_t n_coarse, int32_t group, int32_t n_bands,
                           float fill, void* out_bf16, int32_t* out_labels, void* stream) {
    if (n < 0 || d < 1 || n_coarse < 0 || n_coarse > d || group < 1 || n_bands < 1 ||
        (int64_t)group * n_bands != n_coarse)
        return LSP_EINVAL;
    if (n > 0 && (!x_bf16 || !labels || !shifts || !out_bf16 || !out_labels)) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::shift_bands_kernel, lsp::grid_for((n * d + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint16_t*>(x_bf16),
                       labels, shifts, n, d, n_coarse, group, n_bands, lsp::f32_to_bf16_bits(fill),
                       static_cast<uint16_t*>(out_bf16), out_labels);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_peak_bands(const lsp_peak* peaks, int64_t n, int64_t band_bins, int32_t n_bands,
                          int32_t* labels, void* stream) {
    if (n < 0 || band_bins < 1 || n_bands < 1 || (n > 0 && (!peaks || !labels))) return LSP_EINVAL;
    if (n == 0) return LSP_OK;
    hipLaunchKernelGGL(lsp::peak_bands_kernel, lsp::grid_for((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), peaks, n, band_bins, n_bands, labels);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

lsp_status lsp_select_fallback(const lsp_peak* peaks, const float* mass, int64_t n,
                               float mass_min, float power_min, int32_t* objects, int32_t* count,
                               void* stream) {
    if (n < 0 || n > INT32_MAX || !count || (n > 0 && (!peaks || !objects))) return LSP_EINVAL;
    hipLaunchKernelGGL(lsp::select_kernel, dim3(1), dim3(lsp::kSelThreads), 0,
                       static_cast<hipStream_t>(stream), peaks, mass, n, mass_min, power_min,
                       objects, count);
    return hipGetLastError() == hipSuccess ? LSP_OK : LSP_EHIP;
}

}  // extern "C"
