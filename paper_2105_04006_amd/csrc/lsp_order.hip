// lsp_order.hip -- longest-first order of a batch's rows.
//
// A batch's work items are (row, frequency chunk) pairs whose cost is
// proportional to the row's observation count N_t.  Handed out in input
// order, the last items a queue gives out can be long ones, and the chip
// idles while they finish.  Graham's longest-processing-time-first rule
// (largest jobs first, each to the least loaded machine) bounds that tail by
// the shortest jobs instead.  Here the rows are sorted by descending N_t with
// a counting sort on the device, and position s of the sorted order is dealt
// to XCD s % 8, so that each XCD's queue is balanced and runs longest first.
//
// Three small kernels: count rows per cost bucket, an exclusive scan of the
// buckets in descending cost order, and a scatter that places each row.
// Counts below 1,024 have a bucket each; above, 64 buckets per octave (cost
// within 1.6%).  Rows of one bucket land in no particular order (the scatter
// takes positions with atomics); no result depends on the order.
#include "lsp_common.h"

namespace lsp {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kPerThread = (kOrderBuckets + kScanThreads - 1) / kScanThreads;

__device__ __forceinline__ int cost_bucket(int64_t n) {
    if (n <= 0) return 0;
    if (n < 1024) return (int)n;
    const int e = 63 - __clzll((unsigned long long)n);  // 10..62
    return 1024 + (e - 10) * 64 + (int)((n >> (e - 6)) & 63);
}

// Slot of a row's bucket in the histogram: descending cost comes first.
__device__ __forceinline__ int row_slot(const OrderParams& P, int64_t r) {
    const int64_t o = P.row_obj ? (int64_t)P.row_obj[r] : r / P.rows_per_group;
    int b = 0;
    if (o >= 0 && o < P.n_obj && !(P.row_band && P.row_band[r] < 0))
        b = cost_bucket(P.offsets[o + 1] - P.offsets[o]);
    return kOrderBuckets - 1 - b;
}

__global__ __launch_bounds__(256) void order_count_kernel(const OrderParams P) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < P.n_rows; r += stride)
        atomicAdd(&P.hist[row_slot(P, r)], 1u);
}

// Exclusive prefix sum of the bucket counts, in place (one workgroup).
__global__ __launch_bounds__(kScanThreads) void order_scan_kernel(const OrderParams P) {
    __shared__ unsigned int s_sum[kScanThreads];
    const int b0 = threadIdx.x * kPerThread;
    unsigned int v[kPerThread];
    unsigned int own = 0u;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        v[q] = b0 + q < kOrderBuckets ? P.hist[b0 + q] : 0u;
        own += v[q];
    }
    s_sum[threadIdx.x] = own;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const unsigned int add = threadIdx.x >= d ? s_sum[threadIdx.x - d] : 0u;
        __syncthreads();
        s_sum[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned int run = s_sum[threadIdx.x] - own;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        if (b0 + q < kOrderBuckets) P.hist[b0 + q] = run;
        run += v[q];
    }
}

// Row r takes the next position s of its bucket; s is dealt to XCD s % 8,
// whose rows occupy ranks [xcd_first_rank(x), xcd_first_rank(x + 1)).
__global__ __launch_bounds__(256) void order_place_kernel(const OrderParams P) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < P.n_rows; r += stride) {
        const int64_t s = (int64_t)atomicAdd(&P.hist[row_slot(P, r)], 1u);
        const int x = (int)(s % kXcds);
        P.perm[xcd_first_rank(x, P.n_rows) + s / kXcds] = (int32_t)r;
    }
}

}  // namespace

hipError_t launch_row_order(const OrderParams& p, hipStream_t s) {
    if (p.n_rows <= 0) return hipSuccess;
    hipError_t e = launch_fill_u32(p.hist, kOrderBuckets, 0u, s);
    if (e != hipSuccess) return e;
    int64_t blocks = (p.n_rows + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(order_count_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, p);
    hipLaunchKernelGGL(order_place_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace lsp
