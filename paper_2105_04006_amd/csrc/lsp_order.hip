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
// Counts below 1,024 have a bucket each; above, 64 buckets per octave (cost
// within 1.6%).  Rows with no work at all -- a negative band or an object
// index outside the batch -- get a bucket of their own after every other, so
// that they end each XCD's run and the first position of that bucket (n_work)
// tells the main kernels where their queues can stop.  (A row of an empty or
// degenerate object is not such a row: it still writes its fill values.)  The sort is two-level, so that no global counter is shared
// by many rows (the rows of a batch crowd into a few hundred buckets):
//   count : each of kOrderBlocks workgroups histograms its contiguous share
//           of the rows in LDS and writes the histogram out as one row of a
//           [kOrderBlocks x kOrderBuckets] matrix;
//   split : one thread per bucket turns its column of the matrix into each
//           workgroup's offset within the bucket (workgroups in order) and
//           the bucket's total;
//   scan  : one workgroup turns the totals into each bucket's first
//           position (buckets in descending cost);
//   place : each workgroup places its rows from those positions through LDS
//           cursors.
// Rows of one bucket and one workgroup land in no particular order (LDS
// atomics); no result depends on the order.
#include "lsp_common.h"

namespace lsp {
namespace {

constexpr int kOrderThreads = 256;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ int cost_bucket(int64_t n) {
    if (n <= 0) return 0;
    if (n < 1024) return (int)n;
    const int e = 63 - __clzll((unsigned long long)n);  // 10..62
    return 1024 + (e - 10) * 64 + (int)((n >> (e - 6)) & 63);
}

// Slot of a row's bucket: descending cost comes first, rows with no work last.
__device__ __forceinline__ int row_slot(const OrderParams& P, int64_t r) {
    const int64_t o = P.row_obj ? (int64_t)P.row_obj[r] : r / P.rows_per_group;
    if (o < 0 || o >= P.n_obj || (P.row_band && P.row_band[r] < 0)) return kOrderBuckets - 1;
    return kOrderBuckets - 2 - cost_bucket(P.offsets[o + 1] - P.offsets[o]);
}

// Workgroup g's share of the rows: [g * per, min((g + 1) * per, n_rows)).
__device__ __forceinline__ void share(const OrderParams& P, int64_t* lo, int64_t* hi) {
    const int64_t per = (P.n_rows + kOrderBlocks - 1) / kOrderBlocks;
    *lo = (int64_t)blockIdx.x * per;
    *hi = *lo + per < P.n_rows ? *lo + per : P.n_rows;
}

__global__ __launch_bounds__(kOrderThreads) void order_count_kernel(const OrderParams P) {
    __shared__ unsigned int s_hist[kOrderBuckets];
    for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderThreads) s_hist[b] = 0u;
    __syncthreads();
    int64_t lo, hi;
    share(P, &lo, &hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kOrderThreads)
        atomicAdd(&s_hist[row_slot(P, r)], 1u);
    __syncthreads();
    unsigned int* out = P.hist + (int64_t)blockIdx.x * kOrderBuckets;
    for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderThreads) out[b] = s_hist[b];
}

// Column b of the matrix, in place: hist[g][b] becomes the number of rows
// of bucket b in workgroups before g; total[b] receives the bucket's count.
__global__ __launch_bounds__(kOrderThreads) void order_split_kernel(const OrderParams P) {
    const int b = blockIdx.x * kOrderThreads + threadIdx.x;
    if (b >= kOrderBuckets) return;
    unsigned int run = 0u;
#pragma unroll 16
    for (int g = 0; g < kOrderBlocks; ++g) {
        unsigned int* h = P.hist + (int64_t)g * kOrderBuckets + b;
        const unsigned int c = *h;
        *h = run;
        run += c;
    }
    P.total[b] = run;
}

// Exclusive prefix sum of the bucket totals, in place (one workgroup): each
// bucket's first position.
__global__ __launch_bounds__(kScanThreads) void order_scan_kernel(const OrderParams P) {
    constexpr int kPer = (kOrderBuckets + kScanThreads - 1) / kScanThreads;
    __shared__ unsigned int s_sum[kScanThreads];
    const int b0 = threadIdx.x * kPer;
    unsigned int v[kPer];
    unsigned int own = 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        v[q] = b0 + q < kOrderBuckets ? P.total[b0 + q] : 0u;
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
    for (int q = 0; q < kPer; ++q) {
        if (b0 + q < kOrderBuckets) P.total[b0 + q] = run;
        run += v[q];
    }
}

// Row r takes the next position s of its workgroup's share of its bucket;
// s is dealt to XCD s % 8, whose rows occupy ranks [xcd_first_rank(x),
// xcd_first_rank(x + 1)).
__global__ __launch_bounds__(kOrderThreads) void order_place_kernel(const OrderParams P) {
    __shared__ unsigned int s_next[kOrderBuckets];
    const unsigned int* within = P.hist + (int64_t)blockIdx.x * kOrderBuckets;
    for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderThreads)
        s_next[b] = P.total[b] + within[b];
    __syncthreads();
    int64_t lo, hi;
    share(P, &lo, &hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kOrderThreads) {
        const int64_t s = (int64_t)atomicAdd(&s_next[row_slot(P, r)], 1u);
        const int x = (int)(s % kXcds);
        P.perm[xcd_first_rank(x, P.n_rows) + s / kXcds] = (int32_t)r;
    }
}

}  // namespace

hipError_t launch_row_order(const OrderParams& p, hipStream_t s) {
    if (p.n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_count_kernel, dim3(kOrderBlocks), dim3(kOrderThreads), 0, s, p);
    hipLaunchKernelGGL(order_split_kernel, dim3((kOrderBuckets + kOrderThreads - 1) / kOrderThreads),
                       dim3(kOrderThreads), 0, s, p);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, p);
    hipLaunchKernelGGL(order_place_kernel, dim3(kOrderBlocks), dim3(kOrderThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace lsp
