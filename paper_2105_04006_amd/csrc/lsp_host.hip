// lsp_host.hip -- returning whole periodograms to host memory (Section 3.5).
//
// The paper copies batch periodograms to the host through small pinned
// staging buffers on three streams, then has several host threads move each
// staged piece into its final pageable location, instead of one large copy
// that the driver stages itself.  Here the same idea is a pipeline over
// chunks of objects:
//   - objects are cut into chunks whose periodograms hold about chunk_bytes;
//   - chunk c belongs to lane c % n_streams.  A lane has a compute stream, a
//     copy stream, two device chunk buffers and a pinned staging buffer of
//     two halves; its driver thread keeps the kernels of the next chunk
//     queued on the compute stream while it drains the current one: the copy
//     stream moves the chunk to staging in pieces (the DMA fills one half
//     while host threads empty the other) and a pool of copy threads writes
//     each staged piece to the caller's array;
//   - the lanes run concurrently, so kernels, device-to-host copies and host
//     copies of different chunks all overlap.
// The full [n_obj x n_f] periodogram is never resident on the device.
//
// A pipe owns its streams (default priority), pinned staging buffers, copy
// threads and (grown on demand) device buffers; calls on one pipe must not
// overlap.
#include <emmintrin.h>
#include <stdint.h>
#include <string.h>

#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "lsp_common.h"

namespace lsp {
namespace {

constexpr int kMaxStreams = 8;
constexpr int kMaxCopyThreads = 64;

// Copy with streaming (non-temporal) stores: the destination is written once
// and not read back here, so its lines need not be fetched into the caches
// first, which saves a quarter of the host-memory traffic of a staged piece
// (DMA write, read, destination write, no read-for-ownership).
void stream_copy(char* dst, const char* src, size_t n) {
    size_t head = (16 - ((uintptr_t)dst & 15)) & 15;
    if (head > n) head = n;
    memcpy(dst, src, head);
    dst += head;
    src += head;
    n -= head;
    const size_t body = n & ~(size_t)63;
    for (size_t i = 0; i < body; i += 64) {
        const __m128i a = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i));
        const __m128i b = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 16));
        const __m128i c = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 32));
        const __m128i d = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 48));
        _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i), a);
        _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 16), b);
        _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 32), c);
        _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 48), d);
    }
    memcpy(dst + body, src + body, n - body);
    _mm_sfence();
}

// Fixed set of host threads running copy jobs; copy() splits one copy into
// `parts` jobs and returns when all of them are done.
class CopyPool {
  public:
    explicit CopyPool(int n) {
        for (int i = 0; i < n; ++i) threads_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : threads_) t.join();
    }
    int size() const { return (int)threads_.size(); }

    void copy(char* dst, const char* src, size_t n, int parts) {
        if (parts <= 1 || threads_.empty() || n < ((size_t)1 << 20)) {
            stream_copy(dst, src, n);
            return;
        }
        struct Done {
            std::mutex mu;
            std::condition_variable cv;
            int left;
        } done;
        done.left = parts;
        const size_t step = (n + parts - 1) / parts;
        {
            std::lock_guard<std::mutex> g(mu_);
            for (int i = 0; i < parts; ++i) {
                const size_t a = (size_t)i * step;
                const size_t b = a + step < n ? a + step : n;
                jobs_.push_back([dst, src, a, b, &done] {
                    if (b > a) stream_copy(dst + a, src + a, b - a);
                    std::lock_guard<std::mutex> h(done.mu);
                    if (--done.left == 0) done.cv.notify_all();
                });
            }
        }
        cv_.notify_all();
        std::unique_lock<std::mutex> w(done.mu);
        done.cv.wait(w, [&] { return done.left == 0; });
    }

  private:
    void loop() {
        for (;;) {
            std::function<void()> job;
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [this] { return stop_ || !jobs_.empty(); });
                if (stop_ && jobs_.empty()) return;
                job = std::move(jobs_.front());
                jobs_.pop_front();
            }
            job();
        }
    }
    std::vector<std::thread> threads_;
    std::deque<std::function<void()>> jobs_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool stop_ = false;
};

struct Lane {
    hipStream_t stream = nullptr;  // kernels
    hipStream_t copy = nullptr;    // device-to-host copies
    hipEvent_t half_done[2] = {nullptr, nullptr};
    hipEvent_t computed[2] = {nullptr, nullptr};
    char* staging = nullptr;  // pinned, staging_bytes
    void* d_pgram[2] = {nullptr, nullptr};  // device chunk periodograms (double buffer)
    size_t d_pgram_bytes[2] = {0, 0};
    void* d_peaks[2] = {nullptr, nullptr};  // device chunk peak records
    size_t d_peaks_bytes[2] = {0, 0};
    void* d_ws = nullptr;     // device workspace of the batch call
    size_t d_ws_bytes = 0;
};

bool grow(void** p, size_t* have, size_t want) {
    if (*have >= want) return true;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, want) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    *have = want;
    return true;
}

}  // namespace
}  // namespace lsp

struct lsp_pipe_s {
    int n_streams = 0;
    size_t staging_bytes = 0;
    size_t chunk_bytes = 0;
    int copy_parts = 1;
    lsp::Lane lanes[lsp::kMaxStreams];
    lsp::CopyPool* pool = nullptr;
};

namespace {

void destroy_pipe(lsp_pipe p) {
    if (!p) return;
    delete p->pool;
    for (int i = 0; i < p->n_streams; ++i) {
        lsp::Lane& l = p->lanes[i];
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.copy) (void)hipStreamSynchronize(l.copy);
        for (int b = 0; b < 2; ++b) {
            if (l.half_done[b]) (void)hipEventDestroy(l.half_done[b]);
            if (l.computed[b]) (void)hipEventDestroy(l.computed[b]);
            if (l.d_pgram[b]) (void)hipFree(l.d_pgram[b]);
            if (l.d_peaks[b]) (void)hipFree(l.d_peaks[b]);
        }
        if (l.staging) (void)hipHostFree(l.staging);
        if (l.d_ws) (void)hipFree(l.d_ws);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.copy) (void)hipStreamDestroy(l.copy);
    }
    delete p;
}

// One stream's share of a call: chunks lane, lane + n_streams, ...
lsp_status run_lane(lsp_pipe p, int lane, const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                    const double* t, const double* y, const double* dy, bool gen,
                    const lsp_grid* grid, const lsp_options* opt, size_t bin_bytes,
                    int64_t chunk_objs, char* host_pgram, lsp_peak* host_peaks) {
    lsp::Lane& L = p->lanes[lane];
    const size_t half = p->staging_bytes / 2;
    const size_t row_bytes = bin_bytes * (size_t)grid->n_f;
    const int64_t n_chunks = (n_obj + chunk_objs - 1) / chunk_objs;
    std::vector<int64_t> mine;
    for (int64_t c = lane; c < n_chunks; c += p->n_streams) mine.push_back(c);
    // Kernels of the lane's i-th chunk into buffer i % 2, then an event the
    // copy stream waits for.
    auto launch = [&](size_t i) -> lsp_status {
        const int b = (int)(i & 1);
        const int64_t o0 = mine[i] * chunk_objs;
        const int64_t m = o0 + chunk_objs < n_obj ? chunk_objs : n_obj - o0;
        lsp_status st = lsp::batch_call(offsets + o0, m, n_obs, t, y, dy, gen, grid, opt,
                                        host_pgram ? L.d_pgram[b] : nullptr,
                                        static_cast<lsp_peak*>(L.d_peaks[b]), L.d_ws,
                                        L.d_ws_bytes, L.stream, n_obj == 1);
        if (st != LSP_OK) return st;
        return hipEventRecord(L.computed[b], L.stream) == hipSuccess ? LSP_OK : LSP_EHIP;
    };
    for (size_t i = 0; i < mine.size() && i < 2; ++i) {
        lsp_status st = launch(i);
        if (st != LSP_OK) return st;
    }
    for (size_t i = 0; i < mine.size(); ++i) {
        const int b = (int)(i & 1);
        const int64_t o0 = mine[i] * chunk_objs;
        const int64_t m = o0 + chunk_objs < n_obj ? chunk_objs : n_obj - o0;
        if (hipStreamWaitEvent(L.copy, L.computed[b], 0) != hipSuccess) return LSP_EHIP;
        // Pieces of the chunk's periodograms through the two staging halves,
        // then its peak records: the DMA fills one half while the copy
        // threads drain the other.
        struct Piece {
            const char* src;
            char* dst;
            size_t n;
        };
        std::vector<Piece> pieces;
        if (host_pgram) {
            const size_t total = row_bytes * (size_t)m;
            for (size_t a = 0; a < total; a += half)
                pieces.push_back({static_cast<const char*>(L.d_pgram[b]) + a,
                                  host_pgram + row_bytes * (size_t)o0 + a,
                                  total - a < half ? total - a : half});
        }
        if (host_peaks)
            pieces.push_back({static_cast<const char*>(L.d_peaks[b]),
                              reinterpret_cast<char*>(host_peaks + o0), sizeof(lsp_peak) * m});
        auto issue = [&](size_t k) -> bool {
            char* dst = L.staging + (k & 1) * half;
            return hipMemcpyAsync(dst, pieces[k].src, pieces[k].n, hipMemcpyDeviceToHost,
                                  L.copy) == hipSuccess &&
                   hipEventRecord(L.half_done[k & 1], L.copy) == hipSuccess;
        };
        for (size_t k = 0; k < pieces.size() && k < 2; ++k)
            if (!issue(k)) return LSP_EHIP;
        for (size_t k = 0; k < pieces.size(); ++k) {
            if (hipEventSynchronize(L.half_done[k & 1]) != hipSuccess) return LSP_EHIP;
            p->pool->copy(pieces[k].dst, L.staging + (k & 1) * half, pieces[k].n, p->copy_parts);
            if (k + 2 < pieces.size() && !issue(k + 2)) return LSP_EHIP;
        }
        // every piece of buffer b has arrived: it takes the chunk after next
        if (i + 2 < mine.size()) {
            lsp_status st = launch(i + 2);
            if (st != LSP_OK) return st;
        }
    }
    return LSP_OK;
}

}  // namespace

extern "C" {

lsp_status lsp_pipe_create(int32_t n_streams, size_t staging_bytes, size_t chunk_bytes,
                           int32_t copy_threads, lsp_pipe* pipe) {
    if (!pipe) return LSP_EINVAL;
    *pipe = nullptr;
    // Defaults measured on 4 GB of FP32 periodograms (10,000 objects x 1e5
    // bins): with two chunk buffers per lane, one lane keeps the DMA engine
    // busy, and more lanes interleave their copies and run slower.
    if (n_streams == 0) n_streams = 1;
    if (staging_bytes == 0) staging_bytes = (size_t)16 << 20;
    if (chunk_bytes == 0) chunk_bytes = (size_t)128 << 20;
    if (copy_threads == 0) copy_threads = 12;
    if (n_streams < 1 || n_streams > lsp::kMaxStreams || copy_threads < 1 ||
        copy_threads > lsp::kMaxCopyThreads || staging_bytes < ((size_t)2 << 10) ||
        staging_bytes % 512)
        return LSP_EINVAL;
    lsp_pipe p = new (std::nothrow) lsp_pipe_s;
    if (!p) return LSP_EHIP;
    p->n_streams = n_streams;
    p->staging_bytes = staging_bytes;
    p->chunk_bytes = chunk_bytes;
    // each stream's copies are split over the pool so that the streams
    // together keep every copy thread busy
    p->copy_parts = (copy_threads + n_streams - 1) / n_streams;
    for (int i = 0; i < n_streams; ++i) {
        lsp::Lane& l = p->lanes[i];
        if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&l.copy, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l.half_done[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&l.half_done[1], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&l.computed[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&l.computed[1], hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&l.staging), staging_bytes,
                          hipHostMallocDefault) != hipSuccess) {
            p->n_streams = i + 1;
            destroy_pipe(p);
            return LSP_EHIP;
        }
    }
    try {
        p->pool = new lsp::CopyPool(copy_threads);
    } catch (...) {  // thread creation or allocation failed
        p->pool = nullptr;
    }
    if (!p->pool) {
        destroy_pipe(p);
        return LSP_EHIP;
    }
    *pipe = p;
    return LSP_OK;
}

void lsp_pipe_destroy(lsp_pipe pipe) { destroy_pipe(pipe); }

static lsp_status batch_to_host(lsp_pipe pipe, const int64_t* offsets, int64_t n_obj,
                                int64_t n_obs, const double* t, const double* y, const double* dy,
                                int32_t generalized, const lsp_grid* grid,
                                const lsp_options* opt_in, void* host_pgram, lsp_peak* host_peaks,
                                void* stream) {
    if (!pipe || !offsets || !grid || n_obj < 1 || n_obs < 0) return LSP_EINVAL;
    if (!(generalized == 0 || generalized == 1)) return LSP_EINVAL;
    if (!generalized && dy) return LSP_EINVAL;
    if (!host_pgram && !host_peaks) return LSP_EINVAL;
    const lsp_options opt = opt_in ? *opt_in : lsp_default_options();
    if (opt.t_split > 1) return LSP_EUNSUPPORTED;
    const bool gen = generalized != 0;
    if (lsp::batch_workspace_bytes(1, n_obs, grid, &opt, gen, n_obj == 1) == 0) return LSP_EINVAL;
    const size_t bin_bytes = opt.pgram_dtype == LSP_PGRAM_F64 ? 8 : 4;
    const size_t row_bytes = bin_bytes * (size_t)grid->n_f;
    // Objects per chunk: about chunk_bytes of periodogram (at least one
    // object), and the peak records of a chunk fit in half a staging buffer.
    int64_t chunk = (int64_t)(pipe->chunk_bytes / row_bytes);
    if (chunk < 1) chunk = 1;
    const int64_t peak_cap = (int64_t)(pipe->staging_bytes / 2 / sizeof(lsp_peak));
    if (chunk > peak_cap) chunk = peak_cap;
    if (chunk > n_obj) chunk = n_obj;
    // Every chunk runs with the launch configuration of the whole batch (so
    // its results are lsp_batch's bit for bit); a chunk of the largest size
    // needs the most workspace.
    const size_t ws = lsp::batch_workspace_bytes(chunk, n_obs, grid, &opt, gen, n_obj == 1);
    if (ws == 0) return LSP_EUNSUPPORTED;
    // Device buffers for one chunk per stream (kept for later calls).
    for (int i = 0; i < pipe->n_streams; ++i) {
        lsp::Lane& l = pipe->lanes[i];
        for (int b = 0; b < 2; ++b)
            if ((host_pgram &&
                 !lsp::grow(&l.d_pgram[b], &l.d_pgram_bytes[b], row_bytes * (size_t)chunk)) ||
                !lsp::grow(&l.d_peaks[b], &l.d_peaks_bytes[b], sizeof(lsp_peak) * (size_t)chunk))
                return LSP_EHIP;
        if (!lsp::grow(&l.d_ws, &l.d_ws_bytes, ws)) return LSP_EHIP;
    }
    // The inputs are ready once the caller's stream reaches this point.
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return LSP_EHIP;
    lsp_status st = LSP_OK;
    if (hipEventRecord(ready, static_cast<hipStream_t>(stream)) != hipSuccess) st = LSP_EHIP;
    for (int i = 0; i < pipe->n_streams && st == LSP_OK; ++i)
        if (hipStreamWaitEvent(pipe->lanes[i].stream, ready, 0) != hipSuccess ||
            hipStreamWaitEvent(pipe->lanes[i].copy, ready, 0) != hipSuccess)
            st = LSP_EHIP;
    if (st == LSP_OK) {
        // No C++ exception may leave this C entry point: a lane that cannot
        // allocate, or a driver thread that cannot start, reports LSP_EHIP.
        std::vector<lsp_status> res(pipe->n_streams, LSP_OK);
        std::vector<std::thread> drivers;
        auto lane = [&](int i) {
            try {
                res[i] = run_lane(pipe, i, offsets, n_obj, n_obs, t, y, dy, gen, grid, &opt,
                                  bin_bytes, chunk, static_cast<char*>(host_pgram), host_peaks);
            } catch (...) {
                res[i] = LSP_EHIP;
            }
        };
        for (int i = 1; i < pipe->n_streams; ++i) {
            try {
                drivers.emplace_back(lane, i);
            } catch (...) {
                lane(i);  // no thread: run this lane's share here
            }
        }
        lane(0);
        for (auto& d : drivers) d.join();
        for (int i = 0; i < pipe->n_streams; ++i) {
            if ((hipStreamSynchronize(pipe->lanes[i].stream) != hipSuccess ||
                 hipStreamSynchronize(pipe->lanes[i].copy) != hipSuccess) &&
                st == LSP_OK)
                st = LSP_EHIP;
            if (res[i] != LSP_OK && st == LSP_OK) st = res[i];
        }
    }
    (void)hipEventDestroy(ready);
    return st;
}

lsp_status lsp_batch_to_host(lsp_pipe pipe, const int64_t* offsets, int64_t n_obj, int64_t n_obs,
                             const double* t, const double* y, const double* dy,
                             int32_t generalized, const lsp_grid* grid, const lsp_options* opt_in,
                             void* host_pgram, lsp_peak* host_peaks, void* stream) {
    try {
        return batch_to_host(pipe, offsets, n_obj, n_obs, t, y, dy, generalized, grid, opt_in,
                             host_pgram, host_peaks, stream);
    } catch (...) {  // allocation failure before any thread started
        return LSP_EHIP;
    }
}

}  // extern "C"
