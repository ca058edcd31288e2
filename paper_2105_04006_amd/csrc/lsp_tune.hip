// lsp_tune.hip -- launch-shape autotuner for the FP32 form (host code).
//
// The best frequencies-per-lane K, wavefronts per workgroup, recurrence,
// schedule and (single object) observation split depend on N_t, N_f and the
// number of objects.  lsp_autotune times candidate shapes on the caller's own
// data -- for a batch, on a prefix of its objects large enough to fill the
// device many times over -- and keeps the fastest candidate whose peaks agree
// with the FP64 form on the same objects (within one bin on >= 99.9% of
// objects, |dP| <= 1e-3 at the peaks).  Results can be cached per shape class
// in a JSON-lines file.  The call is synchronous and allocates no device
// memory: it runs in the caller's workspace and peak scratch.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lsp_common.h"

namespace lsp {
namespace {

std::mutex g_cache_mutex;

int log2_bucket(double v) { return v <= 1.0 ? 0 : (int)floor(log2(v)); }

std::string shape_key(const char* arch, int single, int64_t n_obj, int64_t n_obs, int64_t n_f) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s/%s/obj%d/nt%d/nf%d", arch, single ? "single" : "batch",
             log2_bucket((double)n_obj), log2_bucket((double)n_obs / (double)n_obj),
             log2_bucket((double)n_f));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, lsp_options* o) {
    if (!path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[256];
        int kk, w, rec, sched, split, wsp;
        if (sscanf(line,
                   "{\"key\": \"%255[^\"]\", \"k_per_lane\": %d, \"waves_per_wg\": %d, "
                   "\"recurrence\": %d, \"schedule\": %d, \"t_split\": %d, "
                   "\"wave_split\": %d",
                   k, &kk, &w, &rec, &sched, &split, &wsp) == 7 &&
            key == k) {
            o->k_per_lane = kk;
            o->waves_per_wg = w;
            o->recurrence = rec;
            o->schedule = sched;
            o->t_split = split;
            o->wave_split = wsp;
            found = true;  // the last entry for a key wins
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const lsp_options& o, double ms) {
    if (!path) return;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"key\": \"%s\", \"k_per_lane\": %d, \"waves_per_wg\": %d, \"recurrence\": %d, "
            "\"schedule\": %d, \"t_split\": %d, \"wave_split\": %d, \"ms\": %.6f}\n",
            key.c_str(), o.k_per_lane, o.waves_per_wg, o.recurrence, o.schedule, o.t_split,
            o.wave_split, ms);
    fclose(f);
}

std::vector<lsp_options> candidates(const lsp_options& base, bool single) {
    std::vector<lsp_options> out;
    const int ks[] = {8, 10, 12, 16, 32};
    // (eight waves per workgroup exist only with the in-workgroup wave split,
    // which only a single object's search covers)
    const int ws[] = {1, 2, 4, 8};
    // One object: the recurrence is fixed to the three-term form (as accurate
    // and cheaper) and the search covers how the object is split instead.
    std::vector<int> recs = single ? std::vector<int>{LSP_REC_CHEBYSHEV}
                                   : std::vector<int>{LSP_REC_ROTATION, LSP_REC_CHEBYSHEV};
    std::vector<int> scheds = single ? std::vector<int>{LSP_SCHED_GRID}
                                     : std::vector<int>{LSP_SCHED_GRID, LSP_SCHED_PERSISTENT};
    std::vector<int> splits = single ? std::vector<int>{0, 1, 2, 4, 8, 16} : std::vector<int>{1};
    for (int k : ks)
        for (int w : ws)
            for (int r : recs)
                for (int sc : scheds)
                    for (int sp : splits)
                        for (int wsp = 0; wsp < (single && w > 1 ? 2 : 1); ++wsp) {
                            if (w == 8 && !wsp) continue;
                            lsp_options o = base;
                            o.form = LSP_FORM_FP32P;
                            o.k_per_lane = k;
                            o.waves_per_wg = w;
                            o.recurrence = r;
                            o.schedule = sc;
                            o.t_split = sp;
                            o.wave_split = wsp ? LSP_WSPLIT_ON : LSP_WSPLIT_OFF;
                            out.push_back(o);
                        }
    return out;
}

bool peaks_agree(const std::vector<lsp_peak>& a, const std::vector<lsp_peak>& ref) {
    int64_t n_ok = 0, agree = 0;
    for (size_t o = 0; o < ref.size(); ++o) {
        if (ref[o].status != LSP_OBJ_OK) {
            if (a[o].status != ref[o].status) return false;
            continue;
        }
        ++n_ok;
        const int64_t d = a[o].index - ref[o].index;
        if (d >= -1 && d <= 1) ++agree;
        if (!(fabs(a[o].power - ref[o].power) <= 1e-3)) return false;
    }
    return n_ok == 0 || (double)agree >= 0.999 * (double)n_ok;
}

}  // namespace
}  // namespace lsp

extern "C" {

size_t lsp_autotune_workspace_bytes(int64_t n_obj, int64_t n_obs, const lsp_grid* grid,
                                    const lsp_options* base_in) {
    const lsp_options base = base_in ? *base_in : lsp_default_options();
    size_t need = 0;
    lsp_options ref = base;
    ref.form = LSP_FORM_FP64;
    ref.k_per_lane = ref.waves_per_wg = ref.t_split = 0;
    ref.schedule = LSP_SCHED_AUTO;
    ref.recurrence = LSP_REC_AUTO;
    need = lsp_workspace_bytes(n_obj, n_obs, grid, &ref);
    if (need == 0) return 0;
    for (const lsp_options& o : lsp::candidates(base, n_obj == 1))
        need = std::max(need, lsp_workspace_bytes(n_obj, n_obs, grid, &o));
    return need;
}

lsp_status lsp_autotune(const int64_t* offsets, int64_t n_obj, int64_t n_obs, const double* t,
                        const double* y, const lsp_grid* grid, const lsp_options* base_in,
                        lsp_options* tuned, lsp_peak* peak_scratch, void* workspace,
                        size_t workspace_bytes, const char* cache_path, int32_t repeats,
                        void* stream) {
    if (!tuned || !peak_scratch || !workspace || !grid) return LSP_EINVAL;
    if (!offsets && n_obj != 1) return LSP_EINVAL;
    if (n_obj < 1 || n_obs < 0 || repeats < 1) return LSP_EINVAL;
    const lsp_options base = base_in ? *base_in : lsp_default_options();
    const bool single = offsets == nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return LSP_EHIP;
    const std::string key = lsp::shape_key(prop.gcnArchName, single, n_obj, n_obs, grid->n_f);
    *tuned = base;
    tuned->form = LSP_FORM_FP32P;
    if (lsp::cache_lookup(cache_path, key, tuned)) return LSP_OK;

    // Tune on a prefix of the batch holding about 1e11 evaluations (tens of
    // milliseconds of FP32 work): enough items to fill the device many times.
    int64_t m = n_obj, m_obs = n_obs;
    if (!single) {
        std::vector<int64_t> off(n_obj + 1);
        if (hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * (n_obj + 1), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return LSP_EHIP;
        const double target = 1e11;
        m = 1;
        while (m < n_obj && (double)(off[m] - off[0]) * (double)grid->n_f < target) ++m;
        m_obs = std::min<int64_t>(std::max<int64_t>(off[m], 0), n_obs);
    }

    std::vector<lsp_peak> ref(m), got(m);
    lsp_options ref_opt = base;
    ref_opt.form = LSP_FORM_FP64;
    ref_opt.k_per_lane = ref_opt.waves_per_wg = ref_opt.t_split = 0;
    ref_opt.schedule = LSP_SCHED_AUTO;
    ref_opt.recurrence = LSP_REC_AUTO;
    lsp_status st = single ? lsp_single(t, y, m_obs, grid, &ref_opt, nullptr, peak_scratch,
                                        workspace, workspace_bytes, stream)
                           : lsp_batch(offsets, m, m_obs, t, y, grid, &ref_opt, nullptr,
                                       peak_scratch, workspace, workspace_bytes, stream);
    if (st != LSP_OK) return st;
    if (hipMemcpyAsync(ref.data(), peak_scratch, sizeof(lsp_peak) * m, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LSP_EHIP;

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LSP_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LSP_EHIP;
    }
    double best_ms = 1e300;
    bool any = false;
    for (const lsp_options& o : lsp::candidates(base, single)) {
        const size_t need = lsp_workspace_bytes(m, m_obs, grid, &o);
        if (need == 0 || need > workspace_bytes) continue;
        auto call = [&]() {
            return single ? lsp_single(t, y, m_obs, grid, &o, nullptr, peak_scratch, workspace,
                                       workspace_bytes, stream)
                          : lsp_batch(offsets, m, m_obs, t, y, grid, &o, nullptr, peak_scratch,
                                      workspace, workspace_bytes, stream);
        };
        if (call() != LSP_OK) continue;
        if (hipMemcpyAsync(got.data(), peak_scratch, sizeof(lsp_peak) * m, hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = LSP_EHIP;
            break;
        }
        if (!lsp::peaks_agree(got, ref)) continue;
        if (hipEventRecord(e0, s) != hipSuccess) {
            st = LSP_EHIP;
            break;
        }
        for (int r = 0; r < repeats; ++r) call();
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = LSP_EHIP;
            break;
        }
        const double per = (double)ms / repeats;
        if (per < best_ms) {
            best_ms = per;
            *tuned = o;
            any = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LSP_OK) return st;
    if (!any) return LSP_EUNSUPPORTED;
    lsp::cache_store(cache_path, key, *tuned, best_ms);
    return LSP_OK;
}

}  // extern "C"
