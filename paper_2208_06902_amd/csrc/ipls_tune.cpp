// Autotuner of the batched (segmented) form: times the segmented sort of a window of the batch
// under candidate parameters and keeps the fastest, one parameter at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/ipls.h"
#include "ipls_engine.h"

namespace {

constexpr uint64_t kWindowKeys = 1ull << 25;
constexpr int kReps = 2;

struct Trial {
    ipls::Engine* e;
    hipStream_t s;
    const void* src;       // caller's window (read only)
    void* keys;            // private copy sorted by every trial
    uint32_t* pay;         // zero payload when the batch carries one
    uint64_t* offs;        // window offsets (device)
    uint64_t nseg, len, kb;
    ipls_dtype dtype;
    void* ws;
    size_t ws_bytes;
    hipEvent_t a, b;
};

// Best-of-kReps milliseconds of one segmented sort of the window, or a negative value on error.
double time_params(Trial& t, const ipls_params& p) {
    float best = -1.f;
    for (int r = 0; r < kReps; ++r) {
        if (hipMemcpyAsync(t.keys, t.src, t.len * t.kb, hipMemcpyDeviceToDevice, t.s) != hipSuccess) return -1.0;
        if (hipEventRecord(t.a, t.s) != hipSuccess) return -1.0;
        ipls_status st = ipls::engine_sort_segmented(*t.e, t.keys, t.pay, t.offs, t.nseg, t.dtype, &p, t.ws,
                                                     t.ws_bytes, nullptr, t.s);
        if (st != IPLS_OK) return -1.0;
        if (hipEventRecord(t.b, t.s) != hipSuccess || hipEventSynchronize(t.b) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) return -1.0;
        if (best < 0.f || ms < best) best = ms;
    }
    return best;
}

}  // namespace

extern "C" ipls_status ipls_autotune_segmented(const void* keys, const uint64_t* seg_offsets, size_t nseg,
                                               ipls_dtype dtype, int has_payload, const ipls_params* base,
                                               ipls_params* out, ipls_tune_report* report, void* stream) {
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    if (!keys || !seg_offsets || !out || nseg == 0) return IPLS_ERR_INVALID;
    ipls_params p0;
    if (base) p0 = *base;
    else ipls_default_params(&p0);
    if (p0.tile_keys == 0) p0.tile_keys = 4096;  // the library default, named
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint64_t> off(nseg + 1);
    if (hipMemcpyAsync(off.data(), seg_offsets, (nseg + 1) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return IPLS_ERR_HIP;
    for (size_t i = 0; i < nseg; ++i)
        if (off[i + 1] < off[i]) return IPLS_ERR_INVALID;
    // window: the leading segments, at least kWindowKeys keys (or the whole batch)
    size_t w = 0;
    while (w < nseg && off[w] - off[0] < kWindowKeys) ++w;
    Trial t{};
    t.kb = dtype == IPLS_F32 ? 4 : 8;
    t.nseg = w;
    t.len = off[w] - off[0];
    t.dtype = dtype;
    t.s = s;
    t.src = (const char*)keys + off[0] * t.kb;
    *out = p0;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->window_segments = (uint32_t)w;
        report->window_keys = t.len;
    }
    if (t.len < 2) return IPLS_OK;
    std::vector<uint64_t> woff(w + 1);
    for (size_t i = 0; i <= w; ++i) woff[i] = off[i] - off[0];
    t.ws_bytes = ipls_workspace_bytes(t.len, dtype, has_payload, &p0);
    const size_t kbytes = (t.len * t.kb + 255) & ~(size_t)255;
    const size_t pbytes = has_payload ? ((t.len * 4 + 255) & ~(size_t)255) : 0;
    const size_t obytes = (woff.size() * 8 + 255) & ~(size_t)255;
    char* mem = nullptr;
    if (hipMalloc((void**)&mem, kbytes + pbytes + obytes + t.ws_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return IPLS_ERR_OOM;
    }
    t.keys = mem;
    t.pay = has_payload ? (uint32_t*)(mem + kbytes) : nullptr;
    t.offs = (uint64_t*)(mem + kbytes + pbytes);
    t.ws = mem + kbytes + pbytes + obytes;
    ipls_status st = IPLS_OK;
    t.e = ipls::engine_new();
    if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) st = IPLS_ERR_HIP;
    if (st == IPLS_OK && has_payload && hipMemsetAsync(t.pay, 0, t.len * 4, s) != hipSuccess) st = IPLS_ERR_HIP;
    if (st == IPLS_OK &&
        hipMemcpyAsync(t.offs, woff.data(), woff.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        st = IPLS_ERR_HIP;
    if (st == IPLS_OK && hipStreamSynchronize(s) != hipSuccess) st = IPLS_ERR_HIP;

    uint32_t trials = 0;
    ipls_params best = p0;
    double best_ms = -1.0, default_ms = -1.0;
    if (st == IPLS_OK) {
        time_params(t, p0);  // warm the context's buffers
        best_ms = default_ms = time_params(t, p0);
        trials = 1;
        if (best_ms < 0) st = IPLS_ERR_HIP;
    }
    const uint32_t tiles[] = {4096, 2048}, thresholds[] = {4096, 2048, 1024}, buckets[] = {256, 128, 64};
    for (int dim = 0; dim < 3 && st == IPLS_OK; ++dim) {
        const uint32_t* cand = dim == 0 ? tiles : dim == 1 ? thresholds : buckets;
        const int nc = dim == 0 ? 2 : 3;
        ipls_params round_best = best;
        for (int c = 0; c < nc; ++c) {
            ipls_params q = best;
            if (dim == 0) q.tile_keys = cand[c];
            else if (dim == 1) q.base_case_max = cand[c];
            else q.num_buckets = cand[c];
            if (std::memcmp(&q, &best, sizeof(q)) == 0) continue;
            const uint64_t smin = q.sample_min ? q.sample_min : (q.sample_policy == 1 ? 0 : 2ull * q.num_buckets);
            if (smin > q.base_case_max) continue;  // not a valid combination
            const double ms = time_params(t, q);
            ++trials;
            if (ms >= 0 && ms < best_ms) {
                best_ms = ms;
                round_best = q;
            }
        }
        best = round_best;
    }
    (void)hipStreamSynchronize(s);
    if (t.a) (void)hipEventDestroy(t.a);
    if (t.b) (void)hipEventDestroy(t.b);
    ipls::engine_free(t.e);
    (void)hipFree(mem);
    if (st != IPLS_OK) return st;
    *out = best;
    if (report) {
        report->trials = trials;
        report->default_ms = default_ms;
        report->best_ms = best_ms;
    }
    return IPLS_OK;
}
