// Host side of the IPLS library: level-synchronous orchestration of the distribution kernels
// and the C ABI declared in include/ipls.h.
//
// One sort = a loop of levels.  Each level partitions every bucket of more than T keys at once
// (all buckets of the level share every launch), reading one buffer and writing the other; the
// base case finishes buckets of at most T keys into the caller's buffer.  The host reads back a
// small plan (item count, tile and sample totals) once per level to size the next launches.
// Samples are sorted by the same engine one nesting level down (the Machine Learning Models
// chapter notes that an ML-enhanced sort can sort its own sample), or straight by the base case
// when every sample has at most T keys.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/ipls.h"
#include "ipls_engine.h"
#include "ipls_kernels.h"

namespace ipls {
namespace {

constexpr uint64_t kWorklistFewItems = 1024;  // up to this many items: four a k_worklist workgroup
constexpr uint32_t kSmallS = kFitLds;  // samples up to this size are fitted in one workgroup's LDS
constexpr uint64_t kDeferBaseItems = 2048;  // levels of at least this many items run before the previous level's base case
constexpr uint64_t kDeferBaseShare = 64;    // ... and levels of at least 1/64 of its keys

// IPLS_DEBUG_CHECKS in the environment: 1 checks the sort's invariants after every pass and at
// the end (ipls_debug.h); 2 does the same and plants a mismatch in the final multiset comparison,
// so that a test sees the error reported.  Read on every top-level sort.
int debug_checks() {
    const char* v = std::getenv("IPLS_DEBUG_CHECKS");
    if (!v || !*v || *v == '0') return 0;
    return *v == '2' ? 2 : 1;
}
constexpr uint32_t kFitChunk = 2048;   // windows per workgroup in the multi-round fit
constexpr uint32_t kCand = 15;         // candidate widths per fit round
constexpr uint32_t kSmallTile = 4 * kWave * kPassIPT;  // 2048 keys: 4 waves
constexpr uint32_t kTile = 8 * kWave * kPassIPT;       // 4096 keys: 8 waves

// Keys per distribution tile: 4096 (8 waves, the default) or 2048 (4 waves); 8 keys a thread.
inline uint32_t tile_keys_of(const ipls_params& p) { return p.tile_keys == kSmallTile ? kSmallTile : kTile; }
constexpr int kMaxLevels = 4096;
constexpr int kMaxDepth = 16;

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

// A call of the allocation-free entry point carves every buffer from its GPU's static scratch
// array instead of allocating: t_arena is set for the duration of that call on its thread.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
};
thread_local Arena* t_arena = nullptr;

ipls_status ensure(Buf& b, size_t bytes) {
    if (b.p && bytes <= b.cap) return IPLS_OK;
    size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    if (t_arena) {
        want = (want + 255) & ~(size_t)255;
        if (want > t_arena->cap - t_arena->off) return IPLS_ERR_OOM;  // the scratch array is full
        b.p = t_arena->base + t_arena->off;
        b.cap = want;
        t_arena->off += want;
        return IPLS_OK;
    }
    if (b.p) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return IPLS_ERR_OOM;
    }
    b.cap = want;
    return IPLS_OK;
}


struct Depth {
    Buf scratch, spay, items[2], base[2], sample_base, counters, plan, tile_off, sample_off, fit_off, chunk_off, tile_map,
        fit_map, chunk_map, models, masks, hist, bstart, tile_pref, chunk_sum, chunk_pref, sample, leaves, seg, roots,
        leaf_first, leaf_last, eqinfo, rsample, copy, copy_off, copy_map, treeflag, sample2, children[2], spans, cls, wide,
        dbg_all, dbg_acc;
    Plan* plan_h = nullptr;     // pinned, coherent: k_plan writes it directly
    Plan* plan_hd = nullptr;    // its device address (null: the plan is copied into plan_copy)
    uint64_t plan_seq = 0;      // k_plan launches so far
    Plan plan_copy;             // host copy of the plan for contexts that allocate nothing
};

template <class F>
void for_each_buf(Depth& D, F&& f) {
    for (Buf* b : {&D.scratch, &D.spay, &D.items[0], &D.items[1], &D.base[0], &D.base[1], &D.sample_base, &D.counters,
                   &D.plan, &D.tile_off, &D.sample_off, &D.fit_off, &D.chunk_off, &D.tile_map, &D.fit_map,
                   &D.chunk_map, &D.models, &D.masks, &D.hist, &D.bstart, &D.tile_pref, &D.chunk_sum, &D.chunk_pref,
                   &D.sample, &D.leaves, &D.seg, &D.roots, &D.leaf_first, &D.leaf_last, &D.eqinfo, &D.rsample,
                   &D.copy, &D.copy_off, &D.copy_map, &D.treeflag, &D.sample2, &D.children[0], &D.children[1],
                   &D.spans, &D.cls, &D.wide, &D.dbg_all, &D.dbg_acc})
        f(*b);
}

// One engine context: the cached buffers of every nesting depth.  Calls on one context are
// serialised by its mutex; separate contexts (the server's lanes) run concurrently.
struct Device {
    Depth depth[kMaxDepth];
    std::mutex mu;
    // The top-level sort's base case runs on a stream of its own (non-blocking, default priority),
    // beside the next level's partition; ev_base[parity] marks the end of a level's base launch.
    hipStream_t side = nullptr;
    hipEvent_t ev_base[2] = {nullptr, nullptr};
    hipEvent_t ev_defer = nullptr;  // a level's worklist, which a deferred base launch waits for
    // The allocation-free entry point's context: buffers come from the scratch array, the plan is
    // copied back, and everything runs on the caller's stream (no side stream, no events).
    bool noalloc = false;
};

void release(Buf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

void release_device(Device& dv) {
    for (Depth& D : dv.depth) {
        for_each_buf(D, [](Buf& b) { release(b); });
        if (D.plan_h && D.plan_h != &D.plan_copy) (void)hipHostFree(D.plan_h);
        D.plan_h = nullptr;
        D.plan_hd = nullptr;
    }
    for (hipEvent_t* e : {&dv.ev_base[0], &dv.ev_base[1], &dv.ev_defer}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
    if (dv.side) (void)hipStreamDestroy(dv.side);
    dv.side = nullptr;
}

struct Prof {
    std::atomic<int> mask{0};  // bit k: record kernel id k
    static constexpr int kLevels = 16;  // per-level figures for levels 0..15 (deeper ones count in 15)
    struct Rec {
        hipEvent_t a, b;
        int kernel, level;
        double bytes;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    uint64_t launches[3] = {0, 0, 0};
    double ms[3] = {0, 0, 0}, bytes[3] = {0, 0, 0};
    uint64_t lv_launches[3][kLevels] = {};
    double lv_ms[3][kLevels] = {}, lv_bytes[3][kLevels] = {};
};

std::mutex g_mu;         // the map of default contexts
std::mutex g_prof_mu;    // profiling records
std::mutex g_status_mu;  // last status per stream
std::unordered_map<int, Device*> g_devices;
std::unordered_map<void*, ipls_status> g_stream_status;
Prof g_prof;

// The default context of the current device (used by the plain entry points).
Device& device_ctx() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_devices.find(dev);
    if (it != g_devices.end()) return *it->second;
    Device* d = new Device();
    g_devices[dev] = d;
    return *d;
}

hipEvent_t prof_event() {
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr;
    int kernel, level;
    double bytes;
    hipStream_t s;
    // level: the recursion level of the launch (for the base case, the level whose pass made its
    // buckets)
    ProfScope(int k, int lv, double by, hipStream_t st) : kernel(k), level(lv), bytes(by), s(st) {
        if ((g_prof.mask & (1 << k)) && !t_arena) {
            {
                std::lock_guard<std::mutex> g(g_prof_mu);
                a = prof_event();
            }
            (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b;
            {
                std::lock_guard<std::mutex> g(g_prof_mu);
                b = prof_event();
            }
            (void)hipEventRecord(b, s);
            std::lock_guard<std::mutex> g(g_prof_mu);
            g_prof.pending.push_back({a, b, kernel, level, bytes});
        }
    }
};

static int prof_level(int level) { return level < 0 ? 0 : level < Prof::kLevels ? level : Prof::kLevels - 1; }

// Bytes of a kernel known only after its launch was recorded (the class bytes a scatter wrote).
void prof_add_bytes(int kernel, int level, double bytes) {
    if (!(g_prof.mask & (1 << kernel))) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.bytes[kernel] += bytes;
    g_prof.lv_bytes[kernel][prof_level(level)] += bytes;
}

// Accumulates the finished records (the caller has synchronised the streams they were on).
void prof_collect() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    std::vector<Prof::Rec> keep;
    for (auto& r : g_prof.pending) {
        if (hipEventQuery(r.b) != hipSuccess) {  // still running on another context's stream
            (void)hipGetLastError();
            keep.push_back(r);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof.launches[r.kernel] += 1;
            g_prof.ms[r.kernel] += ms;
            g_prof.bytes[r.kernel] += r.bytes;
            const int lv = prof_level(r.level);
            g_prof.lv_launches[r.kernel][lv] += 1;
            g_prof.lv_ms[r.kernel][lv] += ms;
            g_prof.lv_bytes[r.kernel][lv] += r.bytes;
        }
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.pending.swap(keep);
}

// With IPLS_VERBOSE set in the environment, a failed HIP call is reported on stderr (source line
// and HIP's error name) before the entry point returns IPLS_ERR_HIP.
void report_hip_failure(int line, hipError_t e) {
    static const bool verbose = std::getenv("IPLS_VERBOSE") != nullptr;
    if (verbose) std::fprintf(stderr, "ipls: HIP call at ipls_lib.hip:%d failed: %s\n", line, hipGetErrorName(e));
}

// The runtime keeps a thread's last error until it is read, including a "not ready" from the
// caller's own queries; each entry point reads it off before its first launch check.
inline void clear_stale_error() { (void)hipGetLastError(); }

#define HIP_TRY(x)                                 \
    do {                                           \
        const hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) {                    \
            report_hip_failure(__LINE__, e_);      \
            (void)hipGetLastError();               \
            return IPLS_ERR_HIP;                   \
        }                                          \
    } while (0)
#define ST_TRY(x)                     \
    do {                              \
        ipls_status st_ = (x);        \
        if (st_ != IPLS_OK) return st_; \
    } while (0)
#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

// Waits until stream s has run the k_plan launch numbered seq.  The host polls the plan's number in
// the pinned buffer, which k_plan writes last (a stream synchronisation wakes the host some tens of
// microseconds after the kernel ends); every 256 polls it asks the stream, which ends the wait on an
// error, or once the stream has drained without the number showing (the caller then copies the
// plan instead).
static hipError_t wait_plan(hipStream_t s, const volatile Plan* ph, uint64_t seq) {
    for (uint32_t i = 1;; ++i) {
        if (ph->seq == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return hipSuccess;
        }
        if ((i & 255) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q != hipErrorNotReady) return q;
            (void)hipGetLastError();  // the runtime keeps "not ready" as the thread's last error
        }
    }
}

int fit_rounds(uint64_t max_S) {
    uint64_t L = max_S / 3;
    int r = 0;
    while (L > 0) {
        ++r;
        L = (L <= kCand) ? 0 : L / (kCand + 1);
    }
    return r;
}

size_t key_bytes(int dt) { return dt == IPLS_F32 ? 4 : 8; }

struct Run {
    ipls_params p;
    hipStream_t s;
    ipls_stats st;
    int dtype;
    // ipls_partition: stop after the first level and export its result
    uint64_t* part_counts = nullptr;
    ipls_linear_model* part_model = nullptr;
    bool single_pass = false;
};

// FMCD fit of every item's sorted sample: one workgroup per small sample, rounds of candidate
// widths over chunks of the large samples.
template <int DT>
ipls_status fit_level(Depth& D, hipStream_t s, uint64_t ni, uint64_t max_S, uint64_t total_fit_chunks,
                      const typename Key<DT>::T* sample, const uint64_t* sample_off, const uint64_t* fit_off,
                      Model* models, uint32_t K, const EqInfo* eq = nullptr, FitGate gate = {nullptr, nullptr, 0}) {
    if (max_S <= (uint64_t)kFitLdsTiny)
        k_fmcd_small<DT, kFitLdsTiny><<<(unsigned)ni, 256, 0, s>>>(sample, sample_off, ni, models, K, kSmallS, eq, gate);
    else if (max_S <= (uint64_t)kFitLdsSmall)
        k_fmcd_small<DT, kFitLdsSmall><<<(unsigned)ni, 256, 0, s>>>(sample, sample_off, ni, models, K, kSmallS, eq,
                                                                   gate);
    else
        k_fmcd_small<DT, kFitLds><<<(unsigned)ni, 256, 0, s>>>(sample, sample_off, ni, models, K, kSmallS, eq, gate);
    LAUNCH_CHECK();
    if (max_S <= kSmallS) return IPLS_OK;
    const int R = fit_rounds(max_S);
    ST_TRY(ensure(D.masks, ni * R * 8));
    ST_TRY(ensure(D.fit_map, total_fit_chunks * 4));
    HIP_TRY(hipMemsetAsync(D.masks.p, 0, ni * R * 8, s));
    k_expand<<<(unsigned)((total_fit_chunks + 255) / 256), 256, 0, s>>>(fit_off, ni, total_fit_chunks,
                                                                        (uint32_t*)D.fit_map.p);
    LAUNCH_CHECK();
    for (int r = 0; r < R; ++r) {
        k_fmcd_round<DT><<<(unsigned)total_fit_chunks, 256, 0, s>>>(sample, sample_off, fit_off,
                                                                    (const uint32_t*)D.fit_map.p,
                                                                    (uint64_t*)D.masks.p, R, r, K, kFitChunk, kCand,
                                                                    eq);
        LAUNCH_CHECK();
    }
    k_fmcd_finish<DT><<<(unsigned)((ni + 255) / 256), 256, 0, s>>>(sample, sample_off, ni, (const uint64_t*)D.masks.p,
                                                                   R, models, K, kSmallS, kCand, eq);
    LAUNCH_CHECK();
    return IPLS_OK;
}

// Two-level model of every item whose FMCD fit is usable: root fit onto M leaves, leaf ranges,
// per-leaf training (one wave per leaf), envelope, and the max sample loads of both models.
// grad mode (ab_in set): one item, evaluate the loss gradient at ab_in instead of training.
template <int DT>
ipls_status train_l2pl(Depth& D, hipStream_t s, uint64_t ni, uint64_t max_S, uint64_t total_fit_chunks,
                       const typename Key<DT>::T* sample, const uint64_t* sample_off, const uint64_t* fit_off,
                       Model* models, uint32_t K, uint32_t M, uint32_t iters, const double* ab_in = nullptr,
                       double* grad_out = nullptr, double* loss_out = nullptr, double* ab_out = nullptr,
                       const Item* items = nullptr, uint32_t gate_T = 0) {
    ST_TRY(ensure(D.roots, ni * sizeof(Model)));
    ST_TRY(ensure(D.leaf_first, ni * (M + 1) * 4));
    ST_TRY(ensure(D.leaves, ni * 4 * kMaxLeaves * 8));
    ST_TRY(ensure(D.leaf_last, ni * kMaxLeaves * 8));
    Model* roots = (Model*)D.roots.p;
    ST_TRY((fit_level<DT>(D, s, ni, max_S, total_fit_chunks, sample, sample_off, fit_off, roots, M, nullptr,
                          FitGate{models, items, items ? gate_T : 0u})));
    k_l2pl_bounds<DT><<<(unsigned)ni, 256, 0, s>>>(sample, sample_off, ni, models, roots, M,
                                                   (uint32_t*)D.leaf_first.p, items, items ? gate_T : 0u);
    LAUNCH_CHECK();
    k_l2pl_train<DT><<<(unsigned)((ni * M + 3) / 4), 256, 0, s>>>(
        sample, sample_off, ni, models, roots, (const uint32_t*)D.leaf_first.p, K, M, iters, (double*)D.leaves.p,
        (double*)D.leaf_last.p, ab_in, grad_out, loss_out, ab_out);
    LAUNCH_CHECK();
    if (ab_in) return IPLS_OK;
    k_l2pl_envelope<<<(unsigned)ni, 64, 0, s>>>(ni, models, roots, (const uint32_t*)D.leaf_first.p, M,
                                                (double*)D.leaves.p, (const double*)D.leaf_last.p);
    LAUNCH_CHECK();
    k_l2pl_load<DT><<<(unsigned)ni, 256, 0, s>>>(sample, sample_off, ni, models, roots, (const double*)D.leaves.p, K,
                                                 M);
    LAUNCH_CHECK();
    return IPLS_OK;
}

template <int DT, bool PAY>
ipls_status sort_segments(Device& dv, Run& run, int d, typename Key<DT>::T* keys, uint32_t* pay, uint64_t len,
                          const uint64_t* seg_off, uint64_t nseg, void* ws_keys, bool top);

// Base-case sort of `count` buckets of size class cls (<= 64 * 2^cls keys).  Classes 0..3: merge sort, 16 keys per thread,
// NT = 4 * 2^cls threads per bucket, 256 / NT buckets per workgroup.
template <int DT, bool PAY, int NT>
ipls_status launch_base_nt(hipStream_t s, const BaseItem* list, uint64_t count, typename Key<DT>::T* keys,
                           uint32_t* pay, const typename Key<DT>::T* sk, const uint32_t* sp) {
    constexpr uint64_t G = kBlock / NT;
    k_base_sort<DT, PAY, NT><<<(unsigned)((count + G - 1) / G), kBlock, 0, s>>>(list, count, keys, pay, sk, sp);
    LAUNCH_CHECK();
    return IPLS_OK;
}

// VMAP (keys only): the large classes count skewed buckets again by value (used for samples).
template <int DT, bool PAY, bool VMAP = false>
ipls_status launch_base(hipStream_t s, int cls, const BaseItem* list, uint64_t count, typename Key<DT>::T* keys,
                        uint32_t* pay, const typename Key<DT>::T* sk, const uint32_t* sp) {
    if (count == 0) return IPLS_OK;
    switch (cls) {
        case 0: return launch_base_nt<DT, PAY, 4>(s, list, count, keys, pay, sk, sp);
        case 1: return launch_base_nt<DT, PAY, 8>(s, list, count, keys, pay, sk, sp);
        case 2: return launch_base_nt<DT, PAY, 16>(s, list, count, keys, pay, sk, sp);
        case 3: return launch_base_nt<DT, PAY, 32>(s, list, count, keys, pay, sk, sp);
        case 4:
            k_base_large<DT, PAY, 2, 8, VMAP><<<(unsigned)count, 128, 0, s>>>(list, count, keys, pay, sk, sp);
            LAUNCH_CHECK();
            return IPLS_OK;
        case 5:
            k_base_large<DT, PAY, 4, 8, VMAP><<<(unsigned)count, 256, 0, s>>>(list, count, keys, pay, sk, sp);
            LAUNCH_CHECK();
            return IPLS_OK;
        default:
            k_base_large<DT, PAY, 8, 8, VMAP><<<(unsigned)count, 512, 0, s>>>(list, count, keys, pay, sk, sp);
            LAUNCH_CHECK();
            return IPLS_OK;
    }
}

// The merge-sort classes 0..3 of a level's base-case lists (at list + off[c], count[c] buckets each)
// in one launch.
template <int DT, bool PAY>
ipls_status launch_base_small(hipStream_t s, const BaseItem* list, const BaseLayout& bl, const uint64_t* count,
                              typename Key<DT>::T* keys, uint32_t* pay, const typename Key<DT>::T* sk,
                              const uint32_t* sp) {
    static_assert(kBaseClasses > 4, "classes 0..3 are the merge sorts");
    BaseSmall a;
    uint64_t g = 0;
    for (int c = 0; c < 4; ++c) {
        const uint64_t G = (uint64_t)kBlock / (4u << c);  // buckets per workgroup
        a.list[c] = list + bl.off[c];
        a.count[c] = count[c];
        a.first[c] = g;
        g += (count[c] + G - 1) / G;
    }
    a.first[4] = g;
    if (g == 0) return IPLS_OK;
    k_base_sort_small<DT, PAY><<<(unsigned)g, kBlock, 0, s>>>(a, keys, pay, sk, sp);
    LAUNCH_CHECK();
    return IPLS_OK;
}

// Sort the samples of a level: base case when every sample fits, else the engine one level deeper.
template <int DT>
ipls_status sort_samples(Device& dv, Run& run, int d, const Plan& pl, typename Key<DT>::T* sample) {
    Depth& D = dv.depth[d];
    hipStream_t s = run.s;
    if (pl.max_S <= run.p.base_case_max) {
        // k_plan has written every sample as a base-case bucket of the sample buffer
        return launch_base<DT, false, true>(s, base_class((uint32_t)pl.max_S), (const BaseItem*)D.sample_base.p,
                                      pl.num_items, sample, nullptr, nullptr, nullptr);
    }
    if (d + 1 >= kMaxDepth) return IPLS_ERR_DEVICE;
    run.st.sample_depth = std::max<uint32_t>(run.st.sample_depth, (uint32_t)(d + 1));
    return sort_segments<DT, false>(dv, run, d + 1, sample, nullptr, pl.total_samples,
                                    (const uint64_t*)D.sample_off.p, pl.num_items, nullptr, false);
}

template <int DT, bool PAY>
ipls_status sort_segments(Device& dv, Run& run, int d, typename Key<DT>::T* keys, uint32_t* pay, uint64_t len,
                          const uint64_t* seg_off, uint64_t nseg, void* ws_keys, bool top) {
    using T = typename Key<DT>::T;
    Depth& D = dv.depth[d];
    const ipls_params& P = run.p;
    hipStream_t s = run.s;
    const uint32_t K = P.num_buckets, T_ = P.base_case_max;
    const size_t kb = sizeof(T);
    const uint64_t item_cap = len / (T_ + 1) + 1;
    BaseLayout bl;
    bl.off[0] = 0;
    for (int c = 0; c < kBaseClasses; ++c) {
        bl.cap[c] = c == 0 ? std::min<uint64_t>(len, item_cap * K + nseg) + 1 : len / (32ull << c) + 1;
        bl.off[c + 1] = bl.off[c] + bl.cap[c];
    }
    const uint64_t base_cap = bl.off[kBaseClasses];

    T* scratch;
    uint32_t* spay = nullptr;
    if (ws_keys) {
        scratch = (T*)ws_keys;
        if (PAY) spay = (uint32_t*)((char*)ws_keys + ((len * kb + 255) & ~(size_t)255));
    } else {
        ST_TRY(ensure(D.scratch, len * kb));
        scratch = (T*)D.scratch.p;
        if (PAY) {
            ST_TRY(ensure(D.spay, len * 4));
            spay = (uint32_t*)D.spay.p;
        }
    }
    ST_TRY(ensure(D.items[0], item_cap * sizeof(Item)));
    ST_TRY(ensure(D.items[1], item_cap * sizeof(Item)));
    const uint64_t copy_cap = P.equality ? item_cap * kMaxHeavy + 1 : 1;  // equality buckets per level
    ST_TRY(ensure(D.copy, copy_cap * sizeof(CopyItem)));
    ST_TRY(ensure(D.copy_off, (copy_cap + 1) * 8));
    ST_TRY(ensure(D.base[0], base_cap * sizeof(BaseItem)));
    ST_TRY(ensure(D.base[1], base_cap * sizeof(BaseItem)));
    // Base-case lists alternate by level parity: level L's worklist writes base[L & 1], which the
    // base launch of level L + 1 reads (the seeds count as level -1).  The top-level sort runs those
    // launches on the side stream; the main stream waits for them only before the list is written
    // again, two levels later, and at the end of the sort.
    const bool overlap = top && !dv.noalloc;
    if (overlap && !dv.side) {
        HIP_TRY(hipStreamCreateWithFlags(&dv.side, hipStreamNonBlocking));
        for (hipEvent_t* e : {&dv.ev_base[0], &dv.ev_base[1], &dv.ev_defer})
            HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    }
    hipStream_t sb = overlap ? dv.side : s;  // stream of the base-case launches
    bool base_pending[2] = {false, false};   // a side-stream base launch read base[parity]
    auto join = [&]() -> ipls_status {       // the main stream continues after the base case
        for (int q = 0; q < 2; ++q)
            if (base_pending[q]) {
                if (hipStreamWaitEvent(s, dv.ev_base[q], 0) != hipSuccess) return IPLS_ERR_HIP;
                base_pending[q] = false;
            }
        return IPLS_OK;
    };
    ST_TRY(ensure(D.counters, C_N * sizeof(uint64_t)));
    ST_TRY(ensure(D.plan, sizeof(Plan)));
    ST_TRY(ensure(D.tile_off, (item_cap + 1) * 8));
    ST_TRY(ensure(D.sample_off, (item_cap + 1) * 8));
    ST_TRY(ensure(D.fit_off, (item_cap + 1) * 8));
    ST_TRY(ensure(D.chunk_off, (item_cap + 1) * 8));
    ST_TRY(ensure(D.sample_base, item_cap * sizeof(BaseItem)));
    ST_TRY(ensure(D.wide, item_cap * 4));
    if (!D.plan_h && dv.noalloc) {
        D.plan_h = &D.plan_copy;
        D.plan_hd = nullptr;
    } else if (!D.plan_h) {
        HIP_TRY(hipHostMalloc((void**)&D.plan_h, sizeof(Plan), hipHostMallocMapped | hipHostMallocCoherent));
        std::memset(D.plan_h, 0, sizeof(Plan));
        HIP_TRY(hipHostGetDevicePointer((void**)&D.plan_hd, D.plan_h, 0));
    }
    uint64_t* cnt = (uint64_t*)D.counters.p;
    // sample inheritance: samples and child lists alternate between two buffers by level parity
    // (a level reads its parent level's); one class byte per key
    const bool inherit = P.inherit && !run.single_pass;
    const uint64_t thr = std::max<uint64_t>(3, P.sample_min ? P.sample_min : 2ull * K);
    if (inherit) ST_TRY(ensure(D.cls, len + 16));  // the counting pass reads whole aligned words
    uint8_t* cls = inherit ? (uint8_t*)D.cls.p : nullptr;

    HIP_TRY(hipMemsetAsync(cnt, 0, C_N * sizeof(uint64_t), s));
    // IPLS_DEBUG_CHECKS: the input's multiset hash before anything moves (top-level sorts that may
    // allocate; the checks' buffers come from the cache)
    const int dbg = (top && !dv.noalloc) ? debug_checks() : 0;
    const unsigned dbg_grid = (unsigned)std::min<uint64_t>((len + 255) / 256, 4096);
    if (dbg) {
        ST_TRY(ensure(D.dbg_all, 4 * sizeof(uint64_t)));
        k_dbg_zero<<<1, 64, 0, s>>>((uint64_t*)D.dbg_all.p, 4);
        k_dbg_hash_all<DT, PAY><<<dbg_grid, 256, 0, s>>>(keys, pay, len, (uint64_t*)D.dbg_all.p);
        LAUNCH_CHECK();
    }
    k_seed<<<(unsigned)((nseg + 255) / 256), 256, 0, s>>>(seg_off, nseg, T_, (Item*)D.items[0].p,
                                                          (BaseItem*)D.base[1].p, bl, cnt, item_cap);
    LAUNCH_CHECK();

    LevelArgs A;
    A.K = K;
    A.T = T_;
    A.M = P.leaves;
    A.div = P.sample_divisor;
    A.smin = P.sample_min ? P.sample_min : (P.sample_policy == 1 ? 0 : 2ull * K);
    A.smax = P.sample_max;
    // the bucket policy: the plain FMCD line of a sort (a single pass keeps K)
    const bool adapt = P.bucket_policy && P.model == 0 && !P.equality && !inherit && !run.single_pass;
    A.adapt = adapt ? 1u : 0u;
    A.smin_param = P.sample_min;
    A.policy = P.sample_policy;
    A.seed = P.seed;
    const uint32_t tile = tile_keys_of(P);
    static_assert((kTile & (kTile - 1)) == 0 && (kSmallTile & (kSmallTile - 1)) == 0 &&
                      (kChunk & (kChunk - 1)) == 0 && (kFitChunk & (kFitChunk - 1)) == 0,
                  "k_plan divides by shifts");
    A.tile_keys = tile;
    A.small_S = kSmallS;
    A.fit_chunk = kFitChunk;
    A.cand = kCand;
    A.chunk = kChunk;

    int cur = 0;
    uint64_t prev_items = 0, prev_sum_n = 0, prev_closed = 0, prev_closed_keys = 0;
    for (int level = 0;; ++level) {
        const int par = level & 1;
        const Child* prev_children = (inherit && level > 0) ? (const Child*)D.children[par ^ 1].p : nullptr;
        k_plan<<<1, 256, 0, s>>>((const Item*)D.items[cur].p, cnt, cur, (Plan*)D.plan.p, (uint64_t*)D.tile_off.p, (uint64_t*)D.sample_off.p,
                                  (uint64_t*)D.fit_off.p, (uint64_t*)D.chunk_off.p, A, item_cap, bl,
                                  (const CopyItem*)D.copy.p, (uint64_t*)D.copy_off.p, copy_cap, prev_children,
                                  D.plan_hd, ++D.plan_seq, (BaseItem*)D.sample_base.p, (uint32_t*)D.wide.p);
        LAUNCH_CHECK();
        if (D.plan_hd) HIP_TRY(wait_plan(s, (const volatile Plan*)D.plan_h, D.plan_seq));
        if (((volatile Plan*)D.plan_h)->seq != D.plan_seq) {
            // not visible yet through the mapped buffer: copy the device's plan instead
            HIP_TRY(hipMemcpyAsync(D.plan_h, D.plan.p, sizeof(Plan), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (D.plan_h->seq != D.plan_seq) {
                ST_TRY(join());
                return IPLS_ERR_DEVICE;
            }
        }
        const Plan pl = *D.plan_h;
        if (pl.err) {
            ST_TRY(join());
            return IPLS_ERR_DEVICE;
        }
        if (top && inherit) prof_add_bytes(0, level - 1, (double)pl.inh_n);  // class bytes the last scatter wrote
        if (top && level > 0) {
            // the previous level's buckets that were not closed were partitioned
            const uint64_t closed_now = pl.closed - prev_closed;
            if (prev_items > closed_now) {
                run.st.levels = level;
                run.st.passes += prev_items - closed_now;
                run.st.keys_partitioned += prev_sum_n - (pl.closed_keys - prev_closed_keys);
            }
            run.st.closed = pl.closed + pl.eq_closed;
            run.st.inherited = pl.inherited;
            if (level == 1) run.st.level1_max_load = pl.l1max;
            run.st.fallback = pl.digit;
            run.st.l2pl_used = pl.l2pl;
            prev_closed = pl.closed;
            prev_closed_keys = pl.closed_keys;
        }
        if (pl.copy_count) {
            // equality buckets the previous level left in the scratch buffer
            ST_TRY(ensure(D.copy_map, pl.copy_tiles * 4));
            k_expand<<<(unsigned)((pl.copy_tiles + 255) / 256), 256, 0, s>>>((const uint64_t*)D.copy_off.p,
                                                                             pl.copy_count, pl.copy_tiles,
                                                                             (uint32_t*)D.copy_map.p);
            LAUNCH_CHECK();
            k_copy<DT, PAY><<<(unsigned)pl.copy_tiles, 256, 0, s>>>((const CopyItem*)D.copy.p,
                                                                    (const uint64_t*)D.copy_off.p,
                                                                    (const uint32_t*)D.copy_map.p, pl.copy_tiles,
                                                                    keys, pay, scratch, spay);
            LAUNCH_CHECK();
        }
        // the previous level's buckets of <= T keys: base[(level - 1) & 1], complete (the host has
        // just seen the plan, so the main stream's earlier work is done)
        const int bp = (level + 1) & 1;
        auto launch_level_base = [&](hipStream_t sl) -> ipls_status {
            ProfScope ps(2, level - 1, (double)pl.base_keys * 2.0 * (kb + (PAY ? 4 : 0)), sl);
            ST_TRY((launch_base_small<DT, PAY>(sl, (const BaseItem*)D.base[bp].p, bl, pl.cls_count, keys, pay, scratch,
                                               spay)));
            for (int c = 4; c < kBaseClasses; ++c)
                ST_TRY((launch_base<DT, PAY>(sl, c, (const BaseItem*)D.base[bp].p + bl.off[c], pl.cls_count[c], keys,
                                             pay, scratch, spay)));
            return IPLS_OK;
        };
        // They go to the side stream while another level follows on the main stream; the last
        // level's go to the main stream, beside the side stream's earlier (larger) base-case
        // launch, whose tail leaves most of the device idle.  The launch waits for the coming
        // level's worklist when that level has many items (its latency-bound per-item kernels
        // would otherwise wait for CUs held by the base case's large-LDS workgroups) or holds at
        // least 1/64 as many keys as the base case (its counting and scatter then stream at the
        // device's full bandwidth instead of sharing it); a level of a few keys runs beside it.
        const bool side = overlap && pl.num_items > 0;
        const bool defer_base = side && pl.num_base &&
                                (pl.num_items >= kDeferBaseItems || pl.sum_n * kDeferBaseShare >= pl.base_keys);
        if (pl.num_base && !defer_base) {
            ST_TRY(launch_level_base(side ? sb : s));
            if (side) {
                HIP_TRY(hipEventRecord(dv.ev_base[bp], sb));
                base_pending[bp] = true;
            }
        }
        if (top) run.st.base_buckets += pl.num_base;
        if (pl.num_items == 0) break;
        if (level + 1 > kMaxLevels) {
            ST_TRY(join());
            return IPLS_ERR_DEVICE;
        }
        const bool src_scratch = (level & 1) != 0;
        T* src = src_scratch ? scratch : keys;
        T* dst = src_scratch ? keys : scratch;
        uint32_t* psrc = src_scratch ? spay : pay;
        uint32_t* pdst = src_scratch ? pay : spay;
        prev_items = pl.num_items;
        prev_sum_n = pl.sum_n;

        const uint64_t ni = pl.num_items, nt = pl.total_tiles;
        ST_TRY(ensure(D.tile_map, nt * sizeof(TileInfo)));
        Buf& sbuf = (inherit && par) ? D.sample2 : D.sample;
        ST_TRY(ensure(sbuf, pl.total_samples * kb));
        T* sample = (T*)sbuf.p;
        const T* prev_sample = (inherit && level > 0) ? (const T*)(par ? D.sample.p : D.sample2.p) : nullptr;
        ST_TRY(ensure(D.models, ni * sizeof(Model)));
        ST_TRY(ensure(D.hist, ni * K * 8));
        ST_TRY(ensure(D.bstart, ni * K * 8));
        const uint64_t nc = pl.total_chunks;
        ST_TRY(ensure(D.chunk_map, nc * 4));
        ST_TRY(ensure(D.tile_pref, nt * K * 4));
        ST_TRY(ensure(D.chunk_sum, nc * K * 4));
        ST_TRY(ensure(D.chunk_pref, nc * K * 8));
        const Item* items = (const Item*)D.items[cur].p;
        Model* models = (Model*)D.models.p;

        const uint64_t eb = (std::max(nt, nc) + 255) / 256;
        const EqInfo* eq = nullptr;
        const uint32_t* tree = nullptr;
        if (P.model == 0 && !P.equality && !inherit && pl.max_S <= (uint64_t)kFitLdsFused) {
            // the plain FMCD line on samples of at most 2048 keys (the deeper levels' items): gather,
            // sort and fit in one launch, with the tile and chunk maps (a workgroup's bitonic sort of
            // a larger sample takes longer than the three launches)
            auto ksf = pl.max_S <= (uint64_t)kFitLdsTiny ? k_sample_fit<DT, kFitLdsTiny> : k_sample_fit<DT, kFitLdsFused>;
            ksf<<<(unsigned)(eb + ni), 256, 0, s>>>(
                items, ni, (const uint64_t*)D.sample_off.p, src, P.seed, models, K, eb, (const uint64_t*)D.tile_off.p,
                nt, (TileInfo*)D.tile_map.p, tile, (const uint64_t*)D.chunk_off.p, nc, (uint32_t*)D.chunk_map.p,
                adapt ? T_ : 0u);
            LAUNCH_CHECK();
        } else {
            // the sample gather and the tile and chunk maps, in one launch
            k_sample<DT><<<(unsigned)(eb + (pl.total_samples + 255) / 256), 256, 0, s>>>(
                items, ni, (const uint64_t*)D.sample_off.p, pl.total_samples, src, sample, P.seed, prev_children,
                prev_sample, eb, (const uint64_t*)D.tile_off.p, nt, (TileInfo*)D.tile_map.p, tile,
                (const uint64_t*)D.chunk_off.p, nc, (uint32_t*)D.chunk_map.p);
            LAUNCH_CHECK();
            ST_TRY(sort_samples<DT>(dv, run, d, pl, sample));

            // FMCD fit (with equality buckets: on the sample without the heavy values' runs)
            if (P.equality) {
                ST_TRY(ensure(D.eqinfo, ni * sizeof(EqInfo)));
                ST_TRY(ensure(D.rsample, pl.total_samples * kb));
                k_heavy<DT><<<(unsigned)ni, 256, 0, s>>>((const T*)sample, (const uint64_t*)D.sample_off.p, ni, K,
                                                         (EqInfo*)D.eqinfo.p, (T*)D.rsample.p);
                LAUNCH_CHECK();
                eq = (const EqInfo*)D.eqinfo.p;
            }
            ST_TRY((fit_level<DT>(D, s, ni, pl.max_S, pl.total_fit_chunks,
                                  eq ? (const T*)D.rsample.p : (const T*)sample, (const uint64_t*)D.sample_off.p,
                                  (const uint64_t*)D.fit_off.p, models, K, eq,
                                  FitGate{nullptr, items, 0u, adapt ? T_ : 0u})));
            if (P.model == 3) {
                ST_TRY(ensure(D.leaves, ni * 4 * kMaxLeaves * 8));
                ST_TRY(ensure(D.treeflag, ni * 4));
                k_tree<DT><<<(unsigned)ni, 256, 0, s>>>((const T*)sample, (const uint64_t*)D.sample_off.p, ni, K,
                                                        (double*)D.leaves.p, (uint32_t*)D.treeflag.p);
                LAUNCH_CHECK();
                tree = (const uint32_t*)D.treeflag.p;
            }
            // the auto policy trains an item only if D n > T S.  D <= S/3 + 1 and every sample holds
            // at least s0 keys (the sample minimum, or the cap below it; items have more than
            // T >= s0 keys), so a level whose largest item has n (s0 + 3) <= 3 T s0 trains none and
            // skips the launches
            uint64_t s0 = P.sample_min ? P.sample_min : 2ull * K;
            if (P.sample_max && P.sample_max < s0) s0 = P.sample_max;
            const bool none_trained = P.model == 1 && P.sample_policy == 0 && s0 > 0 &&
                                      pl.max_n * (s0 + 3) <= 3ull * T_ * s0;
            if ((P.model == 1 && !none_trained) || P.model == 2)
                ST_TRY((train_l2pl<DT>(D, s, ni, pl.max_S, pl.total_fit_chunks, (const T*)sample,
                                       (const uint64_t*)D.sample_off.p, (const uint64_t*)D.fit_off.p, models, K, P.leaves,
                                       P.train_iters, nullptr, nullptr, nullptr, nullptr, items,
                                       P.model == 1 ? T_ : 0u)));
        }

        // degenerate buckets and final model
        k_minmax<DT><<<(unsigned)nc, 256, 0, s>>>(items, (const uint64_t*)D.chunk_off.p, (const uint32_t*)D.chunk_map.p,
                                                  models, src, tile, kChunk);
        LAUNCH_CHECK();
        k_finalize<DT><<<(unsigned)((ni + 255) / 256), 256, 0, s>>>(items, models, (const Model*)D.roots.p, ni, K,
                                                                src_scratch ? 1 : 0, P.model,
                                                                cnt + C_STATS, eq, tree, prev_children);
        LAUNCH_CHECK();

        // classify + per-tile counts, scan of the counts, bucket starts
        {
            ProfScope ps(1, level, (double)(pl.sum_n - pl.inh_n) * kb + (double)pl.inh_n, s);
            if (!cls) {
                // a workgroup per tile, then the prefixes inside each chunk
                auto kt = tile == kTile ? k_count_tile<DT, 8, kPassIPT> : k_count_tile<DT, 4, kPassIPT>;
                kt<<<(unsigned)nt, tile / kPassIPT, 0, s>>>((const TileInfo*)D.tile_map.p, nt,
                                                            models, (const double*)D.leaves.p, src,
                                                            (uint32_t*)D.tile_pref.p, K, P.leaves);
                LAUNCH_CHECK();
                k_chunk_prefix<<<(unsigned)nc, 256, 0, s>>>((const uint64_t*)D.tile_off.p, (const uint64_t*)D.chunk_off.p, (const uint32_t*)D.chunk_map.p, nc,
                                                            (uint32_t*)D.tile_pref.p, (uint32_t*)D.chunk_sum.p, K);
                LAUNCH_CHECK();
            } else {
                auto kc = tile == kTile ? k_classify_hist<DT, 8, kPassIPT> : k_classify_hist<DT, 4, kPassIPT>;
                kc<<<(unsigned)nc, tile / kPassIPT, 0, s>>>(
                    items, (const uint64_t*)D.tile_off.p, (const uint64_t*)D.chunk_off.p, (const uint32_t*)D.chunk_map.p,
                    nc, models, (const double*)D.leaves.p, src, (uint32_t*)D.tile_pref.p, (uint32_t*)D.chunk_sum.p, K,
                    P.leaves, cls);
                LAUNCH_CHECK();
            }
        }
        // chunk prefixes, bucket sizes and bucket starts: a workgroup per item; wide items by a
        // workgroup per (item, bucket), then their starts
        k_scan_chunks<<<(unsigned)ni, 256, 0, s>>>((const uint64_t*)D.chunk_off.p, K, (const uint32_t*)D.chunk_sum.p,
                                                   (uint64_t*)D.chunk_pref.p, (uint64_t*)D.hist.p,
                                                   (uint64_t*)D.bstart.p);
        LAUNCH_CHECK();
        if (pl.n_wide) {
            k_scan_chunks_wide<<<(unsigned)(pl.n_wide * K), 256, 0, s>>>(
                (const uint64_t*)D.chunk_off.p, (const uint32_t*)D.wide.p, K, (const uint32_t*)D.chunk_sum.p,
                (uint64_t*)D.chunk_pref.p, (uint64_t*)D.hist.p);
            LAUNCH_CHECK();
            k_bucket_starts<<<(unsigned)pl.n_wide, 256, 0, s>>>((const uint64_t*)D.hist.p, (uint64_t*)D.bstart.p, K,
                                                                (const uint32_t*)D.wide.p);
            LAUNCH_CHECK();
        }

        // children that inherit their part of the sample: ranges, then their lines (before the scatter,
        // which writes the class bytes).  Each entry holds at least thr sample keys and more than T
        // keys, which bounds the list.
        const ChildSpan* spans = nullptr;
        Child* children = nullptr;
        if (inherit) {
            const uint64_t ccap = std::min<uint64_t>(pl.total_samples / thr, pl.sum_n / ((uint64_t)T_ + 1)) + 1;
            ST_TRY(ensure(D.children[par], ccap * sizeof(Child)));
            ST_TRY(ensure(D.spans, ni * sizeof(ChildSpan)));
            children = (Child*)D.children[par].p;
            spans = (const ChildSpan*)D.spans.p;
            k_child_split<DT><<<(unsigned)ni, 256, 0, s>>>(ni, models, sample, (const uint64_t*)D.sample_off.p,
                                                           (const uint64_t*)D.hist.p, K, T_, thr,
                                                           (ChildSpan*)D.spans.p, children, cnt, ccap);
            LAUNCH_CHECK();
            k_child_fit<DT><<<(unsigned)ccap, 256, 0, s>>>(children, cnt, ccap, sample, K);
            LAUNCH_CHECK();
        }

        // scatter
        {
            ProfScope ps(0, level, (double)pl.sum_n * 2.0 * (kb + (PAY ? 4 : 0)), s);
            auto ks = inherit ? (tile == kTile ? k_scatter<DT, PAY, 8, kPassIPT, true> : k_scatter<DT, PAY, 4, kPassIPT, true>)
                              : (tile == kTile ? k_scatter<DT, PAY, 8, kPassIPT, false>
                                               : k_scatter<DT, PAY, 4, kPassIPT, false>);
            ks<<<(unsigned)nt, tile / kPassIPT, 0, s>>>(
                items, (const TileInfo*)D.tile_map.p, nt, (const uint64_t*)D.chunk_off.p,
                nc, models, (const double*)D.leaves.p, (const uint64_t*)D.bstart.p, (const uint64_t*)D.chunk_pref.p,
                (const uint32_t*)D.tile_pref.p, src, psrc, dst, pdst, K, P.leaves, spans, children, cls);
            LAUNCH_CHECK();
        }
        if (dbg) {
            // the pass's invariants; a failure shows in the next level's plan
            ST_TRY(ensure(D.dbg_acc, ni * 4 * sizeof(uint64_t)));
            uint64_t* acc = (uint64_t*)D.dbg_acc.p;
            k_dbg_zero<<<(unsigned)((4 * ni + 255) / 256), 256, 0, s>>>(acc, 4 * ni);
            k_dbg_hash_tiles<DT, PAY><<<(unsigned)nt, 256, 0, s>>>((const TileInfo*)D.tile_map.p, nt, models, src, psrc,
                                                                   acc);
            k_dbg_hash_tiles<DT, PAY><<<(unsigned)nt, 256, 0, s>>>((const TileInfo*)D.tile_map.p, nt, models, dst, pdst,
                                                                   acc + 2 * ni);
            k_dbg_place<DT><<<(unsigned)nt, 256, 0, s>>>((const TileInfo*)D.tile_map.p, nt, items, models,
                                                        (const double*)D.leaves.p, dst, (const uint64_t*)D.bstart.p,
                                                        K, P.leaves, cnt + C_ERR);
            k_dbg_level<<<(unsigned)((ni + 255) / 256), 256, 0, s>>>(items, ni, models, (const uint64_t*)D.hist.p, K,
                                                                     acc, acc + 2 * ni, cnt + C_ERR);
            LAUNCH_CHECK();
        }
        if (top && level == 0 && run.single_pass) {
            k_export_model<<<1, 1, 0, s>>>(models, run.part_model, K);
            LAUNCH_CHECK();
            HIP_TRY(hipMemcpyAsync(run.part_counts, D.hist.p, K * 8, hipMemcpyDeviceToDevice, s));
            Model m0;
            HIP_TRY(hipMemcpyAsync(&m0, models, sizeof(Model), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ST_TRY(join());
            if (m0.kind != kKindClosedKeep) {
                HIP_TRY(hipMemcpyAsync(keys, scratch, len * kb, hipMemcpyDeviceToDevice, s));
                if (PAY) HIP_TRY(hipMemcpyAsync(pay, spay, len * 4, hipMemcpyDeviceToDevice, s));
            }
            return IPLS_OK;
        }

        // next level; this level's base-case list is base[level & 1], whose last reader may still run
        if (base_pending[par]) {
            HIP_TRY(hipStreamWaitEvent(s, dv.ev_base[par], 0));
            base_pending[par] = false;
        }
        // a wave per item; levels of many items take 16 a workgroup, so that fewer workgroups queue
        // on the same few device counters
        {
            auto kw = ni <= kWorklistFewItems ? k_worklist<4> : k_worklist<16>;
            const uint32_t W = ni <= kWorklistFewItems ? 4 : 16;
            kw<<<(unsigned)((ni + W - 1) / W), kWave * W, 0, s>>>(
                items, ni, models, (const uint64_t*)D.hist.p, (const uint64_t*)D.bstart.p, K, T_, src_scratch ? 0 : 1,
                (Item*)D.items[cur ^ 1].p, (BaseItem*)D.base[par].p, bl, cnt, C_ITEMS0 + (cur ^ 1), item_cap,
                (CopyItem*)D.copy.p, copy_cap, spans, children, (top && level == 0 && ni == 1) ? cnt + C_L1MAX : nullptr);
            LAUNCH_CHECK();
        }
        if (defer_base) {
            HIP_TRY(hipEventRecord(dv.ev_defer, s));
            HIP_TRY(hipStreamWaitEvent(sb, dv.ev_defer, 0));
            ST_TRY(launch_level_base(sb));
            HIP_TRY(hipEventRecord(dv.ev_base[bp], sb));
            base_pending[bp] = true;
        }
        cur ^= 1;
    }
    // the caller's stream completes only after the base case
    ST_TRY(join());
    if (dbg) {
        // the output: sorted segments holding the input's multiset
        uint64_t* all = (uint64_t*)D.dbg_all.p;
        k_dbg_hash_all<DT, PAY><<<dbg_grid, 256, 0, s>>>(keys, pay, len, all + 2);
        k_dbg_sorted<DT><<<dbg_grid, 256, 0, s>>>(keys, len, seg_off, nseg, cnt + C_ERR);
        k_dbg_compare<<<1, 1, 0, s>>>(all, dbg == 2 ? 1 : 0, cnt + C_ERR);
        LAUNCH_CHECK();
        uint64_t e = 0;
        HIP_TRY(hipMemcpyAsync(&e, cnt + C_ERR, sizeof(e), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (e) return IPLS_ERR_DEVICE;
    }
    return IPLS_OK;
}

template <int DT>
ipls_status fit_entry(Device& dv, Run& run, const void* sample, uint64_t S, bool sorted, uint32_t K,
                      ipls_linear_model* out) {
    clear_stale_error();
    using T = typename Key<DT>::T;
    hipStream_t s = run.s;
    Depth& D = dv.depth[0];
    const size_t kb = sizeof(T);
    ST_TRY(ensure(D.sample, std::max<uint64_t>(S, 1) * kb));
    ST_TRY(ensure(D.models, sizeof(Model)));
    ST_TRY(ensure(D.seg, 6 * sizeof(uint64_t)));
    if (S > 0) HIP_TRY(hipMemcpyAsync(D.sample.p, sample, S * kb, hipMemcpyDeviceToDevice, s));
    uint64_t h[4] = {0, S, 0, S > kSmallS ? (S + kFitChunk - 1) / kFitChunk : 0};
    HIP_TRY(hipMemcpyAsync(D.seg.p, h, sizeof(h), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t* off = (const uint64_t*)D.seg.p;
    if (!sorted && S >= 2)
        ST_TRY((sort_segments<DT, false>(dv, run, 1, (T*)D.sample.p, nullptr, S, off, 1, nullptr, false)));
    Model* models = (Model*)D.models.p;
    if (S == 0) {
        k_degenerate_model<<<1, 1, 0, s>>>(models);
        LAUNCH_CHECK();
    } else {
        ST_TRY((fit_level<DT>(D, s, 1, S, h[3], (const T*)D.sample.p, off, off + 2, models, K)));
    }
    k_export_model<<<1, 1, 0, s>>>(models, out, K);
    LAUNCH_CHECK();
    return IPLS_OK;
}

// One sorted fp64 sample x[0..S) as a single item at depth 0: copy it in, fit the placeholder
// FMCD model, then train (or evaluate the gradient of) the two-level model.
ipls_status l2pl_entry(Device& dv, hipStream_t s, const double* x, uint64_t S, uint32_t K, uint32_t M, uint32_t iters,
                       double* root_out, double* leaf_out, double* ab_out, const double* ab_in, double* grad_out,
                       double* loss_out) {
    clear_stale_error();
    Depth& D = dv.depth[0];
    ST_TRY(ensure(D.sample, S * 8));
    ST_TRY(ensure(D.models, sizeof(Model)));
    ST_TRY(ensure(D.seg, 6 * sizeof(uint64_t)));
    HIP_TRY(hipMemcpyAsync(D.sample.p, x, S * 8, hipMemcpyDeviceToDevice, s));
    uint64_t h[4] = {0, S, 0, S > kSmallS ? (S + kFitChunk - 1) / kFitChunk : 0};
    HIP_TRY(hipMemcpyAsync(D.seg.p, h, sizeof(h), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t* off = (const uint64_t*)D.seg.p;
    Model* models = (Model*)D.models.p;
    k_linear_placeholder<<<1, 1, 0, s>>>(models);
    LAUNCH_CHECK();
    ST_TRY((train_l2pl<0>(D, s, 1, S, h[3], (const uint64_t*)D.sample.p, off, off + 2, models, K, M, iters, ab_in,
                          grad_out, loss_out, ab_out)));
    Model root, m;
    HIP_TRY(hipMemcpyAsync(&root, D.roots.p, sizeof(Model), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&m, models, sizeof(Model), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (root.kind != kKindLinear) return IPLS_ERR_DEVICE;  // the root fit is degenerate
    if (ab_in) return IPLS_OK;
    if (!m.l2_ok) return IPLS_ERR_DEVICE;  // a coefficient is not finite
    double r[2] = {root.a, root.b};
    HIP_TRY(hipMemcpyAsync(root_out, r, sizeof(r), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(leaf_out, D.leaves.p, 4 * (size_t)M * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return IPLS_OK;
}

ipls_status check_params(const ipls_params& p) {
    if (p.num_buckets < 4 || p.base_case_max < 1 || p.sample_divisor < 2) return IPLS_ERR_INVALID;
    if (p.sample_policy > 1 || p.equality > 1 || p.inherit > 1 || p.bucket_policy > 1) return IPLS_ERR_INVALID;
    if (p.inherit && (p.model != 0 || p.equality)) return IPLS_ERR_INVALID;  // defined for the FMCD line alone
    if (p.tile_keys != 0 && p.tile_keys != kTile && p.tile_keys != kSmallTile) return IPLS_ERR_INVALID;
    const uint64_t smin = p.sample_min ? p.sample_min : (p.sample_policy == 1 ? 0 : 2ull * p.num_buckets);
    if (smin > p.base_case_max) return IPLS_ERR_INVALID;
    if (p.model > 3) return IPLS_ERR_INVALID;
    if (p.leaves < 4) return IPLS_ERR_INVALID;
    if (p.num_buckets > (uint32_t)kMaxBuckets || p.base_case_max > (uint32_t)kMaxBase ||
        p.leaves > (uint32_t)kMaxLeaves)
        return IPLS_ERR_UNSUPPORTED;
    return IPLS_OK;
}

template <int DT>
ipls_status dispatch_payload(Device& dv, Run& run, void* keys, uint32_t* pay, uint64_t len, const uint64_t* off,
                             uint64_t nseg, void* ws) {
    using T = typename Key<DT>::T;
    if (pay) return sort_segments<DT, true>(dv, run, 0, (T*)keys, pay, len, off, nseg, ws, true);
    return sort_segments<DT, false>(dv, run, 0, (T*)keys, nullptr, len, off, nseg, ws, true);
}

ipls_status dispatch(Device& dv, Run& run, void* keys, uint32_t* pay, uint64_t len, const uint64_t* off,
                     uint64_t nseg, void* ws) {
    switch (run.dtype) {
        case IPLS_F64: return dispatch_payload<0>(dv, run, keys, pay, len, off, nseg, ws);
        case IPLS_F32: return dispatch_payload<1>(dv, run, keys, pay, len, off, nseg, ws);
        case IPLS_U64: return dispatch_payload<2>(dv, run, keys, pay, len, off, nseg, ws);
        default: return IPLS_ERR_DTYPE;
    }
}

ipls_status finish(ipls_status st, hipStream_t s) {
    if (st == IPLS_OK && hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        st = IPLS_ERR_HIP;
    }
    if (g_prof.mask) prof_collect();
    std::lock_guard<std::mutex> g(g_status_mu);
    g_stream_status[(void*)s] = st;
    return st;
}

}  // namespace
}  // namespace ipls

extern "C" size_t ipls_workspace_bytes(size_t n, ipls_dtype dtype, int has_payload, const ipls_params* p);

namespace ipls {

__global__ void k_single_segment(uint64_t* off, uint64_t n) {
    off[0] = 0;
    off[1] = n;
}

ipls_status sort_single(Device& dv, void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                        void* workspace, size_t workspace_bytes, ipls_stats* stats, hipStream_t s) {
    clear_stale_error();
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    if (n > 0 && !keys) return IPLS_ERR_INVALID;
    ipls_params prm;
    if (p) prm = *p;
    else ipls_default_params(&prm);
    ipls_status st = check_params(prm);
    if (st != IPLS_OK) return st;
    if (((uintptr_t)keys % key_bytes(dtype)) != 0 || ((uintptr_t)payload % 4) != 0) return IPLS_ERR_INVALID;
    if (workspace && (workspace_bytes < ipls_workspace_bytes(n, dtype, payload != nullptr, &prm) ||
                      ((uintptr_t)workspace & 255)))
        return IPLS_ERR_INVALID;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n < 2) return IPLS_OK;
    // the allocation-free context is locked by its entry point, which also sets up its buffers
    std::unique_lock<std::mutex> g(dv.mu, std::defer_lock);
    if (!dv.noalloc) g.lock();
    Run run;
    run.p = prm;
    run.s = s;
    run.dtype = dtype;
    std::memset(&run.st, 0, sizeof(run.st));
    Depth& D0 = dv.depth[0];
    st = ensure(D0.seg, 2 * sizeof(uint64_t));
    if (st != IPLS_OK) return st;
    // single segment [0, n): the offsets are written on the stream by a one-thread kernel.  (A copy
    // from a pinned host buffer of default flags, which is not coherent, could read values the CPU
    // had not yet written back to memory, and the buffer's reuse needed a stream synchronisation.)
    k_single_segment<<<1, 1, 0, s>>>((uint64_t*)D0.seg.p, n);
    if (hipGetLastError() != hipSuccess) return IPLS_ERR_HIP;
    st = dispatch(dv, run, keys, payload, n, (const uint64_t*)D0.seg.p, 1, workspace);
    if (st != IPLS_OK && dv.side) (void)hipStreamSynchronize(dv.side);
    st = finish(st, s);
    if (stats) *stats = run.st;
    return st;
}

ipls_status sort_multi(Device& dv, void* keys, uint32_t* payload, const uint64_t* seg_offsets, size_t nseg,
                                  ipls_dtype dtype, const ipls_params* p, void* workspace, size_t workspace_bytes,
                                  ipls_stats* stats, hipStream_t s) {
    clear_stale_error();
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (nseg == 0) return IPLS_OK;
    if (!seg_offsets || !keys) return IPLS_ERR_INVALID;
    ipls_params prm;
    if (p) prm = *p;
    else ipls_default_params(&prm);
    ipls_status st = check_params(prm);
    if (st != IPLS_OK) return st;
    if (((uintptr_t)keys % key_bytes(dtype)) != 0 || ((uintptr_t)payload % 4) != 0) return IPLS_ERR_INVALID;
    std::lock_guard<std::mutex> g(dv.mu);
    uint64_t len = 0;
    if (hipMemcpyAsync(&len, seg_offsets + nseg, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return IPLS_ERR_HIP;
    if (len < 2) return IPLS_OK;
    if (workspace && (workspace_bytes < ipls_workspace_bytes(len, dtype, payload != nullptr, &prm) ||
                      ((uintptr_t)workspace & 255)))
        return IPLS_ERR_INVALID;
    Run run;
    run.p = prm;
    run.s = s;
    run.dtype = dtype;
    std::memset(&run.st, 0, sizeof(run.st));
    st = dispatch(dv, run, keys, payload, len, seg_offsets, nseg, workspace);
    if (st != IPLS_OK && dv.side) (void)hipStreamSynchronize(dv.side);
    st = finish(st, s);
    if (stats) *stats = run.st;
    return st;
}

struct Engine {
    Device dev;
};

// The allocation-free entry point's scratch array and its per-GPU context.  In host code `scratch`
// names a host-side stand-in: its device address on the current GPU comes from
// hipGetSymbolAddress, once per GPU, and only that address is used.
constexpr size_t kNoAllocBytes = IPLS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

struct NoAllocCtx {
    Device dv;
    char* ptr = nullptr;  // scratch's address on this GPU
};
std::unordered_map<int, NoAllocCtx*> g_noalloc;  // by device, guarded by g_mu

ipls_status noalloc_ctx(NoAllocCtx** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return IPLS_ERR_HIP;
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_noalloc.find(dev);
    if (it != g_noalloc.end()) {
        *out = it->second;
        return IPLS_OK;
    }
    char* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return IPLS_ERR_HIP;
    }
    NoAllocCtx* c = new NoAllocCtx();
    c->dv.noalloc = true;
    c->ptr = ptr;
    g_noalloc[dev] = c;
    *out = c;
    return IPLS_OK;
}

Engine* engine_new() { return new Engine(); }

void engine_free(Engine* e) {
    if (!e) return;
    {
        std::lock_guard<std::mutex> g(e->dev.mu);
        (void)hipDeviceSynchronize();
        release_device(e->dev);
    }
    delete e;
}

ipls_status engine_sort(Engine& e, void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                        void* workspace, size_t workspace_bytes, ipls_stats* stats, hipStream_t s) {
    return sort_single(e.dev, keys, payload, n, dtype, p, workspace, workspace_bytes, stats, s);
}

ipls_status engine_sort_segmented(Engine& e, void* keys, uint32_t* payload, const uint64_t* seg_offsets, size_t nseg,
                                  ipls_dtype dtype, const ipls_params* p, void* workspace, size_t workspace_bytes,
                                  ipls_stats* stats, hipStream_t s) {
    return sort_multi(e.dev, keys, payload, seg_offsets, nseg, dtype, p, workspace, workspace_bytes, stats, s);
}

}  // namespace ipls

using namespace ipls;

extern "C" {

void ipls_default_params(ipls_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->num_buckets = 256;
    p->base_case_max = 4096;
    p->sample_divisor = 100;
    p->sample_min = 0;
    p->sample_max = 0;
    p->seed = 0x1F5A220806902000ull;
    p->model = IPLS_MODEL_FMCD;
    p->leaves = 256;
    p->train_iters = 4;
    p->tile_keys = 0;
    p->sample_policy = 0;
    p->equality = 0;
    p->inherit = 0;
    p->bucket_policy = 1;
}

const char* ipls_status_string(ipls_status st) {
    switch (st) {
        case IPLS_OK: return "IPLS_OK";
        case IPLS_ERR_INVALID: return "IPLS_ERR_INVALID";
        case IPLS_ERR_DTYPE: return "IPLS_ERR_DTYPE";
        case IPLS_ERR_OOM: return "IPLS_ERR_OOM";
        case IPLS_ERR_HIP: return "IPLS_ERR_HIP";
        case IPLS_ERR_DEVICE: return "IPLS_ERR_DEVICE";
        case IPLS_ERR_UNSUPPORTED: return "IPLS_ERR_UNSUPPORTED";
    }
    return "IPLS_ERR_UNKNOWN";
}

size_t ipls_workspace_bytes(size_t n, ipls_dtype dtype, int has_payload, const ipls_params* p) {
    (void)p;
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return 0;
    size_t kb = key_bytes(dtype);
    size_t bytes = (n * kb + 255) & ~(size_t)255;
    if (has_payload) bytes += n * 4;
    return bytes;
}

ipls_status ipls_stream_status(void* stream) {
    std::lock_guard<std::mutex> g(g_status_mu);
    auto it = g_stream_status.find(stream);
    return it == g_stream_status.end() ? IPLS_OK : it->second;
}

ipls_status ipls_sort_ex(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                         void* workspace, size_t workspace_bytes, ipls_stats* stats, void* stream) {
    return sort_single(device_ctx(), keys, payload, n, dtype, p, workspace, workspace_bytes, stats,
                       (hipStream_t)stream);
}

ipls_status ipls_sort(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, void* stream) {
    return ipls_sort_ex(keys, payload, n, dtype, nullptr, nullptr, 0, nullptr, stream);
}

ipls_status ipls_sort_segmented(void* keys, uint32_t* payload, const uint64_t* seg_offsets, size_t nseg,
                                ipls_dtype dtype, const ipls_params* p, ipls_stats* stats, void* stream) {
    return sort_multi(device_ctx(), keys, payload, seg_offsets, nseg, dtype, p, nullptr, 0, stats,
                      (hipStream_t)stream);
}

ipls_status ipls_fit_model(const void* sample, size_t S, ipls_dtype dtype, int sample_is_sorted, uint32_t K,
                           ipls_linear_model* out, void* stream) {
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    if (!out || (S > 0 && !sample) || K < 4) return IPLS_ERR_INVALID;
    if (S > 0xffffffffull) return IPLS_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Device& dv = device_ctx();
    std::lock_guard<std::mutex> g(dv.mu);
    Run run;
    ipls_default_params(&run.p);
    run.s = s;
    run.dtype = dtype;
    std::memset(&run.st, 0, sizeof(run.st));
    ipls_status st;
    switch (dtype) {
        case IPLS_F64: st = fit_entry<0>(dv, run, sample, S, sample_is_sorted != 0, K, out); break;
        case IPLS_F32: st = fit_entry<1>(dv, run, sample, S, sample_is_sorted != 0, K, out); break;
        default: st = fit_entry<2>(dv, run, sample, S, sample_is_sorted != 0, K, out); break;
    }
    return finish(st, s);
}

ipls_status ipls_partition(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                           uint64_t* counts, ipls_linear_model* model, void* stream) {
    clear_stale_error();
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    ipls_params prm;
    if (p) prm = *p;
    else ipls_default_params(&prm);
    ipls_status st = check_params(prm);
    if (st != IPLS_OK) return st;
    if (!keys || !counts || n <= prm.base_case_max) return IPLS_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    Device& dv = device_ctx();
    std::lock_guard<std::mutex> g(dv.mu);
    Run run;
    run.p = prm;
    run.s = s;
    run.dtype = dtype;
    std::memset(&run.st, 0, sizeof(run.st));
    run.single_pass = true;
    run.part_counts = counts;
    Depth& D0 = dv.depth[0];
    st = ensure(D0.seg, 2 * sizeof(uint64_t) + sizeof(ipls_linear_model));
    if (st != IPLS_OK) return st;
    run.part_model = model ? model : (ipls_linear_model*)((uint64_t*)D0.seg.p + 2);
    k_single_segment<<<1, 1, 0, s>>>((uint64_t*)D0.seg.p, n);
    LAUNCH_CHECK();
    HIP_TRY(hipMemsetAsync(counts, 0, prm.num_buckets * 8, s));
    st = dispatch(dv, run, keys, payload, n, (const uint64_t*)D0.seg.p, 1, nullptr);
    return finish(st, s);
}

ipls_status ipls_l2pl_train(const double* x, size_t S, uint32_t K, uint32_t M, uint32_t iters, double* root,
                            double* leaf, double* ab, void* stream) {
    if (!x || !root || !leaf || S < 3 || K < 4 || M < 4) return IPLS_ERR_INVALID;
    if (K > (uint32_t)kMaxBuckets || M > (uint32_t)kMaxLeaves || S > 0xffffffffull) return IPLS_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Device& dv = device_ctx();
    std::lock_guard<std::mutex> g(dv.mu);
    ipls_status st = l2pl_entry(dv, s, x, S, K, M, iters, root, leaf, ab, nullptr, nullptr, nullptr);
    return finish(st, s);
}

ipls_status ipls_l2pl_grad(const double* x, size_t S, uint32_t K, uint32_t M, const double* ab, double* grad,
                           double* loss, void* stream) {
    clear_stale_error();
    if (!x || !ab || !grad || S < 3 || K < 4 || M < 4) return IPLS_ERR_INVALID;
    if (K > (uint32_t)kMaxBuckets || M > (uint32_t)kMaxLeaves || S > 0xffffffffull) return IPLS_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Device& dv = device_ctx();
    std::lock_guard<std::mutex> g(dv.mu);
    ipls_status st = l2pl_entry(dv, s, x, S, K, M, 0, nullptr, nullptr, nullptr, ab, grad, loss);
    return finish(st, s);
}

// ------------------------------------------------------------------ allocation-free entry point
// ipls_sort_noalloc: the buffers of a sort (the ping-pong copy of the keys and payload and every
// per-level table) are carved from `scratch`, a static device array that each GPU holds until the
// process ends; the call allocates nothing.
ipls_status ipls_sort_noalloc(void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                              ipls_stats* stats, void* stream) {
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    if (n > IPLS_NOALLOC_MAX_KEYS) return IPLS_ERR_UNSUPPORTED;  // larger than the scratch array serves
    ipls::NoAllocCtx* c = nullptr;
    const ipls_status st0 = ipls::noalloc_ctx(&c);
    if (st0 != IPLS_OK) return st0;
    std::lock_guard<std::mutex> g(c->dv.mu);  // held for the whole sort (sort_single does not take it)
    // every call starts carving from the array's beginning: the previous call's buffers are
    // forgotten (never freed: they are the array's own memory)
    for (ipls::Depth& D : c->dv.depth) ipls::for_each_buf(D, [](ipls::Buf& b) { b = ipls::Buf{}; });
    ipls::Arena arena;
    arena.base = c->ptr;
    arena.cap = ipls::kNoAllocBytes;
    ipls::t_arena = &arena;
    const ipls_status st = ipls::sort_single(c->dv, keys, payload, n, dtype, p, nullptr, 0, stats, (hipStream_t)stream);
    ipls::t_arena = nullptr;
    // a failed call may have left work on the stream: it must not outlive the call on the array
    if (st != IPLS_OK) (void)hipStreamSynchronize((hipStream_t)stream);
    return st;
}

void ipls_profile_enable(int mask) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.mask = mask & 7;
    for (int k = 0; k < 3; ++k) {
        g_prof.launches[k] = 0;
        g_prof.ms[k] = 0;
        g_prof.bytes[k] = 0;
        for (int l = 0; l < Prof::kLevels; ++l) {
            g_prof.lv_launches[k][l] = 0;
            g_prof.lv_ms[k][l] = 0;
            g_prof.lv_bytes[k][l] = 0;
        }
    }
}

void ipls_profile_read(int kernel, uint64_t* launches, double* ms, double* bytes) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (kernel < 0 || kernel > 2) return;
    if (launches) *launches = g_prof.launches[kernel];
    if (ms) *ms = g_prof.ms[kernel];
    if (bytes) *bytes = g_prof.bytes[kernel];
}

void ipls_profile_read_level(int kernel, int level, uint64_t* launches, double* ms, double* bytes) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (kernel < 0 || kernel > 2 || level < 0 || level >= Prof::kLevels) return;
    if (launches) *launches = g_prof.lv_launches[kernel][level];
    if (ms) *ms = g_prof.lv_ms[kernel][level];
    if (bytes) *bytes = g_prof.lv_bytes[kernel][level];
}

}  // extern "C"
