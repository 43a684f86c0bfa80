// Request server: continuous batching of sort requests on one GPU.
//
// Memory.  The caller hands over one device arena: the HBM budget.  A request is admitted when
// its memory fits the arena now (ipls_server_reserve never blocks; it reports IPLS_ERR_OOM and
// the caller retries after a completion frees memory):
//   * a large request (more than batch_max_keys keys) gets its own slot for keys and payload plus
//     the sort's ping-pong workspace;
//   * a small request gets a slot at the end of the open batch buffer of its class (dtype,
//     payload or not).  Slots of one batch are contiguous, so the batch is sorted as one segmented
//     sort in place, with no copy in or out.
// The caller writes the request's input into its slot with work on its own stream and submits
// the request; the server orders its sort after that work with an event.
//
// Execution.  `lanes` worker threads, each with its own stream and engine context, take work in
// submission order: a large request, or the submitted slots of a batch (taking a batch closes it,
// so later small requests open a new one; its slots submitted later are taken afterwards).  Lanes run concurrently, so requests that arrive while others are on
// the GPU start as soon as a lane and memory are free, and their kernels overlap on the device.
// Every request's result is the sort of its own keys alone: a segmented sort never moves a key
// across a segment boundary.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ipls.h"
#include "ipls_engine.h"

namespace {

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
uint64_t key_width(ipls_dtype d) { return d == IPLS_F32 ? 4 : 8; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    void init(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        uint64_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }
    uint64_t used() const { return used_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

enum ReqState { kReserved, kSubmitted, kRunning, kDone };

struct Request {
    uint64_t id = 0, n = 0;
    ipls_dtype dtype = IPLS_F64;
    bool pay = false;
    ReqState state = kReserved;
    int64_t batch = -1;            // batch id, or -1 for a large request
    uint64_t seg_index = 0;        // position inside its batch
    uint64_t alloc_off = 0, alloc_bytes = 0;  // large request: its own allocation
    uint64_t keys_off = 0, pay_off = 0, ws_off = 0, ws_bytes = 0;
    hipEvent_t ready = nullptr;
    double t_reserve = 0, t_submit = 0, t_start = 0, t_done = 0;
    ipls_status status = IPLS_OK;
    bool polled = false, released = false;
    uint32_t batch_size = 1;
};

struct Batch {
    int64_t id = 0;
    int cls = 0;
    ipls_dtype dtype = IPLS_F64;
    bool pay = false;
    uint64_t cap_keys = 0, used_keys = 0;
    uint64_t alloc_off = 0, alloc_bytes = 0;
    uint64_t keys_off = 0, pay_off = 0, ws_off = 0, ws_bytes = 0, offs_off = 0;
    std::vector<uint64_t> reqs;
    bool closed = false, queued = false;
    bool running = false;  // a lane is sorting some of its submitted slots
    uint32_t live = 0;     // requests not yet released
};

struct WorkItem {
    bool is_batch;
    int64_t id;
};

}  // namespace

struct ipls_server {
    char* arena = nullptr;
    ipls_server_config cfg;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Arena alloc;
    uint64_t next_id = 1;
    int64_t next_batch = 0;
    std::unordered_map<uint64_t, Request> reqs;
    std::unordered_map<int64_t, Batch> batches;
    int64_t open_batch[6];  // per class: dtype * 2 + payload
    std::deque<WorkItem> queue;
    std::deque<uint64_t> done_order;
    std::vector<std::thread> lanes;
    bool stop = false;
    int device = 0;
    ipls_server_stats st;

    static int cls_of(ipls_dtype d, bool pay) { return (int)d * 2 + (pay ? 1 : 0); }

    void lane_main(int lane);
    void run_request(ipls::Engine& e, hipStream_t s, uint64_t rid, uint64_t* offs_h);
    void run_batch(ipls::Engine& e, hipStream_t s, int64_t bid, uint64_t* offs_h);
    std::vector<std::vector<Request>> take_batch_locked(int64_t bid);
    void end_batch_locked(int64_t bid);
    void free_batch_locked(Batch& b);
};

// Takes a batch for a lane: closes it (later small requests open a new one) and hands over the
// slots submitted so far, as runs of adjacent slots (each run is contiguous in the batch buffer).
// Slots still only reserved stay behind and are taken when they are submitted, after this lane
// is done with the batch, so a lane never waits for a caller.
std::vector<std::vector<Request>> ipls_server::take_batch_locked(int64_t bid) {
    Batch& b = batches[bid];
    b.closed = true;
    b.queued = false;
    b.running = true;
    if (open_batch[b.cls] == bid) open_batch[b.cls] = -1;
    std::vector<std::vector<Request>> runs;
    bool adjacent = false;
    const double t = now_s();
    for (uint64_t id : b.reqs) {
        Request& q = reqs[id];
        if (q.state != kSubmitted) {
            adjacent = false;
            continue;
        }
        q.state = kRunning;
        q.t_start = t;
        if (!adjacent) runs.emplace_back();
        runs.back().push_back(q);
        adjacent = true;
    }
    return runs;
}

// A lane is done with a batch: slots submitted meanwhile make it queued again.
void ipls_server::end_batch_locked(int64_t bid) {
    Batch& b = batches[bid];
    b.running = false;
    for (uint64_t id : b.reqs) {
        if (reqs[id].state == kSubmitted) {
            b.queued = true;
            queue.push_back({true, bid});
            cv_work.notify_all();
            break;
        }
    }
}

void ipls_server::free_batch_locked(Batch& b) {
    alloc.release(b.alloc_off, b.alloc_bytes);
    batches.erase(b.id);
}

void ipls_server::run_request(ipls::Engine& e, hipStream_t s, uint64_t rid, uint64_t* offs_h) {
    (void)offs_h;
    Request r;
    {
        std::lock_guard<std::mutex> g(mu);
        Request& q = reqs[rid];
        q.state = kRunning;
        q.t_start = now_s();
        r = q;
    }
    ipls_status status = IPLS_OK;
    if (r.ready && hipStreamWaitEvent(s, r.ready, 0) != hipSuccess) status = IPLS_ERR_HIP;
    if (status == IPLS_OK)
        status = ipls::engine_sort(e, arena + r.keys_off, r.pay ? (uint32_t*)(arena + r.pay_off) : nullptr, r.n,
                                   r.dtype, &cfg.params, arena + r.ws_off, r.ws_bytes, nullptr, s);
    const double t = now_s();
    std::lock_guard<std::mutex> g(mu);
    Request& q = reqs[rid];
    q.state = kDone;
    q.status = status;
    q.t_done = t;
    done_order.push_back(rid);
    st.completed += 1;
    st.singles_run += 1;
    st.keys_sorted += r.n;
    cv_done.notify_all();
}

void ipls_server::run_batch(ipls::Engine& e, hipStream_t s, int64_t bid, uint64_t* offs_h) {
    Batch b;
    std::vector<std::vector<Request>> runs;
    {
        std::lock_guard<std::mutex> g(mu);
        runs = take_batch_locked(bid);
        b = batches[bid];
    }
    const uint64_t w = key_width(b.dtype);
    uint64_t* offs_d = (uint64_t*)(arena + b.offs_off);
    for (const std::vector<Request>& rs : runs) {
        // one segmented sort per run of adjacent submitted slots; runs are sorted one after the
        // other on this lane's stream, so they share the batch's workspace and offsets buffer
        // (each engine call returns after its stream has completed)
        ipls_status status = IPLS_OK;
        for (const Request& r : rs) {
            if (status != IPLS_OK) break;
            if (r.ready && hipStreamWaitEvent(s, r.ready, 0) != hipSuccess) status = IPLS_ERR_HIP;
        }
        const uint64_t nseg = rs.size(), k0 = rs[0].keys_off;
        if (status == IPLS_OK) {
            // offs_h is coherent pinned memory: the copy engine reads what the CPU has just written
            for (uint64_t i = 0; i < nseg; ++i) offs_h[i] = (rs[i].keys_off - k0) / w;
            offs_h[nseg] = offs_h[nseg - 1] + rs[nseg - 1].n;
            if (hipMemcpyAsync(offs_d, offs_h, (nseg + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess)
                status = IPLS_ERR_HIP;
            if (status == IPLS_OK)
                status = ipls::engine_sort_segmented(e, arena + k0, b.pay ? (uint32_t*)(arena + rs[0].pay_off) : nullptr,
                                                     offs_d, nseg, b.dtype, &cfg.params, arena + b.ws_off, b.ws_bytes,
                                                     nullptr, s);
        }
        const double t = now_s();
        std::lock_guard<std::mutex> g(mu);
        for (const Request& r : rs) {
            Request& q = reqs[r.id];
            q.state = kDone;
            q.status = status;
            q.t_done = t;
            q.batch_size = (uint32_t)nseg;
            done_order.push_back(r.id);
            st.completed += 1;
            st.keys_sorted += r.n;
        }
        st.batches_run += 1;
        cv_done.notify_all();
    }
    std::lock_guard<std::mutex> g(mu);
    end_batch_locked(bid);
}

void ipls_server::lane_main(int lane) {
    (void)lane;
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    ipls::Engine* e = ipls::engine_new();
    uint64_t* offs_h = nullptr;
    bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
              hipHostMalloc((void**)&offs_h, (cfg.batch_max_requests + 1) * 8, hipHostMallocCoherent) == hipSuccess;
    for (;;) {
        WorkItem w;
        {
            std::unique_lock<std::mutex> g(mu);
            cv_work.wait(g, [&] { return stop || !queue.empty(); });
            if (queue.empty()) break;  // stop requested and nothing left
            w = queue.front();
            queue.pop_front();
        }
        if (!ok) {
            // no stream or staging buffer on this lane: the work it takes fails
            std::lock_guard<std::mutex> g(mu);
            std::vector<uint64_t> ids;
            if (w.is_batch) {
                for (const std::vector<Request>& rs : take_batch_locked(w.id))
                    for (const Request& r : rs) ids.push_back(r.id);
            } else {
                ids.push_back((uint64_t)w.id);
            }
            for (uint64_t id : ids) {
                reqs[id].state = kDone;
                reqs[id].status = IPLS_ERR_HIP;
                reqs[id].t_done = now_s();
                done_order.push_back(id);
            }
            if (w.is_batch) end_batch_locked(w.id);
            cv_done.notify_all();
            continue;
        }
        if (w.is_batch) run_batch(*e, s, w.id, offs_h);
        else run_request(*e, s, (uint64_t)w.id, offs_h);
    }
    if (s) (void)hipStreamSynchronize(s);
    ipls::engine_free(e);
    if (s) (void)hipStreamDestroy(s);
    if (offs_h) (void)hipHostFree(offs_h);
}

extern "C" {

void ipls_server_default_config(ipls_server_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->lanes = 3;
    c->batch_max_keys = 1ull << 18;
    c->batch_keys = 1ull << 22;
    c->batch_max_requests = 1024;
    ipls_default_params(&c->params);
}

ipls_status ipls_server_create(void* arena, size_t arena_bytes, const ipls_server_config* cfg, ipls_server** out) {
    if (!arena || !out || ((uintptr_t)arena & (kAlign - 1))) return IPLS_ERR_INVALID;
    ipls_server_config c;
    if (cfg) c = *cfg;
    else ipls_server_default_config(&c);
    if (c.lanes < 1 || c.lanes > 16 || c.batch_keys < c.batch_max_keys || c.batch_max_requests < 1)
        return IPLS_ERR_INVALID;
    ipls_server* s = new ipls_server();
    s->arena = (char*)arena;
    s->cfg = c;
    s->alloc.init(arena_bytes & ~(kAlign - 1));
    for (int64_t& b : s->open_batch) b = -1;
    std::memset(&s->st, 0, sizeof(s->st));
    s->st.arena_bytes = arena_bytes;
    (void)hipGetDevice(&s->device);
    for (uint32_t i = 0; i < c.lanes; ++i) s->lanes.emplace_back([s, i] { s->lane_main((int)i); });
    *out = s;
    return IPLS_OK;
}

ipls_status ipls_server_reserve(ipls_server* s, size_t n, ipls_dtype dtype, int has_payload, uint64_t* req_id,
                                void** keys, uint32_t** payload) {
    if (!s || !req_id || !keys) return IPLS_ERR_INVALID;
    if (dtype != IPLS_F64 && dtype != IPLS_F32 && dtype != IPLS_U64) return IPLS_ERR_DTYPE;
    const bool pay = has_payload != 0;
    const uint64_t w = key_width(dtype);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return IPLS_ERR_INVALID;
    Request r;
    r.id = s->next_id;
    r.n = n;
    r.dtype = dtype;
    r.pay = pay;
    r.t_reserve = now_s();
    if (n > s->cfg.batch_max_keys) {
        const uint64_t kb = align_up(n * w), pb = pay ? align_up(n * 4) : 0;
        const uint64_t wb = align_up(ipls_workspace_bytes(n, dtype, pay, &s->cfg.params));
        uint64_t off;
        if (!s->alloc.alloc(kb + pb + wb, &off)) {
            s->st.rejected += 1;
            return IPLS_ERR_OOM;
        }
        r.alloc_off = off;
        r.alloc_bytes = kb + pb + wb;
        r.keys_off = off;
        r.pay_off = off + kb;
        r.ws_off = off + kb + pb;
        r.ws_bytes = wb;
    } else {
        const int cls = ipls_server::cls_of(dtype, pay);
        int64_t bid = s->open_batch[cls];
        if (bid >= 0) {
            Batch& b = s->batches[bid];
            if (b.used_keys + n > b.cap_keys || b.reqs.size() >= s->cfg.batch_max_requests) {
                b.closed = true;  // full: stays queued (or is queued at its first submission)
                s->open_batch[cls] = -1;
                bid = -1;
            }
        }
        if (bid < 0) {
            Batch b;
            b.id = s->next_batch;
            b.cls = cls;
            b.dtype = dtype;
            b.pay = pay;
            b.cap_keys = s->cfg.batch_keys;
            const uint64_t kb = align_up(b.cap_keys * w), pb = pay ? align_up(b.cap_keys * 4) : 0;
            const uint64_t wb = align_up(ipls_workspace_bytes(b.cap_keys, dtype, pay, &s->cfg.params));
            const uint64_t ob = align_up((s->cfg.batch_max_requests + 1) * 8);
            uint64_t off;
            if (!s->alloc.alloc(kb + pb + wb + ob, &off)) {
                s->st.rejected += 1;
                return IPLS_ERR_OOM;
            }
            s->next_batch += 1;
            b.alloc_off = off;
            b.alloc_bytes = kb + pb + wb + ob;
            b.keys_off = off;
            b.pay_off = off + kb;
            b.ws_off = off + kb + pb;
            b.ws_bytes = wb;
            b.offs_off = off + kb + pb + wb;
            s->batches[b.id] = b;
            s->open_batch[cls] = b.id;
            bid = b.id;
        }
        Batch& b = s->batches[bid];
        r.batch = bid;
        r.seg_index = b.reqs.size();
        r.keys_off = b.keys_off + b.used_keys * w;
        r.pay_off = b.pay_off + b.used_keys * 4;
        b.used_keys += n;
        b.reqs.push_back(r.id);
        b.live += 1;
    }
    s->next_id += 1;
    s->reqs[r.id] = r;
    s->st.admitted += 1;
    s->st.bytes_in_use = s->alloc.used();
    s->st.peak_bytes_in_use = std::max(s->st.peak_bytes_in_use, s->st.bytes_in_use);
    *req_id = r.id;
    *keys = s->arena + r.keys_off;
    if (payload) *payload = pay ? (uint32_t*)(s->arena + r.pay_off) : nullptr;
    return IPLS_OK;
}

ipls_status ipls_server_submit(ipls_server* s, uint64_t req_id, void* producer_stream) {
    if (!s) return IPLS_ERR_INVALID;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return IPLS_ERR_HIP;
    if (hipEventRecord(ev, (hipStream_t)producer_stream) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return IPLS_ERR_HIP;
    }
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end() || it->second.state != kReserved) {
        (void)hipEventDestroy(ev);
        return IPLS_ERR_INVALID;
    }
    Request& r = it->second;
    r.ready = ev;
    r.state = kSubmitted;
    r.t_submit = now_s();
    if (r.batch < 0) {
        s->queue.push_back({false, (int64_t)r.id});
    } else {
        // a batch a lane is sorting is queued again when that lane is done with it
        Batch& b = s->batches[r.batch];
        if (!b.queued && !b.running) {
            b.queued = true;
            s->queue.push_back({true, b.id});
        }
    }
    s->st.max_queue_depth = std::max<uint64_t>(s->st.max_queue_depth, s->queue.size());
    s->cv_work.notify_all();
    return IPLS_OK;
}

ipls_status ipls_server_wait(ipls_server* s, uint64_t req_id, ipls_server_done* info) {
    if (!s) return IPLS_ERR_INVALID;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end() || it->second.state == kReserved) return IPLS_ERR_INVALID;
    s->cv_done.wait(g, [&] { return s->reqs[req_id].state == kDone; });
    Request& r = s->reqs[req_id];
    if (info) {
        info->req_id = r.id;
        info->status = r.status;
        info->n = r.n;
        info->t_reserve = r.t_reserve;
        info->t_submit = r.t_submit;
        info->t_start = r.t_start;
        info->t_done = r.t_done;
        info->batch_size = r.batch_size;
    }
    return r.status;
}

ipls_status ipls_server_poll(ipls_server* s, ipls_server_done* out, size_t max, size_t* count) {
    if (!s || !count || (max && !out)) return IPLS_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    size_t k = 0;
    while (k < max && !s->done_order.empty()) {
        const uint64_t id = s->done_order.front();
        s->done_order.pop_front();
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || it->second.polled) continue;
        Request& r = it->second;
        r.polled = true;
        out[k].req_id = r.id;
        out[k].status = r.status;
        out[k].n = r.n;
        out[k].t_reserve = r.t_reserve;
        out[k].t_submit = r.t_submit;
        out[k].t_start = r.t_start;
        out[k].t_done = r.t_done;
        out[k].batch_size = r.batch_size;
        ++k;
    }
    *count = k;
    return IPLS_OK;
}

ipls_status ipls_server_release(ipls_server* s, uint64_t req_id) {
    if (!s) return IPLS_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end() || it->second.state != kDone) return IPLS_ERR_INVALID;
    Request r = it->second;
    if (r.ready) (void)hipEventDestroy(r.ready);
    s->reqs.erase(it);
    if (r.batch < 0) {
        s->alloc.release(r.alloc_off, r.alloc_bytes);
    } else {
        Batch& b = s->batches[r.batch];
        b.live -= 1;
        if (b.live == 0 && b.closed) s->free_batch_locked(b);
    }
    s->st.bytes_in_use = s->alloc.used();
    return IPLS_OK;
}

ipls_status ipls_server_stats_get(ipls_server* s, ipls_server_stats* out) {
    if (!s || !out) return IPLS_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    s->st.bytes_in_use = s->alloc.used();
    s->st.queue_depth = s->queue.size();
    *out = s->st;
    return IPLS_OK;
}

ipls_status ipls_server_destroy(ipls_server* s) {
    if (!s) return IPLS_ERR_INVALID;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->lanes) t.join();
    for (auto& kv : s->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    delete s;
    return IPLS_OK;
}

}  // extern "C"
