// HIP kernels of one IPLS distribution level on gfx950.
//
// A level partitions every "item" (a bucket of more than T keys) of the current source buffer
// into K sub-buckets of the other buffer:
//   plan -> expand -> sample gather -> (sort samples) -> FMCD fit [-> two-level model, splitter
//   tree, equality buckets] -> min/max of degenerate buckets -> finalize -> classify + per-tile
//   counts -> scan of the chunk totals -> bucket starts [-> children's inherited lines]
//   -> scatter (stable; destinations from the scanned counts) -> worklist (next items, base-case
//   buckets)
// and the base case sorts the small buckets in LDS into the caller's buffer.  The paper's
// IPS4o framework does the same steps with threads and in-place block permutation (Background,
// IPS4o section); here the GPU's many workgroups replace the task scheduler and the level's
// buckets are processed together in every launch.
#pragma once

#include "../../include/ipls.h"
#include "ipls_device.h"

namespace ipls {

// Items of more than kScanSerial chunks have their chunk totals scanned by a workgroup per bucket.
constexpr uint64_t kScanSerial = 64;

struct LevelArgs {
    uint32_t K, T, M;
    uint64_t div, smin, smax, seed;
    uint32_t policy;
    uint32_t tile_keys, small_S, fit_chunk, cand, chunk;
    uint32_t adapt;       // bucket policy: an item's K is bucket_count(n) (and its sample's 2K minimum)
    uint64_t smin_param;  // the caller's sample minimum (0: 2K, none under policy 1)
};

// ------------------------------------------------------------------ plan
// One workgroup of 256 threads (small enough to start beside a running base case): per-item prefix sums of tiles, samples and large-sample fit
// chunks; totals and maxima for the host.  Consumes the item and base-case counters of the
// previous level and resets the counters the coming level appends to.
// One item's share of a level: {chunks, tiles, sample keys, fit chunks, keys, keys with an
// inherited line, 1 if its chunk scan takes a workgroup per bucket}.
// The tile, chunk and fit-chunk sizes are powers of two (the host checks): shifts, not divisions.
__device__ inline void plan_item(const Item& it, const Child* prev_children, const LevelArgs& A, uint64_t (&w)[7]) {
    const uint64_t n = it.n;
    const uint32_t ts = __builtin_ctz(A.tile_keys), cs = __builtin_ctz(A.chunk), fs = __builtin_ctz(A.fit_chunk);
    const uint64_t nt = (n + A.tile_keys - 1) >> ts;
    const uint64_t nc = (nt + A.chunk - 1) >> cs;
    const uint32_t Ki = bucket_count(n, A.K, A.T, A.adapt);
    const uint64_t smin = A.adapt ? (A.smin_param ? A.smin_param : (A.policy == 1 ? 0 : 2ull * Ki)) : A.smin;
    const uint64_t ns = (it.inh && prev_children) ? prev_children[it.inh - 1].s_len
                                                  : sample_size(n, A.div, smin, A.smax, A.policy, Ki);
    w[0] = nc;
    w[1] = nt;
    w[2] = ns;
    w[3] = ns > A.small_S ? (ns + A.fit_chunk - 1) >> fs : 0;
    w[4] = n;
    w[5] = (it.inh && prev_children) ? n : 0;
    w[6] = nc > kScanSerial ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_plan(const Item* items, uint64_t* cnt, int cur, Plan* plan, uint64_t* tile_off,
                                               uint64_t* sample_off, uint64_t* fit_off, uint64_t* chunk_off,
                                               LevelArgs A, uint64_t item_cap, BaseLayout bl, const CopyItem* copy,
                                               uint64_t* copy_off, uint64_t copy_cap, const Child* prev_children,
                                               Plan* plan_host, uint64_t seq, BaseItem* sample_base,
                                               uint32_t* wide_items) {
    __shared__ uint64_t sc[16];
    __shared__ uint64_t sc6[16 * 7];
    __shared__ uint64_t s_max[4];
    __shared__ uint64_t s_cnt[C_N];  // the counters, read once, all in parallel
    constexpr int kPlanWords = (int)(sizeof(Plan) / 8);
    static_assert(sizeof(Plan) % 8 == 0 && offsetof(Plan, seq) == sizeof(Plan) - 8, "seq is the plan's last word");
    __shared__ uint64_t s_plan[kPlanWords];
    constexpr int kPlanIPT = 8;  // items per thread and round
    // an item's chunks, tiles, samples, fit chunks; entry j at j + j/8, so that the 16-byte reads
    // of kPlanIPT consecutive items per thread (144 bytes apart) hit distinct LDS banks
    __shared__ uint4 s_w[kPlanIPT * 256 + kPlanIPT * 256 / 8];
    if (threadIdx.x < (uint32_t)C_N) s_cnt[threadIdx.x] = cnt[threadIdx.x];
    if (threadIdx.x == 0) { s_max[0] = s_max[1] = s_max[2] = s_max[3] = 0; }
    __syncthreads();
    const uint64_t num = s_cnt[C_ITEMS0 + cur];
    uint64_t nb = 0;
    bool base_over = false;
    for (int c = 0; c < kBaseClasses; ++c) {
        nb += s_cnt[C_CLS + c];
        base_over |= s_cnt[C_CLS + c] > bl.cap[c];
    }
    uint64_t run_t = 0, run_s = 0, run_f = 0, run_c = 0, run_w = 0, sum_n = 0, sum_inh = 0;
    const uint64_t use = num < item_cap ? num : item_cap;
    const uint32_t t = threadIdx.x, per = kPlanIPT * blockDim.x;
    // a round of kPlanIPT * 256 items: every thread reads kPlanIPT of them, 256 apart (coalesced,
    // all in flight) and keeps their figures in LDS; then thread t sums the kPlanIPT consecutive
    // items from kPlanIPT t, one block scan gives their offsets, and it writes them
    for (uint64_t base = 0; base < use; base += per) {
        uint64_t mS = 0, mN = 0, pn = 0, pinh = 0;
        uint64_t its_n[kPlanIPT], its_inh[kPlanIPT];  // the fields plan_item reads
#pragma unroll
        for (int k = 0; k < kPlanIPT; ++k) {
            const uint64_t i = base + (uint64_t)k * blockDim.x + t;
            its_n[k] = i < use ? items[i].n : 0;
            its_inh[k] = i < use ? items[i].inh : 0;
        }
#pragma unroll 1
        for (int k = 0; k < kPlanIPT; ++k) {
            const uint32_t j = (uint32_t)k * blockDim.x + t;
            if (base + j >= use) break;
            uint64_t w[7];
            Item it = {0, 0, 0, 0};
            // a register array is indexed by constants only
#pragma unroll
            for (int q = 0; q < kPlanIPT; ++q)
                if (q == k) {
                    it.n = its_n[q];
                    it.inh = its_inh[q];
                }
            plan_item(it, prev_children, A, w);
            mS = w[2] > mS ? w[2] : mS;
            mN = w[4] > mN ? w[4] : mN;
            pn += w[4];
            pinh += w[5];
            // each fits 32 bits: an item has fewer than 2^44 keys, its sample fewer than 2^32
            s_w[j + (j >> 3)] = make_uint4((uint32_t)w[0], (uint32_t)w[1], (uint32_t)w[2], (uint32_t)w[3]);
        }
        // maxima: one LDS atomic per wave
        mS = wave_max<uint64_t>(mS);
        mN = wave_max<uint64_t>(mN);
        if (lane_id() == 0) {
            atomicMax((unsigned long long*)&s_max[0], (unsigned long long)mS);
            atomicMax((unsigned long long*)&s_max[1], (unsigned long long)mN);
        }
        __syncthreads();
        const uint64_t i0 = base + (uint64_t)t * kPlanIPT;
        uint64_t v[7] = {0, 0, 0, 0, pn, pinh, 0};
#pragma unroll 1
        for (int k = 0; k < kPlanIPT; ++k) {
            if (i0 + k >= use) break;
            const uint4 q = s_w[t * (kPlanIPT + 1) + k];
            v[0] += q.x;
            v[1] += q.y;
            v[2] += q.z;
            v[3] += q.w;
            v[6] += q.x > kScanSerial ? 1u : 0u;
        }
        uint64_t ex[7], tot[7];
        block_exclusive_sums<7>(v, ex, tot, sc6);
        uint64_t at_c = run_c + ex[0], at_t = run_t + ex[1], at_s = run_s + ex[2], at_f = run_f + ex[3],
                 at_w = run_w + ex[6];
        // the thread's kPlanIPT offsets of each array are one aligned 64-byte run (the arrays are
        // 256-byte aligned): written with 16-byte stores when the run is whole
        uint64_t oc[kPlanIPT], ot[kPlanIPT], os[kPlanIPT], of[kPlanIPT];
        uint32_t nsam[kPlanIPT];
#pragma unroll
        for (int k = 0; k < kPlanIPT; ++k) {
            const bool in = i0 + k < use;
            const uint4 q = in ? s_w[t * (kPlanIPT + 1) + k] : make_uint4(0u, 0u, 0u, 0u);
            oc[k] = at_c;
            ot[k] = at_t;
            os[k] = at_s;
            of[k] = at_f;
            nsam[k] = q.z;
            if (q.x > kScanSerial) wide_items[at_w++] = (uint32_t)(i0 + k);  // items whose chunks a workgroup per bucket scans
            at_c += q.x;
            at_t += q.y;
            at_s += q.z;
            at_f += q.w;
        }
        if (i0 + kPlanIPT <= use) {
#pragma unroll
            for (int k = 0; k < kPlanIPT; k += 2) {
                *(ulonglong2*)&chunk_off[i0 + k] = make_ulonglong2(oc[k], oc[k + 1]);
                *(ulonglong2*)&tile_off[i0 + k] = make_ulonglong2(ot[k], ot[k + 1]);
                *(ulonglong2*)&sample_off[i0 + k] = make_ulonglong2(os[k], os[k + 1]);
                *(ulonglong2*)&fit_off[i0 + k] = make_ulonglong2(of[k], of[k + 1]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPlanIPT; ++k)
                if (i0 + k < use) {
                    chunk_off[i0 + k] = oc[k];
                    tile_off[i0 + k] = ot[k];
                    sample_off[i0 + k] = os[k];
                    fit_off[i0 + k] = of[k];
                }
        }
        // the samples as base-case buckets of the sample buffer (used when every sample has <= T keys)
        if (sample_base)
#pragma unroll
            for (int k = 0; k < kPlanIPT; ++k)
                if (i0 + k < use) sample_base[i0 + k] = BaseItem{os[k], nsam[k], 0};
        run_c += tot[0];
        run_t += tot[1];
        run_s += tot[2];
        run_f += tot[3];
        sum_n += tot[4];
        sum_inh += tot[5];
        run_w += tot[6];
        __syncthreads();  // s_w is refilled by the next round
    }
    if (threadIdx.x == 0) {
        s_max[2] = sum_n;
        s_max[3] = sum_inh;
    }
    // tiles of the equality buckets the previous level left in the scratch buffer
    const uint64_t ncopy_all = s_cnt[C_COPY], ncopy = ncopy_all < copy_cap ? ncopy_all : copy_cap;
    uint64_t run_k = 0;
    for (uint64_t base = 0; base < ncopy; base += blockDim.x) {
        const uint64_t q = base + threadIdx.x;
        const uint64_t nt = q < ncopy ? (copy[q].n + kCopyTile - 1) / kCopyTile : 0;
        uint64_t tk;
        const uint64_t ek = block_exclusive_sum<uint64_t>(nt, sc, &tk);
        if (q < ncopy) copy_off[q] = run_k + ek;
        run_k += tk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Plan& P = *(Plan*)s_plan;
        copy_off[ncopy] = run_k;
        P.copy_count = ncopy;
        P.copy_tiles = run_k;
        P.eq_closed = s_cnt[C_EQCLOSED];
        P.inherited = s_cnt[C_INHERITED];
        P.l1max = s_cnt[C_L1MAX];
        tile_off[use] = run_t;
        sample_off[use] = run_s;
        fit_off[use] = run_f;
        chunk_off[use] = run_c;
        P.total_chunks = run_c;
        uint64_t e = s_cnt[C_ERR];
        if (num > item_cap || base_over || ncopy_all > copy_cap) e |= kErrCapacity;
        cnt[C_ERR] = e;
        P.num_items = use;
        P.num_base = nb;
        P.total_tiles = run_t;
        P.total_samples = run_s;
        P.total_fit_chunks = run_f;
        P.max_S = s_max[0];
        P.max_n = s_max[1];
        P.sum_n = s_max[2];
        P.inh_n = s_max[3];
        P.n_wide = run_w;
        P.err = e;
        P.closed = s_cnt[C_STATS + 0];
        P.digit = s_cnt[C_STATS + 1];
        P.l2pl = s_cnt[C_STATS + 2];
        P.closed_keys = s_cnt[C_STATS + 3];
        P.base_keys = s_cnt[C_BASEKEYS];
        for (int c = 0; c < kBaseClasses; ++c) {
            const uint64_t k = s_cnt[C_CLS + c];
            P.cls_count[c] = k < bl.cap[c] ? k : bl.cap[c];
        }
        P.seq = seq;
    }
    // counters the coming level appends to start from zero; this level's list is consumed
    if (t == C_CHILD || t == C_COPY || t == C_COPYKEYS || t == C_BASEKEYS || t == C_BASE ||
        t == (uint32_t)(C_ITEMS0 + cur) || t == (uint32_t)(C_ITEMS0 + (cur ^ 1)) ||
        (t >= (uint32_t)C_CLS && t < (uint32_t)(C_CLS + kBaseClasses)))
        cnt[t] = 0;
    __syncthreads();
    // the plan, word by word in parallel, to the device copy and to the host's pinned (coherent)
    // buffer; the host's copy gets its number last
    if (t < (uint32_t)kPlanWords) {
        ((uint64_t*)plan)[t] = s_plan[t];
        if (plan_host && t + 1 < (uint32_t)kPlanWords) ((uint64_t*)plan_host)[t] = s_plan[t];
    }
    if (plan_host) {
        __threadfence_system();
        __syncthreads();
        if (t == 0) plan_host->seq = seq;
    }
}

// map[t] = the item whose range [off[i], off[i+1]) holds t (items with empty ranges are skipped)
__global__ void k_expand(const uint64_t* off, uint64_t num_items, uint64_t total, uint32_t* map) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    uint64_t lo = 0, hi = num_items;  // largest i with off[i] <= t
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    map[t] = (uint32_t)lo;
}

// Two maps from one workgroup index: the tiles over [0, total1) from off1 (each item's tiles of
// `tile` keys, the last one ragged), and map2 over [0, total2) from off2 (both with num_items
// ranges).
__device__ inline void expand2(uint64_t block, const uint64_t* off1, uint64_t total1, TileInfo* map1,
                               const Item* items, uint32_t tile, const uint64_t* off2, uint64_t total2,
                               uint32_t* map2, uint64_t num_items) {
    const uint64_t t = block * blockDim.x + threadIdx.x;
    auto find = [&](const uint64_t* off) {
        uint64_t lo = 0, hi = num_items;  // largest i with off[i] <= t
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (off[mid] <= t) lo = mid;
            else hi = mid;
        }
        return (uint32_t)lo;
    };
    if (t < total1) {
        const uint32_t i = find(off1);
        const Item it = items[i];
        const uint64_t first = (t - off1[i]) * tile, rem = it.n - first;
        map1[t] = TileInfo{it.lo + first, i, rem < (uint64_t)tile ? (uint32_t)rem : tile};
    }
    if (t < total2) map2[t] = find(off2);
}

// ------------------------------------------------------------------ seeds
// Segments of an array (or of the sample buffer) become level-1 items (> T keys) or base-case
// buckets (2..T keys, sorted in place).
__global__ __launch_bounds__(256) void k_seed(const uint64_t* off, uint64_t nseg, uint32_t T, Item* items,
                                              BaseItem* base, BaseLayout bl, uint64_t* cnt, uint64_t item_cap) {
    __shared__ AppendScratch sc;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t a = 0, n = 0;
    if (s < nseg) {
        a = off[s];
        const uint64_t b = off[s + 1];
        if (b < a) atomicOr((unsigned long long*)&cnt[C_ERR], (unsigned long long)kErrOffsets);
        else n = b - a;
    }
    const int cls = base_class((uint32_t)(n <= T ? n : 1));
    const int ch = n > T ? 0 : (n >= 2 ? 1 + cls : -1);
    const uint64_t q = block_append(ch, n, sc, &cnt[C_ITEMS0], &cnt[C_CLS], &cnt[C_BASEKEYS]);
    if (ch == 0 && q < item_cap) items[q] = Item{a, n, 0, 0};
    if (ch > 0 && q < bl.cap[cls]) base[bl.off[cls] + q] = BaseItem{a, (uint32_t)n, 0};
}

// ------------------------------------------------------------------ sample gather
// One key per stratum j = [floor(j n / S), floor((j+1) n / S)) of every item, moved inside the
// stratum by mix64(stream + (j+1) gamma), stream = mix64(seed ^ mix64(lo_rel gamma + n)).
// floor(j n / S) = j q + floor(j r / S) with n = q S + r keeps the arithmetic in 64 bits (S < 2^32).
// An item that inherits copies its restricted sample (already sorted) from the previous level's
// sample buffer instead.
// The same launch also builds the tile and chunk maps (expand2) in its first expand_blocks
// workgroups.
template <int DT>
__global__ void k_sample(const Item* items, uint64_t num_items, const uint64_t* sample_off, uint64_t total,
                         const typename Key<DT>::T* src, typename Key<DT>::T* sample, uint64_t seed,
                         const Child* prev_children, const typename Key<DT>::T* prev_sample, uint64_t expand_blocks,
                         const uint64_t* tile_off, uint64_t total_tiles, TileInfo* tile_map, uint32_t tile,
                         const uint64_t* chunk_off, uint64_t total_chunks, uint32_t* chunk_map) {
    if (blockIdx.x < expand_blocks) {
        expand2(blockIdx.x, tile_off, total_tiles, tile_map, items, tile, chunk_off, total_chunks, chunk_map,
                num_items);
        return;
    }
    uint64_t s = (uint64_t)(blockIdx.x - expand_blocks) * blockDim.x + threadIdx.x;
    if (s >= total) return;
    uint64_t lo = 0, hi = num_items;
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) >> 1;
        if (sample_off[mid] <= s) lo = mid;
        else hi = mid;
    }
    const Item it = items[lo];
    const uint64_t S = sample_off[lo + 1] - sample_off[lo];
    const uint64_t j = s - sample_off[lo];
    if (it.inh && prev_children) {
        sample[s] = prev_sample[prev_children[it.inh - 1].s_lo + j];
        return;
    }
    const uint64_t q = it.n / S, r = it.n % S;
    const uint64_t a = j * q + (j * r) / S;
    const uint64_t b = (j + 1) * q + ((j + 1) * r) / S;
    const uint64_t stream = mix64(seed ^ mix64(it.lo_rel * kGamma + it.n));
    const uint64_t h = mix64(stream + (j + 1) * kGamma);
    sample[s] = src[it.lo + a + h % (b - a)];
}

// ------------------------------------------------------------------ FMCD fit (Linear Models section)
// FMCD returns the smallest window width D >= 1 for which every window x[i..i+D] of the sorted
// sample spans at least u(D) = (x[S-1-D] - x[D]) / (K-2), giving up once 3D > S (then the spread
// of floor(S/3) is kept and D = floor(S/3) + 1).  The window test is monotone in D (a wider
// window spans more, u(D) shrinks as D grows, and fp64 rounding is monotone), so a search over D
// finds the same D as the paper's left-to-right walk; the kernels search in parallel.
__device__ inline double fmcd_spread(double hi, double lo, uint32_t K) { return (hi - lo) / (double)(K - 2); }

// a = 1/u, b = (K - a (x[S-1-D] + x[D])) / 2, in this order of fp64 operations.
__device__ inline void fmcd_line(double u, double xh, double xl, uint32_t K, double* a, double* b) {
    double aa = 1.0 / u;
    double mid = xh + xl;
    double am = aa * mid;
    *a = aa;
    *b = ((double)K - am) / 2.0;
}

__device__ inline bool fit_usable(double a, double b) { return (a > 0.0) && isfinite(a) && isfinite(b); }

__device__ inline void model_degenerate(Model& m) {
    m.kind = kKindPending;
    m.umin = ~0ull;
    m.umax = 0ull;
}

// x[0..S) = val(sample[0..S)) into LDS, eight loads in flight per thread.
template <int DT>
__device__ inline void fill_sample_lds(double* x, const typename Key<DT>::T* xs, uint64_t S) {
    constexpr int U = 8;
    for (uint64_t j0 = threadIdx.x; j0 < S; j0 += (uint64_t)U * blockDim.x) {
        typename Key<DT>::T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t j = j0 + (uint64_t)u * blockDim.x;
            if (j < S) v[u] = xs[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t j = j0 + (uint64_t)u * blockDim.x;
            if (j < S) x[j] = Key<DT>::val(v[u]);
        }
    }
}

// Binary search for FMCD's D over [1, S/3 + 1] by the whole block, x(j) the j-th value of a sorted
// sample of S >= 3 keys (fewer than 2^32, in LDS) with finite ends; then the line.  Every thread
// gets the same result.  A probe tests its windows four at a time (the test is an OR, so the order
// does not matter), which keeps several LDS loads in flight.
template <typename X>
__device__ inline void fmcd_search(const X& x, uint64_t S, uint32_t K, double* a, double* b, uint64_t* Dout) {
    const uint64_t Dmax = S / 3;
    uint64_t lo = 1, hi = Dmax + 1;
    const uint32_t nt = blockDim.x;
    while (lo < hi) {
        const uint64_t D = lo + ((hi - lo) >> 1);
        const double u = fmcd_spread(x(S - 1 - D), x(D), K);
        const uint32_t d = (uint32_t)D, nw = (uint32_t)(S - D);  // windows [w, w + D], w < S - D
        bool fail = false;
        uint32_t w = threadIdx.x;
        for (; w + 3 * nt < nw; w += 4 * nt) {
            const double g0 = x(w + d) - x(w), g1 = x(w + nt + d) - x(w + nt);
            const double g2 = x(w + 2 * nt + d) - x(w + 2 * nt), g3 = x(w + 3 * nt + d) - x(w + 3 * nt);
            fail |= !(g0 >= u) | !(g1 >= u) | !(g2 >= u) | !(g3 >= u);
        }
        for (; w < nw; w += nt) fail |= !(x(w + d) - x(w) >= u);
        if (__syncthreads_or(fail)) lo = D + 1;
        else hi = D;
    }
    const uint64_t D = lo;
    const uint64_t Du = D <= Dmax ? D : Dmax;
    const double u = fmcd_spread(x(S - 1 - Du), x(Du), K);
    fmcd_line(u, x(S - 1 - D), x(D), K, a, b);
    *Dout = D;
}

// Small samples (S <= small_S <= LDS_KEYS): one workgroup per item, the sample in LDS as fp64,
// binary search.  LDS_KEYS is kFitLds, or 4096 or 1024 when every sample of the level is that
// small: a 32 KB workgroup finds room beside other kernels' workgroups (a 128 KB one waits for an
// empty CU), and levels of many small items (samples of 2K keys) fit more 8 KB workgroups per CU.
constexpr int kFitLds = 16384;
constexpr int kFitLdsSmall = 4096;
constexpr int kFitLdsTiny = 1024;
constexpr int kFitLdsFused = 2048;  // the largest sample k_sample_fit takes

// Per-item options of k_fmcd_small: the auto policy's gate for the learned model's root fit (an
// item whose FMCD line lines[i] gives D n <= T S is not trained, and its root is left unusable;
// k_l2pl_bounds applies the same rule), and the bucket policy's K of each item.
struct FitGate {
    const Model* lines;
    const Item* items;
    uint32_t T;        // 0: no gate
    uint32_t adapt_T;  // bucket policy: an item's K is bucket_count(n, K, adapt_T) (0: K for every item)
};

template <int DT, int LDS_KEYS>
__global__ __launch_bounds__(256) void k_fmcd_small(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                    uint64_t num_items, Model* models, uint32_t K_all, uint32_t small_S,
                                                    const EqInfo* eq, FitGate gate) {
    __shared__ double sx[LDS_KEYS];
    const uint64_t i = blockIdx.x;
    if (i >= num_items) return;
    // with equality buckets: the sample without heavy runs, and K - 2E buckets
    const uint64_t off = sample_off[i], S = eq ? eq[i].sr : sample_off[i + 1] - off;
    const uint32_t K = eq ? eq[i].km : (gate.adapt_T ? bucket_count(gate.items[i].n, K_all, gate.adapt_T, 1) : K_all);
    if (S > small_S) return;
    if (gate.T && !(gate.lines[i].kind == kKindLinear && gate.lines[i].D > (uint64_t)gate.T * S / gate.items[i].n)) {
        if (threadIdx.x == 0) {
            Model m = {};
            model_degenerate(m);
            models[i] = m;
        }
        return;
    }
    fill_sample_lds<DT>(sx, sample + off, S);
    __syncthreads();
    Model m = {};
    m.S = S;
    m.kb = K != K_all && !eq ? K : 0u;
    bool usable = S >= 3 && isfinite(sx[0]) && isfinite(sx[S - 1]);
    if (usable) {
        fmcd_search([&](uint64_t j) { return sx[j]; }, S, K, &m.a, &m.b, &m.D);
        usable = fit_usable(m.a, m.b);
    }
    if (!usable) model_degenerate(m);
    if (threadIdx.x == 0) models[i] = m;
}

// ------------------------------------------------------------------ sample, sort and fit in one launch
// For a level whose samples all hold at most CAP keys and whose items take the plain FMCD line (no
// equality buckets, no inherited samples), one workgroup per item does what k_sample, the sample
// sort and k_fmcd_small do in three launches: it gathers the item's sample (the same strata and
// offsets as k_sample), sorts it in LDS by the keys' order-preserving integers (a bitonic network,
// padded to a power of two with the largest integer, which sorts after every key or ties with one
// of the same bits) and fits the line on the sorted values.  Nothing else reads the sorted sample
// on this path, so it is not written back.  The first expand_blocks workgroups build the tile and
// chunk maps, as in k_sample.
template <int DT, int CAP>
__global__ __launch_bounds__(256) void k_sample_fit(const Item* items, uint64_t num_items, const uint64_t* sample_off,
                                                    const typename Key<DT>::T* src, uint64_t seed, Model* models,
                                                    uint32_t K, uint64_t expand_blocks, const uint64_t* tile_off,
                                                    uint64_t total_tiles, TileInfo* tile_map, uint32_t tile,
                                                    const uint64_t* chunk_off, uint64_t total_chunks,
                                                    uint32_t* chunk_map, uint32_t adapt_T) {
    using KT = Key<DT>;
    static_assert((CAP & (CAP - 1)) == 0, "power of two");
    __shared__ uint64_t s_o[CAP];
    if (blockIdx.x < expand_blocks) {
        expand2(blockIdx.x, tile_off, total_tiles, tile_map, items, tile, chunk_off, total_chunks, chunk_map,
                num_items);
        return;
    }
    const uint64_t i = blockIdx.x - expand_blocks;
    if (i >= num_items) return;
    const Item it = items[i];
    const uint64_t off = sample_off[i];
    const uint32_t S = (uint32_t)(sample_off[i + 1] - off);  // 1 <= S <= CAP (the host checks the level's maximum)
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    uint32_t P = 1;
    while (P < S) P <<= 1;
    // gather: stratum j = [floor(j n / S), floor((j+1) n / S)), offset mix64(stream + (j+1) gamma)
    const uint64_t q = it.n / S, r = it.n % S;
    const uint64_t stream = mix64(seed ^ mix64(it.lo_rel * kGamma + it.n));
    for (uint32_t j = tid; j < P; j += nt) {
        uint64_t o = ~0ull;
        if (j < S) {
            const uint64_t a = j * q + ((uint64_t)j * r) / S;
            const uint64_t b = (uint64_t)(j + 1) * q + ((uint64_t)(j + 1) * r) / S;
            const uint64_t h = mix64(stream + (uint64_t)(j + 1) * kGamma);
            o = (uint64_t)KT::ord(src[it.lo + a + h % (b - a)]);
        }
        s_o[j] = o;
    }
    __syncthreads();
    // bitonic sort of s_o[0, P): stage (k, h) compares elements h apart inside blocks of k
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t h = k >> 1; h > 0; h >>= 1) {
            const uint32_t hs = (uint32_t)__builtin_ctz(h);
            for (uint32_t t = tid; t < P / 2; t += nt) {
                const uint32_t lo = ((t >> hs) << (hs + 1)) | (t & (h - 1));
                const uint64_t x = s_o[lo], y = s_o[lo + h];
                if ((x > y) == ((lo & k) == 0)) {
                    s_o[lo] = y;
                    s_o[lo + h] = x;
                }
            }
            __syncthreads();
        }
    }
    // the fit reads the sorted values as fp64, in place of their integers
    double* sx = (double*)s_o;
    for (uint32_t j = tid; j < S; j += nt) sx[j] = KT::val(KT::from_ord(s_o[j]));
    __syncthreads();
    const uint32_t Ki = adapt_T ? bucket_count(it.n, K, adapt_T, 1) : K;
    Model m = {};
    m.S = S;
    m.kb = Ki != K ? Ki : 0u;
    bool usable = S >= 3 && isfinite(sx[0]) && isfinite(sx[S - 1]);
    if (usable) {
        fmcd_search([&](uint64_t j) { return sx[j]; }, S, Ki, &m.a, &m.b, &m.D);
        usable = fit_usable(m.a, m.b);
    }
    if (!usable) model_degenerate(m);
    if (tid == 0) models[i] = m;
}

// ------------------------------------------------------------------ sample inheritance
// Children of every item partitioned by the FMCD line (one workgroup per item, thread c: bucket
// c): the sorted sample's keys the line sends to bucket c form the range [lb(c), lb(c+1)), lb(c)
// being the first sample position of class >= c (a binary search: the line is monotone in the key
// order).  A child that will be partitioned itself (more than T keys) and whose range holds at
// least `thr` keys is appended to the level's child list, its FMCD line still to fit.
template <int DT>
__global__ __launch_bounds__(256) void k_child_split(uint64_t num_items, const Model* models,
                                                     const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                     const uint64_t* hist, uint32_t K, uint32_t T, uint64_t thr,
                                                     ChildSpan* spans, Child* children, uint64_t* cnt, uint64_t cap) {
    using KT = Key<DT>;
    __shared__ uint64_t s_lb[kMaxBuckets + 1];
    __shared__ uint64_t s_scan[16];
    __shared__ uint64_t s_base;
    const uint64_t i = blockIdx.x;
    const uint32_t c = threadIdx.x;
    if (i >= num_items) return;
    const Model m = models[i];
    if (m.kind != kKindLinear || m.neq != 0) {
        if (c == 0) spans[i] = ChildSpan{0u, 0u};
        return;
    }
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    const typename KT::T* xs = sample + off;
    if (c == 0) s_lb[K] = S;
    if (c < K) {
        uint64_t lo = 0, hi = S;  // first position whose class is >= c
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            const typename KT::T u = xs[mid];
            if (classify_linear(m.a, m.b, K, KT::val(u), KT::neg(u)) < c) lo = mid + 1;
            else hi = mid;
        }
        s_lb[c] = lo;
    }
    __syncthreads();
    const uint64_t len = c < K ? s_lb[c + 1] - s_lb[c] : 0;
    const bool take = c < K && hist[i * K + c] > T && len >= thr;
    uint64_t nt;
    const uint64_t rank = block_exclusive_sum<uint64_t>(take ? 1u : 0u, s_scan, &nt);
    if (c == 0) s_base = nt ? atomicAdd((unsigned long long*)&cnt[C_CHILD], (unsigned long long)nt) : 0;
    __syncthreads();
    const uint64_t base = s_base;
    const bool fits = base + nt <= cap;
    if (take && fits) children[base + rank] = Child{0.0, 0.0, 0, off + s_lb[c], (uint32_t)len, c};
    if (c == 0) {
        spans[i] = ChildSpan{(uint32_t)base, fits ? (uint32_t)nt : 0u};
        if (!fits) atomicOr((unsigned long long*)&cnt[C_ERR], (unsigned long long)kErrCapacity);
    }
}

// FMCD line of every entry of the child list (one workgroup each; the sample in LDS when it fits,
// else read from the sample buffer).  An unusable fit leaves a = 0: that child draws a fresh
// sample at its level.
template <int DT>
__global__ __launch_bounds__(256) void k_child_fit(Child* children, const uint64_t* cnt, uint64_t cap,
                                                   const typename Key<DT>::T* sample, uint32_t K) {
    using KT = Key<DT>;
    __shared__ double sx[kFitLds];
    const uint64_t g = blockIdx.x;
    if (g >= cnt[C_CHILD] || g >= cap) return;
    const Child ch = children[g];
    const uint64_t S = ch.s_len;
    const typename KT::T* xs = sample + ch.s_lo;
    double a = 0.0, b = 0.0;
    uint64_t D = 0;
    bool usable;
    if (S <= (uint64_t)kFitLds) {
        fill_sample_lds<DT>(sx, xs, S);
        __syncthreads();
        usable = S >= 3 && isfinite(sx[0]) && isfinite(sx[S - 1]);
        if (usable) fmcd_search([&](uint64_t j) { return sx[j]; }, S, K, &a, &b, &D);
    } else {
        usable = isfinite(KT::val(xs[0])) && isfinite(KT::val(xs[S - 1]));
        if (usable) fmcd_search([&](uint64_t j) { return KT::val(xs[j]); }, S, K, &a, &b, &D);
    }
    usable = usable && fit_usable(a, b);
    if (threadIdx.x == 0) {
        children[g].a = usable ? a : 0.0;
        children[g].b = usable ? b : 0.0;
        children[g].D = D;
    }
}

// Large samples: rounds of `cand` candidate widths spread over the open interval [lo, hi] of D,
// each round one launch over all chunks of all large samples; a failing window sets the
// candidate's bit.  Every workgroup replays the earlier rounds to find the interval.
__device__ inline uint64_t fmcd_candidate(uint64_t lo, uint64_t L, uint64_t m, uint64_t k) {
    return m == L ? lo + k : lo + ((k + 1) * L) / (m + 1);
}

__device__ inline void fmcd_replay(const uint64_t* masks, int rounds, uint64_t Dmax, uint32_t cand, uint64_t* plo,
                                   uint64_t* phi) {
    uint64_t lo = 1, hi = Dmax + 1;
    for (int r = 0; r < rounds; ++r) {
        const uint64_t L = hi - lo;
        if (L == 0) break;
        const uint64_t m = L < cand ? L : cand;
        const uint64_t bits = masks[r];
        uint64_t nhi = hi;
        for (uint64_t k = 0; k < m; ++k)
            if (!((bits >> k) & 1)) {
                nhi = fmcd_candidate(lo, L, m, k);
                break;
            }
        uint64_t nlo = lo;
        for (uint64_t k = 0; k < m; ++k) {
            const uint64_t c = fmcd_candidate(lo, L, m, k);
            if (((bits >> k) & 1) && c < nhi) nlo = c + 1;
        }
        lo = nlo;
        hi = nhi;
    }
    *plo = lo;
    *phi = hi;
}

template <int DT>
__global__ __launch_bounds__(256) void k_fmcd_round(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                    const uint64_t* fit_off, const uint32_t* fit_map, uint64_t* masks,
                                                    int max_rounds, int round, uint32_t K_all, uint32_t chunk,
                                                    uint32_t cand, const EqInfo* eq) {
    using KT = Key<DT>;
    __shared__ uint64_t s_bits;
    const uint32_t i = fit_map[blockIdx.x];
    const uint64_t w = blockIdx.x - fit_off[i];
    const uint64_t off = sample_off[i], S = eq ? eq[i].sr : sample_off[i + 1] - off;
    const uint32_t K = eq ? eq[i].km : K_all;
    if (S < 3) return;
    const typename KT::T* xs = sample + off;
    if (!(isfinite(KT::val(xs[0])) && isfinite(KT::val(xs[S - 1])))) return;
    uint64_t* mk = masks + (uint64_t)i * max_rounds;
    uint64_t lo, hi;
    fmcd_replay(mk, round, S / 3, cand, &lo, &hi);
    const uint64_t L = hi - lo;
    if (L == 0) return;
    const uint64_t m = L < cand ? L : cand;
    if (threadIdx.x == 0) s_bits = 0;
    __syncthreads();
    uint64_t bits = 0;
    const uint64_t w0 = w * chunk, w1 = (w0 + chunk < S) ? w0 + chunk : S;
    for (uint64_t k = 0; k < m; ++k) {
        const uint64_t D = fmcd_candidate(lo, L, m, k);
        const double u = fmcd_spread(KT::val(xs[S - 1 - D]), KT::val(xs[D]), K);
        int fail = 0;
        for (uint64_t t = w0 + threadIdx.x; t < w1 && t + D < S; t += blockDim.x)
            fail |= !(KT::val(xs[t + D]) - KT::val(xs[t]) >= u);
        if (__ballot(fail)) bits |= 1ull << k;
    }
    if (bits && lane_id() == 0) atomicOr((unsigned long long*)&s_bits, (unsigned long long)bits);
    __syncthreads();
    if (threadIdx.x == 0 && s_bits) atomicOr((unsigned long long*)&mk[round], (unsigned long long)s_bits);
}

template <int DT>
__global__ void k_fmcd_finish(const typename Key<DT>::T* sample, const uint64_t* sample_off, uint64_t num_items,
                              const uint64_t* masks, int rounds, Model* models, uint32_t K_all, uint32_t small_S,
                              uint32_t cand, const EqInfo* eq) {
    using KT = Key<DT>;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_items) return;
    const uint64_t off = sample_off[i], S = eq ? eq[i].sr : sample_off[i + 1] - off;
    const uint32_t K = eq ? eq[i].km : K_all;
    if (S <= small_S) return;
    const typename KT::T* xs = sample + off;
    Model m = {};
    m.S = S;
    bool usable = isfinite(KT::val(xs[0])) && isfinite(KT::val(xs[S - 1]));
    if (usable) {
        const uint64_t Dmax = S / 3;
        uint64_t lo, hi;
        fmcd_replay(masks + i * rounds, rounds, Dmax, cand, &lo, &hi);
        const uint64_t D = lo;
        const uint64_t Du = D <= Dmax ? D : Dmax;
        const double u = fmcd_spread(KT::val(xs[S - 1 - Du]), KT::val(xs[Du]), K);
        fmcd_line(u, KT::val(xs[S - 1 - D]), KT::val(xs[D]), K, &m.a, &m.b);
        m.D = D;
        usable = fit_usable(m.a, m.b) && lo == hi;
    }
    if (!usable) model_degenerate(m);
    models[i] = m;
}

// the public view of a fitted model: FMCD's (a, b, D) and whether the fit is unusable
__global__ void k_export_model(const Model* m, ipls_linear_model* out, uint32_t K) {
    const Model x = m[0];
    ipls_linear_model r;
    r.a = x.a;
    r.b = x.b;
    r.D = x.D;
    r.K = K;
    r.degenerate = (x.kind == kKindLinear || x.kind == kKindL2pl) ? 0u : 1u;
    *out = r;
}

__global__ void k_linear_placeholder(Model* m) {
    Model x = {};
    x.kind = kKindLinear;
    m[0] = x;
}

__global__ void k_degenerate_model(Model* m) {
    Model x = {};
    model_degenerate(x);
    m[0] = x;
}

// ------------------------------------------------------------------ two-level model (RMI section)
// A two-level piecewise-linear CDF model: the root is FMCD onto M leaves (a linear model, routed
// like classify_linear); each leaf is a line predicting K times the eCDF of the sorted sample,
// y_j = K (j + 1/2) / S (the Machine Learning Models chapter: an eCDF model becomes a partition
// model through floor(k F(x))).  Because the root is monotone, each leaf owns a contiguous range
// of the sorted sample.  A leaf is trained in its centred coordinate u = (v - c) / h (c the mean
// of its samples, h their largest distance to it) by gradient steps on its mean-squared error;
// the steps are scaled per coordinate by the inverse Hessian diagonal halved (alpha by 1/(4 m2),
// m2 = mean u^2; beta by 1/4).  Sums use 64 strided partials (lane p takes samples p, p+64, ...
// of the leaf in increasing order) and the fixed 64-way tree of wave_tree_sum, so results are
// reproducible bit for bit.  Export: A = alpha / h, B = beta - A c, and a monotone envelope
// [LO, HI] per leaf (LO = HI of the previous leaf, HI = max(LO, min(K, prediction at the leaf's
// last sample))).

__device__ inline double l2pl_target(uint64_t j, uint64_t S, uint32_t K) {
    return (double)K * ((double)j + 0.5) / (double)S;
}

// first[i][l] = first sample of leaf l of item i (M + 1 entries; empty leaves get zero-length ranges)
template <int DT>
// gate_T (the auto policy): an item whose FMCD conflict degree D gives D n <= T S (the line
// leaves no bucket of more than about T keys) keeps its line: its root is marked unusable, which
// every later kernel of the two-level model skips.
__global__ __launch_bounds__(256) void k_l2pl_bounds(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                     uint64_t num_items, const Model* models, Model* roots,
                                                     uint32_t M, uint32_t* first, const Item* items,
                                                     uint32_t gate_T) {
    using KT = Key<DT>;
    const uint64_t i = blockIdx.x;
    if (i >= num_items || models[i].kind != kKindLinear || roots[i].kind != kKindLinear) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    if (gate_T && !(models[i].D > (uint64_t)gate_T * S / items[i].n)) {
        if (threadIdx.x == 0) roots[i].kind = kKindPending;
        return;
    }
    const double ra = roots[i].a, rb = roots[i].b;
    uint32_t* f = first + i * (M + 1);
    for (uint64_t j = threadIdx.x; j <= S; j += blockDim.x) {
        const int lp = j == 0 ? -1 : (int)classify_linear(ra, rb, M, KT::val(sample[off + j - 1]), false);
        const int lc = j == S ? (int)M : (int)classify_linear(ra, rb, M, KT::val(sample[off + j]), false);
        for (int l = lp + 1; l <= lc; ++l) f[l] = (uint32_t)j;
    }
}

// One wave per (item, leaf): geometry, interpolation start, `iters` gradient steps, export.
// grad mode (ab_in != nullptr): evaluate the loss and its gradient at ab_in instead of training.
template <int DT>
__global__ __launch_bounds__(256) void k_l2pl_train(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                    uint64_t num_items, const Model* models, const Model* roots,
                                                    const uint32_t* first, uint32_t K, uint32_t M, uint32_t iters,
                                                    double* leaves, double* lastp, const double* ab_in,
                                                    double* grad_out, double* loss_out, double* ab_out) {
    using KT = Key<DT>;
    const uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t lane = lane_id();
    const uint64_t i = w / M;
    const uint32_t l = (uint32_t)(w % M);
    if (i >= num_items || models[i].kind != kKindLinear || roots[i].kind != kKindLinear) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    const typename KT::T* xs = sample + off;
    const uint32_t* f = first + i * (M + 1);
    const uint64_t j0 = f[l], j1 = f[l + 1];
    double* lv = leaves + i * 4 * kMaxLeaves + 4 * l;
    if (j1 == j0) {
        if (lane == 0) {
            lv[0] = 0.0;
            lv[1] = 0.0;
            lastp[i * kMaxLeaves + l] = 0.0;
            if (ab_out) ab_out[2 * l] = ab_out[2 * l + 1] = 0.0;
            if (grad_out) grad_out[2 * l] = grad_out[2 * l + 1] = 0.0;
            if (loss_out) loss_out[l] = 0.0;
        }
        return;
    }
    const double cnt = (double)(j1 - j0);
    double acc = 0.0;
    for (uint64_t j = j0 + lane; j < j1; j += kWave) acc = acc + KT::val(xs[j]);
    const double mean = __shfl(wave_tree_sum(acc), 0, kWave) / cnt;
    const double x0 = KT::val(xs[j0]), x1 = KT::val(xs[j1 - 1]);
    const double d0 = fabs(x0 - mean), d1 = fabs(x1 - mean);
    double h = d0 > d1 ? d0 : d1;
    if (!(h > 0.0)) h = 1.0;
    acc = 0.0;
    for (uint64_t j = j0 + lane; j < j1; j += kWave) {
        const double u = (KT::val(xs[j]) - mean) / h;
        acc = __builtin_fma(u, u, acc);
    }
    const double m2 = __shfl(wave_tree_sum(acc), 0, kWave) / cnt;
    double alpha = 0.0, beta;
    {
        const double y0 = l2pl_target(j0, S, K), y1 = l2pl_target(j1 - 1, S, K);
        const double u0 = (x0 - mean) / h, u1 = (x1 - mean) / h;
        if (u1 > u0) alpha = (y1 - y0) / (u1 - u0);
        beta = y0 - alpha * u0;
    }
    const double inv = 2.0 / cnt;
    if (ab_in) {
        alpha = ab_in[2 * l];
        beta = ab_in[2 * l + 1];
        double pa = 0.0, pb = 0.0, pl = 0.0;
        for (uint64_t j = j0 + lane; j < j1; j += kWave) {
            const double u = (KT::val(xs[j]) - mean) / h;
            const double r = __builtin_fma(alpha, u, beta) - l2pl_target(j, S, K);
            pa = __builtin_fma(r, u, pa);
            pb = pb + r;
            pl = __builtin_fma(r, r, pl);
        }
        const double ga = wave_tree_sum(pa) * inv, gb = wave_tree_sum(pb) * inv, ls = wave_tree_sum(pl) / cnt;
        if (lane == 0) {
            grad_out[2 * l] = ga;
            grad_out[2 * l + 1] = gb;
            if (loss_out) loss_out[l] = ls;
        }
        return;
    }
    // A leaf of at most 64 samples keeps its lane's (u, y) in registers across the steps (the
    // same values the loop below recomputes).
    const bool one_per_lane = j1 - j0 <= (uint64_t)kWave;
    const bool mine = j0 + lane < j1;
    double u1l = 0.0, y1l = 0.0;
    if (one_per_lane && mine) {
        u1l = (KT::val(xs[j0 + lane]) - mean) / h;
        y1l = l2pl_target(j0 + lane, S, K);
    }
    for (uint32_t it = 0; it < iters; ++it) {
        double pa = 0.0, pb = 0.0;
        if (one_per_lane) {
            if (mine) {
                const double r = __builtin_fma(alpha, u1l, beta) - y1l;
                pa = __builtin_fma(r, u1l, pa);
                pb = pb + r;
            }
        } else {
            for (uint64_t j = j0 + lane; j < j1; j += kWave) {
                const double u = (KT::val(xs[j]) - mean) / h;
                const double r = __builtin_fma(alpha, u, beta) - l2pl_target(j, S, K);
                pa = __builtin_fma(r, u, pa);
                pb = pb + r;
            }
        }
        const double ga = __shfl(wave_tree_sum(pa), 0, kWave) * inv;
        const double gb = __shfl(wave_tree_sum(pb), 0, kWave) * inv;
        // Newton step: with u centred the loss's Hessian is diag(2 m2, 2)
        double na = 0.0;
        if (m2 > 0.0) {
            const double q = 0.5 / m2;
            na = alpha - q * ga;
            if (!(na > 0.0)) na = 0.0;
        }
        alpha = na;
        beta = beta - 0.5 * gb;
    }
    if (lane == 0) {
        const double A = alpha / h;
        const double B = beta - A * mean;
        double last = __builtin_fma(A, x1, B);
        if (last > (double)K) last = (double)K;
        lv[0] = A;
        lv[1] = B;
        lastp[i * kMaxLeaves + l] = last;
        if (ab_out) {
            ab_out[2 * l] = alpha;
            ab_out[2 * l + 1] = beta;
        }
    }
}

// Monotone envelope of every item's leaves (one thread per item, leaves in order) and the check
// that every coefficient is finite; an empty leaf is the constant LO (A = 0, B = LO = HI).
__global__ __launch_bounds__(64) void k_l2pl_envelope(uint64_t num_items, Model* models, const Model* roots,
                                                      const uint32_t* first, uint32_t M, double* leaves,
                                                      const double* lastp) {
    // One wave per item.  Leaf l's HI is the running max, from 0, of the last-sample values of the
    // non-empty leaves up to l (a NaN never wins); LO_l = HI_(l-1).  The running max keeps the
    // earliest of equal values, as the sequential walk does, so a parallel prefix over the lanes
    // (4 consecutive leaves each) gives the same bits.
    const uint64_t i = blockIdx.x;
    const uint32_t lane = lane_id();
    if (i >= num_items) return;
    Model m = models[i];
    if (m.kind != kKindLinear || roots[i].kind != kKindLinear) {
        if (lane == 0) {
            m.l2_ok = 0;
            models[i] = m;
        }
        return;
    }
    const uint32_t* f = first + i * (M + 1);
    double* lv = leaves + i * 4 * kMaxLeaves;
    constexpr int LPL = kMaxLeaves / kWave;  // leaves per lane
    const double kAbsent = __builtin_nan("");
    // combine(a, b): b follows a; b wins only if a is absent or b > a
    auto combine = [](double a, double b) { return (a != a || b > a) ? b : a; };
    double c[LPL], own = kAbsent;
#pragma unroll
    for (int q = 0; q < LPL; ++q) {
        const uint32_t l = lane * LPL + q;
        c[q] = kAbsent;
        if (l < M && f[l + 1] > f[l]) c[q] = lastp[i * kMaxLeaves + l];
        own = combine(own, c[q]);
    }
    // exclusive prefix over the lanes
    double inc = own;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const double o = __shfl_up(inc, d, kWave);
        if (lane >= (uint32_t)d) inc = combine(o, inc);
    }
    double ex = __shfl_up(inc, 1, kWave);
    if (lane == 0) ex = kAbsent;
    double prev = combine(0.0, ex);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < LPL; ++q) {
        const uint32_t l = lane * LPL + q;
        if (l < M) {
            double A = 0.0, B = prev, lo = prev, hi = prev;
            if (f[l + 1] > f[l]) {
                A = lv[4 * l];
                B = lv[4 * l + 1];
                const double last = lastp[i * kMaxLeaves + l];
                hi = last > lo ? last : lo;
            }
            ok = ok && isfinite(A) && isfinite(B) && isfinite(hi);
            lv[4 * l] = A;
            lv[4 * l + 1] = B;
            lv[4 * l + 2] = lo;
            lv[4 * l + 3] = hi;
            prev = hi;
        }
    }
    const bool all_ok = __all(ok);
    if (lane == 0) {
        m.l2_ok = all_ok ? 1u : 0u;
        models[i] = m;
    }
}

// Max sample load of every item under FMCD and under the two-level model (one workgroup per item).
// The FMCD line stays in the model's (a, b) until k_finalize picks the two-level model and moves
// the root there, where classification reads it.
template <int DT>
__global__ __launch_bounds__(256) void k_l2pl_load(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                   uint64_t num_items, Model* models, const Model* roots,
                                                   const double* leaves, uint32_t K, uint32_t M) {
    using KT = Key<DT>;
    __shared__ uint32_t h1[kMaxBuckets], h2[kMaxBuckets];
    __shared__ double s_leaf[4 * kMaxLeaves];
    __shared__ uint32_t s_max[2];
    const uint64_t i = blockIdx.x;
    if (i >= num_items) return;
    const Model m = models[i];
    if (m.kind != kKindLinear || !m.l2_ok) return;
    const double ra = roots[i].a, rb = roots[i].b;
    for (uint32_t q = threadIdx.x; q < 4 * M; q += blockDim.x) s_leaf[q] = leaves[i * 4 * kMaxLeaves + q];
    for (uint32_t b = threadIdx.x; b < kMaxBuckets; b += blockDim.x) h1[b] = h2[b] = 0;
    if (threadIdx.x < 2) s_max[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    for (uint64_t j = threadIdx.x; j < S; j += blockDim.x) {
        const double v = KT::val(sample[off + j]);
        atomicAdd(&h1[classify_linear(m.a, m.b, K, v, false)], 1u);
        atomicAdd(&h2[classify_l2pl(ra, rb, M, s_leaf, K, v, false)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < K; b += blockDim.x) {
        atomicMax(&s_max[0], h1[b]);
        atomicMax(&s_max[1], h2[b]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        models[i].load_lin = s_max[0];
        models[i].load_l2 = s_max[1];
    }
}

// ------------------------------------------------------------------ degenerate buckets
// min and max ord of every bucket whose fit was degenerate (homogeneity check, Learned Sort
// section; digit fallback, IPS4o section).  One workgroup per chunk of `chunk` tiles: a block
// reduction, then one atomic pair per chunk (a bucket of 10^8 equal keys would otherwise send
// hundreds of thousands of atomics to the same two words).
template <int DT>
__global__ __launch_bounds__(256) void k_minmax(const Item* items, const uint64_t* chunk_off, const uint32_t* chunk_map,
                                                Model* models, const typename Key<DT>::T* src, uint32_t tile_keys,
                                                uint32_t chunk) {
    using KT = Key<DT>;
    __shared__ uint64_t s_mn[kBlock / kWave], s_mx[kBlock / kWave];
    const uint32_t i = chunk_map[blockIdx.x];
    if (models[i].kind != kKindPending) return;
    const Item it = items[i];
    const uint64_t span = (uint64_t)tile_keys * chunk;
    const uint64_t base = (blockIdx.x - chunk_off[i]) * span;
    const uint64_t end = (base + span < it.n) ? base + span : it.n;
    const typename KT::T* p = src + it.lo;
    uint64_t mn = ~0ull, mx = 0;
    constexpr int U = 8;  // loads in flight per thread
    for (uint64_t j0 = base + threadIdx.x; j0 < end; j0 += (uint64_t)U * blockDim.x) {
        uint64_t o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t j = j0 + (uint64_t)u * blockDim.x;
            o[u] = j < end ? KT::ord(__builtin_nontemporal_load(&p[j])) : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j0 + (uint64_t)u * blockDim.x < end) {
                mn = o[u] < mn ? o[u] : mn;
                mx = o[u] > mx ? o[u] : mx;
            }
        }
    }
    mx = wave_max(mx);
    mn = ~wave_max(~mn);
    const uint32_t wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_mn[wave] = mn;
        s_mx[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / kWave; ++w) {
            mn = s_mn[w] < mn ? s_mn[w] : mn;
            mx = s_mx[w] > mx ? s_mx[w] : mx;
        }
        atomicMin((unsigned long long*)&models[i].umin, (unsigned long long)mn);
        atomicMax((unsigned long long*)&models[i].umax, (unsigned long long)mx);
    }
}

// Final model of every item: closes homogeneous buckets, sets the digit fallback, and picks the
// two-level model when the policy and the sample loads ask for it.
// stat_counts: [0] closed buckets, [1] digit splits, [2] two-level models, [3] keys in closed buckets
// Splitter tree of every item: from the sorted sample, splitters s_i = x[floor(i S / K)],
// i = 1 .. K-1 (ords, into the item's leaf table), compared strictly unless every splitter is
// the sample's largest value.  tree[i] = 1 (strict), 2 (non-strict), or 0 when the sample holds
// a single value (the degenerate rule decides).
template <int DT>
__global__ __launch_bounds__(256) void k_tree(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                              uint64_t num_items, uint32_t K, double* leaves, uint32_t* tree) {
    using KT = Key<DT>;
    const uint64_t i = blockIdx.x;
    if (i >= num_items) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    const typename KT::T* xs = sample + off;
    const bool usable = S >= 1 && KT::ord(xs[0]) != KT::ord(xs[S - 1]);
    uint64_t* split = (uint64_t*)(leaves + i * 4 * kMaxLeaves);
    if (usable)
        for (uint32_t q = threadIdx.x; q + 1 < K; q += blockDim.x)
            split[q] = KT::ord(xs[((uint64_t)(q + 1) * S) / K]);
    if (threadIdx.x == 0)
        tree[i] = !usable ? 0u : (KT::ord(xs[S / K]) < KT::ord(xs[S - 1]) ? 1u : 2u);
}

// Equality buckets: the heavy values of every item's sorted sample and the sample without their
// runs (one workgroup per item).  A value whose run is longer than S/K (run * K > S) spans at
// least S/K + 1 positions, so it sits at one of the positions 0, m, 2m, ... with m = floor(S/K)+1;
// each such candidate that starts a new value is measured by two binary searches.  The first
// min(16, (K-4)/2) heavy values in ascending order are kept; the sample keeps its order with their
// runs removed (written to rsample at the same offset).  A sample of a single value keeps E = 0
// (the degenerate rule handles it).
template <int DT>
__global__ __launch_bounds__(256) void k_heavy(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                               uint64_t num_items, uint32_t K, EqInfo* eq,
                                               typename Key<DT>::T* rsample) {
    using KT = Key<DT>;
    __shared__ uint64_t s_val[kMaxHeavy], s_lo[kMaxHeavy], s_hi[kMaxHeavy];
    __shared__ uint32_t s_cnt;
    __shared__ uint64_t s_scan[16];
    const uint64_t i = blockIdx.x;
    if (i >= num_items) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    const typename KT::T* xs = sample + off;
    uint32_t emax = (K - 4) / 2;
    emax = emax < (uint32_t)kMaxHeavy ? emax : (uint32_t)kMaxHeavy;
    const uint64_t step = S / K + 1;
    const uint64_t ncand = S ? (S + step - 1) / step : 0;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // candidates in rounds of 256, compacted in order
    for (uint64_t base = 0; base < ncand; base += blockDim.x) {
        const uint64_t c = base + threadIdx.x;
        uint32_t flag = 0;
        uint64_t v = 0, lo = 0, hi = 0;
        if (c < ncand) {
            v = KT::ord(xs[c * step]);
            const bool first = c == 0 || KT::ord(xs[(c - 1) * step]) != v;
            if (first) {
                uint64_t a = 0, b = S;  // lower bound of v
                while (a < b) {
                    const uint64_t mid = (a + b) >> 1;
                    if (KT::ord(xs[mid]) < v) a = mid + 1;
                    else b = mid;
                }
                lo = a;
                b = S;  // upper bound of v
                while (a < b) {
                    const uint64_t mid = (a + b) >> 1;
                    if (KT::ord(xs[mid]) <= v) a = mid + 1;
                    else b = mid;
                }
                hi = a;
                flag = (hi - lo) * (uint64_t)K > S ? 1u : 0u;
            }
        }
        uint64_t tot;
        const uint32_t before = (uint32_t)block_exclusive_sum<uint64_t>(flag, s_scan, &tot);
        const uint32_t at = s_cnt + before;
        if (flag && at < emax) {
            s_val[at] = v;
            s_lo[at] = lo;
            s_hi[at] = hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_cnt = s_cnt + (uint32_t)tot;
        __syncthreads();
    }
    uint32_t E = s_cnt < emax ? s_cnt : emax;
    uint64_t heavy_keys = 0;
    for (uint32_t e = 0; e < E; ++e) heavy_keys += s_hi[e] - s_lo[e];
    if (E == 1 && heavy_keys == S) E = 0;  // a single value: the degenerate rule decides
    if (E == 0) heavy_keys = 0;
    for (uint64_t j = threadIdx.x; j < S; j += blockDim.x) {
        uint64_t shift = 0;
        bool drop = false;
        for (uint32_t e = 0; e < E; ++e) {
            if (j >= s_hi[e]) shift += s_hi[e] - s_lo[e];
            else if (j >= s_lo[e]) drop = true;
        }
        if (!drop) rsample[off + j - shift] = xs[j];
    }
    if (threadIdx.x == 0) {
        EqInfo q;
        q.neq = E;
        q.km = K - 2 * E;
        q.sr = S - heavy_keys;
        for (int e = 0; e < kMaxHeavy; ++e) q.heavy[e] = (uint32_t)e < E ? s_val[e] : 0;
        eq[i] = q;
    }
}

template <int DT>
__global__ void k_finalize(const Item* items, Model* models, const Model* roots, uint64_t num_items, uint32_t K,
                           int src_is_scratch, uint32_t policy, uint64_t* stat_counts, const EqInfo* eq,
                           const uint32_t* tree, const Child* prev_children) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_items) return;
    const uint64_t inh = items[i].inh;
    if (inh && prev_children) {
        // the line fitted on the inherited sample before the parent's scatter wrote the class bytes
        const Child ch = prev_children[inh - 1];
        Model m = {};
        m.kind = kKindLinear;
        m.a = ch.a;
        m.b = ch.b;
        m.D = ch.D;
        m.S = ch.s_len;
        m.inh = 1;
        models[i] = m;
        atomicAdd((unsigned long long*)&stat_counts[C_INHERITED - C_STATS], 1ull);
        return;
    }
    Model m = models[i];
    m.neq = 0;
    if (tree && tree[i]) {  // splitter tree: its splitters are in the item's leaf table
        m.kind = kKindTree;
        m.shift = tree[i] == 1 ? 1u : 0u;
        models[i] = m;
        return;
    }
    if (eq && eq[i].neq) {
        // equality buckets: the linear part (fitted without the heavy runs) or a constant bucket 0
        m.neq = eq[i].neq;
        m.km = eq[i].km;
        for (uint32_t e = 0; e < kMaxHeavy; ++e) m.heavy[e] = e < m.neq ? eq[i].heavy[e] : 0;
        m.const0 = m.kind == kKindPending ? 1u : 0u;
        m.kind = kKindLinear;
        for (uint32_t e = 0; e < kMaxHeavy; ++e)
            m.eqb[e] = e < m.neq ? (uint8_t)classify_equality<DT>(m, Key<DT>::from_ord(m.heavy[e])) : (uint8_t)0;
        models[i] = m;
        return;
    }
    if (m.kind == kKindPending) {
        if (m.umin == m.umax) {
            m.kind = src_is_scratch ? kKindClosedMove : kKindClosedKeep;
            atomicAdd((unsigned long long*)&stat_counts[0], 1ull);
            atomicAdd((unsigned long long*)&stat_counts[3], (unsigned long long)items[i].n);
        } else {
            const uint32_t Kb = m.kb ? m.kb : K;
            const int sh = (int)bit_length(m.umax - m.umin) - (int)(31 - __clz((int)Kb));
            m.kind = kKindDigit;
            m.shift = sh > 0 ? (uint32_t)sh : 0u;
            atomicAdd((unsigned long long*)&stat_counts[1], 1ull);
        }
    } else if (m.kind == kKindLinear && (policy == 1 || policy == 2) && m.l2_ok) {
        const bool splits = m.load_l2 < m.S;
        if (splits && (policy == 2 || m.load_l2 < m.load_lin)) {
            m.kind = kKindL2pl;
            m.a = roots[i].a;  // classification reads the root from (a, b)
            m.b = roots[i].b;
            atomicAdd((unsigned long long*)&stat_counts[2], 1ull);
        }
    }
    models[i] = m;
}

// ------------------------------------------------------------------ tiles and chunks
// A level's keys are cut into tiles of 64 NW IPT keys (NW waves of 8 keys a thread: 2048 keys with
// 4 waves, or 4096 with 8, the default; tiles never cross items); kChunk
// consecutive tiles of an item form a chunk.  Counting, the prefix scan and the scatter all use
// this layout:
//   k_classify_hist: per chunk, the count of every (tile, bucket) -> the tile's exclusive prefix
//                    inside its chunk, and the chunk's totals;
//   k_scan_chunks:   per (item, bucket), the exclusive prefix of the chunk totals, and the item's
//                    bucket sizes (its histogram);
//   k_bucket_starts: per item, bucket starts (exclusive prefix over buckets);
//   k_scatter:       per tile, destination = item start + bucket start + chunk prefix + tile
//                    prefix + rank inside the tile.
// Nothing waits on another workgroup: on MI355X a decoupled look-back chain between tiles pays a
// cross-XCD round trip per step, which measured at half the pass time.
constexpr int kPassIPT = 8;  // keys per thread of the counting and scatter kernels
constexpr int kChunk = 8;

// Wave-level counting of one tile's keys: wave w owns keys [w * 64 * IPT, (w+1) * 64 * IPT) of the
// tile, row r = 64 consecutive keys.  Lanes of a row holding the same bucket are found with 8
// ballots on the bucket bits (four vector instructions a bit); the row's leader lane adds their number to the wave's LDS counter of
// that bucket with an atomic that returns the previous count.  LDS executes a wave's operations in
// order, so the 16 rows' atomics are issued back to back and each returns the count of the wave's
// earlier rows; the leaders' values are then broadcast to their lanes.  rk (when RANKS) receives
// each key's rank among the wave's earlier keys of its bucket, i.e. its stable position.  wc holds
// the wave's 256 counters (zero on entry).
template <int IPT, bool RANKS>
__device__ inline void wave_count(const uint32_t (&bk)[IPT], uint32_t tn, uint32_t wbase, uint32_t* wc,
                                  uint32_t (&rk)[IPT]) {
    const uint32_t lane = lane_id();
    const bool full = wbase + (uint32_t)(IPT * kWave) <= tn;  // the same for the whole wave
    uint32_t prev[IPT], lead[IPT], below[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = full || wbase + r * kWave + lane < tn;
        const uint32_t b = bk[r];
        // diff: lanes whose bucket differs from this lane's in some bit (or that hold no key).
        // Per bit: m = 0 or ~0 from this lane's bit, ones = the lanes with the bit set, and
        // diff |= ones ^ m in one three-input logic op (truth table 0xF6 over (diff, ones, m)).
        const uint64_t vm = full ? ~0ull : __ballot(valid);
        uint32_t diff_lo = ~(uint32_t)vm, diff_hi = ~(uint32_t)(vm >> 32);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)b, (uint32_t)bit, 1u);
            asm("" : "+v"(m));  // keeps the compare on m: one bit extract serves both uses
            const uint64_t ones = __ballot(m != 0u);
            diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)ones, m, 0xF6);
            diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(ones >> 32), m, 0xF6);
        }
        const uint64_t same = ~(((uint64_t)diff_hi << 32) | diff_lo);
        below[r] = count_below(same);
        lead[r] = valid ? (uint32_t)(__ffsll((unsigned long long)same) - 1) : lane;
        prev[r] = 0;
        if (valid && below[r] == 0) {
            if (RANKS) prev[r] = atomicAdd(&wc[b], (uint32_t)__popcll(same));
            else atomicAdd(&wc[b], (uint32_t)__popcll(same));
        }
    }
    if (RANKS) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) rk[r] = (uint32_t)__shfl((int)prev[r], (int)lead[r], kWave) + below[r];
    }
}

// Issues the loads of one tile (wave w owns keys [w * 64 * IPT, (w+1) * 64 * IPT), row r = 64
// consecutive keys), all before any use.
template <int DT, bool PAY, int IPT>
__device__ inline void load_tile(const typename Key<DT>::T* src, const uint32_t* src_pay, uint64_t base, uint32_t tn,
                                 uint32_t wbase, typename Key<DT>::T (&k)[IPT], uint32_t (&p)[PAY ? IPT : 1]) {
    const uint32_t lane = lane_id();
    // streamed once: non-temporal loads (non-temporal stores measured slower: the scatter's
    // partial-line runs need the L2 to combine them).  Lanes past the tile's end get key 0.
    if (wbase + (uint32_t)(IPT * kWave) <= tn) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            k[r] = __builtin_nontemporal_load(&src[base + wbase + r * kWave + lane]);
            if (PAY) p[r] = __builtin_nontemporal_load(&src_pay[base + wbase + r * kWave + lane]);
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t idx = wbase + r * kWave + lane;
        k[r] = 0;
        if (PAY) p[r] = 0u;
        if (idx < tn) {
            k[r] = __builtin_nontemporal_load(&src[base + idx]);
            if (PAY) p[r] = __builtin_nontemporal_load(&src_pay[base + idx]);
        }
    }
}

// Calls f(r, bucket) for every row r of a tile's keys held by this thread.  The model's kind is the
// same for every key of the tile, so it is dispatched once and each kind's row loop is
// straight-line code.  Keys past the tile's end are classified too (every classifier reads only
// its own tables); f masks them.
template <int DT, int IPT, class F>
__device__ inline void classify_rows(const Model& m, const double* leaf, uint32_t K, uint32_t M,
                                     const typename Key<DT>::T (&k)[IPT], F&& f) {
    using KT = Key<DT>;
    switch (m.kind) {
        case kKindClosedMove:
#pragma unroll
            for (int r = 0; r < IPT; ++r) f(r, 0u);
            break;
        case kKindDigit:
#pragma unroll
            for (int r = 0; r < IPT; ++r) f(r, (uint32_t)((KT::ord(k[r]) - m.umin) >> m.shift));
            break;
        case kKindTree:
#pragma unroll
            for (int r = 0; r < IPT; ++r) f(r, classify_tree((const uint64_t*)leaf, K, KT::ord(k[r]), m.shift != 0));
            break;
        case kKindL2pl:
#pragma unroll
            for (int r = 0; r < IPT; ++r) f(r, classify_l2pl(m.a, m.b, M, leaf, K, KT::val(k[r]), KT::neg(k[r])));
            break;
        default:
            if (m.neq) {
#pragma unroll
                for (int r = 0; r < IPT; ++r) f(r, classify_equality<DT>(m, k[r]));
            } else {
#pragma unroll
                for (int r = 0; r < IPT; ++r) f(r, classify_linear(m.a, m.b, m.kb ? m.kb : K, KT::val(k[r]), KT::neg(k[r])));
            }
            break;
    }
}

// The buckets of a tile's keys (0 for lanes past the tile's end).
template <int DT, int IPT>
__device__ inline void classify_tile(uint32_t tn, uint32_t wbase, const Model& m, const double* leaf, uint32_t K,
                                     uint32_t M, const typename Key<DT>::T (&k)[IPT], uint32_t (&bk)[IPT]) {
    const uint32_t lane = lane_id();
    const bool full = wbase + (uint32_t)(IPT * kWave) <= tn;
    classify_rows<DT, IPT>(m, leaf, K, M, k, [&](int r, uint32_t b) {
        bk[r] = (full || wbase + r * kWave + lane < tn) ? b : 0u;
    });
}

// ------------------------------------------------------------------ classify + histogram
// One workgroup per chunk.  For every tile of the chunk: classify, count per bucket, write the
// tile's exclusive prefix inside the chunk (tile_pref[t][b]); at the end the chunk's totals
// (chunk_sum[c][b]).
template <int DT, int NW, int IPT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(6))) void k_classify_hist(const Item* items, const uint64_t* tile_off,
                                                       const uint64_t* chunk_off, const uint32_t* chunk_map,
                                                       uint64_t total_chunks, const Model* models,
                                                       const double* leaves, const typename Key<DT>::T* src,
                                                       uint32_t* tile_pref, uint32_t* chunk_sum, uint32_t K,
                                                       uint32_t M, const uint8_t* src_cls) {
    // Every tile of the chunk has its own LDS histogram, so the waves count tile after tile (the
    // next tile's keys are loaded while this one is counted) with no barrier in between; one
    // barrier at the end, then thread b turns bucket b's counts into the tiles' prefixes.
    using T = typename Key<DT>::T;
    constexpr int NT = kWave * NW, TILE = NT * IPT;
    __shared__ uint32_t h[kChunk][kMaxBuckets];
    __shared__ double s_leaf[4 * kMaxLeaves];
    const uint32_t tid = threadIdx.x, wave = tid / kWave;
    const uint64_t c = blockIdx.x;
    const uint32_t i = chunk_map[c];
    const Item it = items[i];
    const Model m = models[i];
    const uint64_t t0 = tile_off[i];
    const uint64_t t_first = t0 + (c - chunk_off[i]) * kChunk;
    const uint64_t t_end = (t_first + kChunk < tile_off[i + 1]) ? t_first + kChunk : tile_off[i + 1];
    const uint32_t wbase = wave * kWave * IPT;
    auto tile_n = [&](uint64_t t) -> uint32_t {
        const uint64_t rem = it.n - (t - t0) * TILE;
        return rem < (uint64_t)TILE ? (uint32_t)rem : (uint32_t)TILE;
    };
    // an inherited line: the parent's scatter already wrote every key's class (one byte a key)
    const bool bytes = m.inh && src_cls;
    const bool counting = m.kind != kKindClosedKeep && m.kind != kKindClosedMove && !bytes;
    T cur[IPT], nxt[IPT];
    uint32_t nop[1];
    if (counting) load_tile<DT, false, IPT>(src, nullptr, it.lo + (t_first - t0) * TILE, tile_n(t_first), wbase, cur, nop);
    for (uint32_t q = tid, nq = model_table_size(m.kind, K, M); q < nq; q += NT)
        s_leaf[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
    for (uint32_t b = tid; b < kChunk * kMaxBuckets; b += NT) (&h[0][0])[b] = 0;
    __syncthreads();
    if (bytes) {
        // the chunk's class bytes [A0, A1) as aligned 32-bit words, all loads issued first; the
        // class buffer holds at least 3 bytes past the last key
        const uint64_t r0 = (t_first - t0) * TILE;
        const uint64_t r1 = (r0 + (t_end - t_first) * TILE < it.n) ? r0 + (t_end - t_first) * TILE : it.n;
        const uint64_t A0 = it.lo + r0, A1 = it.lo + r1;
        const uint64_t w0 = A0 >> 2, w1 = (A1 + 3) >> 2;
        const uint32_t* cw = (const uint32_t*)src_cls;
        constexpr int NWORD = (kChunk * TILE) / (4 * NT) + 1;
        uint32_t v[NWORD];
#pragma unroll
        for (int q = 0; q < NWORD; ++q) {
            const uint64_t w = w0 + tid + (uint64_t)q * NT;
            v[q] = w < w1 ? cw[w] : 0u;
        }
#pragma unroll
        for (int q = 0; q < NWORD; ++q) {
            const uint64_t w = w0 + tid + (uint64_t)q * NT;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint64_t pos = w * 4 + b;
                if (pos >= A0 && pos < A1)
                    atomicAdd(&h[(uint32_t)((pos - A0) / TILE)][(v[q] >> (8 * b)) & 0xffu], 1u);
            }
        }
    }
    for (uint64_t t = t_first; t < t_end; ++t) {
        const uint32_t tn = tile_n(t), q = (uint32_t)(t - t_first);
        if (counting && t + 1 < t_end)
            load_tile<DT, false, IPT>(src, nullptr, it.lo + (t + 1 - t0) * TILE, tile_n(t + 1), wbase, nxt, nop);
        if (counting) {
            const uint32_t lane = lane_id();
            classify_rows<DT, IPT>(m, s_leaf, K, M, cur, [&](int r, uint32_t b) {
                if (wbase + r * kWave + lane < tn) atomicAdd(&h[q][b], 1u);
            });
        } else if (m.kind == kKindClosedMove && tid == 0) {
            h[q][0] = tn;
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) cur[r] = nxt[r];
    }
    __syncthreads();
    if (tid < K) {
        uint32_t run = 0;  // bucket tid's running count over the chunk's tiles
        for (uint64_t t = t_first; t < t_end; ++t) {
            tile_pref[t * K + tid] = run;
            run += h[t - t_first][tid];
        }
        chunk_sum[c * K + tid] = run;
    }
}

// The same counts with one workgroup per tile (levels without inherited class bytes): every
// workgroup loads its whole tile at once and exits, which streams the keys faster than a
// workgroup walking the 8 tiles of a chunk (6.9 against 7.3 TB/s for a plain read with these
// layouts), and writes the tile's counts to tile_pref[t][b]; k_chunk_prefix then turns them into
// the prefixes inside each chunk and the chunk totals, as k_classify_hist leaves them.
// The tile's keys are loaded before its model is read (a homogeneous item's tiles are read and
// not counted).
template <int DT, int NW, int IPT>
__global__ __launch_bounds__(64 * NW) void k_count_tile(const TileInfo* tile_map, uint64_t total_tiles,
                                                        const Model* models, const double* leaves,
                                                        const typename Key<DT>::T* src, uint32_t* tile_cnt,
                                                        uint32_t K, uint32_t M) {
    using T = typename Key<DT>::T;
    constexpr int NT = kWave * NW;
    __shared__ uint32_t h[kMaxBuckets];
    __shared__ double s_leaf[4 * kMaxLeaves];
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint64_t t = blockIdx.x;
    if (t >= total_tiles) return;
    const TileInfo ti = tile_map[t];
    const uint32_t i = ti.item, tn = ti.n;
    const uint32_t wbase = wave * kWave * IPT;
    T k[IPT];
    uint32_t nop[1];
    load_tile<DT, false, IPT>(src, nullptr, ti.base, tn, wbase, k, nop);
    const Model m = models[i];
    const bool counting = m.kind != kKindClosedKeep && m.kind != kKindClosedMove;
    for (uint32_t q = tid, nq = model_table_size(m.kind, K, M); q < nq; q += NT)
        s_leaf[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
    for (uint32_t b = tid; b < kMaxBuckets; b += NT) h[b] = 0;
    __syncthreads();
    if (counting) {
        classify_rows<DT, IPT>(m, s_leaf, K, M, k, [&](int r, uint32_t b) {
            if (wbase + r * kWave + lane < tn) atomicAdd(&h[b], 1u);
        });
    } else if (m.kind == kKindClosedMove && tid == 0) {
        h[0] = tn;
    }
    __syncthreads();
    for (uint32_t b = tid; b < K; b += NT) tile_cnt[t * K + b] = h[b];
}

// Per chunk (a workgroup, thread b: bucket b): the tile counts of bucket b become exclusive prefixes
// inside the chunk, in place, and their total the chunk's.
__global__ __launch_bounds__(256) void k_chunk_prefix(const uint64_t* tile_off, const uint64_t* chunk_off,
                                                      const uint32_t* chunk_map, uint64_t total_chunks,
                                                      uint32_t* tile_pref, uint32_t* chunk_sum, uint32_t K) {
    const uint64_t c = blockIdx.x;
    if (c >= total_chunks) return;
    const uint32_t i = chunk_map[c];
    const uint64_t t_first = tile_off[i] + (c - chunk_off[i]) * kChunk;
    const uint64_t t_end = (t_first + kChunk < tile_off[i + 1]) ? t_first + kChunk : tile_off[i + 1];
    for (uint32_t b = threadIdx.x; b < K; b += blockDim.x) {
        uint32_t v[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) v[q] = t_first + q < t_end ? tile_pref[(t_first + q) * K + b] : 0u;
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            if (t_first + q < t_end) tile_pref[(t_first + q) * K + b] = run;
            run += v[q];
        }
        chunk_sum[c * K + b] = run;
    }
}

// Exclusive prefix of every item's chunk totals, per bucket (chunk_pref[c][b]); the total is the
// item's bucket size hist[i][b].  Items of at most kScanSerial chunks: one thread per (item, bucket)
// walks the chunks (neighbouring threads read neighbouring buckets).  Larger items (only at the
// first levels of big arrays): one workgroup per (item, bucket).

__global__ __launch_bounds__(256) void k_scan_chunks(const uint64_t* chunk_off, uint32_t K, const uint32_t* chunk_sum,
                                                     uint64_t* chunk_pref, uint64_t* hist, uint64_t* bstart) {
    // one workgroup per item, thread b walks bucket b's chunks; then the bucket starts
    __shared__ uint64_t sc[16];
    const uint64_t i = blockIdx.x;
    const uint32_t b = threadIdx.x;
    const uint64_t c0 = chunk_off[i], c1 = chunk_off[i + 1];
    if (c1 - c0 > kScanSerial) return;  // a wide item: k_scan_chunks_wide, then k_bucket_starts
    uint64_t run = 0;
    if (b < K) {
        for (uint64_t c = c0; c < c1; ++c) {
            const uint64_t v = chunk_sum[c * K + b];
            chunk_pref[c * K + b] = run;
            run += v;
        }
        hist[i * K + b] = run;
    }
    uint64_t tot;
    const uint64_t e = block_exclusive_sum<uint64_t>(b < K ? run : 0, sc, &tot);
    if (b < K) bstart[i * K + b] = e;
}

__global__ __launch_bounds__(256) void k_scan_chunks_wide(const uint64_t* chunk_off, const uint32_t* wide_items,
                                                          uint32_t K, const uint32_t* chunk_sum, uint64_t* chunk_pref,
                                                          uint64_t* hist) {
    // one workgroup per (wide item, bucket): thread t sums a contiguous run of the item's chunks,
    // one block scan of those sums, then each thread writes its run's prefixes
    __shared__ uint64_t sc[16];
    const uint64_t g = blockIdx.x;
    const uint64_t i = wide_items[g / K], b = g % K;
    const uint64_t c0 = chunk_off[i], c1 = chunk_off[i + 1];
    const uint64_t C = c1 - c0;
    if (C <= kScanSerial) return;
    const uint64_t per = (C + blockDim.x - 1) / blockDim.x;
    const uint64_t lo = c0 + threadIdx.x * per;
    const uint64_t hi = lo + per < c1 ? lo + per : c1;
    uint64_t sum = 0;
    constexpr int U = 8;  // loads in flight
    for (uint64_t c = lo; c < hi; c += U) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = c + u < hi ? chunk_sum[(c + u) * K + b] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u) sum += v[u];
    }
    uint64_t total;
    uint64_t run = block_exclusive_sum<uint64_t>(sum, sc, &total);
    for (uint64_t c = lo; c < hi; ++c) {
        const uint64_t v = chunk_sum[c * K + b];
        chunk_pref[c * K + b] = run;
        run += v;
    }
    if (threadIdx.x == 0) hist[i * K + b] = total;
}

// Bucket starts of the wide items (the others get theirs in k_scan_chunks): exclusive prefix of
// the K counts.
__global__ __launch_bounds__(256) void k_bucket_starts(const uint64_t* hist, uint64_t* bstart, uint32_t K,
                                                       const uint32_t* wide_items) {
    __shared__ uint64_t sc[16];
    const uint64_t i = wide_items[blockIdx.x];
    const uint64_t v = threadIdx.x < K ? hist[i * K + threadIdx.x] : 0;
    uint64_t tot;
    const uint64_t e = block_exclusive_sum<uint64_t>(v, sc, &tot);
    if (threadIdx.x < K) bstart[i * K + threadIdx.x] = e;
}

// ------------------------------------------------------------------ scatter
// Stable distribution of one tile (Proposed Algorithm; the Worked Example's contiguous layout is
// the stable one): classify and rank the keys in registers, stage them in LDS in bucket order,
// then write each bucket's run of the tile to one contiguous, coalesced span of the destination.
// Workgroups are mapped to tiles so that each of the 8 XCDs (workgroups are dealt to XCDs round
// robin) walks one contiguous range of tiles: neighbouring tiles, whose runs of a bucket are
// adjacent in the destination, then write through the same L2.
__device__ inline uint64_t xcd_tile(uint64_t g, uint64_t nt) {
    const uint64_t q = nt / 8, r = nt % 8, x = g % 8;
    return x * q + (x < r ? x : r) + g / 8;
}

// CLS: the level has children with inherited lines (sample inheritance).  Their lines are set in
// the staging buffer while the keys are classified (the FMCD line reads no leaf table), each key of
// such a child gets its class under the child's line in registers, the class is staged beside the
// key and written to dst_cls at the key's destination.  No barrier is added.
template <int DT, bool PAY, int NW, int IPT, bool CLS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(CLS && !PAY && NW == 8 ? 6 : 1))) void k_scatter(const Item* items, const TileInfo* tile_map,
                                                 uint64_t total_tiles, const uint64_t* chunk_off,
                                                 uint64_t total_chunks, const Model* models, const double* leaves,
                                                 const uint64_t* bstart, const uint64_t* chunk_pref,
                                                 const uint32_t* tile_pref, const typename Key<DT>::T* src,
                                                 const uint32_t* src_pay, typename Key<DT>::T* dst, uint32_t* dst_pay,
                                                 uint32_t K, uint32_t M, const ChildSpan* spans,
                                                 const Child* children, uint8_t* dst_cls) {
    using T = typename Key<DT>::T;
    using KT = Key<DT>;
    constexpr int NT = kWave * NW, TILE = NT * IPT;
    __shared__ uint32_t s_wcnt[NW][kMaxBuckets];
    __shared__ uint64_t s_base[kMaxBuckets];
    __shared__ uint64_t s_scan[16];
    // The two-level model's leaves (or the children's lines) are only read by the classification,
    // which ends (two barriers) before the first staging write: they share memory with the staged
    // keys.
    constexpr int kStageBytes = TILE * (int)sizeof(T), kLeafBytes = 4 * kMaxLeaves * (int)sizeof(double);
    __shared__ __align__(16) unsigned char s_stage[kStageBytes > kLeafBytes ? kStageBytes : kLeafBytes];
    T* s_keys = (T*)s_stage;
    const double* s_leaf = (const double*)s_stage;
    double2* s_line = (double2*)s_stage;  // CLS: child lines, a = 0 where a child has none
    __shared__ uint8_t s_bkt[TILE];
    __shared__ uint8_t s_cls[CLS ? TILE : 1];
    __shared__ uint32_t s_has[CLS ? kMaxBuckets / 32 : 1];  // CLS: children with a line
    __shared__ uint32_t s_pay[PAY ? TILE : 1];

    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint64_t t = xcd_tile(blockIdx.x, total_tiles);
    const TileInfo ti = tile_map[t];
    const uint32_t i = ti.item, tn = ti.n;
    // issue the tile's loads, then read the model and the destination bases, then one barrier (a
    // homogeneous item already in place has its tiles read and left)
    T k[IPT];
    uint32_t p[PAY ? IPT : 1];
    uint32_t bk[IPT], rk[IPT];
    const uint32_t wbase = wave * kWave * IPT;
    load_tile<DT, PAY, IPT>(src, src_pay, ti.base, tn, wbase, k, p);
    const Model m = models[i];
    if (m.kind == kKindClosedKeep) return;
    const Item it = items[i];
    const uint64_t c = chunk_off[i] + (ti.base - it.lo) / TILE / kChunk;
    const ChildSpan sp = CLS ? spans[i] : ChildSpan{0u, 0u};
    Child ch = {};
    if (CLS && tid < sp.count) ch = children[sp.base + tid];
    uint64_t dbase = 0;
    if (tid < K)
        dbase = it.lo + bstart[(uint64_t)i * K + tid] + chunk_pref[c * K + tid] +
                tile_pref[t * K + tid];
    for (uint32_t q = tid, nq = model_table_size(m.kind, K, M); q < nq; q += NT)
        ((double*)s_stage)[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
    if (CLS && sp.count) {
        if (tid < K) s_line[tid] = make_double2(0.0, 0.0);
        if (tid < kMaxBuckets / 32) s_has[tid] = 0u;
    }
    for (uint32_t b = tid; b < NW * kMaxBuckets; b += NT) (&s_wcnt[0][0])[b] = 0;
    __syncthreads();
    classify_tile<DT, IPT>(tn, wbase, m, s_leaf, K, M, k, bk);
    if (CLS && tid < sp.count && ch.a != 0.0) {
        s_line[ch.c] = make_double2(ch.a, ch.b);
        atomicOr(&s_has[ch.c >> 5], 1u << (ch.c & 31));
    }
    wave_count<IPT, true>(bk, tn, wbase, s_wcnt[wave], rk);
    __syncthreads();

    // classes under the children's lines (registers), before the staging overwrites the lines
    uint32_t cc[CLS ? IPT : 1];
    if (CLS && sp.count) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const double2 ln = s_line[bk[r]];
            cc[r] = ln.x != 0.0 ? classify_linear(ln.x, ln.y, K, KT::val(k[r]), KT::neg(k[r])) : 0u;
        }
    }

    // per-wave offsets and tile-local bucket offsets (bucket order)
    const uint32_t b = tid;
    uint32_t cnt = 0;
    if (b < K) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t cw = s_wcnt[w][b];
            s_wcnt[w][b] = cnt;
            cnt += cw;
        }
    }
    uint32_t tot;  // a tile's counts fit 32 bits
    const uint32_t loc = block_exclusive_sum<uint32_t>(cnt, (uint32_t*)s_scan, &tot);
    if (b < K) {
        // each wave's first slot of bucket b in the staging buffer: one LDS read per key below
#pragma unroll
        for (int w = 0; w < NW; ++w) s_wcnt[w][b] += loc;
        // keys only: the destination address of the bucket's staging slot 0 (one add per key below)
        s_base[b] = (!PAY && !CLS) ? (uint64_t)(uintptr_t)(dst + (dbase - loc)) : dbase - loc;
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t idx = wbase + r * kWave + lane;
        if (idx < tn) {
            const uint32_t pos = s_wcnt[wave][bk[r]] + rk[r];
            s_keys[pos] = k[r];
            s_bkt[pos] = (uint8_t)bk[r];
            if (CLS) s_cls[pos] = (uint8_t)cc[r];
            if (PAY) s_pay[pos] = p[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t j = tid + r * NT;
        if (j < tn) {
            const uint32_t bj = s_bkt[j];
            if constexpr (!PAY && !CLS) {
                ((T*)(uintptr_t)s_base[bj])[j] = s_keys[j];
                continue;
            }
            const uint64_t d = s_base[bj] + j;
            dst[d] = s_keys[j];
            if (PAY) dst_pay[d] = s_pay[j];
            if (CLS && sp.count && ((s_has[bj >> 5] >> (bj & 31)) & 1u)) dst_cls[d] = s_cls[j];
        }
    }
}

// ------------------------------------------------------------------ worklist
// Children of every item: > T keys -> next level's items; equality buckets are closed (moved back
// if they sit in the scratch buffer).  Buckets of T/2 < n <= T keys go to the base case alone.
// Runs of adjacent smaller buckets (1 <= n <= T/2, not separated by a bucket with keys of another
// kind) are sorted together: buckets are in key order and a key's bucket is a function of the key,
// so sorting the run as one range gives the same result.  Inside a run, bucket b joins group
// floor(p_b / (T/2)) (p_b: the keys of the run before it), so a group holds fewer than T keys; the
// group's first bucket emits it.  A group of a single key already in the caller's buffer needs no
// work.
//
// One wave per item (lane l: buckets 4l .. 4l+3), W items a workgroup.  Every step over the
// item's buckets is a scan inside the wave (no workgroup barrier); the workgroup only gathers its
// entries' counts per class, reserves its ranges with one device atomic per class and writes.
// Entries are ranked item by item, bucket by bucket, so the lists are the same on every run.

// Inclusive max-scan over the wave (identity lo).
template <typename V>
__device__ inline V wave_inclusive_max(V v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const V o = __shfl_up(v, s, kWave);
        if (lane >= (uint32_t)s) v = o > v ? o : v;
    }
    return v;
}

template <int W>
__global__ __launch_bounds__(kWave * W) void k_worklist(const Item* items, uint64_t num_items, const Model* models,
                                                        const uint64_t* hist, const uint64_t* bstart, uint32_t K,
                                                        uint32_t T, int dst_is_scratch, Item* next, BaseItem* base,
                                                        BaseLayout bl, uint64_t* cnt, int next_slot, uint64_t next_cap,
                                                        CopyItem* copy, uint64_t copy_cap, const ChildSpan* spans,
                                                        const Child* children, uint64_t* l1max) {
    constexpr int NC = kBaseClasses + 1;  // class 0: next-level items; 1 + c: base-case class c
    static_assert(kMaxBuckets == 4 * kWave, "four buckets a lane");
    __shared__ uint64_t s_sum[W][kMaxBuckets];  // a group's keys, at its first bucket
    __shared__ int s_ent[W][kMaxBuckets];       // bucket -> its child-list entry with a usable line, or -1
    __shared__ uint32_t s_wc[W][NC];            // the wave's entries per class
    __shared__ uint64_t s_gb[NC];
    __shared__ uint64_t s_wkeys[W];             // the wave's base-case keys
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint64_t i = (uint64_t)blockIdx.x * W + w;
    const bool live = i < num_items;  // the same for the whole wave
    const uint64_t half = T / 2 > 0 ? T / 2 : 1;

    int ch[4] = {-1, -1, -1, -1};
    uint64_t nn[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
    uint64_t rel0 = 0, it_lo = 0;
    int ent[4] = {-1, -1, -1, -1};
    if (live) {
        const Model& m = models[i];
        const uint32_t kind = m.kind;
        const Item it = items[i];
        rel0 = it.lo_rel;
        it_lo = it.lo;
        const ChildSpan sp = spans ? spans[i] : ChildSpan{0u, 0u};
        if (sp.count) {
#pragma unroll
            for (int q = 0; q < 4; ++q) s_ent[w][4 * lane + q] = -1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t u = lane; u < sp.count; u += kWave) {
                const Child chd = children[sp.base + u];
                if (chd.a != 0.0) s_ent[w][chd.c] = (int)(sp.base + u);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 4; ++q) ent[q] = s_ent[w][4 * lane + q];
        }
        const bool open = kind != kKindClosedKeep && kind != kKindClosedMove;
        const uint32_t neq = kind == kKindLinear ? m.neq : 0u;
        uint64_t c[4];
        bool brk[4];
        uint64_t mx = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t b = 4 * lane + q;
            c[q] = 0;
            brk[q] = false;
            if (b < K) {
                const uint64_t h = hist[i * K + b];
                mx = h > mx ? h : mx;
                if (open) {
                    c[q] = h;
                    lo[q] = it.lo + bstart[i * K + b];
                    // an equality bucket holds one value: closed here; moved back if it sits in the
                    // scratch buffer
                    bool is_eq = false;
                    for (uint32_t e = 0; e < neq; ++e) is_eq |= m.eqb[e] == b;
                    if (is_eq && c[q] > 0) {
                        atomicAdd((unsigned long long*)&cnt[C_EQCLOSED], 1ull);
                        if (dst_is_scratch) {
                            const uint64_t qq = atomicAdd((unsigned long long*)&cnt[C_COPY], 1ull);
                            if (qq < copy_cap) copy[qq] = CopyItem{lo[q], c[q]};
                            atomicAdd((unsigned long long*)&cnt[C_COPYKEYS], (unsigned long long)c[q]);
                        }
                        c[q] = 0;  // neither an item nor a base-case bucket
                        brk[q] = true;
                    }
                }
            }
        }
        if (l1max) {  // the first level of a single array: its largest bucket, for the statistics
            mx = wave_max<uint64_t>(mx);
            if (lane == 0) *l1max = mx;
        }
        // e: keys of the small buckets before b; eb: e at the last breaker up to b; rs: one past
        // the last breaker before b (the start of b's run)
        bool small[4];
        uint64_t e[4], run_e = 0, lane_brk_e = 0;
        int lane_brk = -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            small[q] = c[q] >= 1 && c[q] <= half;
            brk[q] = brk[q] || c[q] > half;
            e[q] = run_e;
            if (brk[q]) {
                lane_brk = (int)(4 * lane + q);
                lane_brk_e = run_e;
            }
            run_e += small[q] ? c[q] : 0;
        }
        const uint64_t e_in = wave_inclusive_sum<uint64_t>(run_e) - run_e;
        // the last breaker before this lane, and its e (e is nondecreasing: a max-scan finds it)
        int brk_in = wave_inclusive_max<int>(lane_brk);
        uint64_t eb_in = wave_inclusive_max<uint64_t>(lane_brk >= 0 ? e_in + lane_brk_e : 0);
        brk_in = __shfl_up(brk_in, 1, kWave);
        eb_in = __shfl_up(eb_in, 1, kWave);
        if (lane == 0) {
            brk_in = -1;
            eb_in = 0;
        }
        uint64_t eb[4];
        int rs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            e[q] += e_in;
            if (brk[q]) {
                eb_in = e[q];
                brk_in = (int)(4 * lane + q);
            }
            eb[q] = eb_in;
            rs[q] = brk_in + 1;
        }
        // group key of a small bucket, (run start + 1) << 32 | floor(p / half), p = e - eb (p < K
        // half): nondecreasing over the small buckets, so the previous small bucket's key comes
        // from a max-scan; a small bucket whose key is larger starts a group
        uint64_t key[4], run_key = 0;
        uint64_t prevk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t p = small[q] ? e[q] - eb[q] : 0;
            key[q] = small[q] ? (((uint64_t)(rs[q] + 1) << 32) | (p / half)) : 0;
            prevk[q] = run_key;
            run_key = key[q] > run_key ? key[q] : run_key;
        }
        uint64_t key_in = wave_inclusive_max<uint64_t>(run_key);
        key_in = __shfl_up(key_in, 1, kWave);
        if (lane == 0) key_in = 0;
        bool leader[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t pk = prevk[q] > key_in ? prevk[q] : key_in;
            leader[q] = small[q] && pk < key[q];
        }
        // each small bucket adds its keys to its group's first bucket (the last leader up to it)
        int run_lead = -1, lead[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (leader[q]) run_lead = (int)(4 * lane + q);
            lead[q] = run_lead;
        }
        int lead_in = wave_inclusive_max<int>(run_lead);
        lead_in = __shfl_up(lead_in, 1, kWave);
        if (lane == 0) lead_in = -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (lead[q] < 0) lead[q] = lead_in;
            s_sum[w][4 * lane + q] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (small[q]) atomicAdd((unsigned long long*)&s_sum[w][lead[q]], (unsigned long long)c[q]);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (c[q] > T) {
                ch[q] = 0;
                nn[q] = c[q];
            } else if (c[q] > half) {
                nn[q] = c[q];
                ch[q] = 1 + base_class((uint32_t)c[q]);
            } else if (leader[q]) {
                nn[q] = s_sum[w][4 * lane + q];
                if (nn[q] >= 2 || dst_is_scratch) ch[q] = 1 + base_class((uint32_t)nn[q]);
            }
        }
    }
    // ranks inside the wave, class by class (bucket order), and the wave's counts
    uint32_t rk[4] = {0, 0, 0, 0};
    uint64_t bkeys = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) bkeys += ch[q] > 0 ? nn[q] : 0;
    for (int cl = 0; cl < NC; ++cl) {
        uint32_t mine = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) mine += ch[q] == cl ? 1u : 0u;
        const uint32_t inc = wave_inclusive_sum<uint32_t>(mine);
        uint32_t at = inc - mine;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (ch[q] == cl) rk[q] = at++;
        }
        if (lane == kWave - 1) s_wc[w][cl] = inc;
    }
    bkeys = wave_inclusive_sum<uint64_t>(bkeys);
    if (lane == kWave - 1) s_wkeys[w] = bkeys;
    __syncthreads();
    // the workgroup's ranges: one device atomic per class, one for the base-case keys
    if (threadIdx.x < (uint32_t)NC) {
        const int cl = threadIdx.x;
        uint32_t tot = 0;
        for (int v = 0; v < W; ++v) tot += s_wc[v][cl];
        uint64_t* ctr = cl == 0 ? &cnt[next_slot] : &cnt[C_CLS + cl - 1];
        s_gb[cl] = tot ? atomicAdd((unsigned long long*)ctr, (unsigned long long)tot) : 0;
    }
    if (threadIdx.x == 0) {
        uint64_t keys = 0;
        for (int v = 0; v < W; ++v) keys += s_wkeys[v];
        if (keys) atomicAdd((unsigned long long*)&cnt[C_BASEKEYS], (unsigned long long)keys);
    }
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cl = ch[q];
        if (cl < 0) continue;
        uint64_t at = s_gb[cl] + rk[q];
        for (uint32_t v = 0; v < w; ++v) at += s_wc[v][cl];
        const int bc = cl > 0 ? cl - 1 : 0;
        if (cl == 0 && at < next_cap) next[at] = Item{lo[q], nn[q], rel0 + (lo[q] - it_lo), (uint64_t)(ent[q] + 1)};
        if (cl > 0 && at < bl.cap[bc]) base[bl.off[bc] + at] = BaseItem{lo[q], (uint32_t)nn[q], (uint32_t)dst_is_scratch};
    }
}

// Equality buckets a level wrote to the scratch buffer move back to the caller's buffer: every key
// of such a bucket is the same value (the same bits: the key map is one to one), so the keys are
// filled from its first one and only the payloads (in stable order) are copied.  One workgroup per
// tile of kCopyTile keys, tile t of copy item map[t].
template <int DT, bool PAY>
__global__ __launch_bounds__(256) void k_copy(const CopyItem* copy, const uint64_t* copy_off, const uint32_t* map,
                                              uint64_t total_tiles, typename Key<DT>::T* keys, uint32_t* pay,
                                              const typename Key<DT>::T* skeys, const uint32_t* spay) {
    const uint64_t t = blockIdx.x;
    if (t >= total_tiles) return;
    const uint32_t q = map[t];
    const CopyItem ci = copy[q];
    const uint64_t base = (t - copy_off[q]) * kCopyTile;
    const uint64_t rem = ci.n - base;
    const uint32_t n = rem < kCopyTile ? (uint32_t)rem : kCopyTile;
    const typename Key<DT>::T v = skeys[ci.lo];
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
        keys[ci.lo + base + j] = v;
        if (PAY) pay[ci.lo + base + j] = __builtin_nontemporal_load(&spay[ci.lo + base + j]);
    }
}

}  // namespace ipls

// The base case (buckets of at most T keys) lives in its own header.
#include "ipls_base.h"
// Invariant checks (IPLS_DEBUG_CHECKS).
#include "ipls_debug.h"
