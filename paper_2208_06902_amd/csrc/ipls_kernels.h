// HIP kernels of one IPLS distribution level on gfx950.
//
// A level partitions every "item" (a bucket of more than T keys) of the current source buffer
// into K sub-buckets of the other buffer:
//   plan -> expand -> sample gather -> (sort samples) -> FMCD fit [-> two-level model]
//   -> min/max of degenerate buckets -> finalize -> classify + histogram -> bucket starts
//   -> scatter (stable, decoupled look-back) -> worklist (next items, base-case buckets)
// and the base case sorts the small buckets in LDS into the caller's buffer.  The paper's
// IPS4o framework does the same steps with threads and in-place block permutation (Background,
// IPS4o section); here the GPU's many workgroups replace the task scheduler and the level's
// buckets are processed together in every launch.
#pragma once

#include "../../include/ipls.h"
#include "ipls_device.h"

namespace ipls {

struct LevelArgs {
    uint32_t K, T, M;
    uint64_t div, smin, smax, seed;
    uint32_t tile_keys, small_S, fit_chunk, cand;
};

// ------------------------------------------------------------------ plan
// One workgroup of 1024 threads: per-item prefix sums of tiles, samples and large-sample fit
// chunks; totals and maxima for the host.  Consumes the item and base-case counters of the
// previous level and resets the counters the coming level appends to.
__global__ __launch_bounds__(1024) void k_plan(const Item* items, uint64_t* item_count_cur, uint64_t* item_count_next,
                                               uint64_t* base_count, uint64_t* err_word, const uint64_t* stat_counts,
                                               Plan* plan, uint64_t* tile_off,
                                               uint64_t* sample_off, uint64_t* fit_off, LevelArgs A, uint64_t item_cap,
                                               uint64_t base_cap) {
    __shared__ uint64_t sc[16];
    __shared__ uint64_t s_max[3];
    const uint64_t num = *item_count_cur;
    const uint64_t nb = *base_count;
    if (threadIdx.x == 0) { s_max[0] = s_max[1] = s_max[2] = 0; }
    __syncthreads();
    uint64_t run_t = 0, run_s = 0, run_f = 0;
    const uint64_t use = num < item_cap ? num : item_cap;
    for (uint64_t base = 0; base < use; base += blockDim.x) {
        uint64_t i = base + threadIdx.x;
        uint64_t nt = 0, ns = 0, nf = 0, n = 0;
        if (i < use) {
            n = items[i].n;
            nt = (n + A.tile_keys - 1) / A.tile_keys;
            ns = sample_size(n, A.div, A.smin, A.smax);
            nf = ns > A.small_S ? (ns + A.fit_chunk - 1) / A.fit_chunk : 0;
            atomicMax((unsigned long long*)&s_max[0], (unsigned long long)ns);
            atomicMax((unsigned long long*)&s_max[1], (unsigned long long)n);
            atomicAdd((unsigned long long*)&s_max[2], (unsigned long long)n);
        }
        uint64_t tt, ts, tf;
        uint64_t et = block_exclusive_sum<uint64_t>(nt, sc, &tt);
        uint64_t es = block_exclusive_sum<uint64_t>(ns, sc, &ts);
        uint64_t ef = block_exclusive_sum<uint64_t>(nf, sc, &tf);
        if (i < use) {
            tile_off[i] = run_t + et;
            sample_off[i] = run_s + es;
            fit_off[i] = run_f + ef;
        }
        run_t += tt;
        run_s += ts;
        run_f += tf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tile_off[use] = run_t;
        sample_off[use] = run_s;
        fit_off[use] = run_f;
        uint64_t e = *err_word;
        if (num > item_cap || nb > base_cap) e |= kErrCapacity;
        *err_word = e;
        plan->num_items = use;
        plan->num_base = nb < base_cap ? nb : base_cap;
        plan->total_tiles = run_t;
        plan->total_samples = run_s;
        plan->total_fit_chunks = run_f;
        plan->max_S = s_max[0];
        plan->max_n = s_max[1];
        plan->sum_n = s_max[2];
        plan->err = e;
        plan->closed = stat_counts[0];
        plan->digit = stat_counts[1];
        plan->l2pl = stat_counts[2];
        plan->closed_keys = stat_counts[3];
        *item_count_cur = 0;  // this level's list is consumed
        *item_count_next = 0;
        *base_count = 0;
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

// ------------------------------------------------------------------ seeds
// Segments of an array (or of the sample buffer) become level-1 items (> T keys) or base-case
// buckets (2..T keys, sorted in place).
__global__ void k_seed(const uint64_t* off, uint64_t nseg, uint32_t T, Item* items, uint64_t* item_count,
                       BaseItem* base, uint64_t* base_count, uint64_t* err_word, uint64_t item_cap,
                       uint64_t base_cap) {
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    uint64_t a = off[s], b = off[s + 1];
    if (b < a) {
        atomicOr((unsigned long long*)err_word, (unsigned long long)kErrOffsets);
        return;
    }
    uint64_t n = b - a;
    if (n > T) {
        uint64_t i = atomicAdd((unsigned long long*)item_count, 1ull);
        if (i < item_cap) items[i] = Item{a, n, 0, 0};
    } else if (n >= 2) {
        uint64_t i = atomicAdd((unsigned long long*)base_count, 1ull);
        if (i < base_cap) base[i] = BaseItem{a, (uint32_t)n, 0};
    }
}

// ------------------------------------------------------------------ sample gather
// One key per stratum j = [floor(j n / S), floor((j+1) n / S)) of every item, moved inside the
// stratum by mix64(stream + (j+1) gamma), stream = mix64(seed ^ mix64(lo_rel gamma + n)).
// floor(j n / S) = j q + floor(j r / S) with n = q S + r keeps the arithmetic in 64 bits (S < 2^32).
template <int DT>
__global__ void k_sample(const Item* items, uint64_t num_items, const uint64_t* sample_off, uint64_t total,
                         const typename Key<DT>::T* src, typename Key<DT>::T* sample, uint64_t seed) {
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    const uint64_t q = it.n / S, r = it.n % S;
    const uint64_t a = j * q + (j * r) / S;
    const uint64_t b = (j + 1) * q + ((j + 1) * r) / S;
    const uint64_t stream = mix64(seed ^ mix64(it.lo_rel * kGamma + it.n));
    const uint64_t h = mix64(stream + (j + 1) * kGamma);
    sample[s] = src[it.lo + a + h % (b - a)];
}

// sample segments as base-case buckets of the sample buffer (when every sample has <= T keys)
__global__ void k_sample_base(const uint64_t* sample_off, uint64_t num_items, BaseItem* base) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_items) return;
    base[i] = BaseItem{sample_off[i], (uint32_t)(sample_off[i + 1] - sample_off[i]), 0};
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

// Small samples (S <= small_S): one workgroup per item, the sample in LDS as fp64, binary search.
template <int DT>
__global__ __launch_bounds__(256) void k_fmcd_small(const typename Key<DT>::T* sample, const uint64_t* sample_off,
                                                    uint64_t num_items, Model* models, uint32_t K, uint32_t small_S) {
    extern __shared__ double sx[];
    using KT = Key<DT>;
    const uint64_t i = blockIdx.x;
    if (i >= num_items) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
    if (S > small_S) return;
    for (uint64_t j = threadIdx.x; j < S; j += blockDim.x) sx[j] = KT::val(sample[off + j]);
    __syncthreads();
    Model m = {};
    m.S = S;
    bool usable = S >= 3 && isfinite(sx[0]) && isfinite(sx[S - 1]);
    if (usable) {
        const uint64_t Dmax = S / 3;
        uint64_t lo = 1, hi = Dmax + 1;
        while (lo < hi) {
            const uint64_t D = lo + ((hi - lo) >> 1);
            const double u = fmcd_spread(sx[S - 1 - D], sx[D], K);
            int fail = 0;
            for (uint64_t w = threadIdx.x; w + D < S; w += blockDim.x) fail |= !(sx[w + D] - sx[w] >= u);
            if (__syncthreads_or(fail)) lo = D + 1;
            else hi = D;
        }
        const uint64_t D = lo;
        const uint64_t Du = D <= Dmax ? D : Dmax;
        const double u = fmcd_spread(sx[S - 1 - Du], sx[Du], K);
        fmcd_line(u, sx[S - 1 - D], sx[D], K, &m.a, &m.b);
        m.D = D;
        usable = fit_usable(m.a, m.b);
    }
    if (!usable) model_degenerate(m);
    if (threadIdx.x == 0) models[i] = m;
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
                                                    int max_rounds, int round, uint32_t K, uint32_t chunk,
                                                    uint32_t cand) {
    using KT = Key<DT>;
    __shared__ uint64_t s_bits;
    const uint32_t i = fit_map[blockIdx.x];
    const uint64_t w = blockIdx.x - fit_off[i];
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
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
                              const uint64_t* masks, int rounds, Model* models, uint32_t K, uint32_t small_S,
                              uint32_t cand) {
    using KT = Key<DT>;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_items) return;
    const uint64_t off = sample_off[i], S = sample_off[i + 1] - off;
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

__global__ void k_degenerate_model(Model* m) {
    Model x = {};
    model_degenerate(x);
    m[0] = x;
}

// ------------------------------------------------------------------ degenerate buckets
// min and max ord of every bucket whose fit was degenerate (homogeneity check, Learned Sort
// section; digit fallback, IPS4o section).
template <int DT>
__global__ __launch_bounds__(256) void k_minmax(const Item* items, const uint64_t* tile_off, const uint32_t* tile_map,
                                                Model* models, const typename Key<DT>::T* src, uint32_t tile_keys) {
    using KT = Key<DT>;
    const uint32_t i = tile_map[blockIdx.x];
    if (models[i].kind != kKindPending) return;
    const Item it = items[i];
    const uint64_t base = (blockIdx.x - tile_off[i]) * tile_keys;
    const uint64_t end = (base + tile_keys < it.n) ? base + tile_keys : it.n;
    uint64_t mn = ~0ull, mx = 0;
    for (uint64_t j = base + threadIdx.x; j < end; j += blockDim.x) {
        const uint64_t o = KT::ord(src[it.lo + j]);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
    }
    mx = wave_max(mx);
    mn = ~wave_max(~mn);
    if (lane_id() == 0) {
        atomicMin((unsigned long long*)&models[i].umin, (unsigned long long)mn);
        atomicMax((unsigned long long*)&models[i].umax, (unsigned long long)mx);
    }
}

// Final model of every item: closes homogeneous buckets, sets the digit fallback, and picks the
// two-level model when the policy and the sample loads ask for it.
// stat_counts: [0] closed buckets, [1] digit splits, [2] two-level models, [3] keys in closed buckets
__global__ void k_finalize(const Item* items, Model* models, uint64_t num_items, uint32_t K, int src_is_scratch,
                           uint32_t policy, uint64_t* stat_counts) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= num_items) return;
    Model m = models[i];
    if (m.kind == kKindPending) {
        if (m.umin == m.umax) {
            m.kind = src_is_scratch ? kKindClosedMove : kKindClosedKeep;
            atomicAdd((unsigned long long*)&stat_counts[0], 1ull);
            atomicAdd((unsigned long long*)&stat_counts[3], (unsigned long long)items[i].n);
        } else {
            const int sh = (int)bit_length(m.umax - m.umin) - (int)(31 - __clz((int)K));
            m.kind = kKindDigit;
            m.shift = sh > 0 ? (uint32_t)sh : 0u;
            atomicAdd((unsigned long long*)&stat_counts[1], 1ull);
        }
    } else if (m.kind == kKindLinear && policy != 0 && m.l2_ok) {
        const bool splits = m.load_l2 < m.S;
        if (splits && (policy == 2 || m.load_l2 < m.load_lin)) {
            m.kind = kKindL2pl;
            atomicAdd((unsigned long long*)&stat_counts[2], 1ull);
        }
    }
    models[i] = m;
}

// ------------------------------------------------------------------ classify + histogram
// Every workgroup classifies a run of `tiles_per_group` consecutive tiles with per-wave LDS
// histograms and adds them to the item's global counts when the run leaves an item.
template <int DT>
__global__ __launch_bounds__(256) void k_classify_hist(const Item* items, const uint64_t* tile_off,
                                                       const uint32_t* tile_map, uint64_t total_tiles,
                                                       uint32_t tiles_per_group, const Model* models,
                                                       const double* leaves, const typename Key<DT>::T* src,
                                                       uint64_t* hist, uint32_t K, uint32_t M, uint32_t tile_keys) {
    __shared__ uint32_t h[4][kMaxBuckets];
    __shared__ double s_leaf[4 * kMaxLeaves];
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t t0 = (uint64_t)blockIdx.x * tiles_per_group;
    if (t0 >= total_tiles) return;
    const uint64_t t1 = (t0 + tiles_per_group < total_tiles) ? t0 + tiles_per_group : total_tiles;
    for (uint32_t b = threadIdx.x; b < 4 * kMaxBuckets; b += blockDim.x) (&h[0][0])[b] = 0;
    uint64_t t = t0;
    while (t < t1) {
        const uint32_t i = tile_map[t];
        const Item it = items[i];
        const Model m = models[i];
        const uint64_t tend_item = tile_off[i + 1];
        const uint64_t te = tend_item < t1 ? tend_item : t1;
        if (m.kind == kKindL2pl) {
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < 4 * M; q += blockDim.x) s_leaf[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
        }
        __syncthreads();
        if (m.kind != kKindClosedKeep) {
            const uint64_t k0 = (t - tile_off[i]) * tile_keys;
            uint64_t k1 = (te - tile_off[i]) * tile_keys;
            if (k1 > it.n) k1 = it.n;
            if (m.kind == kKindClosedMove) {
                if (threadIdx.x == 0) h[0][0] += (uint32_t)(k1 - k0);
            } else {
                for (uint64_t j = k0 + threadIdx.x; j < k1; j += blockDim.x) {
                    const uint32_t c = classify_key<DT>(m, s_leaf, K, M, src[it.lo + j]);
                    atomicAdd(&h[wave][c], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < K; b += blockDim.x) {
            const uint32_t v = h[0][b] + h[1][b] + h[2][b] + h[3][b];
            h[0][b] = h[1][b] = h[2][b] = h[3][b] = 0;
            if (v) atomicAdd((unsigned long long*)&hist[(uint64_t)i * K + b], (unsigned long long)v);
        }
        t = te;
    }
}

// Bucket starts of every item: exclusive prefix of its K counts.
__global__ __launch_bounds__(256) void k_bucket_starts(const uint64_t* hist, uint64_t* bstart, uint32_t K) {
    __shared__ uint64_t sc[16];
    const uint64_t i = blockIdx.x;
    const uint64_t v = threadIdx.x < K ? hist[i * K + threadIdx.x] : 0;
    uint64_t tot;
    const uint64_t e = block_exclusive_sum<uint64_t>(v, sc, &tot);
    if (threadIdx.x < K) bstart[i * K + threadIdx.x] = e;
}

// ------------------------------------------------------------------ scatter
// Stable distribution of one tile of 256 * IPT keys (Proposed Algorithm; the Worked Example's
// contiguous layout is the stable one).  Steps:
//   1. dynamic tile id (tiles only wait on tiles that started earlier, so the look-back always
//      makes progress);
//   2. classify in registers; wave w ranks its 64 * IPT keys row by row: lanes with the same
//      bucket are found with 8 ballots on the bucket bits, the running per-wave bucket count
//      lives in LDS;
//   3. per-bucket tile counts are published and a decoupled look-back over the item's earlier
//      tiles (one bucket per thread, flag and count packed in one 64-bit word) gives the tile's
//      offset inside each bucket;
//   4. keys are staged in LDS in bucket order and written out in runs, so each bucket's keys of
//      the tile land in one contiguous, coalesced span.
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62, kCountMask = (1ull << 62) - 1;

template <int DT, bool PAY, int IPT>
__global__ __launch_bounds__(256) void k_scatter(const Item* items, const uint64_t* tile_off, const uint32_t* tile_map,
                                                 const Model* models, const double* leaves, const uint64_t* bstart,
                                                 const typename Key<DT>::T* src, const uint32_t* src_pay,
                                                 typename Key<DT>::T* dst, uint32_t* dst_pay, uint64_t* status,
                                                 uint32_t* tile_counter, uint32_t K, uint32_t M) {
    using KT = Key<DT>;
    using T = typename KT::T;
    constexpr int TILE = kBlock * IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wcnt[4][kMaxBuckets];
    __shared__ uint32_t s_loc[kMaxBuckets];
    __shared__ uint64_t s_base[kMaxBuckets];
    __shared__ uint64_t s_scan[16];
    __shared__ T s_keys[TILE];
    __shared__ uint8_t s_bkt[TILE];
    __shared__ uint32_t s_pay[PAY ? TILE : 1];
    __shared__ double s_leaf[4 * kMaxLeaves];

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (uint32_t b = tid; b < 4 * kMaxBuckets; b += kBlock) (&s_wcnt[0][0])[b] = 0;
    __syncthreads();
    const uint32_t t = s_tile;
    const uint32_t i = tile_map[t];
    const Model m = models[i];
    if (m.kind == kKindClosedKeep) return;
    const Item it = items[i];
    const uint64_t tau = t - tile_off[i];
    const uint64_t base = it.lo + tau * TILE;
    const uint64_t rem = it.n - tau * TILE;
    const uint32_t tn = rem < (uint64_t)TILE ? (uint32_t)rem : (uint32_t)TILE;
    if (m.kind == kKindL2pl) {
        for (uint32_t q = tid; q < 4 * M; q += kBlock) s_leaf[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
        __syncthreads();
    }

    // 1-2: load, classify, rank within the wave
    T k[IPT];
    uint32_t p[PAY ? IPT : 1];
    uint32_t bk[IPT], rk[IPT];
    const uint32_t wbase = wave * kWave * IPT;
    volatile uint32_t* wc = s_wcnt[wave];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t idx = wbase + r * kWave + lane;
        const bool valid = idx < tn;
        uint32_t b = 0;
        if (valid) {
            k[r] = src[base + idx];
            if (PAY) p[r] = src_pay[base + idx];
            b = classify_key<DT>(m, s_leaf, K, M, k[r]);
        }
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t ones = __ballot((b >> bit) & 1u);
            same &= ((b >> bit) & 1u) ? ones : ~ones;
        }
        const uint32_t below = count_below(same);
        const uint32_t prev = valid ? wc[b] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wc[b] = prev + (uint32_t)__popcll(same);
        __builtin_amdgcn_wave_barrier();
        bk[r] = b;
        rk[r] = prev + below;
    }
    __syncthreads();

    // 3: tile counts, per-wave offsets, tile-local bucket offsets, look-back
    const uint32_t b = tid;  // one bucket per thread (K <= 256)
    uint32_t cnt = 0;
    if (b < K) {
        const uint32_t c0 = s_wcnt[0][b], c1 = s_wcnt[1][b], c2 = s_wcnt[2][b], c3 = s_wcnt[3][b];
        s_wcnt[0][b] = 0;
        s_wcnt[1][b] = c0;
        s_wcnt[2][b] = c0 + c1;
        s_wcnt[3][b] = c0 + c1 + c2;
        cnt = c0 + c1 + c2 + c3;
    }
    uint64_t tot;
    const uint32_t loc = (uint32_t)block_exclusive_sum<uint64_t>(cnt, s_scan, &tot);
    if (b < K) {
        s_loc[b] = loc;
        uint64_t* st = status + (uint64_t)t * K + b;
        uint64_t excl = 0;
        if (tau == 0) {
            __hip_atomic_store(st, kFlagInc | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st, kFlagAgg | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t pt = t - 1;
            for (;;) {
                uint64_t v;
                do {
                    v = __hip_atomic_load(status + pt * K + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while ((v & ~kCountMask) == 0);
                excl += v & kCountMask;
                if (v & kFlagInc) break;
                --pt;
            }
            __hip_atomic_store(st, kFlagInc | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_base[b] = it.lo + bstart[(uint64_t)i * K + b] + excl - loc;
    }
    __syncthreads();

    // 4: stage in bucket order, write runs
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t idx = wbase + r * kWave + lane;
        if (idx < tn) {
            const uint32_t pos = s_loc[bk[r]] + s_wcnt[wave][bk[r]] + rk[r];
            s_keys[pos] = k[r];
            s_bkt[pos] = (uint8_t)bk[r];
            if (PAY) s_pay[pos] = p[r];
        }
    }
    __syncthreads();
    for (uint32_t j = tid; j < tn; j += kBlock) {
        const uint64_t d = s_base[s_bkt[j]] + j;
        dst[d] = s_keys[j];
        if (PAY) dst_pay[d] = s_pay[j];
    }
}

// ------------------------------------------------------------------ worklist
// Children of every item: > T keys -> next level's items; otherwise -> base case (a single key
// needs the base case only to move out of the scratch buffer).  Closed buckets have no children.
__global__ void k_worklist(const Item* items, uint64_t num_items, const Model* models, const uint64_t* hist,
                           const uint64_t* bstart, uint32_t K, uint32_t T, int dst_is_scratch, Item* next,
                           uint64_t* next_count, BaseItem* base, uint64_t* base_count, uint64_t next_cap,
                           uint64_t base_cap) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= num_items * K) return;
    const uint64_t i = g / K;
    const uint32_t kind = models[i].kind;
    if (kind == kKindClosedKeep || kind == kKindClosedMove) return;
    const uint64_t c = hist[g];
    if (c == 0) return;
    const Item it = items[i];
    const uint64_t start = bstart[g];
    if (c > T) {
        const uint64_t q = atomicAdd((unsigned long long*)next_count, 1ull);
        if (q < next_cap) next[q] = Item{it.lo + start, c, it.lo_rel + start, 0};
    } else if (c >= 2 || dst_is_scratch) {
        const uint64_t q = atomicAdd((unsigned long long*)base_count, 1ull);
        if (q < base_cap) base[q] = BaseItem{it.lo + start, (uint32_t)c, (uint32_t)dst_is_scratch};
    }
}

// ------------------------------------------------------------------ base case
// Buckets of <= T keys (Proposed Algorithm: a radix sort below 2^12 keys in the paper; here an
// LDS bitonic sort) sorted by ord and written into the caller's buffer.  With a payload the sort
// key is (ord, position), which makes it stable.
template <int DT, bool PAY>
__global__ __launch_bounds__(256) void k_base_case(const BaseItem* list, typename Key<DT>::T* keys, uint32_t* pay,
                                                   const typename Key<DT>::T* skeys, const uint32_t* spay) {
    using KT = Key<DT>;
    __shared__ uint64_t so[kMaxBase];
    __shared__ uint16_t si[PAY ? kMaxBase : 1];
    __shared__ uint32_t sp[PAY ? kMaxBase : 1];
    const BaseItem bi = list[blockIdx.x];
    const typename KT::T* src = bi.from_scratch ? skeys : keys;
    const uint32_t* psrc = bi.from_scratch ? spay : pay;
    const uint32_t n = bi.n;
    if (n == 1) {
        if (threadIdx.x == 0) {
            keys[bi.lo] = src[bi.lo];
            if (PAY) pay[bi.lo] = psrc[bi.lo];
        }
        return;
    }
    uint32_t P = 2;
    while (P < n) P <<= 1;
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) {
        so[j] = j < n ? KT::ord(src[bi.lo + j]) : ~0ull;
        if (PAY) {
            si[j] = (uint16_t)j;
            if (j < n) sp[j] = psrc[bi.lo + j];
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = threadIdx.x; q < (P >> 1); q += blockDim.x) {
                const uint32_t a = (q / j) * 2 * j + (q % j), c = a + j;
                const bool up = (a & k) == 0;
                const uint64_t oa = so[a], oc = so[c];
                bool swap;
                if (PAY) {
                    const uint16_t ia = si[a], ic = si[c];
                    const bool gt = oa > oc || (oa == oc && ia > ic);
                    swap = gt == up;
                    if (swap) {
                        si[a] = ic;
                        si[c] = ia;
                    }
                } else {
                    swap = (oa > oc) == up && oa != oc;
                }
                if (swap) {
                    so[a] = oc;
                    so[c] = oa;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
        keys[bi.lo + j] = KT::from_ord(so[j]);
        if (PAY) pay[bi.lo + j] = sp[si[j]];
    }
}

}  // namespace ipls
