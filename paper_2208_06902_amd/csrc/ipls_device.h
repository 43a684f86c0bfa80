// Device-side building blocks of the IPLS library for gfx950 (wave64, 160 KB LDS per CU).
//
// Key map (Experimental Evaluation chapter: doubles are sorted through an order-preserving map to
// unsigned integers), the counter-based hash that jitters sample positions, the clamped linear
// partition model (Linear Models section), and the per-bucket state that flows between kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipls {

constexpr int kWave = 64;
constexpr int kBlock = 256;        // threads of every distribution kernel
constexpr int kMaxBuckets = 256;   // K <= 256: a bucket index is one byte
constexpr int kMaxBase = 4096;     // T <= 4096: a base-case bucket fits one workgroup's LDS
constexpr int kMaxLeaves = 256;

enum : uint32_t {
    kKindLinear = 0,      // FMCD line
    kKindDigit = 1,       // degenerate fit: most-significant digit of ord - umin
    kKindClosedKeep = 2,  // homogeneous bucket already in the caller's buffer: nothing to do
    kKindClosedMove = 3,  // homogeneous bucket in the scratch buffer: copied through bucket 0
    kKindL2pl = 4,        // two-level piecewise-linear CDF model
    kKindPending = 5,     // degenerate fit awaiting the bucket's min/max ord
    kKindTree = 6         // splitter tree over K-1 sample quantiles (shift = 1: strict comparison)
};

// Number of leaf-table doubles a model's classification reads from LDS (two-level model: 4 M
// coefficients; splitter tree: K - 1 splitter ords).
__device__ inline uint32_t model_table_size(uint32_t kind, uint32_t K, uint32_t M) {
    return kind == kKindL2pl ? 4 * M : (kind == kKindTree ? K - 1 : 0u);
}

// One bucket to partition at the current level: keys [lo, lo+n) of the level's source buffer;
// lo_rel is its offset inside its top-level segment (sample positions hash it).  inh: 1 + the
// index of its entry in the previous level's child list when it inherits its part of the parent's
// sorted sample (and the model fitted on it), else 0.
struct Item {
    uint64_t lo, n, lo_rel, inh;
};

// Sample inheritance: a child bucket of a partition by the FMCD line that will be partitioned
// itself reuses the parent's sorted sample restricted to it (a contiguous range, since the line
// is monotone).  Its line is fitted before the parent's scatter, which then also writes each
// key's class under that line (one byte per key), so the child's counting pass reads bytes
// instead of keys.
struct Child {
    double a, b;         // FMCD line of the restricted sample; a = 0 when the fit is unusable
    uint64_t D;          // its conflict degree
    uint64_t s_lo;       // the restricted sample: [s_lo, s_lo + s_len) of the level's sample buffer
    uint32_t s_len, c;   // c: the parent's bucket it is
};

// An item's entries in its level's child list: [base, base + count).
struct ChildSpan {
    uint32_t base, count;
};

// A pass tile: its first key's position in the level's source buffer, its item and its key count,
// so that a pass's workgroup can issue its key loads after one dependent read.
struct TileInfo {
    uint64_t base;
    uint32_t item, n;
};

// A bucket of <= T keys for the base case, at [lo, lo+n) of the caller's buffer (from_scratch = 0)
// or of the scratch buffer (1).  The result always lands in the caller's buffer.
struct BaseItem {
    uint64_t lo;
    uint32_t n;
    uint32_t from_scratch;
};

// Model of one bucket, produced by the fit kernels, read by classification.
constexpr int kMaxHeavy = 16;  // equality buckets per partitioned bucket

struct Model {
    uint32_t kind, shift;
    double a, b;                 // linear: t = fma(a, val, b); also the two-level model's root
    uint64_t D, S;               // FMCD conflict degree, sample size
    uint64_t umin, umax;         // ord range (degenerate fits only)
    uint64_t load_lin, load_l2;  // max sample load of FMCD and of the two-level model
    uint32_t l2_ok;
    uint32_t inh;                // 1: inherited line; the level's counts come from the class bytes
    // equality buckets: neq heavy values (ords, ascending); the linear part has km buckets, or
    // sends every other key to bucket 0 (const0)
    uint32_t neq, km, const0;
    uint32_t kb;  // buckets of this item's line when they differ from the level's K (0: K)
    uint64_t heavy[kMaxHeavy];
    uint8_t eqb[kMaxHeavy];  // the bucket of each heavy value
};

// An equality bucket whose keys a level wrote to the scratch buffer: moved back as they are.
struct CopyItem {
    uint64_t lo, n;
};

// Heavy values of an item's sorted sample and the length of the sample without their runs.
struct EqInfo {
    uint32_t neq, km;
    uint64_t sr;
    uint64_t heavy[kMaxHeavy];
};

// Level plan, computed on the device from the item list and read back by the host.
constexpr int kBaseClasses = 7;  // base-case size classes: n <= 64 * 2^c keys, c = 0..6

struct Plan {
    uint64_t num_items, num_base, total_tiles, total_samples, total_fit_chunks, max_S, max_n, sum_n;
    uint64_t err;
    uint64_t closed, digit, l2pl;  // buckets closed / split by digit / by the two-level model so far
    uint64_t closed_keys;          // keys of closed buckets so far
    uint64_t base_keys;            // keys in this level's base-case buckets
    uint64_t cls_count[kBaseClasses];
    uint64_t total_chunks;
    uint64_t eq_closed;                // equality buckets closed so far
    uint64_t copy_count, copy_tiles;   // equality buckets to move back, in tiles of kCopyTile keys
    uint64_t inherited;                // partitions whose model was inherited, so far
    uint64_t inh_n;                    // keys of this level's items with inherited lines
    uint64_t l1max;                    // largest bucket of the first level (single-array sorts)
    uint64_t n_wide;                   // items of more than kScanSerial chunks
    uint64_t seq;                      // the host's number of the k_plan launch that wrote it
};

constexpr uint32_t kCopyTile = 4096;

// counters of one nesting depth (uint64 slots)
enum : int {
    C_ITEMS0 = 0, C_ITEMS1 = 1, C_BASE = 2, C_ERR = 3, C_TILE = 4,
    C_STATS = 5,      // 4 slots: closed buckets, digit splits, two-level models, closed keys
    C_BASEKEYS = 9,   // keys appended to the base-case list
    C_CLS = 10,       // 7 slots: base-case buckets per size class
    C_EQCLOSED = 17,  // equality buckets closed where they were made (all levels)
    C_COPY = 18,      // equality buckets of this level to move from the scratch buffer
    C_COPYKEYS = 19,  // ... and their keys
    C_CHILD = 20,     // entries of this level's child list
    C_INHERITED = 21, // partitions with an inherited model (all levels)
    C_L1MAX = 22,     // largest bucket of the first level (single-array sorts)
    C_N = 32
};

// Base-case buckets are appended to one list split into a fixed region per size class.  A bucket
// of class c >= 1 holds more than 32 * 2^c keys, so at most len / (32 * 2^c) of them exist;
// class 0 gets the general bound.
struct BaseLayout {
    uint64_t off[kBaseClasses + 1];
    uint64_t cap[kBaseClasses];
};

// size class of a base-case bucket: the smallest c with n <= 64 * 2^c
__device__ __host__ inline int base_class(uint32_t n) {
    int c = 0;
    uint32_t cap = 64;
    while (cap < n && c < kBaseClasses - 1) {
        cap <<= 1;
        ++c;
    }
    return c;
}

// Buckets of the partition of an item of n keys under the bucket policy (adapt != 0): the smallest
// power of two k >= 8n/T within [min(K, 64), K] (a bucket then expects at most T/8 keys);
// otherwise K.
__device__ __host__ inline uint32_t bucket_count(uint64_t n, uint32_t K, uint32_t T, uint32_t adapt) {
    if (!adapt) return K;
    // k < ceil(8n/T) exactly when k T < 8n (k an integer): no 64-bit division
    uint32_t k = 1;
    while (k < K && (uint64_t)k * T < 8 * n) k <<= 1;
    const uint32_t lo = K < 64 ? K : 64;
    return k < lo ? lo : (k > K ? K : k);
}

// Error bits of the device error word.
enum : uint64_t { kErrOffsets = 1, kErrCapacity = 2, kErrProgress = 4, kErrInvariant = 8 };

// ------------------------------------------------------------------ key map
// ord(): IEEE 754 totalOrder as an unsigned integer (flip a negative number's bits, set a positive
// number's sign bit); val(): the fp64 value the model sees (fp32 widened exactly, u64 rounded to
// nearest even); neg(): the sign bit, which sends a NaN to the matching end.
template <int DT>
struct Key;

template <>
struct Key<0> {  // fp64
    using T = uint64_t;
    using O = uint64_t;  // ord type
    __device__ static inline uint64_t ord(T u) { return (u >> 63) ? ~u : (u | 0x8000000000000000ull); }
    __device__ static inline T from_ord(uint64_t o) { return (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o; }
    __device__ static inline double val(T u) { return __longlong_as_double((long long)u); }
    __device__ static inline bool neg(T u) { return (u >> 63) != 0; }
};

template <>
struct Key<1> {  // fp32
    using T = uint32_t;
    using O = uint32_t;
    __device__ static inline uint64_t ord(T u) { return (u & 0x80000000u) ? (uint64_t)(uint32_t)~u : (uint64_t)(u | 0x80000000u); }
    __device__ static inline T from_ord(uint64_t o) {
        uint32_t u = (uint32_t)o;
        return (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    }
    __device__ static inline double val(T u) { return (double)__uint_as_float(u); }
    __device__ static inline bool neg(T u) { return (u >> 31) != 0; }
};

template <>
struct Key<2> {  // uint64
    using T = uint64_t;
    using O = uint64_t;
    __device__ static inline uint64_t ord(T u) { return u; }
    __device__ static inline T from_ord(uint64_t o) { return o; }
    __device__ static inline double val(T u) { return __ull2double_rn(u); }
    __device__ static inline bool neg(T) { return false; }
};

// ------------------------------------------------------------------ sample hash
// SplitMix64's output function (Steele, Lea, Flood 2014) used as a counter-based hash.
__device__ __host__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

// Binary logarithm of n >= 1: exponent plus 24 fractional bits, each bit read off by squaring
// the mantissa in [1, 2) and halving it when it reaches 2.
__device__ __host__ inline double log2_bits(uint64_t n) {
    int e = 63 - __builtin_clzll(n);
    double m = (double)n * __builtin_bit_cast(double, (uint64_t)(1023 - e) << 52);
    if (m >= 2.0) {  // (double)n rounded up to 2^(e+1)
        m *= 0.5;
        e += 1;
    }
    double frac = 0.0, bit = 0.5;
    for (int i = 0; i < 24; ++i) {
        m = m * m;
        if (m >= 2.0) {
            m *= 0.5;
            frac += bit;
        }
        bit *= 0.5;
    }
    return (double)e + frac;
}

// Sample size of a bucket of n keys.  Policy 0: ceil(n / div), at least smin.  Policy 1 (the
// paper's IPLS): alpha*K - 1 with alpha = 0.2 log2(n), rounded to nearest (halves down), at
// least smin, at most ceil(n/2).  Then at most smax (if non-zero) and never above n.
__device__ __host__ inline uint64_t sample_size(uint64_t n, uint64_t div, uint64_t smin, uint64_t smax,
                                                uint32_t policy, uint32_t K) {
    uint64_t s;
    if (policy == 1) {
        double t = 0.2 * log2_bits(n ? n : 1) * (double)K - 0.5;
        s = t > 0.0 ? (uint64_t)t : 0;
        if (s < smin) s = smin;
        if (s > (n + 1) / 2) s = (n + 1) / 2;
    } else {
        // ceil(n / div); in 32 bits when it fits (the same quotient, far fewer instructions)
        const uint64_t t = n + div - 1;
        s = (t >> 32) == 0 ? (uint64_t)((uint32_t)t / (uint32_t)div) : t / div;
        if (s < smin) s = smin;
    }
    if (smax && s > smax) s = smax;
    if (s > n) s = n;
    return s;
}

// ------------------------------------------------------------------ partition models
// Clamped linear model (Linear Models section): comparing t is the same as comparing floor(t)
// with 0 and K; a NaN t (NaN key) goes to the end its sign gives.  One explicit fp64 fma.
__device__ inline uint32_t classify_linear(double a, double b, uint32_t K, double v, bool neg) {
    // straight-line form of: t < 0 -> 0; t >= K -> K - 1; else floor(t) (t in [K - 1, K) floors to
    // K - 1, so clamping t to [0, K - 1] first gives the same bucket); a NaN t (a NaN key) -> the
    // end its sign bit names.  fmax returns 0 for a NaN t, so the conversion is always in range.
    const double t = __builtin_fma(a, v, b);
    const uint32_t c = (uint32_t)__builtin_fmin(__builtin_fmax(t, 0.0), (double)(K - 1u));
    return t == t ? c : (neg ? 0u : K - 1u);
}

// Two-level model: root routes to a leaf, the leaf's line is clipped to its envelope [LO, HI].
__device__ inline uint32_t classify_l2pl(double ra, double rb, uint32_t M, const double* leaf, uint32_t K, double v,
                                         bool neg) {
    // leaf from the root line (a NaN key reads the last leaf and is sent to its end below), then
    // the leaf's line clamped to its envelope [q[2], q[3]], then the bucket as classify_linear
    const double* q = leaf + 4 * classify_linear(ra, rb, M, v, false);
    const double t = __builtin_fmin(__builtin_fmax(__builtin_fma(q[0], v, q[1]), q[2]), q[3]);
    const uint32_t c = (uint32_t)__builtin_fmin(__builtin_fmax(t, 0.0), (double)(K - 1u));
    return v == v ? c : (neg ? 0u : K - 1u);
}

// Equality buckets (IPS4o's): with heavy values h_0 < ... < h_(E-1) a key goes to
// linear bucket (of km) + 2 #{e : h_e < key} + [key is some h_e]; the buckets stay in key order
// and each heavy value has one of its own.
template <int DT>
__device__ inline uint32_t classify_equality(const Model& m, typename Key<DT>::T u) {
    using KT = Key<DT>;
    const uint64_t o = KT::ord(u);
    uint32_t less = 0, eq = 0;
#pragma unroll
    for (int e = 0; e < kMaxHeavy; ++e) {
        if ((uint32_t)e < m.neq) {
            less += m.heavy[e] < o ? 1u : 0u;
            eq |= m.heavy[e] == o ? 1u : 0u;
        }
    }
    const uint32_t b = m.const0 ? 0u : classify_linear(m.a, m.b, m.km, KT::val(u), KT::neg(u));
    return b + 2u * less + eq;
}

// Splitter tree (the Decision Trees section: IPS4o's classifier): the number of splitters below
// the key (strict) or at most the key, by a branchless search over the sorted K-1 splitters.
__device__ inline uint32_t classify_tree(const uint64_t* split, uint32_t K, uint64_t o, bool strict) {
    const uint32_t ns = K - 1;
    uint32_t step = 1u << (31 - __clz((int)ns)), b = 0;
    for (; step; step >>= 1) {
        if (b + step <= ns) {
            const uint64_t sv = split[b + step - 1];
            if (strict ? sv < o : sv <= o) b += step;
        }
    }
    return b;
}

template <int DT>
__device__ inline uint32_t classify_key(const Model& m, const double* leaf, uint32_t K, uint32_t M,
                                        typename Key<DT>::T u) {
    using KT = Key<DT>;
    switch (m.kind) {
        case kKindDigit: return (uint32_t)((KT::ord(u) - m.umin) >> m.shift);
        case kKindTree: return classify_tree((const uint64_t*)leaf, K, KT::ord(u), m.shift != 0);
        case kKindClosedMove: return 0u;
        case kKindL2pl: return classify_l2pl(m.a, m.b, M, leaf, K, KT::val(u), KT::neg(u));
        default:
            if (m.neq) return classify_equality<DT>(m, u);
            return classify_linear(m.a, m.b, m.kb ? m.kb : K, KT::val(u), KT::neg(u));
    }
}

// ------------------------------------------------------------------ wave and block primitives
__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of `mask` in lanes below this one
__device__ inline uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename V>
__device__ inline V wave_inclusive_sum(V v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        V o = __shfl_up(v, s, kWave);
        if (lane >= (uint32_t)s) v += o;
    }
    return v;
}

// Exclusive sum over the block (blockDim.x a multiple of 64, at most 1024 threads); *total gets
// the block's sum.  `scratch` holds 16 values.
template <typename V>
__device__ inline V block_exclusive_sum(V v, V* scratch, V* total) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    V inc = wave_inclusive_sum(v);
    if (lane == kWave - 1) scratch[wave] = inc;
    __syncthreads();
    V before = 0, all = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        V s = scratch[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Exclusive sums of NV values per thread over the block in one exchange (blockDim.x a multiple of
// 64, at most 1024 threads); tot gets the block's sums.  `scratch` holds 16 * NV values.
template <int NV>
__device__ inline void block_exclusive_sums(const uint64_t (&v)[NV], uint64_t (&ex)[NV], uint64_t (&tot)[NV],
                                            uint64_t* scratch) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    uint64_t inc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) inc[j] = wave_inclusive_sum<uint64_t>(v[j]);
    if (lane == kWave - 1)
#pragma unroll
        for (int j = 0; j < NV; ++j) scratch[wave * NV + j] = inc[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        uint64_t before = 0, all = 0;
        for (uint32_t w = 0; w < nw; ++w) {
            const uint64_t x = scratch[w * NV + j];
            if (w < wave) before += x;
            all += x;
        }
        ex[j] = before + inc[j] - v[j];
        tot[j] = all;
    }
    __syncthreads();
}

template <typename V>
__device__ inline V wave_max(V v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        V o = __shfl_xor(v, s, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Sum of the 64 lanes' values in the fixed tree (lane p += lane p+s, s = 32, 16, ..., 1); the
// result is valid in lane 0.  The same order as the CPU reference's 64-way pairwise tree.
__device__ inline double wave_tree_sum(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        double o = __shfl_down(v, s, kWave);
        v = v + o;
    }
    return v;
}

// Wave-aggregated append: every lane with `want` gets a distinct slot of `counter`, with one atomic
// per wave.  All active lanes of the wave must call it.
__device__ inline uint64_t wave_append(bool want, uint64_t* counter) {
    const uint64_t m = __ballot(want);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint64_t base = 0;
    if ((int)lane_id() == leader) base = atomicAdd((unsigned long long*)counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, kWave);
    return base + count_below(m);
}

// Block-aggregated append for the worklist and the seeds.  Every thread of the block calls it with
// a channel: -1 (nothing), 0 (a next-level item) or 1 + c (a base-case bucket of size class c);
// it returns the thread's slot in its channel and adds `keys` of base-case buckets to the key
// counter.  One global atomic per channel per block.
struct AppendScratch {
    uint32_t wc[kBaseClasses + 1][kBlock / kWave];
    uint64_t gbase[kBaseClasses + 1];
    unsigned long long keys;
};

__device__ inline uint64_t block_append(int ch, uint64_t keys, AppendScratch& sc, uint64_t* item_counter,
                                        uint64_t* cls_counter, uint64_t* key_counter) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t local = 0;
    if (threadIdx.x == 0) sc.keys = 0;
    for (int c = 0; c <= kBaseClasses; ++c) {
        const uint64_t m = __ballot(ch == c);
        if (lane == 0) sc.wc[c][wave] = (uint32_t)__popcll(m);
        if (ch == c) local = count_below(m);
    }
    uint64_t v = ch > 0 ? keys : 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
    __syncthreads();
    if (lane == 0 && v) atomicAdd(&sc.keys, (unsigned long long)v);
    if (threadIdx.x <= (uint32_t)kBaseClasses) {
        const int c = threadIdx.x;
        uint32_t tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += sc.wc[c][w];
        uint64_t* ctr = c == 0 ? item_counter : &cls_counter[c - 1];
        sc.gbase[c] = tot ? atomicAdd((unsigned long long*)ctr, (unsigned long long)tot) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && sc.keys) atomicAdd((unsigned long long*)key_counter, sc.keys);
    if (ch < 0) return 0;
    uint32_t woff = 0;
    for (uint32_t w = 0; w < wave; ++w) woff += sc.wc[ch][w];
    return sc.gbase[ch] + woff + local;
}

// As block_append, with the workgroup's own counters in LDS (lc: one per class, lkeys: keys of
// base-case buckets): returns the entry's rank among the workgroup's entries of its class so far.
// The workgroup adds its totals to the device counters once, after all its items.
__device__ inline uint32_t block_append_local(int ch, uint64_t keys, AppendScratch& sc, uint32_t* lc,
                                              unsigned long long* lkeys) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t local = 0;
    for (int c = 0; c <= kBaseClasses; ++c) {
        const uint64_t m = __ballot(ch == c);
        if (lane == 0) sc.wc[c][wave] = (uint32_t)__popcll(m);
        if (ch == c) local = count_below(m);
    }
    uint64_t v = ch > 0 ? keys : 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
    __syncthreads();
    if (lane == 0 && v) atomicAdd(lkeys, (unsigned long long)v);
    if (threadIdx.x <= (uint32_t)kBaseClasses) {
        const int c = threadIdx.x;
        uint32_t tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += sc.wc[c][w];
        sc.gbase[c] = lc[c];
        lc[c] += tot;
    }
    __syncthreads();
    if (ch < 0) return 0;
    uint32_t woff = 0;
    for (uint32_t w = 0; w < wave; ++w) woff += sc.wc[ch][w];
    return (uint32_t)sc.gbase[ch] + woff + local;
}

// Inclusive max over the block of int values (blockDim.x a multiple of 64, at most 1024 threads);
// `scratch` holds 16 values.
__device__ inline int block_inclusive_max(int v, int* scratch) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const int o = __shfl_up(v, s, kWave);
        if (lane >= (uint32_t)s) v = o > v ? o : v;
    }
    if (lane == kWave - 1) scratch[wave] = v;
    __syncthreads();
    for (uint32_t w = 0; w < wave && w < nw; ++w) v = scratch[w] > v ? scratch[w] : v;
    __syncthreads();
    return v;
}

__device__ inline uint32_t bit_length(uint64_t v) { return v ? 64u - (uint32_t)__clzll((long long)v) : 0u; }

}  // namespace ipls
