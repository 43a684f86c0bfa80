// Base-case kernels of the IPLS sort on gfx950: buckets of at most T keys sorted in LDS and
// written into the caller's buffer.  Included at the end of ipls_kernels.h.
#pragma once

#include "ipls_device.h"

namespace ipls {

// ------------------------------------------------------------------ base case
// Buckets of <= T keys are sorted by ord and written into the caller's buffer (the paper's base
// case below 2^12 keys, Proposed Algorithm).  A group of NT threads sorts one bucket of up to
// 16 NT keys; 256 / NT buckets share a workgroup.
//   1. every thread sorts 16 keys in registers with a bitonic network;
//   2. log2(NT) rounds merge pairs of sorted runs through LDS.  A thread finds where its 16
//      outputs start in the two runs with a merge-path search, loads the next 16 keys of each
//      run (independent loads), keeps the 16 smallest with one compare-exchange stage (their
//      sequence is bitonic) and sorts them with a 4-stage bitonic merge.
// With a payload every key carries its current position and compares as (ord, position); the
// left run's keys come first on ties, which is exactly the stable order.
// LDS index with one pad slot every 16 elements, so that a thread's 16 consecutive elements start
// in different banks.
__device__ inline int pad16(int j) { return j + (j >> 4); }

template <bool PAY, typename O>
__device__ inline bool key_less(O ka, uint32_t ia, O kb, uint32_t ib) {
    return PAY ? (ka < kb || (ka == kb && ia < ib)) : (ka < kb);
}

// compare-exchange: afterwards (a, b) is in ascending (up) or descending order
template <bool PAY, typename O>
__device__ inline void cex(O& ka, O& kb, uint32_t& ia, uint32_t& ib, uint32_t& pa, uint32_t& pb, bool up) {
    const bool sw = up ? key_less<PAY>(kb, ib, ka, ia) : key_less<PAY>(ka, ia, kb, ib);
    const O k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    ka = k0;
    kb = k1;
    if (PAY) {
        const uint32_t i0 = sw ? ib : ia, i1 = sw ? ia : ib, p0 = sw ? pb : pa, p1 = sw ? pa : pb;
        ia = i0;
        ib = i1;
        pa = p0;
        pb = p1;
    }
}

// Merge sort of CAP = 16 NT keys held in LDS (pad16 layout, positions 0 .. CAP-1, padding keys
// are kPad at the end) by NT threads t = 0 .. NT-1 of one group; the sorted keys are left in LDS.
// Payload sorts (PAY) hold each key's original index in sp (padding slots: indices >= the bucket
// size) and compare (ord, index), which is the stable order; the caller gathers the payloads by
// index afterwards.  Threads of the workgroup that are not among the NT pass active = false: they
// only take part in the barriers.
template <typename O, bool PAY, int NT>
__device__ inline void merge_sort_lds(O* sk, uint32_t* sp, int t_in, bool active = true) {
    const int t = active ? t_in : 0;  // inactive threads read in bounds and write nothing
    constexpr int IPT = 16, CAP = NT * IPT;
    constexpr O kPad = (O)~(O)0;
    O k[IPT];
    uint32_t id[IPT], nop = 0;  // id: original index (payload sorts only)
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        k[i] = sk[pad16(t * IPT + i)];
        id[i] = PAY ? sp[pad16(t * IPT + i)] : 0u;
    }
    // 1: bitonic sort of the thread's 16 keys
#pragma unroll
    for (int kk = 2; kk <= IPT; kk <<= 1)
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int l = i ^ j;
                if (l > i) cex<PAY>(k[i], k[l], id[i], id[l], nop, nop, (i & kk) == 0);
            }
    // 2: merge rounds, runs of L keys -> 2L
#pragma unroll 1
    for (int L = IPT; L < CAP; L <<= 1) {
        __syncthreads();
        if (active) {
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                sk[pad16(t * IPT + i)] = k[i];
                if (PAY) sp[pad16(t * IPT + i)] = id[i];
            }
        }
        __syncthreads();
        const int q = (t * IPT) / (2 * L), d = t * IPT - q * 2 * L;
        const int a0 = q * 2 * L, b0 = a0 + L;  // unpadded starts of the two runs
        int lo = d > L ? d - L : 0, hi = d < L ? d : L;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sk[pad16(a0 + mid)] <= sk[pad16(b0 + d - 1 - mid)]) lo = mid + 1;
            else hi = mid;
        }
        const int ia = lo, ib = d - lo;
        O xa[IPT], xb[IPT];
        uint32_t qa[IPT], qb[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            xa[j] = ia + j < L ? sk[pad16(a0 + ia + j)] : kPad;
            xb[j] = ib + j < L ? sk[pad16(b0 + ib + j)] : kPad;
            if (PAY) {
                // past-the-end slots get indices past every real one, so real keys win ties
                qa[j] = ia + j < L ? sp[pad16(a0 + ia + j)] : (uint32_t)(2 * CAP + j);
                qb[j] = ib + j < L ? sp[pad16(b0 + ib + j)] : (uint32_t)(3 * CAP + j);
            }
        }
        // the 16 smallest of the two sorted windows: min(xa[j], xb[15-j]) is bitonic
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t ua = PAY ? qa[j] : 0u, ub = PAY ? qb[IPT - 1 - j] : 0u;
            const bool takeB = key_less<PAY>(xb[IPT - 1 - j], ub, xa[j], ua);
            k[j] = takeB ? xb[IPT - 1 - j] : xa[j];
            id[j] = takeB ? ub : ua;
        }
#pragma unroll
        for (int j = IPT >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int l = i ^ j;
                if (l > i) cex<PAY>(k[i], k[l], id[i], id[l], nop, nop, true);
            }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            sk[pad16(t * IPT + i)] = k[i];
            if (PAY) sp[pad16(t * IPT + i)] = id[i];
        }
    }
    __syncthreads();
}

// The merge-sort classes' LDS: 256 / NT groups of 16 NT keys and their pad slots, the same size for
// every NT.
constexpr int kBaseSortLds = kBlock * 17;

// One workgroup (block blk of its class) of the merge-sort classes: 256 / NT buckets of at most 16 NT
// keys each, s_k and s_p holding kBaseSortLds slots.
template <int DT, bool PAY, int NT>
__device__ inline void base_sort_block(const BaseItem* list, uint64_t count, uint64_t blk, typename Key<DT>::T* keys,
                                       uint32_t* pay, const typename Key<DT>::T* skeys, const uint32_t* spay,
                                       typename Key<DT>::O* s_k, uint32_t* s_p) {
    using KT = Key<DT>;
    using O = typename KT::O;
    constexpr int IPT = 16, G = kBlock / NT, CAP = NT * IPT, PCAP = CAP + CAP / 16;
    static_assert(G * PCAP == kBaseSortLds, "every class fills the same LDS");
    constexpr O kPad = (O)~(O)0;
    const int g = threadIdx.x / NT, t = threadIdx.x % NT;
    const uint64_t bidx = blk * G + g;
    BaseItem bi = {0, 0, 0};
    if (bidx < count) bi = list[bidx];
    const uint32_t n = bi.n;
    const typename KT::T* src = bi.from_scratch ? skeys : keys;
    const uint32_t* psrc = bi.from_scratch ? spay : pay;
    O* sk = s_k + g * PCAP;
    uint32_t* sp = s_p + (PAY ? g * PCAP : 0);
    {
        typename KT::T v[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int j = t + r * NT;
            if (j < (int)n) v[r] = __builtin_nontemporal_load(&src[bi.lo + j]);
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int j = t + r * NT;
            sk[pad16(j)] = j < (int)n ? (O)KT::ord(v[r]) : kPad;
            if (PAY) sp[pad16(j)] = (uint32_t)j;  // original index
        }
    }
    __syncthreads();
    merge_sort_lds<O, PAY, NT>(sk, sp, t);
    // payloads by original index, all read before any is written (the source may be the output)
    uint32_t pv[PAY ? IPT : 1];
    if (PAY) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const int j = t + r * NT;
            if (j < (int)n) pv[r] = psrc[bi.lo + sp[pad16(j)]];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int j = t + r * NT;
        if (j < (int)n) {
            keys[bi.lo + j] = KT::from_ord((uint64_t)sk[pad16(j)]);
            if (PAY) pay[bi.lo + j] = pv[r];
        }
    }
}

template <int DT, bool PAY, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PAY ? 3 : 1))) void k_base_sort(const BaseItem* list, uint64_t count, typename Key<DT>::T* keys,
                                                   uint32_t* pay, const typename Key<DT>::T* skeys,
                                                   const uint32_t* spay) {
    using O = typename Key<DT>::O;
    __shared__ O s_k[kBaseSortLds];
    __shared__ uint32_t s_p[PAY ? kBaseSortLds : 1];
    base_sort_block<DT, PAY, NT>(list, count, blockIdx.x, keys, pay, skeys, spay, s_k, s_p);
}

// The four merge-sort classes (buckets of at most 64, 128, 256 and 512 keys) in one launch: the
// workgroups [first[c], first[c + 1]) are class c's.  A level's smallest classes hold few buckets
// each, and four launches of a few workgroups run one after another.
struct BaseSmall {
    const BaseItem* list[4];
    uint64_t count[4];
    uint64_t first[5];
};

template <int DT, bool PAY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PAY ? 3 : 1))) void k_base_sort_small(
    BaseSmall a, typename Key<DT>::T* keys, uint32_t* pay, const typename Key<DT>::T* skeys, const uint32_t* spay) {
    using O = typename Key<DT>::O;
    __shared__ O s_k[kBaseSortLds];
    __shared__ uint32_t s_p[PAY ? kBaseSortLds : 1];
    const uint64_t b = blockIdx.x;
    if (b < a.first[1])
        base_sort_block<DT, PAY, 4>(a.list[0], a.count[0], b, keys, pay, skeys, spay, s_k, s_p);
    else if (b < a.first[2])
        base_sort_block<DT, PAY, 8>(a.list[1], a.count[1], b - a.first[1], keys, pay, skeys, spay, s_k, s_p);
    else if (b < a.first[3])
        base_sort_block<DT, PAY, 16>(a.list[2], a.count[2], b - a.first[2], keys, pay, skeys, spay, s_k, s_p);
    else if (b < a.first[4])
        base_sort_block<DT, PAY, 32>(a.list[3], a.count[3], b - a.first[3], keys, pay, skeys, spay, s_k, s_p);
}

// Stable counting of one digit (0..255) per key over a workgroup of NW waves, with the same
// ballot ranking as the scatter.  Afterwards the key of wave w with digit b and rank rk among the
// wave's earlier keys of b belongs at s_loc[b] + s_wcnt[w][b] + rk; s_cnt[b] is digit b's count.
// Returns the largest count.
template <int NW, int IPT>
__device__ inline uint32_t block_count_digits(const uint32_t (&bk)[IPT], uint32_t n, uint32_t wbase,
                                              uint32_t (*s_wcnt)[kMaxBuckets], uint32_t* s_loc, uint32_t* s_cnt,
                                              uint64_t* s_scan, uint32_t* s_max, uint32_t (&rk)[IPT]) {
    constexpr int NT = kWave * NW, DPT = NT >= kMaxBuckets ? 1 : kMaxBuckets / NT;  // digits per thread
    const uint32_t tid = threadIdx.x, wave = tid / kWave;
    for (uint32_t b = tid; b < NW * kMaxBuckets; b += NT) (&s_wcnt[0][0])[b] = 0;
    __syncthreads();
    wave_count<IPT, true>(bk, n, wbase, s_wcnt[wave], rk);
    __syncthreads();
    uint32_t tot[DPT], sum = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const uint32_t dg = tid * DPT + i;
        uint32_t run = 0;
        if (dg < (uint32_t)kMaxBuckets) {
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = s_wcnt[w][dg];
                s_wcnt[w][dg] = run;
                run += c;
            }
        }
        tot[i] = run;
        sum += run;
        mx = run > mx ? run : mx;
    }
    mx = wave_max(mx);
    if (lane_id() == 0) s_max[wave] = mx;
    uint64_t all;
    uint32_t e = (uint32_t)block_exclusive_sum<uint64_t>(sum, s_scan, &all);  // synchronises
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
        const uint32_t dg = tid * DPT + i;
        if (dg < (uint32_t)kMaxBuckets) {
            s_loc[dg] = e;
            s_cnt[dg] = tot[i];
        }
        e += tot[i];
    }
    mx = 0;
    for (int w = 0; w < NW; ++w) mx = s_max[w] > mx ? s_max[w] : mx;
    __syncthreads();
    return mx;
}

// Stable base case (used for payload sorts) for one bucket of at most 64 NW IPT keys per workgroup
// of NW waves (IPT keys a thread).
// The bucket's smallest ord (min) and the low bits z that are zero in every ord - min are found
// first; x = (ord - min) >> z keeps only the bits where the keys differ, nbits of them.
//  * nbits <= 8: one stable counting pass on x sorts the bucket.
//  * otherwise a stable counting pass on the top 8 bits of x splits it into 256 ordered
//    sub-buckets (an MSD radix step, as SkaSort starts); each key's final place is its
//    sub-bucket's start plus the number of keys of its sub-bucket that precede it in (ord,
//    position) order.  A sub-bucket of more than kSubMax keys (skewed buckets) sends the whole
//    bucket to the merge sort instead.
// All paths are stable.
constexpr uint32_t kSubMax = 64;

template <int DT, bool PAY, int NW, int IPT>
__device__ inline void base_large_stable(const BaseItem& bi, typename Key<DT>::T* keys, uint32_t* pay,
                                         const typename Key<DT>::T* skeys, const uint32_t* spay) {
    using KT = Key<DT>;
    using O = typename KT::O;
    constexpr int NT = 64 * NW, CAP = NT * IPT, PCAP = CAP + CAP / 16;
    constexpr int MT = CAP / 16;  // threads of the merge-sort fallback (16 keys each)
    constexpr O kPad = (O)~(O)0;
    __shared__ O s_k[PCAP];
    __shared__ uint32_t s_p[PAY ? PCAP : 1];
    __shared__ uint32_t s_wcnt[NW][kMaxBuckets];
    __shared__ uint32_t s_loc[kMaxBuckets], s_cnt[kMaxBuckets];
    __shared__ uint64_t s_scan[16];
    __shared__ uint32_t s_max[NW];
    __shared__ O s_red[2][NW];
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint32_t n = bi.n;
    const typename KT::T* src = bi.from_scratch ? skeys : keys;
    const uint32_t* psrc = bi.from_scratch ? spay : pay;
    const uint32_t wbase = wave * kWave * IPT;
    O o[IPT];
    uint32_t p[IPT];
    {
        typename KT::T v[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) {
                v[r] = __builtin_nontemporal_load(&src[bi.lo + j]);
                p[r] = PAY ? __builtin_nontemporal_load(&psrc[bi.lo + j]) : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = wbase + r * kWave + lane < n ? (O)KT::ord(v[r]) : kPad;
    }
    // min over the bucket, then the OR of ord - min (its trailing zeros and bit length)
    O mn = kPad;
#pragma unroll
    for (int r = 0; r < IPT; ++r) mn = o[r] < mn ? o[r] : mn;
    mn = (O)~wave_max((O)~mn);
    if (lane == 0) s_red[0][wave] = mn;
    __syncthreads();
    mn = s_red[0][0];
    for (int w = 1; w < NW; ++w) mn = s_red[0][w] < mn ? s_red[0][w] : mn;
    O orv = 0;
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (wbase + r * kWave + lane < n) orv |= (O)(o[r] - mn);
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) orv |= (O)__shfl_xor(orv, sft, kWave);
    if (lane == 0) s_red[1][wave] = orv;
    __syncthreads();
    orv = 0;
    for (int w = 0; w < NW; ++w) orv |= s_red[1][w];
    const int z = orv ? __builtin_ctzll((unsigned long long)orv) : 0;
    const int nbits = orv ? (int)bit_length((uint64_t)(orv >> z)) : 0;

    uint32_t bk[IPT], rk[IPT];
    const int shift = nbits <= 8 ? z : z + nbits - 8;  // the low digit, or the top 8 varying bits
#pragma unroll
    for (int r = 0; r < IPT; ++r) bk[r] = (uint32_t)(((uint64_t)(o[r] - mn) >> shift) & 255u);
    const uint32_t most = block_count_digits<NW, IPT>(bk, n, wbase, s_wcnt, s_loc, s_cnt, s_scan, s_max, rk);

    if (nbits > 8 && most > kSubMax) {
        // merge sort: keys (and original indices) to LDS at their input positions, padding at the
        // end; then sort, and gather the payloads by index (all read before any is written)
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            s_k[pad16(j)] = o[r];
            if (PAY) s_p[pad16(j)] = j;
        }
        __syncthreads();
        merge_sort_lds<O, PAY, MT>(s_k, s_p, (int)tid, tid < (uint32_t)MT);
        uint32_t pv[PAY ? IPT : 1];
        if (PAY) {
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const uint32_t j = wbase + r * kWave + lane;
                if (j < n) pv[r] = psrc[bi.lo + s_p[pad16(j)]];
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) {
                keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[pad16(j)]);
                if (PAY) pay[bi.lo + j] = pv[r];
            }
        }
        return;
    }

    // keys in digit order (stable)
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wbase + r * kWave + lane < n) {
            const uint32_t pos = s_loc[bk[r]] + s_wcnt[wave][bk[r]] + rk[r];
            s_k[pos] = o[r];
            if (PAY) s_p[pos] = p[r];
        }
    }
    __syncthreads();
    if (nbits > 8) {
        // final place inside the sub-bucket: the keys of the sub-bucket that precede this one in
        // (ord, position) order.  Lane j takes position j of the digit order, so the lanes of a
        // wave mostly share a sub-bucket and its LDS reads are broadcasts.
        O xs[IPT];
        uint32_t ps[IPT], np[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) {
                xs[r] = s_k[j];
                ps[r] = PAY ? s_p[j] : 0u;
                const uint32_t d = (uint32_t)(((uint64_t)(xs[r] - mn) >> shift) & 255u);
                const uint32_t start = s_loc[d], cnt = s_cnt[d];
                uint32_t before = 0;
                for (uint32_t q = 0; q < cnt; ++q) {
                    const O x = s_k[start + q];
                    before += (x < xs[r] || (x == xs[r] && start + q < j)) ? 1u : 0u;
                }
                np[r] = start + before;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            if (wbase + r * kWave + lane < n) {
                s_k[np[r]] = xs[r];
                if (PAY) s_p[np[r]] = ps[r];
            }
        }
        __syncthreads();
    }
    // sorted keys at positions 0 .. n-1: write out (coalesced)
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t j = wbase + r * kWave + lane;
        if (j < n) {
            keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[j]);
            if (PAY) pay[bi.lo + j] = s_p[j];
        }
    }
}


// Base case of keys-only sorts for one bucket of at most CAP = 64 NW IPT keys per workgroup.  Keys
// with equal ord are identical, so any order among them is the sorted order and the pass need not
// be stable.  One reduction finds the bucket's min, max and the low bits z shared by all keys
// (the trailing zeros of every key's difference to the bucket's first key); a histogram of
// log2(CAP)-bit digits of (ord - min) >> z, taken from the top of the varying bits, with LDS atomics,
// places every key in its digit's range.  Digits then hold one key on average:
//  * when the varying bits fit the digit, keys of a digit are equal and the bucket is sorted;
//  * otherwise a key's final place is its digit's start plus the keys of the digit before it in
//    (ord, position) order; a digit of more than kSubMax keys (skewed buckets) sends the bucket to
//    the merge sort instead.
// A value that is the same in every lane, moved to scalar registers (frees vector registers).
template <typename V>
__device__ inline V uniform(V v) {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, (uint32_t)__builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
        return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
    }
}

// Digit of a key of the keys-only base case: the bits below the top varying bit of ord - min, or
// (BY_VALUE) a linear map of the value onto [0, ND); t >= 0 since every key is at least min.
template <typename KT, int ND, bool BY_VALUE, typename O>
__device__ inline uint32_t base_digit(O x, O mn, int shift, double vlo, double vscale) {
    if constexpr (BY_VALUE) {
        const double t = (KT::val(KT::from_ord((uint64_t)x)) - vlo) * vscale;
        return t < (double)(ND - 1) ? (uint32_t)t : (uint32_t)(ND - 1);
    } else {
        return (uint32_t)((uint64_t)(x - mn) >> shift);
    }
}

// The keys-only base case's counting: each key's slot among its digit's keys (LDS atomics on s_c,
// which starts at zero), then the digit starts in s_c[0..ND) and n in s_c[ND].  Returns the largest
// digit count.  Thread t owns digits [t CPT, (t+1) CPT).  The digits are not kept: the placement
// computes them again, which holds fewer registers across the scan.
template <typename KT, int NW, int IPT, int ND, bool BY_VALUE, typename O>
__device__ inline uint32_t base_count(const O (&o)[IPT], uint32_t n, uint32_t wbase, O mn, int shift, double vlo,
                                      double vscale, uint32_t (&sl)[IPT], uint32_t* s_c,
                                      uint64_t* s_scan, uint32_t* s_most) {
    constexpr int NT = 64 * NW, CPT = ND / NT;
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wbase + r * kWave + lane < n) sl[r] = atomicAdd(&s_c[base_digit<KT, ND, BY_VALUE>(o[r], mn, shift, vlo, vscale)], 1u);
    }
    __syncthreads();
    uint32_t c[CPT], sum = 0, most = 0;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        c[i] = s_c[tid * CPT + i];
        sum += c[i];
        most = c[i] > most ? c[i] : most;
    }
    most = wave_max(most);
    if (lane == 0) s_most[wave] = most;
    uint64_t all;
    uint32_t e = (uint32_t)block_exclusive_sum<uint64_t>(sum, s_scan, &all);  // synchronises
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        s_c[tid * CPT + i] = e;
        e += c[i];
    }
    if (tid == 0) s_c[ND] = n;
    most = 0;
    for (int w = 0; w < NW; ++w) most = s_most[w] > most ? s_most[w] : most;
    __syncthreads();
    return most;
}

// The keys-only base case's placement: each key to its digit's start plus its slot.
template <typename KT, int IPT, int ND, bool BY_VALUE, typename O>
__device__ inline void base_place(const O (&o)[IPT], const uint32_t (&sl)[IPT], uint32_t n, uint32_t wbase, O mn,
                                  int shift, double vlo, double vscale, O* s_k, const uint32_t* s_c) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (wbase + r * kWave + lane < n) s_k[s_c[base_digit<KT, ND, BY_VALUE>(o[r], mn, shift, vlo, vscale)] + sl[r]] = o[r];
}

// The keys-only base case's last step for a bucket whose digits do not fit the varying bits: each
// key's place is its digit's start plus the keys of its digit before it in (ord, position) order.
template <typename KT, int NW, int IPT, int ND, bool BY_VALUE, typename O>
__device__ inline void base_fixup(uint32_t n, uint32_t wbase, O mn, int shift, double vlo, double vscale, O* s_k,
                                  const uint32_t* s_c) {
    const uint32_t lane = lane_id();
    O xs[IPT];
    uint32_t np[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t j = wbase + r * kWave + lane;
        if (j < n) {
            xs[r] = s_k[j];
            const uint32_t d = base_digit<KT, ND, BY_VALUE>(xs[r], mn, shift, vlo, vscale);
            const uint32_t start = s_c[d], end = s_c[d + 1];
            uint32_t before = 0;
            for (uint32_t q = start; q < end; ++q) {
                const O y = s_k[q];
                before += (y < xs[r] || (y == xs[r] && q < j)) ? 1u : 0u;
            }
            np[r] = start + before;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (wbase + r * kWave + lane < n) s_k[np[r]] = xs[r];
    __syncthreads();
}

// Digit start of the keys-only base case: 16-bit values packed two to a 32-bit LDS word.
__device__ inline uint32_t digit_start16(const uint32_t* w, uint32_t d) { return (w[d >> 1] >> ((d & 1u) * 16u)) & 0xffffu; }

// The keys-only base case of one bucket of at most CAP = 64 NW IPT keys, in one LDS block of
// CAP keys followed by CAP 16-bit digit counters (40 KB for fp64 at CAP = 4096: four workgroups
// fit a CU).  The bucket's varying bits of ord (below its min, max and shared low zero bits) give
// the digit: the top log2(CAP) of them.  Each key takes a slot in its digit with an LDS atomic,
// a block scan turns the counts into digit starts, and the keys are placed.  When the varying bits
// fit the digit that is the sorted order; otherwise a key's place is its digit's start plus the
// keys of the digit before it in (ord, position) order (a digit holds about one key: the first
// four are read at once).  A digit of more than kSubMax keys (a skewed bucket) sends the bucket
// to the merge sort, which uses the whole LDS block in its padded layout.
template <int DT, int NW, int IPT>
__device__ inline void base_large_keys(const BaseItem& bi, typename Key<DT>::T* keys,
                                       const typename Key<DT>::T* skeys) {
    using KT = Key<DT>;
    using O = typename KT::O;
    constexpr int NT = 64 * NW, CAP = NT * IPT, PCAP = CAP + CAP / 16, MT = CAP / 16;
    constexpr int DB = CAP >= 4096 ? 12 : CAP >= 2048 ? 11 : CAP >= 1024 ? 10 : 9;  // digit bits
    constexpr int ND = 1 << DB;
    static_assert(ND == CAP && IPT % 4 == 0, "one digit per key slot, four per 16-byte counter read");
    constexpr int KB = CAP * (int)sizeof(O), CB = ND * 2;  // key and counter bytes
    constexpr int MEM = (KB + CB > PCAP * (int)sizeof(O)) ? KB + CB : PCAP * (int)sizeof(O);
    constexpr O kPad = (O)~(O)0;
    __shared__ __align__(16) unsigned char s_mem[MEM];
    O* s_k = (O*)s_mem;
    uint32_t* s_cw = (uint32_t*)(s_mem + KB);  // digit counters, then digit starts
    // reduction scratch inside the key area, which is first written after the last read of it
    O* s_red = (O*)s_mem;                                  // [3][NW]
    uint32_t* s_scan = (uint32_t*)(s_mem + 3 * NW * sizeof(O));  // [16]
    uint32_t* s_most = s_scan + 16;                        // [NW]
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint32_t n = bi.n;
    const typename KT::T* src = bi.from_scratch ? skeys : keys;
    const uint32_t wbase = wave * kWave * IPT;
    // lanes past the bucket's end load its first key (n >= 1): min, max and the shared low bits
    // need no masking; the merge sort below pads them with kPad
    O o[IPT];
    {
        typename KT::T v[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            v[r] = __builtin_nontemporal_load(&src[bi.lo + (j < n ? j : 0u)]);
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = (O)KT::ord(v[r]);
    }
    const O oref = (O)KT::ord(src[bi.lo]);
    O mn = o[0], mx = o[0], ov = 0;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        mn = o[r] < mn ? o[r] : mn;
        mx = o[r] > mx ? o[r] : mx;
        ov |= (O)(o[r] - oref);
    }
    mn = (O)~wave_max((O)~mn);
    mx = wave_max(mx);
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) ov |= (O)__shfl_xor(ov, sft, kWave);
    for (uint32_t q = tid; q < (uint32_t)(ND / 2); q += NT) s_cw[q] = 0u;
    if (lane == 0) {
        s_red[0 * NW + wave] = mn;
        s_red[1 * NW + wave] = mx;
        s_red[2 * NW + wave] = ov;
    }
    __syncthreads();
    mn = s_red[0];
    mx = s_red[NW];
    ov = s_red[2 * NW];
    for (int w = 1; w < NW; ++w) {
        mn = s_red[w] < mn ? s_red[w] : mn;
        mx = s_red[NW + w] > mx ? s_red[NW + w] : mx;
        ov |= s_red[2 * NW + w];
    }
    const int z = ov ? __builtin_ctzll((unsigned long long)ov) : 0;
    const int nbits = (int)bit_length((uint64_t)((O)(mx - mn) >> z));
    const int shift = z + (nbits > DB ? nbits - DB : 0);
    const bool exact = nbits <= DB;
    // each key's digit (low 16 bits) and slot in its digit (high 16 bits)
    uint32_t ds[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wbase + r * kWave + lane < n) {
            const uint32_t d = (uint32_t)((uint64_t)(o[r] - mn) >> shift), h = (d & 1u) * 16u;
            const uint32_t old = atomicAdd(&s_cw[d >> 1], 1u << h);
            ds[r] = d | (((old >> h) & 0xffffu) << 16);
        }
    }
    __syncthreads();
    // digit starts: thread t owns digits [t IPT, (t+1) IPT), IPT / 2 counter words
    uint32_t c[IPT], sum = 0, most = 0;
#pragma unroll
    for (int i = 0; i < IPT / 4; ++i) {
        const uint2 wv = *(const uint2*)&s_cw[tid * (IPT / 2) + 2 * i];
        c[4 * i + 0] = wv.x & 0xffffu;
        c[4 * i + 1] = wv.x >> 16;
        c[4 * i + 2] = wv.y & 0xffffu;
        c[4 * i + 3] = wv.y >> 16;
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        sum += c[i];
        most = c[i] > most ? c[i] : most;
    }
    most = wave_max(most);
    if (lane == 0) s_most[wave] = most;
    uint32_t all;
    uint32_t e = block_exclusive_sum<uint32_t>(sum, s_scan, &all);  // synchronises
#pragma unroll
    for (int i = 0; i < IPT / 2; ++i) {
        const uint32_t lo16 = e;
        e += c[2 * i];
        s_cw[tid * (IPT / 2) + i] = lo16 | (e << 16);
        e += c[2 * i + 1];
    }
    most = 0;
    for (int w = 0; w < NW; ++w) most = s_most[w] > most ? s_most[w] : most;
    __syncthreads();

    if (!exact && most > kSubMax) {
        // merge sort: keys to LDS at their input positions (padding keys at the end), then sort
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            s_k[pad16(j)] = j < n ? o[r] : kPad;
        }
        __syncthreads();
        merge_sort_lds<O, false, MT>(s_k, nullptr, (int)tid, tid < (uint32_t)MT);
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[pad16(j)]);
        }
        return;
    }
    if constexpr (sizeof(O) == 8) {
        if (!exact && nbits + DB <= 64) {
            // Each key's varying bits above its placement slot, (ord - min) >> z << DB | slot, are
            // unique, so one 64-bit compare orders two keys of a digit (equal keys by slot: any
            // order of equal keys gives the same output).  The thread that placed a key ranks it
            // among its digit's keys, from its own registers.  No digit holds more than kSubMax
            // keys here, so ds packs the digit's start (12 bits), the key's slot (6) and the
            // digit's count (7).
            static_assert(kSubMax <= 64 && DB <= 12, "packing of start, slot and count");
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                if (wbase + r * kWave + lane < n) {
                    const uint32_t d = ds[r] & 0xffffu, slot = ds[r] >> 16;
                    const uint32_t st = digit_start16(s_cw, d);
                    const uint32_t cn = (d + 1 < (uint32_t)ND ? digit_start16(s_cw, d + 1) : n) - st;
                    const uint32_t p = st + slot;
                    s_k[p] = (O)((((uint64_t)(o[r] - mn) >> z) << DB) | p);
                    ds[r] = st | (slot << 12) | (cn << 18);
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                if (wbase + r * kWave + lane < n) {
                    const uint32_t st = ds[r] & 0xfffu, cn = ds[r] >> 18;
                    const O x = (O)((((uint64_t)(o[r] - mn) >> z) << DB) | (st + ((ds[r] >> 12) & 0x3fu)));
                    uint32_t before = 0;
                    if (cn > 1) {  // a key alone in its digit is in place: its lane reads nothing
#pragma unroll
                        for (uint32_t q = 0; q < 4; ++q) {
                            // read unconditionally (the slots past the digit, at most three past
                            // the last key, lie in the counter area), counted only inside the digit
                            const O y = s_k[st + q];
                            before += ((q < cn) & (y < x)) ? 1u : 0u;
                        }
                        for (uint32_t q = 4; q < cn; ++q) before += s_k[st + q] < x ? 1u : 0u;
                    }
                    ds[r] = st + before;
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r)
                if (wbase + r * kWave + lane < n) s_k[ds[r]] = o[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IPT; ++r) {
                const uint32_t j = wbase + r * kWave + lane;
                if (j < n) keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[j]);
            }
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r)
        if (wbase + r * kWave + lane < n) s_k[digit_start16(s_cw, ds[r] & 0xffffu) + (ds[r] >> 16)] = o[r];
    __syncthreads();
    if (!exact) {
        // place inside the digit; s_k holds CAP keys and then the counters, so the reads of the
        // four slots from a digit's start stay inside the block (those past the digit are ignored)
        O xs[IPT];
        uint32_t np[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) {
                xs[r] = s_k[j];
                const uint32_t d = (uint32_t)((uint64_t)(xs[r] - mn) >> shift);
                const uint32_t start = digit_start16(s_cw, d);
                const uint32_t end = d + 1 < (uint32_t)ND ? digit_start16(s_cw, d + 1) : n;
                uint32_t before = 0;
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q) {
                    const O y = s_k[start + q];
                    before += (start + q < end && (y < xs[r] || (y == xs[r] && start + q < j))) ? 1u : 0u;
                }
                for (uint32_t q = start + 4; q < end; ++q) {
                    const O y = s_k[q];
                    before += (y < xs[r] || (y == xs[r] && q < j)) ? 1u : 0u;
                }
                np[r] = start + before;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IPT; ++r)
            if (wbase + r * kWave + lane < n) s_k[np[r]] = xs[r];
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t j = wbase + r * kWave + lane;
        if (j < n) keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[j]);
    }
}

// The keys-only base case for sorted samples, which span their whole bucket: as base_large_keys,
// but when a digit holds more than kSubMax keys (a float range over several binades, whose top
// varying bits are exponent bits) the bucket is counted again with digits from a linear map of the
// key's value over [min, max]; if a digit still holds more than kSubMax keys, the merge sort runs.
template <int DT, int NW, int IPT>
__device__ inline void base_large_keys_vmap(const BaseItem& bi, typename Key<DT>::T* keys,
                                       const typename Key<DT>::T* skeys) {
    using KT = Key<DT>;
    using O = typename KT::O;
    constexpr int NT = 64 * NW, CAP = NT * IPT, PCAP = CAP + CAP / 16, MT = CAP / 16;
    constexpr int DB = CAP >= 4096 ? 12 : CAP >= 2048 ? 11 : CAP >= 1024 ? 10 : 9;  // digit bits
    constexpr int ND = 1 << DB, CPT = ND / NT;                                     // digits, per thread
    static_assert(ND == CAP && CPT == IPT, "one digit per key slot");
    constexpr O kPad = (O)~(O)0;
    __shared__ O s_k[PCAP];
    __shared__ uint32_t s_c[ND + 1];
    __shared__ uint64_t s_scan[16];
    __shared__ O s_red[3][NW];
    __shared__ uint32_t s_most[NW];
    const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const uint32_t n = bi.n;
    const typename KT::T* src = bi.from_scratch ? skeys : keys;
    const uint32_t wbase = wave * kWave * IPT;
    O o[IPT];
    {
        typename KT::T v[IPT];
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) v[r] = __builtin_nontemporal_load(&src[bi.lo + j]);
        }
#pragma unroll
        for (int r = 0; r < IPT; ++r) o[r] = wbase + r * kWave + lane < n ? (O)KT::ord(v[r]) : kPad;
    }
    const O oref = (O)KT::ord(src[bi.lo]);  // n >= 1
    O mn = kPad, mx = 0, ov = 0;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wbase + r * kWave + lane < n) {
            mn = o[r] < mn ? o[r] : mn;
            mx = o[r] > mx ? o[r] : mx;
            ov |= (O)(o[r] - oref);
        }
    }
    mn = (O)~wave_max((O)~mn);
    mx = wave_max(mx);
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) ov |= (O)__shfl_xor(ov, sft, kWave);
    for (uint32_t d = tid; d <= (uint32_t)ND; d += NT) s_c[d] = 0;
    if (lane == 0) {
        s_red[0][wave] = mn;
        s_red[1][wave] = mx;
        s_red[2][wave] = ov;
    }
    __syncthreads();
    mn = s_red[0][0];
    mx = s_red[1][0];
    ov = s_red[2][0];
    for (int w = 1; w < NW; ++w) {
        mn = s_red[0][w] < mn ? s_red[0][w] : mn;
        mx = s_red[1][w] > mx ? s_red[1][w] : mx;
        ov |= s_red[2][w];
    }
    mn = uniform(mn);
    mx = uniform(mx);
    ov = uniform(ov);
    const int z = ov ? __builtin_ctzll((unsigned long long)ov) : 0;
    const int nbits = (int)bit_length((uint64_t)((O)(mx - mn) >> z));
    const int shift = z + (nbits > DB ? nbits - DB : 0);
    const bool exact = nbits <= DB;
    uint32_t sl[IPT];
    uint32_t most = base_count<KT, NW, IPT, ND, false>(o, n, wbase, mn, shift, 0.0, 0.0, sl, s_c, s_scan, s_most);
    // Digits of a float range that spans several binades are mostly exponent bits, and a few digits
    // take most keys.  Such a bucket is counted again with digits from a linear map of the key's
    // value (monotone in the key order, as every digit function must be); a bucket that is still
    // skewed is merge sorted.  The decision is uniform over the block.
    bool by_value = false;
    double vlo = 0.0, vscale = 0.0;
    if (!exact && most > kSubMax) {
        vlo = uniform(KT::val(KT::from_ord((uint64_t)mn)));
        const double vhi = KT::val(KT::from_ord((uint64_t)mx));
        vscale = uniform((double)ND / (vhi - vlo));
        if (__builtin_isfinite(vlo) && __builtin_isfinite(vhi) && vhi > vlo && __builtin_isfinite(vscale)) {
            by_value = true;
            for (uint32_t d = tid; d <= (uint32_t)ND; d += NT) s_c[d] = 0;
            __syncthreads();
            most = base_count<KT, NW, IPT, ND, true>(o, n, wbase, mn, shift, vlo, vscale, sl, s_c, s_scan, s_most);
        }
    }

    if (!exact && most > kSubMax) {
        // merge sort: keys to LDS at their input positions (padding keys at the end), then sort
#pragma unroll
        for (int r = 0; r < IPT; ++r) s_k[pad16(wbase + r * kWave + lane)] = o[r];
        __syncthreads();
        merge_sort_lds<O, false, MT>(s_k, nullptr, (int)tid, tid < (uint32_t)MT);
#pragma unroll
        for (int r = 0; r < IPT; ++r) {
            const uint32_t j = wbase + r * kWave + lane;
            if (j < n) keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[pad16(j)]);
        }
        return;
    }
    if (by_value) base_place<KT, IPT, ND, true>(o, sl, n, wbase, mn, shift, vlo, vscale, s_k, s_c);
    else base_place<KT, IPT, ND, false>(o, sl, n, wbase, mn, shift, vlo, vscale, s_k, s_c);
    __syncthreads();
    if (by_value) base_fixup<KT, NW, IPT, ND, true>(n, wbase, mn, shift, vlo, vscale, s_k, s_c);
    else if (!exact) base_fixup<KT, NW, IPT, ND, false>(n, wbase, mn, shift, vlo, vscale, s_k, s_c);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t j = wbase + r * kWave + lane;
        if (j < n) keys[bi.lo + j] = KT::from_ord((uint64_t)s_k[j]);
    }
}

// VMAP: skewed buckets are counted again by value before the merge sort is taken (sorted samples,
// which span their whole bucket; the bulk of the base case runs without it).
template <int DT, bool PAY, int NW, int IPT, bool VMAP = false>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(PAY ? 4 : VMAP ? 6 : 8))) void k_base_large(
    const BaseItem* list, uint64_t count,
                                                       typename Key<DT>::T* keys, uint32_t* pay,
                                                       const typename Key<DT>::T* skeys, const uint32_t* spay) {
    if (blockIdx.x >= count) return;
    const BaseItem bi = list[blockIdx.x];
    if constexpr (PAY) base_large_stable<DT, true, NW, IPT>(bi, keys, pay, skeys, spay);
    else if constexpr (VMAP) base_large_keys_vmap<DT, NW, IPT>(bi, keys, skeys);
    else base_large_keys<DT, NW, IPT>(bi, keys, skeys);
}

}  // namespace ipls
