// Invariant checks of the sort, run when IPLS_DEBUG_CHECKS is set in the environment (off by
// default).  After every distribution pass: every item's histogram sums to its key count, the
// pass moved the same multiset of keys (and payloads) into the item's range, and every key lies in
// the bucket its model gives it, which with a monotone model means that the bucket boundaries
// respect the key order.  After the sort: every segment is non-decreasing and holds the multiset
// it held before.  A failed check sets kErrInvariant in the device error word.  Included at the
// end of ipls_kernels.h.
#pragma once

#include "ipls_device.h"

namespace ipls {

// A (key, payload) pair as one 64-bit hash; sums and xors of the hashes compare multisets.
__device__ inline uint64_t dbg_pair_hash(uint64_t ord, uint32_t pay, bool has_pay) {
    return mix64(ord ^ (has_pay ? mix64((uint64_t)pay + 0x9e3779b97f4a7c15ull) : 0ull));
}

// The wave's sum and xor of (sum, x), added by its first lane to acc[0] and acc[1].
__device__ inline void dbg_wave_add(uint64_t sum, uint64_t x, uint64_t* acc) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        sum += __shfl_xor(sum, s, kWave);
        x ^= __shfl_xor(x, s, kWave);
    }
    if (lane_id() == 0) {
        atomicAdd((unsigned long long*)&acc[0], (unsigned long long)sum);
        atomicXor((unsigned long long*)&acc[1], (unsigned long long)x);
    }
}

__global__ void k_dbg_zero(uint64_t* p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Multiset hash of every item's range of buf (a workgroup per tile) into acc[2 item], acc[2 item + 1].
// Items closed where they are (homogeneous, not moved by the pass) are left out.
template <int DT, bool PAY>
__global__ __launch_bounds__(256) void k_dbg_hash_tiles(const TileInfo* tiles, uint64_t nt, const Model* models,
                                                        const typename Key<DT>::T* buf, const uint32_t* pay,
                                                        uint64_t* acc) {
    const uint64_t t = blockIdx.x;
    if (t >= nt) return;
    const TileInfo ti = tiles[t];
    if (models[ti.item].kind == kKindClosedKeep) return;
    uint64_t sum = 0, x = 0;
    for (uint32_t j = threadIdx.x; j < ti.n; j += blockDim.x) {
        const uint64_t h = dbg_pair_hash(Key<DT>::ord(buf[ti.base + j]), PAY ? pay[ti.base + j] : 0u, PAY);
        sum += h;
        x ^= h;
    }
    dbg_wave_add(sum, x, acc + 2 * (uint64_t)ti.item);
}

// Every key of a tile of the pass's destination lies in the bucket whose range holds its position.
template <int DT>
__global__ __launch_bounds__(256) void k_dbg_place(const TileInfo* tiles, uint64_t nt, const Item* items,
                                                   const Model* models, const double* leaves,
                                                   const typename Key<DT>::T* dst, const uint64_t* bstart, uint32_t K,
                                                   uint32_t M, uint64_t* err) {
    __shared__ double s_leaf[4 * kMaxLeaves];
    __shared__ uint64_t s_st[kMaxBuckets];
    const uint64_t t = blockIdx.x;
    if (t >= nt) return;
    const TileInfo ti = tiles[t];
    const uint32_t i = ti.item;
    const Model m = models[i];
    if (m.kind == kKindClosedKeep) return;
    for (uint32_t q = threadIdx.x, nq = model_table_size(m.kind, K, M); q < nq; q += blockDim.x)
        s_leaf[q] = leaves[(uint64_t)i * 4 * kMaxLeaves + q];
    for (uint32_t b = threadIdx.x; b < K; b += blockDim.x) s_st[b] = bstart[(uint64_t)i * K + b];
    __syncthreads();
    const uint64_t rel0 = ti.base - items[i].lo;
    int bad = 0;
    for (uint32_t j = threadIdx.x; j < ti.n; j += blockDim.x) {
        const uint64_t r = rel0 + j;
        uint32_t lo = 0, hi = K;  // the last bucket starting at or before r (s_st[0] = 0)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_st[mid] <= r) lo = mid;
            else hi = mid;
        }
        bad |= classify_key<DT>(m, s_leaf, K, M, dst[ti.base + j]) != lo ? 1 : 0;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr((unsigned long long*)err, (unsigned long long)kErrInvariant);
}

// Per item: the histogram sums to the key count and the pass kept the multiset (acc_src, acc_dst).
__global__ void k_dbg_level(const Item* items, uint64_t ni, const Model* models, const uint64_t* hist, uint32_t K,
                            const uint64_t* acc_src, const uint64_t* acc_dst, uint64_t* err) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || models[i].kind == kKindClosedKeep) return;
    uint64_t sum = 0;
    for (uint32_t b = 0; b < K; ++b) sum += hist[i * K + b];
    if (sum != items[i].n || acc_src[2 * i] != acc_dst[2 * i] || acc_src[2 * i + 1] != acc_dst[2 * i + 1])
        atomicOr((unsigned long long*)err, (unsigned long long)kErrInvariant);
}

// Multiset hash of buf[0, n) into acc[0], acc[1].
template <int DT, bool PAY>
__global__ __launch_bounds__(256) void k_dbg_hash_all(const typename Key<DT>::T* buf, const uint32_t* pay, uint64_t n,
                                                      uint64_t* acc) {
    uint64_t sum = 0, x = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t h = dbg_pair_hash(Key<DT>::ord(buf[j]), PAY ? pay[j] : 0u, PAY);
        sum += h;
        x ^= h;
    }
    dbg_wave_add(sum, x, acc);
}

// Every segment [off[s], off[s+1]) of buf is non-decreasing by ord: a descent at j is an error
// unless j + 1 starts a segment.
template <int DT>
__global__ __launch_bounds__(256) void k_dbg_sorted(const typename Key<DT>::T* buf, uint64_t n, const uint64_t* off,
                                                    uint64_t nseg, uint64_t* err) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j + 1 < n; j += (uint64_t)gridDim.x * blockDim.x) {
        if (Key<DT>::ord(buf[j]) <= Key<DT>::ord(buf[j + 1])) continue;
        uint64_t lo = 0, hi = nseg + 1;  // is j + 1 one of off[0 .. nseg]?
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (off[mid] <= j + 1) lo = mid;
            else hi = mid;
        }
        if (off[lo] != j + 1) atomicOr((unsigned long long*)err, (unsigned long long)kErrInvariant);
    }
}

// The sort's output holds the multiset of its input: acc[0..1] before, acc[2..3] after.  plant = 1
// (IPLS_DEBUG_CHECKS=2) compares against a changed input hash, so that a test sees the error
// reported while every kernel runs as usual.
__global__ void k_dbg_compare(const uint64_t* acc, int plant, uint64_t* err) {
    if ((acc[0] ^ (uint64_t)plant) != acc[2] || acc[1] != acc[3])
        atomicOr((unsigned long long*)err, (unsigned long long)kErrInvariant);
}

}  // namespace ipls
