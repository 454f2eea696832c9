// Device hash and scan helpers shared by the lattice build and the LP
// divide and conquer: a 64-bit key mixer for open addressing, block and
// device-wide exclusive scans, and the compaction of occupied hash slots.
#pragma once

#include "dcrf_internal.h"

namespace dcrf {
namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// exclusive scan of one int per thread within a block of kScanThreads
__device__ int block_exclusive_scan(int v, int *lds, int &total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int add = (t >= off) ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    total = lds[kScanThreads - 1];
    int incl = lds[t];
    __syncthreads();
    return incl - v;
}

[[maybe_unused]] __global__ void __launch_bounds__(kScanThreads)
k_count_occupied(const uint64_t *__restrict__ hkeys, size_t cap,
                 int *__restrict__ tile_counts) {
    __shared__ int lds[kScanThreads];
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    int cnt = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < cap && hkeys[base + i] != kEmpty) ++cnt;
    int total;
    block_exclusive_scan(cnt, lds, total);
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = total;
}

// single block: exclusive scan of the tile counts, total written at [ntiles]
__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(int *__restrict__ tile_counts, int ntiles) {
    __shared__ int lds[kScanThreads];
    int carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads) {
        int i = base + threadIdx.x;
        int v = i < ntiles ? tile_counts[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, lds, total);
        if (i < ntiles) tile_counts[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tile_counts[ntiles] = carry;
}

[[maybe_unused]] __global__ void __launch_bounds__(kScanThreads)
k_assign_ids(const uint64_t *__restrict__ hkeys, size_t cap,
             const int *__restrict__ tile_offsets, int *__restrict__ slot_vid,
             uint64_t *__restrict__ vkeys) {
    __shared__ int lds[kScanThreads];
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    int cnt = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < cap && hkeys[base + i] != kEmpty) ++cnt;
    int total;
    int id = tile_offsets[blockIdx.x] + block_exclusive_scan(cnt, lds, total);
    for (int i = 0; i < kScanItems; ++i) {
        size_t s = base + i;
        if (s < cap) {
            uint64_t k = hkeys[s];
            if (k != kEmpty) {
                slot_vid[s] = id;
                vkeys[id] = k;
                ++id;
            } else {
                slot_vid[s] = -1;
            }
        }
    }
}

// ---- generic exclusive scan of n ints (out[n] receives the total) ----------

__global__ void __launch_bounds__(kScanThreads)
k_sum_tiles(const int *__restrict__ in, int n, int *__restrict__ tile_sums) {
    __shared__ int lds[kScanThreads];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const int *__restrict__ in, int n, const int *__restrict__ tile_off,
             int *__restrict__ out) {
    __shared__ int lds[kScanThreads];
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int total;
    int run = tile_off[blockIdx.x] + block_exclusive_scan(s, lds, total);
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) {
            out[base + i] = run;
            run += in[base + i];
        }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1)
        out[n] = tile_off[blockIdx.x] + total;
}

// exclusive scan of n device ints into out (n + 1 entries) with the tile
// counts kept in the context scratch (sized for the largest hash table)
[[maybe_unused]] void scan_ints(dcrf_ctx *ctx, const int *in, int n, int *out) {
    const hipStream_t s = ctx->stream;
    const int ntiles = std::max(1, ceil_div(n, kScanTile));
    int *tiles = reinterpret_cast<int *>(ctx->scratch.as<char>() + 64);
    hipLaunchKernelGGL(k_sum_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, in,
                       n, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tiles,
                       ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, s, in,
                       n, tiles, out);
    DCRF_CHECK_LAUNCH();
}

}  // namespace
}  // namespace dcrf
