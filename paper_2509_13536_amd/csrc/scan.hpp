// Exclusive prefix sums over uint32 values (three launches: per-block sums,
// scan of the block sums in one block, per-block scan with the block prefix).
// Load/Store are device functors, so a scan can gather its input and scatter
// its output (used for stream compaction and for the per-rank tile counts).
#pragma once
#include "common.hpp"

namespace mgs {

constexpr int kScanThreads = 256;
constexpr int kScanRounds = 8;
constexpr int kScanTile = kScanThreads * kScanRounds;  // 2048 values per block

// Exclusive scan of one value per thread across a 256-thread block.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds4, uint32_t *total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds4[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t s = lds4[w];
        before += (w < wave) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

template <class Load>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Load load, int64_t n, uint32_t *sums) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanRounds; ++r) {
        const int64_t i = base + r * kScanThreads + threadIdx.x;
        if (i < n) s += load(i);
    }
    uint32_t tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block scans `nb` block sums in place; the grand total goes to *total.
static __global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *sums, int64_t nb, uint32_t *total) {
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, lds, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (nb >= 0) sums[nb] = carry;
        if (total) *total = carry;
    }
}

template <class Load, class Store>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Load load, Store store, int64_t n,
                                                            const uint32_t *prefix) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t carry = prefix[blockIdx.x];
    for (int r = 0; r < kScanRounds; ++r) {
        const int64_t i = base + r * kScanThreads + threadIdx.x;
        const uint32_t v = i < n ? load(i) : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, lds, &tot);
        if (i < n) store(i, carry + ex, v);
        carry += tot;
    }
}

inline int64_t scan_tmp_words(int64_t n) { return ceil_div(n, kScanTile) + 1; }

// tmp: at least scan_tmp_words(n) uint32; total: device uint32 (nullable).
template <class Load, class Store>
inline hipError_t scan_exclusive(Load load, Store store, int64_t n, uint32_t *tmp, uint32_t *total,
                                 hipStream_t s) {
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb > 0) k_scan_reduce<Load><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(load, n, tmp);
    k_scan_top<<<1, kScanThreads, 0, s>>>(tmp, nb, total);
    if (nb > 0)
        k_scan_down<Load, Store><<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(load, store, n, tmp);
    return hipGetLastError();
}

struct LoadU32 {
    const uint32_t *p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct StoreU32 {
    uint32_t *p;
    __device__ void operator()(int64_t i, uint32_t ex, uint32_t) const { p[i] = ex; }
};

}  // namespace mgs
