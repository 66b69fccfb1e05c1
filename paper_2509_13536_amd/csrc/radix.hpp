// Stable least-significant-digit radix sort of (key, uint32 value) pairs, one
// 8-bit digit per pass.  A pass is three launches: per-block digit histograms
// (a digit-major table), an exclusive scan of each digit's row of that table
// (one block per digit, which also writes the row's total), and a stable
// scatter that adds the scan of the 256 row totals itself.  Inside a block
// (4 waves) each wave ranks its items 64 at a time: eight ballots find the
// lanes sharing a digit, and a per-wave LDS counter per digit carries the
// running rank, so the order of equal digits is the input order.  Both the
// histogram and the scatter issue all of a wave's loads before they rank, so a
// block waits for memory once.  The scatter stages the block's items in LDS in
// digit order and then writes runs of equal digits to consecutive addresses.
#pragma once
#include <algorithm>
#include "common.hpp"
#include "scan.hpp"

namespace mgs {

constexpr int kRadixThreads = 256;
// A wave ranks ROUNDS batches of 64 contiguous items, a block (4 waves) 256 *
// ROUNDS: 4096 items per block for large inputs (long runs of equal digits,
// so the scatter writes longer contiguous pieces), 1024 for small ones and
// 256 (one batch a wave) under 65536 items, so that a small sort still
// spreads over the CUs and each wave's chain of LDS rounds stays short.
constexpr int kRadixRoundsLarge = 16, kRadixRoundsSmall = 4, kRadixRoundsTiny = 1;
constexpr int64_t kRadixSmallN = int64_t(1) << 21, kRadixTinyN = int64_t(1) << 16;

// digit = (key >> shift) & 0xFF.  A digit function whose digit depends on the
// value as well sets kUsesValue (the histogram then loads the values); one
// whose digit of a 64-bit key lies in the key's low 32 bits sets kLowWord (the
// histogram then loads only those).
template <class K>
struct DigitOfKey {
    static constexpr bool kUsesValue = false, kLowWord = false;
    int shift;
    __device__ __forceinline__ uint32_t operator()(K key, uint32_t) const {
        return (uint32_t)(key >> shift) & 0xFFu;
    }
};

// An extra write per scattered item (its output position, key and value): none.
struct NoSide {
    template <class K>
    __device__ __forceinline__ void operator()(int64_t, K, uint32_t) const {}
};

// lanes of the wave (among `valid` ones) whose digit equals this lane's digit
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
    }
    return valid ? peers : 0ull;
}

template <class K, class Digit, int ROUNDS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const K *keys, const uint32_t *vals,
                                                              int64_t n, Digit dig, uint32_t *hist,
                                                              int64_t nb) {
    __shared__ uint32_t h[4][256];
    for (int i = threadIdx.x; i < 4 * 256; i += kRadixThreads) (&h[0][0])[i] = 0;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t base = (int64_t)blockIdx.x * (256 * ROUNDS) + (int64_t)wave * (64 * ROUNDS);
    K key[ROUNDS];
    uint32_t val[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        if constexpr (sizeof(K) == 8 && Digit::kLowWord)
            key[r] = valid ? (K)reinterpret_cast<const uint32_t *>(keys)[2 * i] : K(0);
        else
            key[r] = valid ? keys[i] : K(0);
        if constexpr (Digit::kUsesValue) val[r] = valid ? (vals ? vals[i] : (uint32_t)i) : 0u;
        else val[r] = 0u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint32_t d = valid ? dig(key[r], val[r]) : 0u;
        // counts only (no ranks): one add for a wave whose valid lanes share a
        // digit (runs of equal high digits), else a return-less LDS atomic per lane
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const uint64_t live = ballot(valid);
        if (ballot(valid && d != d0) == 0ull) {
            if (lane == 0 && live) h[wave][d0] += (uint32_t)__popcll(live);
        } else if (valid) {
            atomicAdd(&h[wave][d], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;
    hist[(int64_t)d * nb + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Exclusive scan, in place, of digit blockIdx.x's row of nb block counts; the
// row's total goes to totals[digit].  Each thread takes a contiguous run of the
// row (all its loads in flight), then one block scan joins the runs.
static __global__ __launch_bounds__(kRadixThreads) void k_radix_rowscan(uint32_t *hist, int64_t nb, uint32_t *totals) {
    __shared__ uint32_t lds4[4];
    uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    const int64_t per = (nb + kRadixThreads - 1) / kRadixThreads;
    const int64_t b0 = std::min<int64_t>((int64_t)threadIdx.x * per, nb);
    const int64_t b1 = std::min<int64_t>(b0 + per, nb);
    uint32_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += row[b];
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(sum, lds4, &tot);
    for (int64_t b = b0; b < b1; ++b) {
        const uint32_t c = row[b];
        row[b] = ex;
        ex += c;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// VALS = false: keys only (no value is staged or written)
template <class K, class Digit, int ROUNDS, class Side, bool VALS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const K *keys_in, const uint32_t *vals_in,
                                                                 K *keys_out, uint32_t *vals_out, int64_t n,
                                                                 Digit dig, const uint32_t *hist, int64_t nb,
                                                                 const uint32_t *totals, Side side) {
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t lds4[4];
    constexpr int kTileItems = 256 * ROUNDS;
    __shared__ K skeys[kTileItems];
    __shared__ uint32_t svals[VALS ? kTileItems : 1];
    for (int i = threadIdx.x; i < 4 * 256; i += kRadixThreads) (&wcnt[0][0])[i] = 0;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int64_t bbase = (int64_t)blockIdx.x * kTileItems;
    const int64_t base = bbase + (int64_t)wave * (64 * ROUNDS);
    // this thread's digit: its row total and this block's start within the row
    const uint32_t row_total = totals[threadIdx.x];
    const uint32_t row_start = hist[(int64_t)threadIdx.x * nb + blockIdx.x];
    K key[ROUNDS];
    uint32_t val[ROUNDS];
    uint32_t rank[ROUNDS];
    uint32_t dg[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? keys_in[i] : K(0);
        val[r] = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const bool valid = base + r * 64 + lane < n;
        const uint32_t d = valid ? dig(key[r], val[r]) : 0u;
        dg[r] = valid ? d : 0xFFFFFFFFu;
        const uint64_t peers = match_digit(d, valid);
        const uint32_t before = wcnt[wave][d];
        rank[r] = before + (uint32_t)__popcll(peers & lt_mask);
        if (valid && (int)(__ffsll((long long)peers) - 1) == lane) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(c0 + c1 + c2 + c3, lds4, &tot);
        const uint32_t gex = block_exclusive_scan(row_total, lds4, &tot);
        dstart[d] = ex;
        wcnt[0][d] = ex;
        wcnt[1][d] = ex + c0;
        wcnt[2][d] = ex + c0 + c1;
        wcnt[3][d] = ex + c0 + c1 + c2;
        gbase[d] = gex + row_start;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        if (dg[r] != 0xFFFFFFFFu) {
            const uint32_t pos = wcnt[wave][dg[r]] + rank[r];
            skeys[pos] = key[r];
            if (VALS) svals[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t cnt = (n - bbase) < kTileItems ? (n - bbase) : kTileItems;
    for (int i = threadIdx.x; i < cnt; i += kRadixThreads) {
        const K k = skeys[i];
        const uint32_t v = VALS ? svals[i] : 0u;
        const uint32_t d = dig(k, v);
        const int64_t o = (int64_t)gbase[d] + (i - (int64_t)dstart[d]);
        keys_out[o] = k;
        if (VALS) vals_out[o] = v;
        side(o, k, v);
    }
}

inline int radix_rounds(int64_t n) {
    return n < kRadixTinyN ? kRadixRoundsTiny : (n < kRadixSmallN ? kRadixRoundsSmall : kRadixRoundsLarge);
}
inline int64_t radix_blocks(int64_t n) { return ceil_div(n, 256 * radix_rounds(n)); }
// histogram words enough for any pass over at most n items (the block count
// is monotone within each tile regime, not across the switches): the table
// and the 256 row totals after it
inline int64_t radix_hist_words(int64_t n) {
    const int64_t nb = std::max<int64_t>(std::max<int64_t>(radix_blocks(std::min<int64_t>(n, kRadixTinyN - 1)),
                                                           radix_blocks(std::min<int64_t>(n, kRadixSmallN - 1))),
                                         radix_blocks(n));
    return 256 * std::max<int64_t>(nb, 1) + 256;
}

template <class K, class Digit, int ROUNDS, class Side, bool VALS>
inline void radix_launch(const K *keys_in, const uint32_t *vals_in, K *keys_out, uint32_t *vals_out, int64_t n,
                         Digit dig, uint32_t *hist, int64_t nb, Side side, hipStream_t s) {
    uint32_t *totals = hist + 256 * nb;
    k_radix_hist<K, Digit, ROUNDS><<<dim3((unsigned)nb), dim3(kRadixThreads), 0, s>>>(keys_in, vals_in, n, dig,
                                                                                     hist, nb);
    k_radix_rowscan<<<dim3(256), dim3(kRadixThreads), 0, s>>>(hist, nb, totals);
    k_radix_scatter<K, Digit, ROUNDS, Side, VALS><<<dim3((unsigned)nb), dim3(kRadixThreads), 0, s>>>(
        keys_in, vals_in, keys_out, vals_out, n, dig, hist, nb, totals, side);
}

// One stable pass; vals_in == nullptr means values are the input indices.
// hist: radix_hist_words(n) uint32.  side(o, key, value) runs for every item
// the scatter writes, at its output position o.
template <class K, class Digit, class Side = NoSide>
inline hipError_t radix_pass(const K *keys_in, const uint32_t *vals_in, K *keys_out, uint32_t *vals_out,
                             int64_t n, Digit dig, uint32_t *hist, hipStream_t s, Side side = Side{}) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = radix_blocks(n);
    if (radix_rounds(n) == kRadixRoundsTiny)
        radix_launch<K, Digit, kRadixRoundsTiny, Side, true>(keys_in, vals_in, keys_out, vals_out, n, dig, hist,
                                                             nb, side, s);
    else if (radix_rounds(n) == kRadixRoundsSmall)
        radix_launch<K, Digit, kRadixRoundsSmall, Side, true>(keys_in, vals_in, keys_out, vals_out, n, dig, hist,
                                                              nb, side, s);
    else
        radix_launch<K, Digit, kRadixRoundsLarge, Side, true>(keys_in, vals_in, keys_out, vals_out, n, dig, hist,
                                                              nb, side, s);
    return hipGetLastError();
}

// The same pass over keys alone (the digit must not read the value; the side
// write sees 0 for it).
template <class K, class Digit, class Side = NoSide>
inline hipError_t radix_pass_keys(const K *keys_in, K *keys_out, int64_t n, Digit dig, uint32_t *hist,
                                  hipStream_t s, Side side = Side{}) {
    static_assert(!Digit::kUsesValue, "a keys-only pass has no values");
    if (n <= 0) return hipSuccess;
    const int64_t nb = radix_blocks(n);
    if (radix_rounds(n) == kRadixRoundsTiny)
        radix_launch<K, Digit, kRadixRoundsTiny, Side, false>(keys_in, nullptr, keys_out, nullptr, n, dig, hist,
                                                              nb, side, s);
    else if (radix_rounds(n) == kRadixRoundsSmall)
        radix_launch<K, Digit, kRadixRoundsSmall, Side, false>(keys_in, nullptr, keys_out, nullptr, n, dig, hist,
                                                               nb, side, s);
    else
        radix_launch<K, Digit, kRadixRoundsLarge, Side, false>(keys_in, nullptr, keys_out, nullptr, n, dig, hist,
                                                               nb, side, s);
    return hipGetLastError();
}

}  // namespace mgs
