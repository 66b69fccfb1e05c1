// Blend kernels of the gfx950 rasteriser (MemGS Sec. II-E): alpha compositing
// of the depth-ordered tile lists, forward and backward, and the tile-level
// tests they share with the emission.
#pragma once

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "project.hpp"
#include "scan.hpp"

namespace mgs {

// work-queue heads sit this many words apart, so that no two share a cache line
constexpr int kQueueStride = 64;

// log2(1/255), and the margin (in log2 alpha) that the tile-level culling
// tests keep above the rounding of the per-pixel evaluation
constexpr float kLog2AlphaMin = -7.994353436858858f;
constexpr float kTileTestMargin = 0.02f;

__device__ __forceinline__ int view_of_bin(const ViewDev *views, int V, int64_t t) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].bin_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- work queues
// Eight queues, one per XCD (workgroups are dealt to the eight XCDs round
// robin); queue q holds the work slots q, q + 8, q + 16, ... of one order over
// all bins.  A block drains its own queue, then steals from the others; every
// block exits after at most eight failed grabs.
// The order puts the bins with the longest lists first: a persistent wave
// takes only a few bins, so a heavy bin started last would set the kernel's
// end, and dealing the order round robin starts every XCD on heavy bins.  Bins
// fall into 256 classes of list length, 16 per octave (the count's leading bit
// and the four bits after it; 2^16 instances or more share the top class).
// k_bin_count adds up the class sizes; k_bin_place gives each block a slice of
// every class (global atomics on class cursors) and scatters the bin ids.  The
// order within a class is unspecified, which changes no result (bins are
// independent).  Both blend kernels take this order.
constexpr int kOrderClasses = 256;
// bookkeeping words: class sizes, then class cursors (zeroed before k_bin_count)
constexpr int kBinOrderWords = 2 * kOrderClasses;

__device__ __forceinline__ uint32_t len_class(uint32_t len) {  // 0 = longest
    const uint32_t v = len + 1u;
    const int e = 31 - __clz(v);
    const uint32_t f = e >= 4 ? (v >> (e - 4)) & 15u : (v << (4 - e)) & 15u;
    const uint32_t q = (uint32_t)e * 16u + f;
    return q >= 255u ? 0u : 255u - q;
}

inline unsigned bin_order_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 512));
}

__global__ __launch_bounds__(256) void k_bin_count(const uint2 *range, int64_t n, uint32_t *book) {
    __shared__ uint32_t h[kOrderClasses];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint2 r = range[i];
        atomicAdd(&h[len_class(r.y - r.x)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(book + threadIdx.x, h[threadIdx.x]);
}

// Same grid and items as k_bin_count.
__global__ __launch_bounds__(256) void k_bin_place(const uint2 *range, int64_t n, uint32_t *book, uint32_t *order) {
    __shared__ uint32_t h[kOrderClasses];     // this block's class sizes, then its next slots
    __shared__ uint32_t base[kOrderClasses];  // this block's first slot in each class
    __shared__ uint32_t lds4[4];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint2 r = range[i];
        atomicAdd(&h[len_class(r.y - r.x)], 1u);
    }
    __syncthreads();
    const int c = threadIdx.x;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(book[c], lds4, &tot);
    const uint32_t mine = h[c];
    base[c] = ex + (mine ? atomicAdd(book + kOrderClasses + c, mine) : 0u);
    h[c] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint2 r = range[i];
        const uint32_t c0 = len_class(r.y - r.x);
        order[base[c0] + atomicAdd(&h[c0], 1u)] = (uint32_t)i;
    }
}

// Slot of queue q's next bin in the order (queue q takes slots q, q + 8, ...);
// -1 once all eight queues are empty.
__device__ __forceinline__ int64_t next_item(uint32_t *queues, int64_t n_items, int &q, int &tries) {
    while (tries < 8) {
        uint32_t i = 0;
        if (lane_id() == 0) i = atomicAdd(queues + q * kQueueStride, 1u);
        i = __shfl(i, 0, 64);
        if (q + 8 * (int64_t)i < n_items) return q + 8 * (int64_t)i;
        q = (q + 1) & 7;
        ++tries;
    }
    return -1;
}

// The unclamped alpha o exp(power) = exp2(p2 + log2 o), p2 the power in log2
// units, and the clamped alpha, evaluated identically by the forward and the
// backward kernels (same operations, explicit FMAs).  log2 o (the staged
// conic's w) enters with the dx-only term, so the opacity costs no operation
// per evaluation.
struct AlphaEval {
    float aun, alpha;
};
__device__ __forceinline__ AlphaEval alpha_at(float adx2, float bdx, float cc, float dy) {
    AlphaEval r;
    const float p2 = __builtin_fmaf(dy, __builtin_fmaf(cc, dy, bdx), adx2);
    r.aun = __builtin_amdgcn_exp2f(p2);
    r.alpha = fminf(kAlphaMax, r.aun);
    return r;
}
// The same evaluation for a Gaussian that cannot reach the clamp (may_clamp
// false): min(0.99, a) is a itself, bit for bit.
__device__ __forceinline__ AlphaEval alpha_at_unclamped(float adx2, float bdx, float cc, float dy) {
    AlphaEval r;
    const float p2 = __builtin_fmaf(dy, __builtin_fmaf(cc, dy, bdx), adx2);
    r.aun = __builtin_amdgcn_exp2f(p2);
    r.alpha = r.aun;
    return r;
}
// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}
// per quadrant column: adx2 = a' dx^2 + log2 o, bdx = b' dx
__device__ __forceinline__ void shared_dx(float ca, float cb, float l2o, float dx, float &adx2, float &bdx) {
    adx2 = __builtin_fmaf(ca * dx, dx, l2o);
    bdx = cb * dx;
}

// Can any pixel of the box [bx0, bx1] x [by0, by1] reach alpha >= 1/255?
// The scaled exponent p2(d) = ca dx^2 + cb dx dy + cc dy^2 (d = mean - pixel)
// is concave; its maximum over the box is 0 when the mean lies inside, else
// on an edge, where the 1D maximum is the clamped stationary point.  The test
// keeps a margin of 0.02 in log2 alpha (1.4 %), far above the rounding of the
// per-pixel evaluation, so a culled Gaussian is one every pixel of the box
// would skip: dropping it leaves every output bit unchanged.
__device__ __forceinline__ bool box_may_hit(float u, float v, float ca, float cb, float cc, float l2o, float bx0,
                                            float bx1, float by0, float by1) {
    if (bx0 > bx1 || by0 > by1) return false;  // box outside the image
    const float dxl = u - bx1, dxh = u - bx0, dyl = v - by1, dyh = v - by0;
    float best;
    if (dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f) {
        best = 0.0f;
    } else {
        best = -INFINITY;
        const float ix = -cb / (2.0f * cc), iy = -cb / (2.0f * ca);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float dx = e ? dxh : dxl;
            const float dy = sclamp(ix * dx, dyl, dyh);
            best = fmaxf(best, (ca * dx + cb * dy) * dx + cc * dy * dy);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float dy = e ? dyh : dyl;
            const float dx = sclamp(iy * dy, dxl, dxh);
            best = fmaxf(best, (ca * dx + cb * dy) * dx + cc * dy * dy);
        }
    }
    return best + l2o >= kLog2AlphaMin - kTileTestMargin;
}

// Can the computed alpha of a Gaussian reach the 0.99 clamp anywhere in the
// pixel box [bx0, bx1] x [by0, by1]?  The quadratic form of the exponent is
// negative semidefinite, so the exact exponent never exceeds log2 o, and its
// fp32 evaluation (alpha_at: five rounded operations on terms no larger than
// |a'| dx^2 + |b'| |dx dy| + |c'| dy^2 + |log2 o|, dx and dy bounded by the
// box) errs by less than 2^-19 of that sum (eight times the worst case).  When
// log2 o plus that bound stays below log2 0.99, alpha = min(0.99, a) equals a
// at every pixel, bit for bit, and the clamp and its zero gradient can be
// skipped.  A NaN or infinite bound keeps the clamp.
constexpr float kLog2AlphaMax = -0.014499569695115089f;  // log2 0.99
__device__ __forceinline__ bool may_clamp(float u, float v, float4 cn, float bx0, float bx1, float by0, float by1) {
    const float dx = fmaxf(fabsf(u - bx0), fabsf(u - bx1)), dy = fmaxf(fabsf(v - by0), fabsf(v - by1));
    const float tmax = fabsf(cn.x) * dx * dx + fabsf(cn.y) * dx * dy + fabsf(cn.z) * dy * dy + fabsf(cn.w);
    return !(cn.w + 0x1p-19f * tmax + 1e-6f < kLog2AlphaMax);
}
// bit of a staged Gaussian's quadrant mask word that marks may_clamp
constexpr uint32_t kClampBit = 0x80000000u;

// A bin of BTX x BTY tiles (the unit of a tile list and of one wave's work),
// split into 8x8 quadrants q = qx + QX qy.  Lane l owns pixel (l % 8, l / 8) of
// every quadrant, so a quadrant that a Gaussian cannot reach, that lies
// outside the Gaussian's tile rectangle, or whose 64 pixels have all finished,
// is skipped by the whole wave with one scalar branch.
// SPLIT: the wave takes one quadrant of a 1x1 bin (its offset from bin_geo's
// quad), for calls with too few bins to fill the chip.
template <int BTX, int BTY, bool SPLIT = false>
struct BinGeo {
    static_assert(!SPLIT || (BTX == 1 && BTY == 1), "a split wave takes one quadrant of a one-tile bin");
    static constexpr int QX = SPLIT ? 1 : 2 * BTX, QY = SPLIT ? 1 : 2 * BTY, NQ = QX * QY;
    float qx0[QX], qx1[QX], qy0[QY], qy1[QY];  // quadrant pixel boxes (clipped to the image)
    float fpx[QX], fpy[QY];                    // this lane's pixel coordinates per quadrant column / row
    int px[QX], py[QY];
    int tx[QX], ty[QY];                        // tile coordinates of the quadrant columns / rows
};

template <int BTX, int BTY, bool SPLIT = false>
__device__ __forceinline__ BinGeo<BTX, BTY, SPLIT> bin_geo(int local, const ViewDev &V, int lane, int quad = 0) {
    using G = BinGeo<BTX, BTY, SPLIT>;
    G t;
    const int by = local / V.BX, bx = local - by * V.BX;
    const int ox = SPLIT ? (quad & 1) : 0, oy = SPLIT ? (quad >> 1) : 0;  // quadrant offset of a split wave
#pragma unroll
    for (int h = 0; h < G::QX; ++h) {
        const int x0 = bx * (kTile * BTX) + 8 * (h + ox);
        t.qx0[h] = (float)x0;
        t.qx1[h] = (float)min(x0 + 7, V.W - 1);
        t.px[h] = x0 + (lane & 7);
        t.fpx[h] = (float)t.px[h];
        t.tx[h] = bx * BTX + ((h + ox) >> 1);
    }
#pragma unroll
    for (int h = 0; h < G::QY; ++h) {
        const int y0 = by * (kTile * BTY) + 8 * (h + oy);
        t.qy0[h] = (float)y0;
        t.qy1[h] = (float)min(y0 + 7, V.H - 1);
        t.py[h] = y0 + (lane >> 3);
        t.fpy[h] = (float)t.py[h];
        t.ty[h] = by * BTY + ((h + oy) >> 1);
    }
    return t;
}

template <int BTX, int BTY, bool SPLIT>
__device__ __forceinline__ uint32_t quad_mask(const BinGeo<BTX, BTY, SPLIT> &t, float u, float v, float4 cn,
                                              ushort4 rc) {
    using G = BinGeo<BTX, BTY, SPLIT>;
    const float l2o = cn.w;  // log2 of the opacity
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < G::NQ; ++q) {
        const int hx = q % G::QX, hy = q / G::QX;
        const bool in_rect = (BTX == 1 || (t.tx[hx] >= rc.x && t.tx[hx] < rc.z)) &&
                             (BTY == 1 || (t.ty[hy] >= rc.y && t.ty[hy] < rc.w));
        if (in_rect && box_may_hit(u, v, cn.x, cn.y, cn.z, l2o, t.qx0[hx], t.qx1[hx], t.qy0[hy], t.qy1[hy]))
            m |= 1u << q;
    }
    return m;
}

// The same culling for a bin of several quadrants, from the ellipse where
// the Gaussian can reach alpha >= 1/255 (with the margin above): with
// Q(d) = -(a' dx^2 + b' dx dy + c' dy^2) = d^T M d (M positive definite for a
// valid conic) it is Q(d) <= S, S = log2 o - log2(1/255) + margin.  Over one
// quadrant row (the band of its pixel centres) the ellipse covers an interval
// of x: its extreme points (+-rx at dy = +-yx) when they lie in the band, else
// the conditional extent at the nearest band edge; a quadrant of the row is
// reached exactly when its pixel columns meet that interval.  Per Gaussian
// that is one set-up and two extents per quadrant row instead of four edge
// maxima per quadrant (box_may_hit); the interval is padded for its rounding
// (1e-3 of the radius and 1e-5 of the coordinate, far above the few ulp of the
// square roots), so the test stays conservative and no result bit changes.  A
// conic that is not positive definite (not from a valid projection) reaches
// every quadrant of its rectangle.
template <int BTX, int BTY, bool SPLIT>
__device__ __forceinline__ uint32_t quad_mask_rows(const BinGeo<BTX, BTY, SPLIT> &t, float u, float v, float4 cn,
                                                   ushort4 rc) {
    using G = BinGeo<BTX, BTY, SPLIT>;
    const float S = cn.w - kLog2AlphaMin + kTileTestMargin;
    if (!(S > 0.0f)) return 0u;  // below 1/255 everywhere (or not a number)
    const float m11 = -cn.x, m12 = -0.5f * cn.y, m22 = -cn.z;
    const float det = m11 * m22 - m12 * m12;
    const bool pd = det > 0.0f && m11 > 0.0f && m22 > 0.0f;
    // the ellipse d^T Sigma^-1 d <= S, Sigma = M^-1
    const float idet = __builtin_amdgcn_rcpf(det);
    const float sxx = m22 * idet, sxy = -m12 * idet;
    const float kx = -m12 * __builtin_amdgcn_rcpf(m11);        // sxy / syy
    const float wx = __builtin_amdgcn_sqrtf(__builtin_amdgcn_rcpf(m11));  // sqrt(det Sigma / syy)
    const float iyy = det * __builtin_amdgcn_rcpf(m11);        // 1 / syy
    const float rx = __builtin_amdgcn_sqrtf(S * sxx);
    const float yx = sxy * __builtin_amdgcn_sqrtf(S * __builtin_amdgcn_rcpf(sxx));
    const float ry = __builtin_amdgcn_sqrtf(S * m11 * idet);
    const float padx = 1e-3f * rx + 1e-5f * fabsf(u) + 1e-3f;
    const float pady = 1e-3f * ry + 1e-5f * fabsf(v) + 1e-3f;
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < G::QY; ++r) {
        if (BTY != 1 && !(t.ty[r] >= rc.y && t.ty[r] < rc.w)) continue;  // outside the tile rectangle
        if (t.qy0[r] > t.qy1[r]) continue;                               // below the image
        const float dlo = v - t.qy1[r], dhi = v - t.qy0[r];
        if (pd && (dhi < -(ry + pady) || dlo > ry + pady)) continue;
        // dx extremes over the band (the largest dx, rx, sits at dy = yx, the
        // smallest at -yx; elsewhere the conditional extent is concave, so the
        // band's extreme is at the clamp of that dy); pixels reached: u - dx
        const float ya = sclamp(yx, dlo, dhi), yb = sclamp(-yx, dlo, dhi);
        const float dmax = ya == yx ? rx : kx * ya + wx * __builtin_amdgcn_sqrtf(fmaxf(0.0f, S - ya * ya * iyy));
        const float dmin = yb == -yx ? -rx : kx * yb - wx * __builtin_amdgcn_sqrtf(fmaxf(0.0f, S - yb * yb * iyy));
        const float xlo = pd ? u - dmax - padx : -INFINITY, xhi = pd ? u - dmin + padx : INFINITY;
#pragma unroll
        for (int h = 0; h < G::QX; ++h) {
            const bool in_rect = BTX == 1 || (t.tx[h] >= rc.x && t.tx[h] < rc.z);
            if (in_rect && t.qx0[h] <= t.qx1[h] && xlo <= t.qx1[h] && xhi >= t.qx0[h]) m |= 1u << (h + G::QX * r);
        }
    }
    return m;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Split work: queue q's i-th grab is quadrant i % 4 of the bin at order slot
// q + 8 (i / 4), so a bin's four quadrants go to one XCD (one L2 for its list);
// -1 once all eight queues are past the last bin.
__device__ __forceinline__ int64_t next_split_item(uint32_t *queues, int64_t n_bins, int &q, int &tries, int &quad) {
    while (tries < 8) {
        uint32_t i = 0;
        if (lane_id() == 0) i = atomicAdd(queues + q * kQueueStride, 1u);
        i = __shfl(i, 0, 64);
        const int64_t slot = q + 8 * (int64_t)(i >> 2);
        if (slot < n_bins) {
            quad = (int)(i & 3u);
            return slot;
        }
        q = (q + 1) & 7;
        ++tries;
    }
    return -1;
}

// ---------------------------------------------------------------- blend forward
// The sorted instance keys of the bin lists, in either format of the emission:
// the depth rank is (key >> rshift) & rmask; the backward record slot is
// key >> eshift in the packed format (eshift > 0) and rec[s] in the wide one.
struct InstRef {
    const uint64_t *key;
    const uint32_t *rec;
    int rshift, eshift;
    uint32_t rmask;
    __device__ __forceinline__ uint32_t rank(uint64_t k) const { return (uint32_t)(k >> rshift) & rmask; }
    __device__ __forceinline__ uint32_t slot(uint32_t s, uint64_t k) const {
        return eshift ? (uint32_t)(k >> eshift) : rec[s];
    }
};

struct BlendArgs {
    const ViewDev *views;
    int n_views;
    int64_t n_items;  // bins
    const uint32_t *order;  // work order of the bins (longest lists first, taken strided)
    const uint2 *range;
    InstRef inst;
    const float2 *rxy;
    const float4 *rconic, *rrgbd;
    const ushort4 *rrect;
    float bg0, bg1, bg2, bgd;
    uint32_t *queues;
    const uint32_t *clamp_flag;  // nonzero: some pair may reach the alpha clamp (may_clamp)
    int box_cull;                // nonzero: quadrant culling by box_may_hit everywhere (a check of quad_mask_rows)
    float *out_rgb, *out_depth, *out_T;
    uint32_t *n_contrib;
    uint32_t *n_blend;  // per-pixel blended count (instrumented variant only)
    uint16_t *inst_qm;  // quadrant mask of every staged list entry, for the backward (nullable)
};

// Staged Gaussian of a batch: image mean, scaled conic + log2 opacity, colour +
// depth, list position, quadrant mask.
// One staged Gaussian, its fields side by side (48 bytes, 16-byte aligned),
// so that the reads of one entry share one address register.  pos: its
// position in the bin's list (the forward stores 1 + the position).
struct StagedG {
    float4 cn, cd;
    float2 xy;
    uint32_t pos, qm;
};
static_assert(sizeof(StagedG) == 48, "three 16-byte rows per staged Gaussian");
struct Staged {
    StagedG g[64];
};

// Six waves per SIMD for the 16x16 bin (at most 80 VGPRs, as without the two
// variants of the loop below).
template <bool COUNT, int BTX, int BTY, bool SPLIT = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(BTX * BTY == 1 ? 6 : 1)))
void k_blend_fwd(BlendArgs a) {
    using G = BinGeo<BTX, BTY, SPLIT>;
    constexpr int QX = G::QX, NQ = G::NQ;
    __shared__ Staged sh;
    const int lane = threadIdx.x;
    int q = blockIdx.x & 7, tries = 0;
    // Without a pair that may reach the alpha clamp (the projection's flag),
    // the evaluation skips the clamp: bit for bit the same alpha.
    const bool any_clamp = __builtin_amdgcn_readfirstlane(*a.clamp_flag) != 0u;
    auto run = [&](auto clamp_v) {
    constexpr bool CLAMP = decltype(clamp_v)::value;
    for (;;) {
        int quad = 0;
        const int64_t slot = SPLIT ? next_split_item(a.queues, a.n_items, q, tries, quad)
                                   : next_item(a.queues, a.n_items, q, tries);
        if (slot < 0) break;
        const int64_t item = a.order[slot];  // the bin
        const int v = (int)uniform_u32((uint32_t)view_of_bin(a.views, a.n_views, item));
        const ViewDev &V = a.views[v];
        G t = bin_geo<BTX, BTY, SPLIT>((int)(item - V.bin_base), V, lane, quad);
        // keep the float pixel coordinates in registers: left alone, the
        // compiler converts them from the integer ones again for every staged
        // Gaussian (four conversions per visit, about a tenth of the issue)
#pragma unroll
        for (int h = 0; h < QX; ++h) asm volatile("" : "+v"(t.fpx[h]));
#pragma unroll
        for (int h = 0; h < G::QY; ++h) asm volatile("" : "+v"(t.fpy[h]));
        // T > 0: active; T < 0: finished with transmittance -T
        float T[NQ], C0[NQ], C1[NQ], C2[NQ], D[NQ];
        uint32_t last[NQ], cnt[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            T[i] = (t.px[i % QX] < V.W && t.py[i / QX] < V.H) ? 1.0f : -1.0f;
            C0[i] = C1[i] = C2[i] = D[i] = 0.0f;
            last[i] = 0;
            cnt[i] = 0;
        }
        const uint2 rg = a.range[item];
        for (uint32_t b = rg.x; b < rg.y; b += 64) {
            uint32_t act = 0;
#pragma unroll
            for (int i = 0; i < NQ; ++i) act |= (ballot(T[i] > 0.0f) != 0ull) ? (1u << i) : 0u;
            if (act == 0) break;
            // stage the batch: Gaussians live in some quadrant, compacted in list order
            const uint32_t s = b + lane;
            uint32_t qm = 0;
            float2 xy;
            float4 cn, cd;
            if (s < rg.y) {
                const uint32_t k = a.inst.rank(a.inst.key[s]);
                xy = a.rxy[k];
                cn = a.rconic[k];
                qm = G::NQ >= 4 && !a.box_cull ? quad_mask_rows(t, xy.x, xy.y, cn, a.rrect[k])
                                               : quad_mask(t, xy.x, xy.y, cn, a.rrect[k]);
                if (qm) cd = a.rrgbd[k];
                // the backward stages the same entries with the same mask
                // (bins of several tiles: the one-tile kernel is held to 80
                // VGPRs and would spill for it)
                if (!SPLIT && BTX * BTY > 1 && a.inst_qm) a.inst_qm[s] = (uint16_t)qm;
            }
            const uint64_t m = ballot(qm != 0);
            if (qm) {
                const int slot = __popcll(m & ((1ull << lane) - 1ull));
                StagedG &d = sh.g[slot];
                d.cn = cn;
                d.cd = cd;
                d.xy = xy;
                d.pos = s - rg.x + 1u;  // 1 + the list position: what a blending pixel records
                d.qm = qm;
            }
            const int nb = __popcll(m);
            __syncthreads();
            // lane j holds staged slot j's quadrant mask (its quadrants with an
            // active pixel): a visit takes it with a lane read instead of an LDS
            // round trip
            const uint32_t slot_qm = lane < nb ? sh.g[lane].qm & act : 0u;
            if constexpr (SPLIT) {
                // A split wave (one quadrant, a few waves per SIMD) is bound by
                // its dependent chains: it takes the live entries two at a time,
                // forms both alphas (which do not depend on T), then blends them
                // in list order: the same operations on each pixel, the same bits.
                uint64_t live = ballot(slot_qm != 0u);
                auto alpha_of = [&](const StagedG &sj) {
                    float adx2, bdx;
                    shared_dx(sj.cn.x, sj.cn.y, sj.cn.w, sj.xy.x - t.fpx[0], adx2, bdx);
                    const float dy = sj.xy.y - t.fpy[0];
                    return CLAMP ? alpha_at(adx2, bdx, sj.cn.z, dy) : alpha_at_unclamped(adx2, bdx, sj.cn.z, dy);
                };
                auto blend_one = [&](float alpha, float4 cd4, uint32_t pos1) {
                    const float Tn = __builtin_fmaf(-alpha, T[0], T[0]);
                    const bool ok = alpha >= kAlphaMin;
                    const bool blend = ok && (Tn >= kTMin);
                    const float w = blend ? alpha * T[0] : 0.0f;
                    C0[0] = __builtin_fmaf(w, cd4.x, C0[0]);
                    C1[0] = __builtin_fmaf(w, cd4.y, C1[0]);
                    C2[0] = __builtin_fmaf(w, cd4.z, C2[0]);
                    D[0] = __builtin_fmaf(w, cd4.w, D[0]);
                    T[0] = blend ? Tn : (ok ? -fabsf(T[0]) : T[0]);
                    last[0] = blend ? pos1 : last[0];
                    if (COUNT) cnt[0] += blend ? 1u : 0u;
                };
                constexpr int kAhead = 4;
                while (live) {
                    // the entries chosen first (a missing one repeats the first),
                    // so their reads and alphas need no branch; a missing entry's
                    // blend takes alpha 0, which blends nothing and leaves every
                    // value as it is (the colour and depth sums, never negative,
                    // gain +0)
                    int j[kAhead];
                    bool has[kAhead];
                    j[0] = __ffsll((long long)live) - 1;
                    has[0] = true;
                    live &= live - 1ull;
#pragma unroll
                    for (int u = 1; u < kAhead; ++u) {
                        has[u] = live != 0ull;
                        j[u] = has[u] ? __ffsll((long long)live) - 1 : j[0];
                        if (has[u]) live &= live - 1ull;
                    }
                    float al[kAhead];
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) al[u] = alpha_of(sh.g[j[u]]).alpha;
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) blend_one(has[u] ? al[u] : 0.0f, sh.g[j[u]].cd, sh.g[j[u]].pos);
                }
            } else
            for (int j = 0; j < nb; ++j) {
                const StagedG &sj = sh.g[j];
                const uint32_t mj = __builtin_amdgcn_readlane(slot_qm, j);
                if (mj == 0) continue;
                const float2 g = sj.xy;
                const float4 cn4 = sj.cn;
                const float4 cd4 = sj.cd;
                const uint32_t pos1 = sj.pos;
                // dy once per quadrant row (each row's pixels of a lane share it)
                float dyr[G::QY];
#pragma unroll
                for (int r = 0; r < G::QY; ++r) dyr[r] = g.y - t.fpy[r];
                // One quadrant's evaluation (i = h + QX r: column h, row r).
                auto eval = [&](auto ic, float adx2, float bdx) {
                    constexpr int i = decltype(ic)::value, r = i / QX;
                    const AlphaEval e = CLAMP ? alpha_at(adx2, bdx, cn4.z, dyr[r])
                                              : alpha_at_unclamped(adx2, bdx, cn4.z, dyr[r]);
                    const float Tn = __builtin_fmaf(-e.alpha, T[i], T[i]);  // T (1 - alpha), one rounding
                    // a finished pixel (T < 0) has Tn < 0, so it never blends again,
                    // and -|T| keeps it finished: no separate test of T > 0
                    const bool ok = e.alpha >= kAlphaMin;
                    const bool blend = ok && (Tn >= kTMin);
                    const float w = blend ? e.alpha * T[i] : 0.0f;
                    C0[i] = __builtin_fmaf(w, cd4.x, C0[i]);
                    C1[i] = __builtin_fmaf(w, cd4.y, C1[i]);
                    C2[i] = __builtin_fmaf(w, cd4.z, C2[i]);
                    D[i] = __builtin_fmaf(w, cd4.w, D[i]);
                    T[i] = blend ? Tn : (ok ? -fabsf(T[i]) : T[i]);
                    last[i] = blend ? pos1 : last[i];
                    if (COUNT) cnt[i] += blend ? 1u : 0u;
                };
                // column by column, a column's dx terms only where one of its
                // quadrants is live (each quadrant's pixels are its own, so the
                // order of the quadrants changes no result)
                static_for<QX>([&](auto hc) {
                    constexpr int h = decltype(hc)::value;
                    float adx2, bdx;
                    if constexpr (NQ == 1) {  // a split wave: its one quadrant is live
                        shared_dx(cn4.x, cn4.y, cn4.w, g.x - t.fpx[0], adx2, bdx);
                        eval(std::integral_constant<int, 0>{}, adx2, bdx);
                        return;
                    }
                    uint32_t colm = 0;
#pragma unroll
                    for (int r = 0; r < G::QY; ++r) colm |= 1u << (h + QX * r);
                    if (!(mj & colm)) return;
                    shared_dx(cn4.x, cn4.y, cn4.w, g.x - t.fpx[h], adx2, bdx);
                    static_for<G::QY>([&](auto rc) {
                        constexpr int i = h + QX * decltype(rc)::value;
                        if (mj & (1u << i)) eval(std::integral_constant<int, i>{}, adx2, bdx);
                    });
                });
            }
            __syncthreads();
        }
        const int64_t plane = (int64_t)V.W * V.H;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            // from the kept float coordinates (exact integers), so that the
            // integer ones need not stay live through the loop
            const int px = (int)t.fpx[i % QX], py = (int)t.fpy[i / QX];
            if (px < V.W && py < V.H) {
                const float Tf = fabsf(T[i]);
                const int64_t pix = V.pix_base + (int64_t)py * V.W + px;
                const int64_t pl = (int64_t)py * V.W + px;
                float *rgb = a.out_rgb + 3 * V.pix_base;
                rgb[pl] = C0[i] + Tf * a.bg0;
                rgb[plane + pl] = C1[i] + Tf * a.bg1;
                rgb[2 * plane + pl] = C2[i] + Tf * a.bg2;
                a.out_depth[pix] = D[i] + Tf * a.bgd;
                a.out_T[pix] = Tf;
                a.n_contrib[pix] = last[i];
                if (COUNT) a.n_blend[pix] = cnt[i];
            }
        }
    }
    };
    if (any_clamp) run(std::true_type{});
    else run(std::false_type{});
}

// ---------------------------------------------------------------- blend backward
struct BlendBwdArgs {
    const ViewDev *views;
    int n_views;
    int64_t n_items;  // bins
    const uint32_t *order;  // work order of the bins (longest lists first, taken strided)
    const uint2 *range;
    InstRef inst;
    const float2 *rxy;
    const float4 *rconic, *rrgbd;
    const ushort4 *rrect;
    float bg0, bg1, bg2, bgd;
    uint32_t *queues;
    const float *out_T, *dL_rgb, *dL_depth;
    const uint32_t *n_contrib;
    float *records;  // [M][10]
    int box_cull;    // as in BlendArgs
    const uint16_t *inst_qm;  // the forward's quadrant masks per list entry (bins of several tiles; nullable)
};

__device__ __forceinline__ void zero_record(float *records, uint32_t e) {
    float2 *rec = reinterpret_cast<float2 *>(records + (int64_t)e * kRecord);
#pragma unroll
    for (int c = 0; c < kRecord / 2; ++c) rec[c] = make_float2(0.f, 0.f);
}
// The kRecord = 10 per-lane values of one Gaussian visit are summed over the
// 64 lanes in two stages.
//  (1) wave_fold_record folds them with the CDNA4 cross-row swaps:
//      permlane32_swap exchanges the upper half-wave of one value with the
//      lower half-wave of the next, so one add leaves value 2k summed over lane
//      pairs (l, l+32) in lanes 0-31 and value 2k+1 in lanes 32-63 (five
//      registers); permlane16_swap does the same between rows 0/1 and 2/3 of two
//      such registers.  Three registers remain, each 16-lane row holding one
//      value summed over the four lanes l, l+16, l+32, l+48:
//        z0 rows = values 0, 2, 1, 3;  z1 rows = 4, 6, 5, 7;  z2 rows = 8, 8, 9, 9.
//      17 VALU instructions; the registers go to LDS (three stores a lane).
//  (2) after kFold visits (or at the end of a batch) one flush sums each
//      value's 16 row partials, one lane per (visit, value): 60 of the 64 lanes
//      read 16 floats and add them, and write the record value to its slot.
// The second stage replaces four DPP steps per register and the per-visit
// stores of the row totals (about 18 VALU instructions a visit) by about 20
// instructions per kFold visits.
// ds_swizzle bit mode: and-mask 31, or-mask 0, xor-mask 16 (lane ^ 16 in each 32)
constexpr int kSwizzleXor16 = (16 << 10) | 31;
__device__ __forceinline__ float2 swap32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return make_float2(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float2 swap16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return make_float2(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
static_assert(kRecord == 10, "the record reduction folds exactly ten values");
__device__ __forceinline__ void wave_fold_record(const float *x, float z[3]) {
    float y[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float2 s = swap32(x[2 * k], x[2 * k + 1]);
        y[k] = s.x + s.y;
    }
    float2 s = swap16(y[0], y[1]);
    z[0] = s.x + s.y;
    s = swap16(y[2], y[3]);
    z[1] = s.x + s.y;
    // the last register pairs with itself: rows 0/1 and 2/3 exchanged by a
    // swizzle (lane ^ 16 within each half-wave), which needs no copy of y[4]
    // for the swap's second operand
    z[2] = y[4] + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(y[4]), kSwizzleXor16));
}
// The fold of a tracking call (POSE: the pose gradient alone, maps of SH
// degree 0, whose colour does not depend on the view): of the ten values only
// the six the pose reads, gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2 and the
// depth weight (values 1-5 and 9), folded by the same steps.  Every value is
// summed over the same lanes in the same order whichever register and half
// it sits in ((x_l + x_l+32) + (x_l+16 + x_l+48), then the 16 row partials in
// the flush), so each is bit for bit the full fold's:
//   z0 rows = values 1, 3, 2, 4;  z1 rows = 5, 5, 9, 9.
// 10 VALU instead of 16, two LDS stores instead of three.
__device__ __forceinline__ void wave_fold_pose(const float *x, float z[2]) {  // x: values 1, 2, 3, 4, 5, 9
    const float2 s0 = swap32(x[0], x[1]);
    const float y0 = s0.x + s0.y;
    const float2 s1 = swap32(x[2], x[3]);
    const float y1 = s1.x + s1.y;
    const float2 s2 = swap32(x[4], x[5]);
    const float y2 = s2.x + s2.y;
    const float2 s = swap16(y0, y1);
    z[0] = s.x + s.y;
    z[1] = y2 + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(y2), kSwizzleXor16));
}
// Visits folded before a flush: 10 kFold <= 64 lanes.
constexpr int kFold = 6;
// Where value v of a folded visit sits: register v_reg(v), row v_row(v).
__device__ __forceinline__ int fold_reg(int v) { return v < 4 ? 0 : (v < 8 ? 1 : 2); }
__device__ __forceinline__ int fold_row(int v) {
    const int w = v < 8 ? (v & 3) : 2 * (v - 8);  // z2 holds value 8 in rows 0-1, 9 in rows 2-3
    return v < 8 ? ((w & 1) << 1) | (w >> 1) : w;
}
// A flush lane's source in the folded rows: value v of folded visit ff, 16
// consecutive floats of part[kFold][3][64]; -1 for a value the tracking fold
// leaves out (its record value is zero).
template <bool POSE>
__device__ __forceinline__ int fold_src(int ff, int v) {
    if (!POSE) return (ff * 3 + fold_reg(v)) * 64 + 16 * fold_row(v);
    int reg, row;
    switch (v) {
        case 1: reg = 0; row = 0; break;
        case 3: reg = 0; row = 1; break;
        case 2: reg = 0; row = 2; break;
        case 4: reg = 0; row = 3; break;
        case 5: reg = 1; row = 0; break;
        case 9: reg = 1; row = 2; break;
        default: return -1;
    }
    return (ff * 3 + reg) * 64 + 16 * row;
}

struct StagedBwd {
    StagedG g[64];                 // pos: the position in the bin's list
    uint32_t e[64];                // record slot of each staged Gaussian
    float part[kFold][3][64];      // folded visits awaiting a flush
};

// POSE: a tracking call over maps of SH degree 0 (the pose gradient alone):
// the colour and opacity sums are not formed and their record values are zero.
template <int BTX, int BTY, bool POSE>
__global__ __launch_bounds__(64) void k_blend_bwd(BlendBwdArgs a) {
    using G = BinGeo<BTX, BTY>;
    constexpr int QX = G::QX, NQ = G::NQ;
    __shared__ StagedBwd sh;
    const int lane = threadIdx.x;
    // this lane's share of a flush: value fv of folded visit ff, read from 16
    // consecutive floats of sh.part (lanes 60-63 have none)
    const int ff = lane / kRecord, fv = lane - ff * kRecord;
    const bool flush_lane = ff < kFold;
    const int src = flush_lane ? fold_src<POSE>(ff, fv) : -1;
    const int part_off = src >= 0 ? src : 0;
    int q = blockIdx.x & 7, tries = 0;
    for (;;) {
        const int64_t slot = next_item(a.queues, a.n_items, q, tries);
        if (slot < 0) break;
        const int64_t item = a.order[slot];  // the bin
        const int v = (int)uniform_u32((uint32_t)view_of_bin(a.views, a.n_views, item));
        const ViewDev &V = a.views[v];
        const G t = bin_geo<BTX, BTY>((int)(item - V.bin_base), V, lane);
        const int64_t plane = (int64_t)V.W * V.H;
        // nSg = -(colour, depth) composited behind the current Gaussian, dotted
        // with the pixel's upstream gradient (negated: c.g - S.g is then one
        // chain of four FMAs)
        float Tc[NQ], nSg[NQ], g0[NQ], g1[NQ], g2[NQ], gd[NQ];
        uint32_t nc[NQ];
        uint32_t ncq[NQ];  // per quadrant: the largest last-contributor position
        uint32_t ncmax = 0;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int px = t.px[i % QX], py = t.py[i / QX];
            if (px < V.W && py < V.H) {
                const int64_t pix = V.pix_base + (int64_t)py * V.W + px;
                const int64_t pl = (int64_t)py * V.W + px;
                const float *gr = a.dL_rgb + 3 * V.pix_base;
                Tc[i] = a.out_T[pix];
                nc[i] = a.n_contrib[pix];
                g0[i] = gr[pl];
                g1[i] = gr[plane + pl];
                g2[i] = gr[2 * plane + pl];
                gd[i] = a.dL_depth ? a.dL_depth[pix] : 0.0f;
            } else {
                Tc[i] = 1.0f; nc[i] = 0; g0[i] = g1[i] = g2[i] = gd[i] = 0.0f;
            }
            nSg[i] = -(a.bg0 * g0[i] + a.bg1 * g1[i] + a.bg2 * g2[i] + a.bgd * gd[i]);
            ncq[i] = uniform_u32(wave_max_u32(nc[i]));
            ncmax = ncq[i] > ncmax ? ncq[i] : ncmax;
        }
        const uint2 rg = a.range[item];
        // Gaussians past every pixel's last contributor get zero records.
        for (uint32_t s = rg.x + ncmax + lane; s < rg.y; s += 64) zero_record(a.records, a.inst.slot(s, a.inst.key[s]));
        int hi = (int)ncmax;
        while (hi > 0) {
            const int lo = hi > 64 ? hi - 64 : 0;
            const int nb = hi - lo;
            uint32_t qm = 0, e = 0;
            float2 xy;
            float4 cn, cd;
            if (lane < nb) {
                const uint32_t s = rg.x + lo + lane;
                const uint64_t key = a.inst.key[s];
                const uint32_t k = a.inst.rank(key);
                xy = a.rxy[k];
                cn = a.rconic[k];
                e = a.inst.slot(s, key);
                // the forward's mask of this entry when it kept them (it staged
                // every entry up to the last contributor with the same test)
                qm = a.inst_qm ? (uint32_t)a.inst_qm[s]
                               : (a.box_cull ? quad_mask(t, xy.x, xy.y, cn, a.rrect[k])
                                             : quad_mask_rows(t, xy.x, xy.y, cn, a.rrect[k]));
                if (qm) {
                    cd = a.rrgbd[k];
                    if (may_clamp(xy.x, xy.y, cn, t.qx0[0], t.qx1[QX - 1], t.qy0[0], t.qy1[G::QY - 1])) qm |= kClampBit;
                } else {
                    zero_record(a.records, e);
                }
            }
            const uint64_t m = ballot(qm != 0);
            const int nlive = __popcll(m);
            if (qm) {
                // staged back to front (the last list entry first), so that the
                // loop below walks the slots upwards
                const int slot = nlive - 1 - __popcll(m & ((1ull << lane) - 1ull));
                StagedG &d = sh.g[slot];
                d.cn = cn;
                d.cd = cd;
                d.xy = xy;
                d.pos = (uint32_t)(lo + lane);
                d.qm = qm;
                sh.e[slot] = e;
            }
            __syncthreads();
            // folded visits since the last flush: their staged indices, six bits each
            uint64_t pend = 0;
            int nfold = 0;
            auto flush = [&](int nf) {
                __syncthreads();  // the folded rows are in LDS
                if (ff < nf) {
                    const float4 *p = reinterpret_cast<const float4 *>(&sh.part[0][0][0] + part_off);
                    const float4 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
                    float r = ((p0.x + p0.y) + (p0.z + p0.w)) + ((p1.x + p1.y) + (p1.z + p1.w)) +
                              (((p2.x + p2.y) + (p2.z + p2.w)) + ((p3.x + p3.y) + (p3.z + p3.w)));
                    if (POSE && src < 0) r = 0.0f;
                    const uint32_t js = (uint32_t)(pend >> (6 * ff)) & 63u;
                    a.records[(int64_t)sh.e[js] * kRecord + fv] = r;
                }
                __syncthreads();  // sh.part may be written again
            };
            // lane j holds staged slot j's list position and its live quadrants:
            // those of its mask in which some pixel's last contributor lies at
            // or behind it (tested here for the 64 slots at once, not per
            // visit), so a visit takes them with lane reads
            uint32_t slot_pos = 0, slot_live = 0;
            bool slot_clamp = false;
            if (lane < nlive) {
                slot_pos = sh.g[lane].pos;
                const uint32_t qm = sh.g[lane].qm;
                slot_clamp = (qm & kClampBit) != 0;
#pragma unroll
                for (int i = 0; i < NQ; ++i)
                    if (slot_pos < ncq[i]) slot_live |= qm & (1u << i);
            }
            // the staged Gaussians that some quadrant visits; the others get
            // zero records
            const uint64_t visited = ballot(slot_live != 0);
            // the visit loop, without the clamp when no staged Gaussian of the
            // batch can reach it
            const bool batch_clamp = ballot(slot_clamp && slot_live != 0) != 0ull;
            auto visits = [&](auto clamp_v) {
            constexpr bool CLAMP = decltype(clamp_v)::value;
            for (uint64_t left = visited; left; left &= left - 1ull) {
                const int j = __ffsll((long long)left) - 1;
                const StagedG &sj = sh.g[j];
                const float2 g = sj.xy;
                const float4 cn4 = sj.cn;
                const float4 cd4 = sj.cd;
                const uint32_t pos = __builtin_amdgcn_readlane(slot_pos, j);
                const uint32_t mj = __builtin_amdgcn_readlane(slot_live, j);
                // this lane's sums over its pixels of gp (= dL/dpower) and its
                // moments gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2, and of the
                // dL/dc weights.  dy is one value per quadrant row, so each row
                // keeps only sum gp (P) and sum gp dx (Q), and the dy moments
                // are formed once per visit from them; sum gp dx^2 is kept whole.
                // The sums start at -0: x + (-0) is x for every x, so the
                // compiler drops the additions at a row's first quadrant (with +0
                // it must keep them, for the sign of a zero), and a dead row adds
                // nothing to the per-visit combination.
                constexpr int QY = G::QY;
                float P[QY], Q[QY], dyr[QY];
#pragma unroll
                for (int r = 0; r < QY; ++r) {
                    P[r] = -0.f;
                    Q[r] = -0.f;
                    dyr[r] = g.y - t.fpy[r];
                }
                float sgxx = -0.f;
                float sr = -0.f, sg = -0.f, sb = -0.f, sd = -0.f;
                // One quadrant's evaluation (dx and the column terms from its
                // column).  Without CLAMP (no Gaussian of the batch can reach the
                // 0.99 clamp in this bin: may_clamp) the clamp and its gradient
                // test are skipped, bit for bit the same.
                auto eval = [&](auto qi, float dx, float dx2, float adx2, float bdx) {
                    constexpr int i = decltype(qi)::value;
                    constexpr int r = i / QX;
                    const float dy = dyr[r];
                    const AlphaEval ev = CLAMP ? alpha_at(adx2, bdx, cn4.z, dy) : alpha_at_unclamped(adx2, bdx, cn4.z, dy);
                    const bool ok = (pos < nc[i]) && (ev.alpha >= kAlphaMin);
                    // an entry that does not blend at this pixel has al = 0, and the
                    // hardware reciprocal of exactly 1 is exactly 1: T stays as it is
                    const float al = ok ? ev.alpha : 0.0f;
                    const float Ti = Tc[i] * __builtin_amdgcn_rcpf(1.0f - al);
                    // c.g - S.g
                    const float dd = __builtin_fmaf(cd4.w, gd[i], __builtin_fmaf(cd4.z, g2[i],
                                                    __builtin_fmaf(cd4.y, g1[i], __builtin_fmaf(cd4.x, g0[i], nSg[i]))));
                    const float wk = al * Ti;  // alpha T: the colour weight, and dL/dpower / (c.g - S.g)
                    const float gp = (!CLAMP || ev.aun <= kAlphaMax) ? wk * dd : 0.0f;
                    if constexpr (!POSE) {
                        sr = __builtin_fmaf(wk, g0[i], sr);
                        sg = __builtin_fmaf(wk, g1[i], sg);
                        sb = __builtin_fmaf(wk, g2[i], sb);
                    }
                    sd = __builtin_fmaf(wk, gd[i], sd);
                    P[r] += gp;
                    Q[r] = __builtin_fmaf(gp, dx, Q[r]);
                    sgxx = __builtin_fmaf(gp, dx2, sgxx);
                    nSg[i] = __builtin_fmaf(-al, dd, nSg[i]);
                    Tc[i] = Ti;
                };
                // column by column, a column's dx terms only where one of its
                // quadrants is live
                static_for<QX>([&](auto hc) {
                    constexpr int h = decltype(hc)::value;
                    uint32_t colm = 0;
#pragma unroll
                    for (int r = 0; r < QY; ++r) colm |= 1u << (h + QX * r);
                    if (!(mj & colm)) return;
                    const float dx = g.x - t.fpx[h];
                    const float dx2 = dx * dx;
                    float adx2, bdx;
                    shared_dx(cn4.x, cn4.y, cn4.w, dx, adx2, bdx);
                    static_for<QY>([&](auto rc) {
                        constexpr int i = h + QX * decltype(rc)::value;
                        if (mj & (1u << i)) eval(std::integral_constant<int, i>{}, dx, dx2, adx2, bdx);
                    });
                });
                // the visit's moments from the row sums: sum gp, sum gp dx, and
                // per row dy P (sum gp dy), dy (dy P) (sum gp dy^2) and dy Q (sum
                // gp dx dy).  Without branches: a dead row's sums are -0 and add
                // nothing, so the result is the live rows' alone.
                float sgp = P[0], sgx = Q[0], sgy = dyr[0] * P[0];
                float sgyy = sgy * dyr[0], sgxy = dyr[0] * Q[0];
#pragma unroll
                for (int r = 1; r < QY; ++r) {
                    const float tr = dyr[r] * P[r];
                    sgp += P[r];
                    sgx += Q[r];
                    sgy += tr;
                    sgyy = __builtin_fmaf(tr, dyr[r], sgyy);
                    sgxy = __builtin_fmaf(dyr[r], Q[r], sgxy);
                }
                // (a visit where no pixel blends folds zeros: rarer than the
                // test that would skip it would cost)
                if constexpr (POSE) {
                    const float vals[6] = {sgx, sgy, sgxx, sgxy, sgyy, sd};
                    float z[2];
                    wave_fold_pose(vals, z);
                    sh.part[nfold][0][lane] = z[0];
                    sh.part[nfold][1][lane] = z[1];
                } else {
                    const float vals[kRecord] = {sgp, sgx, sgy, sgxx, sgxy, sgyy, sr, sg, sb, sd};
                    float z[3];
                    wave_fold_record(vals, z);
                    sh.part[nfold][0][lane] = z[0];
                    sh.part[nfold][1][lane] = z[1];
                    sh.part[nfold][2][lane] = z[2];
                }
                pend |= (uint64_t)j << (6 * nfold);
                if (++nfold == kFold) {
                    flush(kFold);
                    nfold = 0;
                    pend = 0;
                }
            }
            };
            if (batch_clamp) visits(std::true_type{});
            else visits(std::false_type{});
            if (nfold) flush(nfold);
            // staged Gaussians that no pixel of the bin reached: zero records
            if (lane < nlive && !((visited >> lane) & 1ull)) zero_record(a.records, sh.e[lane]);
            __syncthreads();
            hi = lo;
        }
    }
}

// ---------------------------------------------------------------- split backward
// For calls with few bins: one workgroup of four waves per 16x16 bin, wave w
// taking quadrant w (one pixel per lane), so four times the waves walk the
// lists.  Wave 0 stages each batch for all four (the masks of all four
// quadrants); each wave then visits the staged Gaussians live in its quadrant
// and folds and flushes its sums as the one-wave kernel does, into a per-wave
// slot of the staged Gaussian's record in LDS; after a block barrier the 256
// threads add the four waves' values in wave order and write the records.
// Deterministic; the sums are grouped differently from the one-wave kernel's.
struct StagedBwdSplit {
    StagedG g[64];
    uint32_t e[64];
    float part[4][kFold][3][64];  // each wave's folded visits awaiting its flush
    float rec[64][4][kRecord];    // each wave's record values per staged Gaussian
    uint64_t folded[4];           // staged Gaussians each wave wrote
    int64_t item;                 // the bin (block broadcast)
    uint32_t ncq[4];              // each quadrant's largest last-contributor position
    int nlive;
};

// one thread's grab for a block: the slot of queue q's next bin, -1 when all
// eight queues are empty
__device__ __forceinline__ int64_t next_item_thread(uint32_t *queues, int64_t n_items, int &q, int &tries) {
    while (tries < 8) {
        const uint32_t i = atomicAdd(queues + q * kQueueStride, 1u);
        if (q + 8 * (int64_t)i < n_items) return q + 8 * (int64_t)i;
        q = (q + 1) & 7;
        ++tries;
    }
    return -1;
}

// LDS written by lanes of this wave, then read by other lanes of it
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool POSE>
__global__ __launch_bounds__(256) void k_blend_bwd_split(BlendBwdArgs a) {
    using G = BinGeo<1, 1, true>;
    constexpr int QX = 2;  // quadrant columns of the bin (staging)
    __shared__ StagedBwdSplit sh;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ff = lane / kRecord, fv = lane - ff * kRecord;
    const bool flush_lane = ff < kFold;
    const int src = flush_lane ? fold_src<POSE>(ff, fv) : -1;
    const int part_off = src >= 0 ? src : 0;
    int q = blockIdx.x & 7, tries = 0;  // thread 0's queue state
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t slot = next_item_thread(a.queues, a.n_items, q, tries);
            sh.item = slot < 0 ? -1 : (int64_t)a.order[slot];
        }
        __syncthreads();
        const int64_t item = sh.item;
        if (item < 0) break;
        const int v = (int)uniform_u32((uint32_t)view_of_bin(a.views, a.n_views, item));
        const ViewDev &V = a.views[v];
        const int local = (int)(item - V.bin_base);
        const G t = bin_geo<1, 1, true>(local, V, lane, w);
        const int64_t plane = (int64_t)V.W * V.H;
        float Tc, nSg, g0, g1, g2, gd;
        uint32_t nc;
        {
            const int px = t.px[0], py = t.py[0];
            if (px < V.W && py < V.H) {
                const int64_t pix = V.pix_base + (int64_t)py * V.W + px;
                const int64_t pl = (int64_t)py * V.W + px;
                const float *gr = a.dL_rgb + 3 * V.pix_base;
                Tc = a.out_T[pix];
                nc = a.n_contrib[pix];
                g0 = gr[pl];
                g1 = gr[plane + pl];
                g2 = gr[2 * plane + pl];
                gd = a.dL_depth ? a.dL_depth[pix] : 0.0f;
            } else {
                Tc = 1.0f; nc = 0; g0 = g1 = g2 = gd = 0.0f;
            }
            nSg = -(a.bg0 * g0 + a.bg1 * g1 + a.bg2 * g2 + a.bgd * gd);
        }
        const uint32_t ncq = uniform_u32(wave_max_u32(nc));
        if (lane == 0) sh.ncq[w] = ncq;
        __syncthreads();
        const uint32_t ncmax = max(max(sh.ncq[0], sh.ncq[1]), max(sh.ncq[2], sh.ncq[3]));
        const uint2 rg = a.range[item];
        // Gaussians past every pixel's last contributor get zero records.
        for (uint32_t s = rg.x + ncmax + threadIdx.x; s < rg.y; s += 256)
            zero_record(a.records, a.inst.slot(s, a.inst.key[s]));
        int hi = (int)ncmax;
        while (hi > 0) {
            const int lo = hi > 64 ? hi - 64 : 0;
            const int nb = hi - lo;
            if (w == 0) {
                // staging, by wave 0 for the bin's four quadrants, back to front
                const BinGeo<1, 1> tb = bin_geo<1, 1>(local, V, lane);
                uint32_t qm = 0, e = 0;
                float2 xy;
                float4 cn, cd;
                if (lane < nb) {
                    const uint32_t s = rg.x + lo + lane;
                    const uint64_t key = a.inst.key[s];
                    const uint32_t k = a.inst.rank(key);
                    xy = a.rxy[k];
                    cn = a.rconic[k];
                    e = a.inst.slot(s, key);
                    qm = a.box_cull ? quad_mask(tb, xy.x, xy.y, cn, a.rrect[k]) : quad_mask_rows(tb, xy.x, xy.y, cn, a.rrect[k]);
                    if (qm) {
                        cd = a.rrgbd[k];
                        if (may_clamp(xy.x, xy.y, cn, tb.qx0[0], tb.qx1[QX - 1], tb.qy0[0], tb.qy1[QX - 1])) qm |= kClampBit;
                    } else {
                        zero_record(a.records, e);
                    }
                }
                const uint64_t m = ballot(qm != 0);
                const int nlive = __popcll(m);
                if (qm) {
                    const int slot = nlive - 1 - __popcll(m & ((1ull << lane) - 1ull));
                    StagedG &d = sh.g[slot];
                    d.cn = cn;
                    d.cd = cd;
                    d.xy = xy;
                    d.pos = (uint32_t)(lo + lane);
                    d.qm = qm;
                    sh.e[slot] = e;
                }
                if (lane == 0) sh.nlive = nlive;
            }
            __syncthreads();
            const int nlive = sh.nlive;
            uint64_t pend = 0;
            int nfold = 0;
            auto flush = [&](int nf) {
                wave_lds_sync();  // this wave's folded rows are in LDS
                if (ff < nf) {
                    const float4 *p = reinterpret_cast<const float4 *>(&sh.part[w][0][0][0] + part_off);
                    const float4 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
                    float r = ((p0.x + p0.y) + (p0.z + p0.w)) + ((p1.x + p1.y) + (p1.z + p1.w)) +
                              (((p2.x + p2.y) + (p2.z + p2.w)) + ((p3.x + p3.y) + (p3.z + p3.w)));
                    if (POSE && src < 0) r = 0.0f;
                    const uint32_t js = (uint32_t)(pend >> (6 * ff)) & 63u;
                    sh.rec[js][w][fv] = r;
                }
                wave_lds_sync();  // sh.part[w] may be written again
            };
            // the staged Gaussians this wave visits: live in its quadrant and
            // at or behind some pixel's last contributor (per batch, not per visit)
            uint32_t slot_pos = 0;
            bool mine = false, slot_clamp = false;
            if (lane < nlive) {
                slot_pos = sh.g[lane].pos;
                const uint32_t qm = sh.g[lane].qm;
                mine = ((qm >> w) & 1u) && slot_pos < ncq;
                slot_clamp = (qm & kClampBit) != 0;
            }
            const uint64_t visited = ballot(mine);
            const bool batch_clamp = ballot(mine && slot_clamp) != 0ull;
            auto visits = [&](auto clamp_v) {
            constexpr bool CLAMP = decltype(clamp_v)::value;
            for (uint64_t left = visited; left; left &= left - 1ull) {
                const int j = __ffsll((long long)left) - 1;
                const StagedG &sj = sh.g[j];
                const float2 g = sj.xy;
                const float4 cn4 = sj.cn;
                const float4 cd4 = sj.cd;
                const uint32_t pos = __builtin_amdgcn_readlane(slot_pos, j);
                const float dx = g.x - t.fpx[0];
                float adx2, bdx;
                shared_dx(cn4.x, cn4.y, cn4.w, dx, adx2, bdx);
                const float dy = g.y - t.fpy[0];
                const AlphaEval ev = CLAMP ? alpha_at(adx2, bdx, cn4.z, dy) : alpha_at_unclamped(adx2, bdx, cn4.z, dy);
                const bool ok = (pos < nc) && (ev.alpha >= kAlphaMin);
                const float al = ok ? ev.alpha : 0.0f;
                const float Ti = Tc * __builtin_amdgcn_rcpf(1.0f - al);
                const float dd = __builtin_fmaf(cd4.w, gd, __builtin_fmaf(cd4.z, g2,
                                                __builtin_fmaf(cd4.y, g1, __builtin_fmaf(cd4.x, g0, nSg))));
                const float wk = al * Ti;
                const float gp = (!CLAMP || ev.aun <= kAlphaMax) ? wk * dd : 0.0f;
                const float gx = gp * dx, gy = gp * dy;
                nSg = __builtin_fmaf(-al, dd, nSg);
                Tc = Ti;
                if constexpr (POSE) {
                    const float vals[6] = {gx, gy, gx * dx, gx * dy, gy * dy, wk * gd};
                    float z[2];
                    wave_fold_pose(vals, z);
                    sh.part[w][nfold][0][lane] = z[0];
                    sh.part[w][nfold][1][lane] = z[1];
                } else {
                    const float vals[kRecord] = {gp, gx, gy, gx * dx, gx * dy, gy * dy, wk * g0, wk * g1, wk * g2, wk * gd};
                    float z[3];
                    wave_fold_record(vals, z);
                    sh.part[w][nfold][0][lane] = z[0];
                    sh.part[w][nfold][1][lane] = z[1];
                    sh.part[w][nfold][2][lane] = z[2];
                }
                pend |= (uint64_t)j << (6 * nfold);
                if (++nfold == kFold) {
                    flush(kFold);
                    nfold = 0;
                    pend = 0;
                }
            }
            };
            if (batch_clamp) visits(std::true_type{});
            else visits(std::false_type{});
            if (nfold) flush(nfold);
            if (lane == 0) sh.folded[w] = visited;
            __syncthreads();
            // records: the four waves' values in wave order; zeros for a staged
            // Gaussian that no pixel of the bin reached
            for (int o = threadIdx.x; o < nlive * kRecord; o += 256) {
                const int j = o / kRecord, vv = o - j * kRecord;
                float r = 0.0f;
#pragma unroll
                for (int ww = 0; ww < 4; ++ww)
                    if ((sh.folded[ww] >> j) & 1ull) r += sh.rec[j][ww][vv];
                a.records[(int64_t)sh.e[j] * kRecord + vv] = r;
            }
            __syncthreads();
            hi = lo;
        }
    }
}

}  // namespace mgs
