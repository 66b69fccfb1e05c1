// Tile-based differentiable rasteriser for gfx950 (MemGS Sec. II-C, II-E).
//
// Forward (one call renders any number of views of any number of maps):
//   k_setup        per-call tables from the kernel arguments; zero the counters
//   k_project      per (Gaussian, view) pair: screen test, key path, conic, SH
//                  colour, tile count; per-block totals (visible pairs,
//                  instances, depth-key range)
//   k_sum_blocks   the totals, written to a pinned host mailbox: the host waits
//                  for this one read-back (the layout of the rest depends on it)
//   compaction     scan of visibility; (depth key, pair) of visible pairs
//   pair sort      stable radix sort on (view, depth key - its minimum)
//                  => depth rank of each visible pair (ties by index); the
//                  last pass writes each rank's tile count
//   rank scan      scan of tile counts in rank order => instance offsets
//   k_emit         per rank: one instance key (bin id, rank and record slot,
//                  packed into 64 bits) per covered list bin, a wave writing
//                  its ranks' keys together (64 ranks, 16 in calls with few;
//                  coalesced); gathers the blend inputs into rank order
//   tile sort      stable keys-only radix sort on the bin id (2 passes), so
//                  each bin's list is in rank = depth order
//   k_tile_ranges  [first, last) of every bin; k_bin_count / k_bin_place
//                  order the bins longest list first
//   k_blend_fwd    persistent, one wave per list bin: a 16x16 tile (4 pixels
//                  per lane), or 2x1 tiles (8 per lane) in calls with many
//                  tiles, or an 8x8 quadrant of a tile (1 per lane) in calls
//                  with few; for a backward call over bins of several tiles
//                  it keeps each list entry's quadrant mask
// Backward:
//   k_blend_bwd    persistent; back to front from each pixel's last
//                  contributor, transmittance recovered by division; per
//                  Gaussian the wave's contributions are summed across lanes
//                  and written once as a 10-float record per (bin, Gaussian)
//   k_rank_reduce  per rank: the sum of its records (contiguous)
//   k_pair_bwd     per visible pair: chain rule to the Gaussian's parameters,
//                  block partial sums of the pose gradient
//   k_gauss_bwd    per Gaussian: its pairs summed over views in view order
//   k_pose_final   fp64 reduction of the pose partials
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "blend.hpp"
#include "api_range.hpp"
#include "common.hpp"
#include "project.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace mgs {

// ---------------------------------------------------------------- counters
// counters[0] Pv (u32), counters[2..3] M (u64); the eight work-queue heads
// from word CNT_Q on, 256 bytes apart so that no two share a cache line
// counters[CNT_CLAMP] != 0: some visible pair may reach the 0.99 alpha clamp
// within its tile rectangle (may_clamp), set by the projection
enum { CNT_PV = 0, CNT_M = 2, CNT_KMIN = 4, CNT_KMAX = 5, CNT_CLAMP = 6, CNT_Q = 64, CNT_WORDS = CNT_Q + 8 * kQueueStride };

__global__ void k_init(uint32_t *counters) {
    for (int i = threadIdx.x; i < CNT_WORDS; i += blockDim.x) counters[i] = 0;
}

// The per-call tables (views, maps, views grouped by map) of a call with at
// most kArgViews views and kArgMaps maps travel in the kernel arguments of
// k_setup, which writes them to the workspace and zeroes the counters: no
// host-to-device copy from pageable memory (each costs a staging copy on the
// host and a copy kernel).  Larger calls copy the tables.
constexpr int kArgViews = 16, kArgMaps = 8;
struct SetupArgs {
    ViewDev views[kArgViews];
    MapDev maps[kArgMaps];
    int32_t vlist[kArgViews];
    int32_t n_views, n_maps;
};
static_assert(sizeof(SetupArgs) <= 4000, "kernel arguments hold at most 4 KB");
static_assert(sizeof(ViewDev) % 4 == 0 && sizeof(MapDev) % 4 == 0, "tables are copied as words");

__device__ __forceinline__ void copy_words(const void *src, void *dst, int words) {
    const uint32_t *s = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    for (int i = threadIdx.x; i < words; i += blockDim.x) d[i] = s[i];
}

__global__ void k_setup(SetupArgs a, ViewDev *views, MapDev *maps, int32_t *vlist, uint32_t *counters) {
    for (int i = threadIdx.x; i < CNT_WORDS; i += blockDim.x) counters[i] = 0;
    copy_words(a.views, views, a.n_views * (int)(sizeof(ViewDev) / 4));
    copy_words(a.maps, maps, a.n_maps * (int)(sizeof(MapDev) / 4));
    copy_words(a.vlist, vlist, a.n_views);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ int view_of_pair(const ViewDev *views, int V, int64_t p) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pair_base <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- emission spans
// A Gaussian reaches alpha >= 1/255 only where d^T Sigma^-1 d <= s with
// s = 2 ln(255 o) (d = mean - pixel centre, Sigma the dilated image
// covariance), here with the tile-test margin added.  Over one tile row, i.e.
// the band dy in [v - py1, v - py0], that ellipse spans an x interval: its
// extreme points (+-rx at dy = +-yx) when they lie in the band, else the
// conditional extent kx dy +- wx sqrt(s - dy^2 / syy) at the nearest band
// edge.  Tiles of the row that miss the padded interval cannot blend the
// Gaussian at any pixel and are not emitted; the rest of the 3-sigma rectangle
// is.  The projection (to count) and the emission (to write) evaluate the same
// functions on the same stored values, so the counts and the writes agree.
// The hardware square root and reciprocal (about 1 ulp) are far inside the
// one-pixel pad.  Rectangles of more than kSpanSoloRows rows are spread over
// the wave, one row per lane.
constexpr int kSpanSoloRows = 8;

__device__ __forceinline__ float nsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float nrcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct SpanGeo {
    float u, v, s, iyy, kx, wx, rx, ry, yx, pad;
};

__device__ __forceinline__ float span_s(float o) {
    return 1.3862943611198906f * (__builtin_amdgcn_logf(o) - kLog2AlphaMin + kTileTestMargin);  // 2 ln 2 (...)
}

__device__ __forceinline__ SpanGeo span_geo(float u, float v, float sxx, float sxy, float syy, float s) {
    SpanGeo g;
    const float sp = fmaxf(s, 0.0f);
    g.u = u;
    g.v = v;
    g.s = s;
    g.iyy = nrcp(syy);
    g.kx = sxy * g.iyy;
    g.wx = nsqrt(fmaxf(0.0f, sxx - sxy * g.kx));  // sqrt(det / syy)
    g.rx = nsqrt(sp * sxx);
    g.yx = sxy * nsqrt(sp * nrcp(sxx));
    // one pixel plus the relative rounding of the extents and coordinates
    g.pad = 1.0f + 1e-3f * g.rx + 1e-5f * fabsf(u);
    const float ry = nsqrt(sp * syy);
    g.ry = ry + 1.0f + 1e-3f * ry + 1e-5f * fabsf(v);
    return g;
}

// Pixel rows of bin row by of a rectangle (tile rows [y0, y1)), clipped to the
// rectangle and the image; false when empty.
__device__ __forceinline__ bool bin_band(int by, int bty, int y0, int y1, int H, float &py0, float &py1) {
    const int lo = max(by * bty * kTile, y0 * kTile);
    const int hi = min(min((by + 1) * bty * kTile, y1 * kTile), H) - 1;
    py0 = (float)lo;
    py1 = (float)hi;
    return lo <= hi;
}

// bin columns [c0, c1) of one bin row (pixel rows [py0, py1]) that the padded
// ellipse reaches within the rectangle's tile columns [x0, x1); bins of btx tiles
__device__ __forceinline__ void span_bins(const SpanGeo &g, float py0, float py1, int x0, int x1, int btx, int &c0,
                                          int &c1) {
    c0 = c1 = x0 / btx;
    const float dlo = g.v - py1, dhi = g.v - py0;
    if (!(g.s > 0.0f) || dhi < -g.ry || dlo > g.ry) return;
    const float ya = sclamp(g.yx, dlo, dhi), yb = sclamp(-g.yx, dlo, dhi);
    const float dmax = ya == g.yx ? g.rx : g.kx * ya + g.wx * nsqrt(fmaxf(0.0f, g.s - ya * ya * g.iyy));
    const float dmin = yb == -g.yx ? -g.rx : g.kx * yb - g.wx * nsqrt(fmaxf(0.0f, g.s - yb * yb * g.iyy));
    // pixel columns reached, within the rectangle's
    const float xlo = fmaxf(g.u - dmax - g.pad, (float)(kTile * x0));
    const float xhi = fminf(g.u - dmin + g.pad, (float)(kTile * x1 - 1));
    if (!(xlo <= xhi)) return;
    // bin c holds pixel columns bw c .. bw c + bw - 1
    const float ibw = 1.0f / (float)(kTile * btx);  // a power of two: exact
    const int a = (int)ceilf((xlo - (float)(kTile * btx - 1)) * ibw);
    const int b = (int)floorf(xhi * ibw) + 1;
    c0 = max(a, x0 / btx);
    c1 = max(c0, min(b, (x1 + btx - 1) / btx));
}

__device__ __forceinline__ SpanGeo span_bcast(const SpanGeo &g, int src) {
    SpanGeo b;
    b.u = readlane_f(g.u, src);
    b.v = readlane_f(g.v, src);
    b.s = readlane_f(g.s, src);
    b.iyy = readlane_f(g.iyy, src);
    b.kx = readlane_f(g.kx, src);
    b.wx = readlane_f(g.wx, src);
    b.rx = readlane_f(g.rx, src);
    b.ry = readlane_f(g.ry, src);
    b.yx = readlane_f(g.yx, src);
    b.pad = readlane_f(g.pad, src);
    return b;
}

// instances of a rectangle: the bins its spans reach, over its bin rows
__device__ __forceinline__ uint32_t span_count(const SpanGeo &g, const ViewDev &V, int x0, int y0, int x1, int y1) {
    uint32_t n = 0;
    for (int by = y0 / V.BTY; by * V.BTY < y1; ++by) {
        float py0, py1;
        if (!bin_band(by, V.BTY, y0, y1, V.H, py0, py1)) continue;
        int c0, c1;
        span_bins(g, py0, py1, x0, x1, V.BTX, c0, c1);
        n += (uint32_t)(c1 - c0);
    }
    return n;
}

// ---------------------------------------------------------------- projection
// Per (Gaussian, view) pair, one 64-byte record with everything the emission
// reads: the depth-sorted emission gathers pairs in random order, and one
// record is one memory segment.
struct alignas(16) PairRec {
    float4 geo;    // image mean u, v; covariance xx, xy
    float4 span;   // covariance yy, span radius s, rectangle (x0 | y0 << 16), (x1 | y1 << 16)
    float4 conic;  // scaled conic a', b', c' and log2 of the opacity (the blend's form)
    float4 rgbd;   // colour, camera z
};

// Gaussians of one map that one projection block screens (for one view):
// 256 x ROUNDS.  Four rounds (1024) amortise
// the block's setup and keep four independent chains per thread; calls with
// few such blocks take one round (256) instead, four times the blocks.
constexpr int kProjRoundsLarge = 4, kProjRoundsSmall = 1;
constexpr int64_t kProjSmallBlocks = 1024;  // fewer 1024-Gaussian blocks than this: 256-Gaussian chunks

struct ProjectArgs {
    const ViewDev *views;
    const MapDev *maps;
    int n_views;
    int64_t P;
    uint32_t *pair_depth;   // [P]
    uint32_t *pair_count;   // [P]
    ushort4 *pair_rect;     // [P]
    float4 *pair_uvr;       // [P] u, v, r, z
    PairRec *pair_rec;      // [P] what the emission reads (written for unculled pairs)
    uint32_t *blk_vis;      // [n_views][cols] visible pairs of each block
    uint64_t *blk_cnt;      // [n_views][cols] tile instances of each block
    uint32_t *blk_kmin;     // [n_views][cols] smallest and largest depth key of a
    uint32_t *blk_kmax;     //   visible pair of each block (~0 and 0 for none)
    int64_t cols;           // chunks of 256 x ROUNDS Gaussians of the largest map
    uint32_t *clamp_flag;   // counters[CNT_CLAMP]
};

// Conservative screen test of one (Gaussian, view) pair: false only for a
// pair that the key path culls.  The camera-frame mean is formed with the key
// path's own operations, so the near-plane test is the same test.  For the
// rest the key path's radius is bounded from above: its lam is at most
// a + c + 0.32 (the eigenvalue, or (a + c) / 2 + sqrt(0.1) when the
// discriminant is clamped), and a + c, the trace of J W Sigma_W W^T J^T plus
// the two dilations, is at most ((fx/z)^2 (1 + limx^2) + (fy/z)^2 (1 + limy^2))
// smax^2 + 0.6 (W has orthonormal rows, Sigma_W's largest eigenvalue is smax^2,
// and the clamped x/z and y/z stay within limx and limy).  The key path's tile
// rectangle is empty unless u + r >= 0 and u - r < 16 TX (and likewise for v);
// the bound, 1 % and two pixels of slack, and a slack for u and v computed with
// a reciprocal keep every visible pair.  Non-finite inputs fall through to the
// key path, which culls them.
__device__ __forceinline__ bool may_be_visible(const float *m, float smax, const ViewDev &V) {
#pragma clang fp contract(off)
    const float *Rc = V.R;
    float p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = ((Rc[3 * a] * m[0] + Rc[3 * a + 1] * m[1]) + Rc[3 * a + 2] * m[2]) + V.t[a];
    const float pz = p[2];
    if (!(pz > V.near_z)) return false;
    const float iz = __builtin_amdgcn_rcpf(pz);
    const float kx = V.fx * iz, ky = V.fy * iz;
    const float tr = (kx * kx * (1.0f + V.limx * V.limx) + ky * ky * (1.0f + V.limy * V.limy)) * (smax * smax) + 0.92f;
    const float rb = 3.03f * __builtin_sqrtf(tr) + 2.0f;
    const float u = V.fx * (p[0] * iz) + V.cx, v = V.fy * (p[1] * iz) + V.cy;
    const float slack = rb + 1e-4f * (fabsf(u) + fabsf(v)) + 2.0f;
    if (!(u + slack >= 0.0f) || !(u - slack < 16.0f * (float)V.TX)) return !(tr == tr && u == u);
    if (!(v + slack >= 0.0f) || !(v - slack < 16.0f * (float)V.TY)) return !(tr == tr && v == v);
    return true;
}

// One block per (chunk of 256 x ROUNDS Gaussians of the view's map, view); view
// and map parameters are uniform per block and come through scalar loads.
// Workgroups are dealt to the eight XCDs round robin (block i on XCD i % 8): the
// blocks of one chunk for all views sit 8 apart, so they run on one XCD close
// in time and the chunk's Gaussians are read from HBM once and then from that
// XCD's L2.  A block first runs the screen test over its chunk (most pairs of a
// view fall outside it) and writes the culled pairs' outputs, then runs the key
// path only over the pairs that passed, packed densely over its threads, so
// waves do not carry culled lanes through the long path.  Each block writes
// its totals to its own slot; k_sum_blocks adds them up (no atomics on one
// shared address from thousands of blocks).
template <int ROUNDS>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a) {
    constexpr int kChunk = 256 * ROUNDS;
    const int64_t rest = blockIdx.x >> 3;  // (chunk / 8) * n_views + view
    const int v = (int)(rest % a.n_views);
    const int64_t chunk = (rest / a.n_views) * 8 + (blockIdx.x & 7);
    if (chunk >= a.cols) return;  // the whole block: past the last chunk
    const int64_t b = (int64_t)v * a.cols + chunk;
    const ViewDev &V = a.views[v];
    const MapDev &Mp = a.maps[V.map];
    const int64_t g0 = chunk * kChunk;
    __shared__ uint16_t cand[kChunk];
    __shared__ uint32_t ncand;
    if (threadIdx.x == 0) ncand = 0;
    __syncthreads();
    // every load of the screen test first, then the tests
    constexpr int kRounds = ROUNDS;
    float mm[kRounds][3], smax[kRounds];
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        const int64_t g = g0 + j * 256 + (int)threadIdx.x;
        if (g < Mp.n) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mm[j][c] = Mp.means[3 * g + c];
            smax[j] = fmaxf(fmaxf(Mp.scales[3 * g], Mp.scales[3 * g + 1]), Mp.scales[3 * g + 2]);
        }
    }
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        const int k = j * 256 + (int)threadIdx.x;
        const int64_t g = g0 + k;
        const bool in = g < Mp.n;
        const bool c = in && may_be_visible(mm[j], smax[j], V);
        if (in && !c) {
            a.pair_depth[V.pair_base + g] = 0xFFFFFFFFu;  // rect and uvr are left unwritten for a culled pair
            a.pair_count[V.pair_base + g] = 0u;
        }
        const uint64_t mc = ballot(c);
        uint32_t base = 0;
        if (lane_id() == 0 && mc) base = atomicAdd(&ncand, (uint32_t)__popcll(mc));
        base = (uint32_t)__shfl((int)base, 0, 64);
        if (c) cand[base + (uint32_t)__popcll(mc & ((1ull << lane_id()) - 1ull))] = (uint16_t)k;
    }
    __syncthreads();
    const uint32_t nc = ncand;
    uint32_t vis = 0, kmn = 0xFFFFFFFFu, kmx = 0u;
    uint64_t tot = 0;
    for (uint32_t k0 = 0; k0 < nc; k0 += 256) {
        const uint32_t kk = k0 + threadIdx.x;
        const bool act = kk < nc;
        const int64_t g = act ? g0 + cand[kk] : 0;
        const int64_t p = V.pair_base + g;
        uint32_t cnt = 0, key = 0u;
        bool coop = false;  // a tall rectangle: its spans are counted by the whole wave
        bool clamp = false;
        SpanGeo sg{};
        int rx0 = 0, ry0 = 0, rx1 = 0, ry1 = 0;
        if (act) {
            float m[3] = {Mp.means[3 * g], Mp.means[3 * g + 1], Mp.means[3 * g + 2]};
            float s[3] = {Mp.scales[3 * g], Mp.scales[3 * g + 1], Mp.scales[3 * g + 2]};
            const float4 q4 = *reinterpret_cast<const float4 *>(Mp.quats + 4 * g);
            float q[4] = {q4.x, q4.y, q4.z, q4.w};
            const float o = Mp.opac[g];
            Proj P;
            if (key_path(m, s, q, o, V, P)) {
                const float sr = span_s(o);
                sg = span_geo(P.u, P.v, P.a, P.b, P.c, sr);
                rx0 = P.x0; ry0 = P.y0; rx1 = P.x1; ry1 = P.y1;
                if (P.y1 - P.y0 <= kSpanSoloRows) cnt = span_count(sg, V, P.x0, P.y0, P.x1, P.y1);
                else coop = true;
                float A, B, C;
                conic_of(P, A, B, C);
                float rgb[3], raw[3];
                switch (Mp.sh_degree) {
                    case 0: sh_colour<0>(Mp, g, m, V, rgb, raw, nullptr, nullptr); break;
                    case 1: sh_colour<1>(Mp, g, m, V, rgb, raw, nullptr, nullptr); break;
                    case 2: sh_colour<2>(Mp, g, m, V, rgb, raw, nullptr, nullptr); break;
                    default: sh_colour<3>(Mp, g, m, V, rgb, raw, nullptr, nullptr); break;
                }
                key = f2u(P.p[2]);
                a.pair_depth[p] = key;
                a.pair_rect[p] = make_ushort4((unsigned short)P.x0, (unsigned short)P.y0, (unsigned short)P.x1,
                                              (unsigned short)P.y1);
                a.pair_uvr[p] = make_float4(P.u, P.v, P.r, P.p[2]);
                PairRec rec;
                rec.geo = make_float4(P.u, P.v, P.a, P.b);
                rec.span = make_float4(P.c, sr, __builtin_bit_cast(float, (uint32_t)P.x0 | ((uint32_t)P.y0 << 16)),
                                       __builtin_bit_cast(float, (uint32_t)P.x1 | ((uint32_t)P.y1 << 16)));
                rec.conic = make_float4(-0.5f * kLog2e * A, -kLog2e * B, -0.5f * kLog2e * C, __builtin_amdgcn_logf(o));
                rec.rgbd = make_float4(rgb[0], rgb[1], rgb[2], P.p[2]);
                a.pair_rec[p] = rec;
                // every pixel the blend evaluates for this pair lies in its tile rectangle
                clamp = may_clamp(P.u, P.v, rec.conic, (float)(kTile * P.x0), (float)(kTile * P.x1 - 1),
                                  (float)(kTile * P.y0), (float)(kTile * P.y1 - 1));
            } else {
                a.pair_depth[p] = 0xFFFFFFFFu;
            }
        }
        uint64_t tall = ballot(coop);
        while (tall) {
            const int src = __ffsll((long long)tall) - 1;
            tall &= tall - 1;
            const SpanGeo sb = span_bcast(sg, src);
            const int x0 = readlane_i(rx0, src), y0 = readlane_i(ry0, src);
            const int x1 = readlane_i(rx1, src), y1 = readlane_i(ry1, src);
            uint32_t c = 0;
            for (int by = y0 / V.BTY + lane_id(); by * V.BTY < y1; by += 64) {
                float py0, py1;
                if (!bin_band(by, V.BTY, y0, y1, V.H, py0, py1)) continue;
                int c0, c1;
                span_bins(sb, py0, py1, x0, x1, V.BTX, c0, c1);
                c += (uint32_t)(c1 - c0);
            }
            c = wave_sum_u32(c);
            if (lane_id() == src) cnt = c;
        }
        if (act) a.pair_count[p] = cnt;
        if (ballot(clamp && cnt > 0) != 0ull && lane_id() == 0) atomicOr(a.clamp_flag, 1u);
        vis += cnt > 0 ? 1u : 0u;
        tot += cnt;
        if (cnt > 0) {
            kmn = min(kmn, key);
            kmx = max(kmx, key);
        }
    }
    // block totals
    __shared__ uint32_t sv[4], smn[4], smx[4];
    __shared__ uint64_t sc[4];
    uint32_t wv = vis;
    uint64_t wc = tot;
    for (int off = 32; off > 0; off >>= 1) {
        wv += __shfl_xor(wv, off, 64);
        wc += __shfl_xor(wc, off, 64);
        kmn = min(kmn, (uint32_t)__shfl_xor((int)kmn, off, 64));
        kmx = max(kmx, (uint32_t)__shfl_xor((int)kmx, off, 64));
    }
    if (lane_id() == 0) {
        sv[threadIdx.x >> 6] = wv;
        sc[threadIdx.x >> 6] = wc;
        smn[threadIdx.x >> 6] = kmn;
        smx[threadIdx.x >> 6] = kmx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.blk_vis[b] = sv[0] + sv[1] + sv[2] + sv[3];
        a.blk_cnt[b] = sc[0] + sc[1] + sc[2] + sc[3];
        a.blk_kmin[b] = min(min(smn[0], smn[1]), min(smn[2], smn[3]));
        a.blk_kmax[b] = max(max(smx[0], smx[1]), max(smx[2], smx[3]));
    }
}

// One block of 1024 threads: Pv and M from the per-block totals.
__global__ __launch_bounds__(1024) void k_sum_blocks(const uint32_t *blk_vis, const uint64_t *blk_cnt,
                                                     const uint32_t *blk_kmin, const uint32_t *blk_kmax, int64_t n,
                                                     uint32_t *counters, uint32_t *mail, uint32_t ticket) {
    uint64_t tv = 0, tc = 0;
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        tv += blk_vis[i];
        tc += blk_cnt[i];
        mn = min(mn, blk_kmin[i]);
        mx = max(mx, blk_kmax[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        tv += __shfl_xor(tv, off, 64);
        tc += __shfl_xor(tc, off, 64);
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, 64));
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
    }
    __shared__ uint64_t sv[16], sc[16];
    __shared__ uint32_t smn[16], smx[16];
    if (lane_id() == 0) {
        sv[threadIdx.x >> 6] = tv;
        sc[threadIdx.x >> 6] = tc;
        smn[threadIdx.x >> 6] = mn;
        smx[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            sv[0] += sv[w];
            sc[0] += sc[w];
            smn[0] = min(smn[0], smn[w]);
            smx[0] = max(smx[0], smx[w]);
        }
        const uint32_t words[6] = {(uint32_t)sv[0], 0u, (uint32_t)sc[0], (uint32_t)(sc[0] >> 32), smn[0], smx[0]};
        counters[CNT_PV] = words[CNT_PV];
        counters[CNT_M] = words[CNT_M];
        counters[CNT_M + 1] = words[CNT_M + 1];
        counters[CNT_KMIN] = words[CNT_KMIN];
        counters[CNT_KMAX] = words[CNT_KMAX];
        if (mail) {  // the host's copy, same word order
            for (int k = 0; k < 6; ++k) mail[k] = words[k];
            mail_flag(mail, ticket);
        }
    }
}

// visibility -> compacted (depth key, pair index)
struct LoadVis {
    const uint32_t *count;
    __device__ uint32_t operator()(int64_t i) const { return count[i] > 0 ? 1u : 0u; }
};
struct StoreCompact {
    const uint32_t *count, *depth;
    uint32_t *keys, *vals;
    __device__ void operator()(int64_t i, uint32_t ex, uint32_t v) const {
        if (v) {
            keys[ex] = depth[i];
            vals[ex] = (uint32_t)i;
        }
    }
};

// Digit of the pair sort: byte `shift / 8` of (view << kbits) | (key - kmin),
// kmin the smallest depth key of a visible pair and kbits the bits of the
// keys' range.  Sorting that composite stably sorts by view, then depth key,
// then compaction order (pair index), in as few bytes as the keys span.
struct PairDigit {
    static constexpr bool kUsesValue = true, kLowWord = false;
    const ViewDev *views;
    int n_views;
    uint32_t kmin;
    int kbits;
    int shift;
    __device__ __forceinline__ uint32_t operator()(uint32_t key, uint32_t pair) const {
        uint64_t c = (uint64_t)(key - kmin);
        if (shift + 8 > kbits) c |= (uint64_t)view_of_pair(views, n_views, pair) << kbits;
        return (uint32_t)(c >> shift) & 0xFFu;
    }
};

// tile counts in rank order
struct LoadRankCount {
    const uint32_t *rank_pair, *pair_count;
    __device__ uint32_t operator()(int64_t k) const { return pair_count[rank_pair[k]]; }
};
// The pair sort's last scatter writes each rank's instance count (the scan
// that follows then reads it in rank order instead of gathering it).
struct SideRankCount {
    const uint32_t *pair_count;
    uint32_t *rank_count;
    __device__ __forceinline__ void operator()(int64_t o, uint32_t, uint32_t pair) const {
        rank_count[o] = pair_count[pair];
    }
};

struct EmitArgs {
    const ViewDev *views;
    int n_views;
    int64_t Pv;
    const uint32_t *rank_pair, *rank_off;  // rank_off: [Pv + 1]
    const PairRec *pair_rec;
    uint32_t *pair_rank;
    float2 *rank_xy;
    float4 *rank_conic, *rank_rgbd;
    ushort4 *rank_rect;
    // instance e of the emission order (the record slot of its (Gaussian, bin)
    // pair in the backward), for depth rank k in global bin b:
    //   packed (bin_bits > 0): b | k << bin_bits | e << (bin_bits + rank_bits)
    //   wide (bin_bits = 0):   b << 32 | k (e travels as the sort's value)
    uint64_t *inst_key;
    int bin_bits, rank_bits;
    uint32_t *zero;  // [n_zero] words cleared on the way (the bin ranges and the ordering counts)
    int64_t n_zero;
    int ranks_per_wave;  // 64, or 16 for calls with few ranks (more waves, shorter chains)
};

__device__ __forceinline__ uint64_t inst_key_of(const EmitArgs &a, int64_t bin, uint32_t k, uint32_t e) {
    return a.bin_bits ? (uint64_t)bin | ((uint64_t)k << a.bin_bits) | ((uint64_t)e << (a.bin_bits + a.rank_bits))
                      : ((uint64_t)bin << 32) | k;
}
constexpr uint64_t kNoTile = ~0ull;  // key of an unused slot: its bin sorts last, owned by no bin

// digit of the packed keys' bin field: `width` (1..8) bits from `shift`, so
// that the rank and slot bits above the bin never take part in the order
struct BinDigit {
    static constexpr bool kUsesValue = false, kLowWord = true;  // the bin field lies in the low 32 bits
    int shift, width;
    __device__ __forceinline__ uint32_t operator()(uint64_t key, uint32_t) const {
        return (uint32_t)(key >> shift) & ((1u << width) - 1u);
    }
};

// A wave takes 64 depth ranks and writes the (bin, rank) instances of their
// spans at rank_off[k] onwards, bin row by bin row (instance e of the emission
// order is the record slot of that (Gaussian, bin) pair in the backward).  The
// wave works on the ranks together, so that its stores are coalesced and no
// lane waits on a larger Gaussian: first its (rank, bin row) items, 64 at a
// time, each lane finding its item's rank by binary lifting over the ranks'
// inclusive row counts and forming that row's span of bins; then the items'
// instances, 64 at a time, each lane finding its item the same way over the
// items' inclusive instance counts.  Consecutive lanes then write consecutive
// slots.  A rank's rows may run over several item chunks: the wave carries the
// count already written for the rank that continues into the next chunk.
__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    // ranks dealt to waves in groups of 8 consecutive ones, the groups of a
    // wave (8, or 2 with 16 ranks a wave) spread over the whole depth order:
    // large Gaussians, which cluster at the near end, land in many waves
    // instead of a few
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int lane = lane_id();
    const int64_t k = (((int64_t)(lane >> 3)) * nw + (t >> 6)) * 8 + (lane & 7);
    const bool in = lane < a.ranks_per_wave && k < a.Pv;
    for (int64_t i = t; i < a.n_zero; i += nw * 64) a.zero[i] = 0u;
    // bins per list bin along x and y: the same for every view of a call
    const int BTX = a.views[0].BTX, BTY = a.views[0].BTY;
    uint32_t o = 0, cnt = 0, rlo = 0, rhi = 0;
    int nrows = 0, by0 = 0, H = 0, BX = 0, bbase = 0;
    SpanGeo g{};
    if (in) {
        const uint32_t p = a.rank_pair[k];
        const int v = view_of_pair(a.views, a.n_views, p);
        const ViewDev &V = a.views[v];
        const PairRec rec = a.pair_rec[p];
        rlo = __builtin_bit_cast(uint32_t, rec.span.z);  // x0 | y0 << 16
        rhi = __builtin_bit_cast(uint32_t, rec.span.w);  // x1 | y1 << 16
        const ushort4 rc = make_ushort4((unsigned short)(rlo & 0xFFFFu), (unsigned short)(rlo >> 16),
                                        (unsigned short)(rhi & 0xFFFFu), (unsigned short)(rhi >> 16));
        g = span_geo(rec.geo.x, rec.geo.y, rec.geo.z, rec.geo.w, rec.span.x, rec.span.y);
        a.pair_rank[p] = (uint32_t)k;
        a.rank_xy[k] = make_float2(rec.geo.x, rec.geo.y);
        a.rank_conic[k] = rec.conic;
        a.rank_rgbd[k] = rec.rgbd;
        a.rank_rect[k] = rc;
        o = a.rank_off[k];
        cnt = a.rank_off[k + 1] - o;
        by0 = rc.y / BTY;
        nrows = cnt ? (rc.w + BTY - 1) / BTY - by0 : 0;
        H = V.H;
        BX = V.BX;
        bbase = V.bin_base;
    }
    const uint32_t incl_r = wave_incl_scan_u32((uint32_t)nrows);
    const uint32_t total_r = (uint32_t)readlane_i((int)incl_r, 63);
    uint32_t carry = 0;  // instances written in earlier chunks for rank lane carry_rank
    int carry_rank = -1;
    for (uint32_t x0 = 0; x0 < total_r; x0 += 64) {
        const uint32_t x = x0 + (uint32_t)lane;
        const bool valid = x < total_r;
        // the item's rank: lane s, the first whose inclusive row count exceeds x
        int s = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
            if ((uint32_t)__shfl((int)incl_r, s + step - 1, 64) <= x) s += step;
        s = min(s, 63);
        const int s_rows = __shfl(nrows, s, 64);
        const uint32_t first_row = (uint32_t)__shfl((int)incl_r, s, 64) - (uint32_t)s_rows;  // item index of its row 0
        const int r = (int)(x - first_row);
        SpanGeo gs;
        gs.u = __shfl(g.u, s, 64);
        gs.v = __shfl(g.v, s, 64);
        gs.s = __shfl(g.s, s, 64);
        gs.iyy = __shfl(g.iyy, s, 64);
        gs.kx = __shfl(g.kx, s, 64);
        gs.wx = __shfl(g.wx, s, 64);
        gs.rx = __shfl(g.rx, s, 64);
        gs.ry = __shfl(g.ry, s, 64);
        gs.yx = __shfl(g.yx, s, 64);
        gs.pad = __shfl(g.pad, s, 64);
        const uint32_t slo = (uint32_t)__shfl((int)rlo, s, 64), shi = (uint32_t)__shfl((int)rhi, s, 64);
        const int sx0 = (int)(slo & 0xFFFFu), sy0 = (int)(slo >> 16), sx1 = (int)(shi & 0xFFFFu), sy1 = (int)(shi >> 16);
        const int by = __shfl(by0, s, 64) + r;
        const int sH = __shfl(H, s, 64), sBX = __shfl(BX, s, 64), sbase = __shfl(bbase, s, 64);
        const uint32_t so = (uint32_t)__shfl((int)o, s, 64), scnt = (uint32_t)__shfl((int)cnt, s, 64);
        const uint32_t sk = (uint32_t)__shfl((int)(uint32_t)k, s, 64);
        int c0 = 0, c1 = 0;
        float py0, py1;
        if (valid && bin_band(by, BTY, sy0, sy1, sH, py0, py1)) span_bins(gs, py0, py1, sx0, sx1, BTX, c0, c1);
        const uint32_t w = (uint32_t)(c1 - c0);
        const uint32_t incl_w = wave_incl_scan_u32(w);
        const uint32_t excl_w = incl_w - w;
        // the rank's instances in this chunk's earlier rows, plus those of
        // earlier chunks when the rank continues from one
        const int f = first_row > x0 ? (int)(first_row - x0) : 0;  // lane of the rank's first item here
        const uint32_t before = excl_w - (uint32_t)__shfl((int)excl_w, f, 64);
        const uint32_t carried = s == carry_rank ? carry : 0u;
        const uint32_t start = so + carried + before;
        // the rank that continues into the next chunk: the last item's
        const int last = (int)min(total_r - 1u - x0, 63u);
        const int s_last = readlane_i(s, last), f_last = readlane_i(f, last);
        const uint32_t run = (uint32_t)readlane_i((int)incl_w, last) - (uint32_t)readlane_i((int)excl_w, f_last);
        carry = (s_last == carry_rank ? carry : 0u) + run;
        carry_rank = s_last;
        // a rank whose spans gave fewer instances than counted (never: the
        // count used the same spans) fills the rest with keys of no bin
        if (valid && r == s_rows - 1)
            for (uint32_t i = start + w; i < so + scnt; ++i) a.inst_key[i] = kNoTile;
        // the chunk's instances, 64 at a time
        const uint32_t total_w = (uint32_t)readlane_i((int)incl_w, 63);
        const uint32_t bin0 = (uint32_t)(sbase + by * sBX + c0);  // bin of the item's first column
        const uint32_t end = so + scnt;
        for (uint32_t y0 = 0; y0 < total_w; y0 += 64) {
            const uint32_t y = y0 + (uint32_t)lane;
            int j = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
                if ((uint32_t)__shfl((int)incl_w, j + step - 1, 64) <= y) j += step;
            j = min(j, 63);
            const uint32_t d = y - (uint32_t)__shfl((int)excl_w, j, 64);  // column within item j's span
            const uint32_t oo = (uint32_t)__shfl((int)start, j, 64) + d;
            const uint32_t bin = (uint32_t)__shfl((int)bin0, j, 64) + d;
            const uint32_t kj = (uint32_t)__shfl((int)sk, j, 64);
            const uint32_t ej = (uint32_t)__shfl((int)end, j, 64);
            if (y < total_w && oo < ej) a.inst_key[oo] = inst_key_of(a, (int64_t)bin, kj, oo);
        }
    }
}

// [first, last) of every bin in the sorted keys: a bin starts where the bin
// differs from the previous key's and ends where it differs from the next.
// half: the 32-bit half of each key that holds the bin (stride 2), mask: the
// bin's bits in it.  Neighbours come from the adjacent lanes; only a wave's
// end lanes load theirs.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t *half, uint32_t mask, int64_t M, int64_t n_bins,
                                                     uint2 *range) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = s < M;
    const uint32_t t = in ? half[2 * s] & mask : 0xFFFFFFFFu;
    const int lane = lane_id();
    uint32_t tp = (uint32_t)__shfl_up((int)t, 1, 64), tn = (uint32_t)__shfl_down((int)t, 1, 64);
    if (lane == 0) tp = s > 0 && in ? half[2 * (s - 1)] & mask : ~t;
    if (lane == 63) tn = s + 1 < M ? half[2 * (s + 1)] & mask : ~t;
    if (!in || (int64_t)t >= n_bins) return;
    if (s == 0 || tp != t) range[t].x = (uint32_t)s;
    if (s == M - 1 || tn != t) range[t].y = (uint32_t)(s + 1);
}

// ---------------------------------------------------------------- per-rank record sums
// One row of 16 lanes per depth rank: the rank's records are contiguous
// (emission order), the row strides over them and reduces with DPP.
__global__ __launch_bounds__(256) void k_rank_reduce(const float *records, const uint32_t *rank_off, int64_t Pv,
                                                     float *grad2d) {
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    float acc[kRecord];
#pragma unroll
    for (int c = 0; c < kRecord; ++c) acc[c] = 0.0f;
    if (k < Pv) {
        const uint32_t e0 = rank_off[k], e1 = rank_off[k + 1];
        for (uint32_t e = e0 + sub; e < e1; e += 16) {
            const float2 *rec = reinterpret_cast<const float2 *>(records + (int64_t)e * kRecord);
#pragma unroll
            for (int c = 0; c < kRecord / 2; ++c) {
                const float2 t = rec[c];
                acc[2 * c] += t.x;
                acc[2 * c + 1] += t.y;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kRecord; ++c) acc[c] = row16_sum(acc[c]);
    if (k < Pv && sub < kRecord / 2) {
        float2 *out = reinterpret_cast<float2 *>(grad2d + k * kRecord);
        float x = acc[0], y = acc[1];
#pragma unroll
        for (int c = 1; c < kRecord / 2; ++c)
            if (sub == c) { x = acc[2 * c]; y = acc[2 * c + 1]; }
        out[sub] = make_float2(x, y);
    }
}

// ---------------------------------------------------------------- per-pair and per-Gaussian backward
// One thread per visible (Gaussian, view) pair, in depth-rank order, so that
// no lane idles on a view where its Gaussian is culled: the chain rule of the
// pair's ten record sums to the Gaussian's parameters (written per pair) and to
// the view's pose (summed per block and view).  A second pass adds each
// Gaussian's pairs over its views in view order.  Both orders are fixed: the
// gradients are deterministic.
constexpr int kPairGradFixed = 11;  // means 3, scales 3, quaternion 4, opacity 1; then SH 3K

struct PairBwdArgs {
    const ViewDev *views;
    const MapDev *maps;
    int n_views;
    int map;
    int64_t Pv;
    const uint32_t *rank_pair;
    const float *grad2d;      // [Pv][10]
    float *pair_grad;         // [Pv][stride]
    int stride;
    float *pose_partial;      // this map's [blocks][n_views][9]
    const int32_t *view_list; // views of this map
    int n_map_views;
};

// POSE_ONLY: the Gaussians' own gradients are not wanted (tracking); the chain
// runs for the pose sums alone and writes nothing per pair, so the compiler
// drops what feeds only the Gaussian parameters.
template <int DEG, bool POSE_ONLY>
__global__ __launch_bounds__(256) void k_pair_bwd(PairBwdArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = -1;
    float pose[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (k < a.Pv) {
        const uint32_t p = a.rank_pair[k];
        const int pv = view_of_pair(a.views, a.n_views, p);
        const ViewDev &V = a.views[pv];
        if (V.map == a.map) {
            v = pv;
            const MapDev &Mp = a.maps[a.map];
            const int64_t g = (int64_t)p - V.pair_base;
            float m[3], sc[3], q[4];
            for (int c = 0; c < 3; ++c) { m[c] = Mp.means[3 * g + c]; sc[c] = Mp.scales[3 * g + c]; }
            const float4 q4 = *reinterpret_cast<const float4 *>(Mp.quats + 4 * g);
            q[0] = q4.x; q[1] = q4.y; q[2] = q4.z; q[3] = q4.w;
            const float o = Mp.opac[g];
            PairGrad rg;
            const float2 *src = reinterpret_cast<const float2 *>(a.grad2d + k * kRecord);
#pragma unroll
            for (int c = 0; c < kRecord / 2; ++c) {
                const float2 t = src[c];
                rg.g[2 * c] = t.x;
                rg.g[2 * c + 1] = t.y;
            }
            float gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0f;
            float gsh[3 * K];
#pragma unroll
            for (int c = 0; c < 3 * K; ++c) gsh[c] = 0.0f;
            Proj P;
            if (key_path(m, sc, q, o, V, P)) chain_pair<DEG>(P, q, sc, o, Mp, g, m, V, rg, gm, gs, gq, &go, gsh, pose);
            if (!POSE_ONLY) {
                float *out = a.pair_grad + k * a.stride;
                for (int c = 0; c < 3; ++c) { out[c] = gm[c]; out[3 + c] = gs[c]; }
                for (int c = 0; c < 4; ++c) out[6 + c] = gq[c];
                out[10] = go;
#pragma unroll
                for (int c = 0; c < 3 * K; ++c) out[kPairGradFixed + c] = gsh[c];
            }
        }
    }
    // this block's pose sums for every view of the map (zero where it has none)
    __shared__ float red[4][9];
    for (int vi = 0; vi < a.n_map_views; ++vi) {
        const int vv = a.view_list[vi];
        float *dst = a.pose_partial + ((int64_t)blockIdx.x * a.n_views + vv) * 9;
        if (!__syncthreads_or(v == vv)) {
            if (threadIdx.x < 9) dst[threadIdx.x] = 0.0f;
            continue;
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const float t = wave_sum(v == vv ? pose[c] : 0.0f);
            if (lane_id() == 0) red[threadIdx.x >> 6][c] = t;
        }
        __syncthreads();
        if (threadIdx.x < 9) dst[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                                red[3][threadIdx.x];
        __syncthreads();
    }
}

struct GaussBwdArgs {
    const ViewDev *views;
    const MapDev *maps;
    int map;
    const int32_t *view_list;  // views of this map
    int n_map_views;
    const uint32_t *pair_rank;   // valid where pair_count > 0
    const uint32_t *pair_count;  // the pair's tile instances (0: in no list)
    const uint32_t *pair_depth;  // 0xFFFFFFFF where the pair was culled
    const float *pair_grad;
    int stride;
    mgs_gaussian_grads gr;
};

template <int DEG>
__global__ __launch_bounds__(256) void k_gauss_bwd(GaussBwdArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int NG = kPairGradFixed + 3 * K;
    const MapDev &Mp = a.maps[a.map];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Mp.n) return;
    const bool stats = a.gr.grad_norm_sum != nullptr;
    float acc[NG];
#pragma unroll
    for (int c = 0; c < NG; ++c) acc[c] = 0.0f;
    // Eq. (3) statistics: per view that keeps the Gaussian after culling, the
    // norm of that view's mean gradient (0 when no tile list holds it)
    float norm_sum = 0.0f;
    uint32_t seen = 0;
    for (int vi = 0; vi < a.n_map_views; ++vi) {
        const ViewDev &V = a.views[a.view_list[vi]];
        if (stats && a.pair_depth[V.pair_base + g] != 0xFFFFFFFFu) ++seen;
        if (a.pair_count[V.pair_base + g] == 0) continue;  // no tile list holds the pair
        const uint32_t k = a.pair_rank[V.pair_base + g];
        const float *src = a.pair_grad + (int64_t)k * a.stride;
#pragma unroll
        for (int c = 0; c < NG; ++c) acc[c] += src[c];
        if (stats) norm_sum += sqrtf(src[0] * src[0] + src[1] * src[1] + src[2] * src[2]);
    }
    if (stats) {
        a.gr.grad_norm_sum[g] += norm_sum;
        a.gr.visible_count[g] += seen;
    }
    if (a.gr.d_means) for (int c = 0; c < 3; ++c) a.gr.d_means[3 * g + c] = acc[c];
    if (a.gr.d_scales) for (int c = 0; c < 3; ++c) a.gr.d_scales[3 * g + c] = acc[3 + c];
    if (a.gr.d_quats) for (int c = 0; c < 4; ++c) a.gr.d_quats[4 * g + c] = acc[6 + c];
    if (a.gr.d_opac) a.gr.d_opac[g] = acc[10];
    if (a.gr.d_sh) {
#pragma unroll
        for (int c = 0; c < 3 * K; ++c) a.gr.d_sh[(int64_t)3 * K * g + c] = acc[kPairGradFixed + c];
    }
}

struct PoseFinalArgs {
    const ViewDev *views;
    int n_views;
    const float *pose_partial;  // [n_maps][nb][n_views][9]
    int64_t nb;                 // pair-backward blocks per map
    float *d_pose;
};

__global__ __launch_bounds__(256) void k_pose_final(PoseFinalArgs a) {
    const int v = blockIdx.x;
    const ViewDev &V = a.views[v];
    const int64_t b0 = (int64_t)V.map * a.nb, nb = a.nb;
    double acc[9];
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
        for (int c = 0; c < 9; ++c) acc[c] += (double)a.pose_partial[((b0 + b) * a.n_views + v) * 9 + c];
    __shared__ double red[256][9];
    for (int c = 0; c < 9; ++c) red[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int c = 0; c < 9; ++c) red[threadIdx.x][c] += red[threadIdx.x + st][c];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double *r = red[0];
        for (int i = 0; i < 3; ++i) {
            const double rot = (double)V.R[3 * i] * r[6] + (double)V.R[3 * i + 1] * r[7] + (double)V.R[3 * i + 2] * r[8];
            a.d_pose[6 * v + i] = (float)(r[i] + rot);
            a.d_pose[6 * v + 3 + i] = (float)r[3 + i];
        }
    }
}

// ---------------------------------------------------------------- host side
namespace {

struct Setup {
    std::vector<ViewDev> views;
    std::vector<MapDev> maps;
    std::vector<int32_t> view_list;      // views grouped by map
    std::vector<int32_t> map_view_off;   // [n_maps + 1]
    int64_t P = 0, B_total = 0, pixels = 0;  // pairs, list bins, pixels
    int btx = 1, bty = 1;                     // tiles per bin
};

// Tiles per list bin of a forward call.  A bin of 2 x 1 tiles makes the
// lists shorter in total (each Gaussian is listed once per bin it touches, not
// per tile: 5.3M instead of 8.1M instances on the 8-view window), so the
// emission, the tile sort and the backward's record sums move less, and the
// backward folds its sums once per bin instead of once per tile; but a lane
// holds twice the pixel state (3 waves per SIMD in the backward, 4 in the
// forward), so the bins must outnumber the resident waves several times over.
// Calls with at least kBin2x1FromTiles tiles therefore take 2 x 1 bins (the
// window: 2.25 -> 2.18 ms per step), smaller ones 1 x 1 (below kSplitBelowBins
// bins also split into quadrant waves).  2 x 2 bins hold 4x the state and are
// slower (about 18 % on the window).  MGS_BIN_TILES = "1x1", "2x1" or "2x2"
// forces a size.
constexpr int64_t kBin2x1FromTiles = 16384;
void choose_bin(const mgs_camera *cams, int32_t n_views, int &btx, int &bty) {
    btx = 1;
    bty = 1;
    if (const char *e = getenv("MGS_BIN_TILES")) {
        if (!strcmp(e, "2x1")) { btx = 2; bty = 1; }
        else if (!strcmp(e, "2x2")) { btx = 2; bty = 2; }
        return;
    }
    if (!cams || n_views < 1 || n_views > 4096) return;  // rejected by the validation
    int64_t tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        const int w = cams[v].width, h = cams[v].height;
        if (w >= 1 && h >= 1 && w <= 16384 && h <= 16384)
            tiles += (int64_t)((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
    }
    if (tiles >= kBin2x1FromTiles) btx = 2;
}

bool bin_supported(int btx, int bty) { return (btx == 1 && bty == 1) || (btx == 2 && (bty == 1 || bty == 2)); }

mgs_status validate_and_setup(const mgs_gaussians *maps, int32_t n_maps, const mgs_camera *cams, int32_t n_views,
                              int btx, int bty, Setup &S) {
    if (!bin_supported(btx, bty)) return MGS_ERR_INVALID_ARG;
    S.btx = btx;
    S.bty = bty;
    if (n_views < 1 || n_views > 4096 || !cams || n_maps < 1 || n_maps > 1024 || !maps) return MGS_ERR_INVALID_ARG;
    S.maps.resize(n_maps);
    for (int m = 0; m < n_maps; ++m) {
        const mgs_gaussians &G = maps[m];
        if (G.n < 0 || G.sh_degree < 0 || G.sh_degree > 3) return MGS_ERR_INVALID_ARG;
        if (G.n > 0 && (!G.means || !G.scales || !G.quats || !G.opac || !G.sh)) return MGS_ERR_INVALID_ARG;
        if (G.quats && (reinterpret_cast<uintptr_t>(G.quats) & 15)) return MGS_ERR_INVALID_ARG;
        MapDev &D = S.maps[m];
        D.means = G.means; D.scales = G.scales; D.quats = G.quats; D.opac = G.opac; D.sh = G.sh;
        D.n = G.n; D.sh_degree = G.sh_degree; D.K = (G.sh_degree + 1) * (G.sh_degree + 1);
        D.pair_first_view = 0;
    }
    S.views.resize(n_views);
    S.map_view_off.assign(n_maps + 1, 0);
    for (int v = 0; v < n_views; ++v) {
        const mgs_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) return MGS_ERR_INVALID_ARG;
        if (!(c.fx > 0) || !(c.fy > 0) || !std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) ||
            !std::isfinite(c.cy))
            return MGS_ERR_INVALID_ARG;
        if (c.map < 0 || c.map >= n_maps) return MGS_ERR_INVALID_ARG;
        ViewDev &V = S.views[v];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) V.R[3 * i + j] = c.Tcw[4 * i + j];
            V.t[i] = c.Tcw[4 * i + 3];
        }
        for (int j = 0; j < 3; ++j)
            V.cam_center[j] = -(V.R[j] * V.t[0] + V.R[3 + j] * V.t[1] + V.R[6 + j] * V.t[2]);
        V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy; V.near_z = c.near_z;
        {
#pragma clang fp contract(off)
            V.limx = kFrustum * ((0.5f * (float)c.width) / c.fx);
            V.limy = kFrustum * ((0.5f * (float)c.height) / c.fy);
        }
        V.W = c.width; V.H = c.height;
        V.TX = (c.width + kTile - 1) / kTile;
        V.TY = (c.height + kTile - 1) / kTile;
        V.map = c.map;
        V.BTX = btx;
        V.BTY = bty;
        V.BX = (V.TX + btx - 1) / btx;
        V.BY = (V.TY + bty - 1) / bty;
        V.pair_base = S.P;
        V.bin_base = (int32_t)S.B_total;
        V.pix_base = S.pixels;
        S.P += maps[c.map].n;
        S.B_total += (int64_t)V.BX * V.BY;
        S.pixels += (int64_t)c.width * c.height;
        S.map_view_off[c.map + 1]++;
    }
    if (S.P >= (int64_t(1) << 31) || S.B_total >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    for (int m = 0; m < n_maps; ++m) S.map_view_off[m + 1] += S.map_view_off[m];
    S.view_list.assign(n_views, 0);
    std::vector<int32_t> fill(S.map_view_off.begin(), S.map_view_off.end() - 1);
    for (int v = 0; v < n_views; ++v) S.view_list[fill[cams[v].map]++] = v;
    return MGS_OK;
}

// Quadrant culling at staging: by the ellipse's interval per quadrant row
// (quad_mask_rows) for bins of four or more quadrants; MGS_QUAD_CULL=box takes
// the per-quadrant edge test everywhere instead, which gives the same bits
// (both are conservative), for checking the one against the other.
bool box_cull() {
    const char *e = getenv("MGS_QUAD_CULL");
    return e && !strcmp(e, "box");
}

// A forward call with fewer bins than this splits each 16x16 bin into its four
// quadrants, one wave each (k_blend_fwd SPLIT): four times the waves, one
// evaluation per visit, the same bits.  MGS_BLEND_SPLIT=0 or 1 forces either.
constexpr int64_t kSplitBelowBins = 4096;
bool split_blend(int btx, int bty, int64_t n_bins) {
    if (btx != 1 || bty != 1) return false;
    if (const char *e = getenv("MGS_BLEND_SPLIT")) {
        if (e[0] == '0') return false;
        if (e[0] == '1') return true;
    }
    return n_bins < kSplitBelowBins;
}

void launch_blend_fwd(bool count, bool split, int btx, int bty, unsigned grid, hipStream_t s, const BlendArgs &ba) {
    if (split) {
        if (count) k_blend_fwd<true, 1, 1, true><<<grid, 64, 0, s>>>(ba);
        else k_blend_fwd<false, 1, 1, true><<<grid, 64, 0, s>>>(ba);
    } else if (btx == 2 && bty == 2) {
        if (count) k_blend_fwd<true, 2, 2><<<grid, 64, 0, s>>>(ba);
        else k_blend_fwd<false, 2, 2><<<grid, 64, 0, s>>>(ba);
    } else if (btx == 2) {
        if (count) k_blend_fwd<true, 2, 1><<<grid, 64, 0, s>>>(ba);
        else k_blend_fwd<false, 2, 1><<<grid, 64, 0, s>>>(ba);
    } else {
        if (count) k_blend_fwd<true, 1, 1><<<grid, 64, 0, s>>>(ba);
        else k_blend_fwd<false, 1, 1><<<grid, 64, 0, s>>>(ba);
    }
}

// pose: a tracking call over maps of SH degree 0 (the blend forms only what the
// pose gradient reads)
template <bool POSE>
void launch_blend_bwd_t(bool split, int btx, int bty, unsigned grid, hipStream_t s, const BlendBwdArgs &bb) {
    if (split) k_blend_bwd_split<POSE><<<grid, 256, 0, s>>>(bb);
    else if (btx == 2 && bty == 2) k_blend_bwd<2, 2, POSE><<<grid, 64, 0, s>>>(bb);
    else if (btx == 2) k_blend_bwd<2, 1, POSE><<<grid, 64, 0, s>>>(bb);
    else k_blend_bwd<1, 1, POSE><<<grid, 64, 0, s>>>(bb);
}
void launch_blend_bwd(bool split, int btx, int bty, unsigned grid, hipStream_t s, const BlendBwdArgs &bb, bool pose) {
    if (pose) launch_blend_bwd_t<true>(split, btx, bty, grid, s, bb);
    else launch_blend_bwd_t<false>(split, btx, bty, grid, s, bb);
}

struct Layout {
    // pre-count
    size_t views, maps, vlist, counters, pair_depth, pair_count, pair_rect, pair_uvr, pair_rec, pair_rank,
        scan_tmp_pre, n_contrib, n_blend, blk_vis, blk_cnt, blk_kmin, blk_kmax, pre_size;
    // post-count
    size_t sk0, sk1, sv0, sv1, rank_off, rank_xy, rank_conic, rank_rgbd, rank_rect, it0, it1, iv0, iv1, hist,
        scan_tmp, tile_range, bin_order, records, grad2d, pair_grad, pose_partial, inst_qm, total;
    int64_t pose_blocks;  // pair-backward blocks per map
    int grad_stride;      // floats per pair gradient
};

// projection grid: chunks of 256 x proj_rounds(S) Gaussians of the largest
// map, one row per view
int64_t proj_max_n(const Setup &S) {
    int64_t max_n = 0;
    for (const ViewDev &V : S.views) max_n = std::max<int64_t>(max_n, S.maps[V.map].n);
    return max_n;
}
int proj_rounds(const Setup &S) {
    const int64_t blocks = ceil_div(proj_max_n(S), 256 * kProjRoundsLarge) * (int64_t)S.views.size();
    return blocks < kProjSmallBlocks ? kProjRoundsSmall : kProjRoundsLarge;
}
int64_t project_cols(const Setup &S) { return ceil_div(proj_max_n(S), 256 * proj_rounds(S)); }

Layout make_layout(const Setup &S, int64_t Pv, int64_t M, bool bwd) {
    Layout L{};
    Bump b;
    const int64_t P = S.P, V = (int64_t)S.views.size(), NM = (int64_t)S.maps.size();
    L.views = b.take(sizeof(ViewDev) * V);
    L.maps = b.take(sizeof(MapDev) * NM);
    L.vlist = b.take(sizeof(int32_t) * V);
    L.counters = b.take(4 * CNT_WORDS);
    L.pair_depth = b.take(4 * P);
    L.pair_count = b.take(4 * P);
    L.pair_rect = b.take(8 * P);
    L.pair_uvr = b.take(16 * P);
    L.pair_rec = b.take(sizeof(PairRec) * P);
    L.pair_rank = b.take(4 * P);
    L.scan_tmp_pre = b.take(4 * scan_tmp_words(P));
    L.n_contrib = b.take(4 * S.pixels);
    L.n_blend = b.take(4 * S.pixels);
    L.blk_vis = b.take(4 * project_cols(S) * V);
    L.blk_cnt = b.take(8 * project_cols(S) * V);
    L.blk_kmin = b.take(4 * project_cols(S) * V);
    L.blk_kmax = b.take(4 * project_cols(S) * V);
    // the compaction's output (the pair sort's input) sits before the count,
    // with room for every pair, so the compaction is queued before the host
    // reads the count back
    L.sk0 = b.take(4 * P);
    L.sv0 = b.take(4 * P);
    L.pre_size = b.size();
    L.sk1 = b.take(4 * Pv);
    L.sv1 = b.take(4 * Pv);
    L.rank_off = b.take(4 * (Pv + 1));
    L.rank_xy = b.take(8 * Pv);
    L.rank_conic = b.take(16 * Pv);
    L.rank_rgbd = b.take(16 * Pv);
    L.rank_rect = b.take(8 * Pv);
    L.it0 = b.take(8 * M); L.it1 = b.take(8 * M);
    L.iv0 = b.take(4 * M); L.iv1 = b.take(4 * M);
    const int64_t nmax = std::max<int64_t>(std::max<int64_t>(Pv, M), 1);
    L.hist = b.take(4 * radix_hist_words(nmax));
    L.scan_tmp = b.take(4 * scan_tmp_words(std::max<int64_t>(radix_hist_words(nmax), Pv + 1)));
    L.tile_range = b.take(8 * S.B_total + 4 * kBinOrderWords);  // ranges, then the bin-order bookkeeping
    L.bin_order = b.take(4 * S.B_total);
    L.pose_blocks = std::max<int64_t>(ceil_div(Pv, 256), 1);
    int kmax = 1;
    for (const MapDev &m : S.maps) kmax = std::max(kmax, m.K);
    L.grad_stride = kPairGradFixed + 3 * kmax;
    if (bwd) {
        L.records = b.take(4 * kRecord * M);
        L.inst_qm = b.take(2 * M);  // the forward's quadrant mask per list entry
        L.grad2d = b.take(4 * kRecord * Pv);
        L.pair_grad = b.take(4 * (size_t)L.grad_stride * Pv);
        L.pose_partial = b.take(4 * 9 * V * NM * L.pose_blocks);
    } else {
        L.records = L.grad2d = L.pair_grad = L.pose_partial = L.inst_qm = 0;
    }
    L.total = b.size();
    return L;
}

// compute units of the current device (queried per call: no cached state)
int num_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    return n;
}

inline unsigned grid_of(int64_t n, int block) { return (unsigned)ceil_div(n, block); }

// resident one-wave blocks per CU for the persistent blend kernels
// (MGS_BLEND_WAVES_PER_CU overrides the default of 24, range 1..64; the
// backward's registers hold it to 16)
int64_t blend_grid(int64_t n_items) {
    int w = 24;
    if (const char *e = getenv("MGS_BLEND_WAVES_PER_CU")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 64) w = v;
    }
    return std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)num_cus() * w));
}

// Optional per-stage timing: events created for this call (stage_ms, the call
// waits) or the caller's events (stage_events, recorded only).
struct StageTimer {
    hipEvent_t ev[6] = {};
    bool own[6] = {};
    int n = 0;
    float *out = nullptr;
    void **ext = nullptr;  // caller's events: record only, never wait
    hipStream_t s = nullptr;
    StageTimer(const mgs_render_opts *o, hipStream_t st)
        : out(o ? o->stage_ms : nullptr), ext(o ? o->stage_events : nullptr), s(st) {}
    void mark() {
        if (n >= 6) return;
        if (ext) {
            if (ext[n]) hipEventRecord(static_cast<hipEvent_t>(ext[n]), s);
        } else if (out && hipEventCreate(&ev[n]) == hipSuccess) {
            own[n] = true;
            hipEventRecord(ev[n], s);
        }
        ++n;
    }
    // stage i = [mark a, mark b); writes out[slot] (own events only)
    void finish(const int (*spans)[3], int nspans) {
        if (!out || ext) return;
        hipEventSynchronize(ev[n - 1]);
        for (int i = 0; i < nspans; ++i) {
            float ms = 0.0f;
            if (spans[i][1] < n && spans[i][2] < n) hipEventElapsedTime(&ms, ev[spans[i][1]], ev[spans[i][2]]);
            out[spans[i][0]] = ms;
        }
    }
    ~StageTimer() {
        for (int i = 0; i < n; ++i)
            if (own[i]) hipEventDestroy(ev[i]);
    }
};

int bits_for(int64_t n_values) {  // bits needed to hold values in [0, n_values)
    int b = 0;
    while ((int64_t(1) << b) < n_values) ++b;
    return b;
}

// MGS_WIDE_INSTANCES=1 keeps the wide instance keys even where the packed ones
// fit (both give the same lists, images and gradients)
bool wide_instances() {
    const char *e = getenv("MGS_WIDE_INSTANCES");
    return e && e[0] == '1';
}

// how the blend kernels read each sorted instance's depth rank and record slot
InstRef instances_of(void *ws, const mgs_forward_info &info) {
    InstRef r;
    r.key = at<uint64_t>(ws, info.off_inst_key);
    if (info.inst_bin_bits > 0) {
        r.rec = nullptr;
        r.rshift = info.inst_bin_bits;
        r.rmask = (uint32_t)((1ull << info.inst_rank_bits) - 1);
        r.eshift = info.inst_bin_bits + info.inst_rank_bits;
    } else {
        r.rec = at<uint32_t>(ws, info.off_inst_rec);
        r.rshift = 0;
        r.rmask = 0xFFFFFFFFu;
        r.eshift = 0;
    }
    return r;
}

}  // namespace
}  // namespace mgs

using namespace mgs;

extern "C" mgs_status mgs_render_forward(const mgs_gaussians *maps, int32_t n_maps, const mgs_camera *cams,
                                         int32_t n_views, const mgs_render_opts *opts, void *ws, size_t ws_bytes,
                                         mgs_forward_info *info, float *out_rgb, float *out_depth, float *out_T,
                                         void *stream) {
    ApiRange api_range("mgs_render_forward");
    if (!info || !out_rgb || !out_depth || !out_T) return MGS_ERR_INVALID_ARG;
    Setup S;
    int btx, bty;
    choose_bin(cams, n_views, btx, bty);
    mgs_status st = validate_and_setup(maps, n_maps, cams, n_views, btx, bty, S);
    if (st != MGS_OK) return st;
    if (ws_bytes > 0 && !ws) return MGS_ERR_INVALID_ARG;
    const bool bwd = opts && opts->need_backward;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = make_layout(S, 0, 0, bwd);
    *info = mgs_forward_info{};
    info->n_pairs = S.P;
    info->n_bins = S.B_total;
    info->bin_tx = S.btx;
    info->bin_ty = S.bty;
    info->n_pixels = S.pixels;
    info->n_views = n_views;
    info->n_maps = n_maps;
    info->need_backward = bwd ? 1 : 0;
    if (ws_bytes < L.pre_size) {
        info->ws_required = L.pre_size;
        return MGS_ERR_WORKSPACE;
    }
    const bool by_args = n_views <= kArgViews && n_maps <= kArgMaps;
    if (!by_args) {
        MGS_HIP(hipMemcpyAsync(at<void>(ws, L.views), S.views.data(), sizeof(ViewDev) * S.views.size(),
                               hipMemcpyHostToDevice, s));
        MGS_HIP(hipMemcpyAsync(at<void>(ws, L.maps), S.maps.data(), sizeof(MapDev) * S.maps.size(),
                               hipMemcpyHostToDevice, s));
        MGS_HIP(hipMemcpyAsync(at<void>(ws, L.vlist), S.view_list.data(), sizeof(int32_t) * S.view_list.size(),
                               hipMemcpyHostToDevice, s));
    }
    StageTimer timer(opts, s);
    timer.mark();  // 0
    uint32_t *counters = at<uint32_t>(ws, L.counters);
    const Mailbox mail = host_mailbox();
    const uint32_t ticket = mailbox_ticket();
    if (by_args) {
        SetupArgs sa;
        memset(&sa, 0, sizeof(sa));
        memcpy(sa.views, S.views.data(), sizeof(ViewDev) * S.views.size());
        memcpy(sa.maps, S.maps.data(), sizeof(MapDev) * S.maps.size());
        memcpy(sa.vlist, S.view_list.data(), sizeof(int32_t) * S.view_list.size());
        sa.n_views = n_views;
        sa.n_maps = n_maps;
        k_setup<<<1, 256, 0, s>>>(sa, at<ViewDev>(ws, L.views), at<MapDev>(ws, L.maps), at<int32_t>(ws, L.vlist),
                                  counters);
    } else {
        k_init<<<1, 64, 0, s>>>(counters);
    }
    ProjectArgs pa;
    pa.views = at<ViewDev>(ws, L.views);
    pa.maps = at<MapDev>(ws, L.maps);
    pa.n_views = n_views;
    pa.P = S.P;
    pa.pair_depth = at<uint32_t>(ws, L.pair_depth);
    pa.pair_count = at<uint32_t>(ws, L.pair_count);
    pa.pair_rect = at<ushort4>(ws, L.pair_rect);
    pa.pair_uvr = at<float4>(ws, L.pair_uvr);
    pa.pair_rec = at<PairRec>(ws, L.pair_rec);
    pa.blk_vis = at<uint32_t>(ws, L.blk_vis);
    pa.blk_cnt = at<uint64_t>(ws, L.blk_cnt);
    pa.blk_kmin = at<uint32_t>(ws, L.blk_kmin);
    pa.blk_kmax = at<uint32_t>(ws, L.blk_kmax);
    pa.clamp_flag = counters + CNT_CLAMP;
    const int64_t cols = project_cols(S);
    pa.cols = cols;
    if (S.P > 0) {
        const unsigned pgrid = (unsigned)(8 * ceil_div(cols, 8) * n_views);
        if (proj_rounds(S) == kProjRoundsSmall) k_project<kProjRoundsSmall><<<pgrid, 256, 0, s>>>(pa);
        else k_project<kProjRoundsLarge><<<pgrid, 256, 0, s>>>(pa);
        MGS_LAUNCHED();
        k_sum_blocks<<<1, 1024, 0, s>>>(pa.blk_vis, pa.blk_cnt, pa.blk_kmin, pa.blk_kmax, cols * n_views, counters,
                                        mail.dev, ticket);
        MGS_LAUNCHED();
    }
    timer.mark();  // 1
    // compaction of visible pairs (its buffers do not depend on the count):
    // queued before the read-back, so the device works while the host turns round
    uint32_t *sk[2] = {at<uint32_t>(ws, L.sk0), nullptr};
    uint32_t *sv[2] = {at<uint32_t>(ws, L.sv0), nullptr};
    if (S.P > 0) {
        MGS_HIP(scan_exclusive(LoadVis{pa.pair_count},
                               StoreCompact{pa.pair_count, pa.pair_depth, sk[0], sv[0]}, S.P,
                               at<uint32_t>(ws, L.scan_tmp_pre), nullptr, s));
    }
    uint32_t host_cnt[6] = {0, 0, 0, 0, 0xFFFFFFFFu, 0};
    if (S.P > 0 && mail.host) {
        MGS_HIP(mailbox_wait(mail, ticket, s));
        const volatile uint32_t *vm = mail.host;
        for (int k = 0; k < 6; ++k) host_cnt[k] = vm[k];
    } else if (S.P > 0) {
        MGS_HIP(hipMemcpyAsync(host_cnt, counters, 24, hipMemcpyDeviceToHost, s));
        MGS_HIP(hipStreamSynchronize(s));
    }
    const int64_t Pv = host_cnt[CNT_PV];
    const uint64_t M64 = (uint64_t)host_cnt[CNT_M] | ((uint64_t)host_cnt[CNT_M + 1] << 32);
    // The two early returns below come after launches that write into ws (the
    // compaction scan): they wait for the stream, so that the caller may free or
    // regrow the workspace as soon as the call returns.
    if (M64 >= (uint64_t(1) << 31)) {
        MGS_HIP(hipStreamSynchronize(s));
        return MGS_ERR_TOO_LARGE;
    }
    const int64_t M = (int64_t)M64;
    L = make_layout(S, Pv, M, bwd);
    info->n_visible = Pv;
    info->n_instances = M;
    info->ws_required = L.total;
    info->off_pair_depth = L.pair_depth;
    info->off_pair_rect = L.pair_rect;
    info->off_pair_uvr = L.pair_uvr;
    info->off_n_contrib = L.n_contrib;
    info->off_n_blend = L.n_blend;
    info->off_bin_range = L.tile_range;
    if (ws_bytes < L.total) {
        MGS_HIP(hipStreamSynchronize(s));
        return MGS_ERR_WORKSPACE;
    }

    uint32_t *tmp = at<uint32_t>(ws, L.scan_tmp);
    uint32_t *hist = at<uint32_t>(ws, L.hist);
    sk[1] = at<uint32_t>(ws, L.sk1);
    sv[1] = at<uint32_t>(ws, L.sv1);
    // pair sort on (view, depth key - kmin): as many bytes as those span
    int cur = 0;
    bool counts_in_rank_order = false;
    if (Pv > 0) {
        uint32_t kmin = host_cnt[CNT_KMIN], kmax = host_cnt[CNT_KMAX];
        if (kmax < kmin) kmin = 0, kmax = 0xFFFFFFFFu;  // not expected with Pv > 0: the full key range
        const int kbits = bits_for((int64_t)kmax - (int64_t)kmin + 1);
        const int passes = (kbits + bits_for(n_views) + 7) / 8;
        for (int p = 0; p < passes; ++p) {
            const PairDigit dig{pa.views, n_views, kmin, kbits, 8 * p};
            if (p + 1 < passes) {
                MGS_HIP(radix_pass<uint32_t>(sk[cur], sv[cur], sk[cur ^ 1], sv[cur ^ 1], Pv, dig, hist, s));
            } else {  // the counts in rank order, for the instance-offset scan
                MGS_HIP(radix_pass<uint32_t>(sk[cur], sv[cur], sk[cur ^ 1], sv[cur ^ 1], Pv, dig, hist, s,
                                             SideRankCount{pa.pair_count, at<uint32_t>(ws, L.rank_off)}));
                counts_in_rank_order = true;
            }
            cur ^= 1;
        }
    }
    uint32_t *rank_pair = sv[cur];
    info->off_rank_pair = cur ? L.sv1 : L.sv0;
    // instance offsets in rank order
    uint32_t *rank_off = at<uint32_t>(ws, L.rank_off);
    if (counts_in_rank_order)  // in place
        MGS_HIP(scan_exclusive(LoadU32{rank_off}, StoreU32{rank_off}, Pv, tmp, rank_off + Pv, s));
    else
        MGS_HIP(scan_exclusive(LoadRankCount{rank_pair, pa.pair_count}, StoreU32{rank_off}, Pv, tmp, rank_off + Pv, s));
    // emit instances
    uint64_t *it[2] = {at<uint64_t>(ws, L.it0), at<uint64_t>(ws, L.it1)};
    uint32_t *iv[2] = {at<uint32_t>(ws, L.iv0), at<uint32_t>(ws, L.iv1)};
    uint32_t *pair_rank = at<uint32_t>(ws, L.pair_rank);
    EmitArgs ea;
    ea.views = pa.views;
    ea.n_views = n_views;
    ea.Pv = Pv;
    ea.rank_pair = rank_pair;
    ea.rank_off = rank_off;
    ea.pair_rec = pa.pair_rec;
    ea.pair_rank = pair_rank;
    ea.rank_xy = at<float2>(ws, L.rank_xy);
    ea.rank_conic = at<float4>(ws, L.rank_conic);
    ea.rank_rgbd = at<float4>(ws, L.rank_rgbd);
    ea.rank_rect = at<ushort4>(ws, L.rank_rect);
    // packed keys (bin, rank and record slot in one word, sorted alone) when
    // the three fit 64 bits, else wide ones with the record slot as the value;
    // enough bin bits that an unused slot's all-ones bin sorts after every bin
    const int tbits = std::max(1, bits_for(S.B_total + 1)), rbits = std::max(1, bits_for(Pv));
    const bool packed = tbits + rbits + bits_for(M) <= 64 && !wide_instances();
    uint2 *range = at<uint2>(ws, L.tile_range);
    ea.zero = reinterpret_cast<uint32_t *>(range);
    ea.n_zero = 2 * S.B_total + kBinOrderWords;
    ea.inst_key = it[0];
    ea.bin_bits = packed ? tbits : 0;
    ea.rank_bits = packed ? rbits : 0;
    // calls with few ranks give each wave 16 of them: four times the waves,
    // each with a quarter of the dependent chunk steps
    ea.ranks_per_wave = Pv < (int64_t(1) << 18) ? 16 : 64;
    if (Pv > 0) k_emit<<<grid_of(Pv * (64 / ea.ranks_per_wave), 256), 256, 0, s>>>(ea);
    MGS_LAUNCHED();
    // stable tile sort on the bin field.  Wide: the values start as the
    // emission index, so at least one pass.
    int ic = 0;
    for (int sh = 0; sh < tbits && M > 0; sh += 8) {
        if (packed)
            MGS_HIP(radix_pass_keys<uint64_t>(it[ic], it[ic ^ 1], M, BinDigit{sh, std::min(8, tbits - sh)}, hist, s));
        else
            MGS_HIP(radix_pass<uint64_t>(it[ic], sh == 0 ? nullptr : iv[ic], it[ic ^ 1], iv[ic ^ 1], M,
                                         DigitOfKey<uint64_t>{32 + sh}, hist, s));
        ic ^= 1;
    }
    info->off_inst_key = ic ? L.it1 : L.it0;
    info->off_inst_rec = packed ? 0 : (ic ? L.iv1 : L.iv0);
    info->inst_bin_bits = ea.bin_bits;
    info->inst_rank_bits = ea.rank_bits;
    if (Pv == 0)  // else cleared by the emission
        k_fill_u32<<<grid_of(ea.n_zero, 256), 256, 0, s>>>(ea.zero, ea.n_zero, 0u);
    if (M > 0)
        k_tile_ranges<<<grid_of(M, 256), 256, 0, s>>>(reinterpret_cast<const uint32_t *>(it[ic]) + (packed ? 0 : 1),
                                                       packed ? (uint32_t)((1ull << tbits) - 1) : 0xFFFFFFFFu, M,
                                                       S.B_total, range);
    uint32_t *bin_order = at<uint32_t>(ws, L.bin_order);
    if (S.B_total > 0) {
        uint32_t *book = reinterpret_cast<uint32_t *>(range + S.B_total);
        k_bin_count<<<bin_order_grid(S.B_total), 256, 0, s>>>(range, S.B_total, book);
        k_bin_place<<<bin_order_grid(S.B_total), 256, 0, s>>>(range, S.B_total, book, bin_order);
    }
    MGS_LAUNCHED();
    // blend
    BlendArgs ba;
    ba.views = pa.views;
    ba.n_views = n_views;
    ba.n_items = S.B_total;
    ba.range = range;
    ba.order = bin_order;
    ba.inst = instances_of(ws, *info);
    ba.rxy = ea.rank_xy;
    ba.rconic = ea.rank_conic;
    ba.rrgbd = ea.rank_rgbd;
    ba.rrect = ea.rank_rect;
    const mgs_render_opts defaults{};
    const mgs_render_opts &o = opts ? *opts : defaults;
    ba.bg0 = o.bg_rgb[0]; ba.bg1 = o.bg_rgb[1]; ba.bg2 = o.bg_rgb[2]; ba.bgd = o.bg_depth;
    ba.queues = counters + CNT_Q;
    ba.clamp_flag = counters + CNT_CLAMP;
    ba.box_cull = box_cull();
    ba.out_rgb = out_rgb;
    ba.out_depth = out_depth;
    ba.out_T = out_T;
    ba.n_contrib = at<uint32_t>(ws, L.n_contrib);
    ba.n_blend = at<uint32_t>(ws, L.n_blend);
    const bool split = split_blend(S.btx, S.bty, S.B_total);
    // the one-wave forward of a backward call over bins of several tiles keeps
    // its quadrant masks for the backward (the same bins, the same decisions)
    ba.inst_qm = bwd && !split && S.btx * S.bty > 1 ? at<uint16_t>(ws, L.inst_qm) : nullptr;
    const int64_t grid = blend_grid(split ? 4 * S.B_total : S.B_total);
    timer.mark();  // 2
    launch_blend_fwd(opts && opts->count_blended, split, S.btx, S.bty, (unsigned)grid, s, ba);
    MGS_LAUNCHED();
    timer.mark();  // 3
    static const int spans[4][3] = {{0, 0, 1}, {1, 1, 2}, {2, 2, 3}, {3, 0, 3}};
    timer.finish(spans, 4);
    return MGS_OK;
}

extern "C" mgs_status mgs_render_backward(const mgs_gaussians *maps, int32_t n_maps, const mgs_camera *cams,
                                          int32_t n_views, const mgs_render_opts *opts,
                                          const mgs_forward_info *info, void *ws, size_t ws_bytes,
                                          const float *out_T, const float *dL_drgb, const float *dL_ddepth,
                                          const mgs_gaussian_grads *grads, float *d_pose, void *stream) {
    ApiRange api_range("mgs_render_backward");
    if (!info || !ws || !out_T || !dL_drgb || !grads) return MGS_ERR_INVALID_ARG;
    Setup S;
    mgs_status st = validate_and_setup(maps, n_maps, cams, n_views, info->bin_tx, info->bin_ty, S);
    if (st != MGS_OK) return st;
    for (int m = 0; m < n_maps; ++m)  // the two statistics come as a pair
        if ((grads[m].grad_norm_sum == nullptr) != (grads[m].visible_count == nullptr)) return MGS_ERR_INVALID_ARG;
    if (!info->need_backward || info->n_pairs != S.P || info->n_views != n_views || info->n_maps != n_maps ||
        info->n_bins != S.B_total)
        return MGS_ERR_INVALID_ARG;
    if (info->inst_bin_bits != 0 &&
        (info->inst_bin_bits < 1 || info->inst_bin_bits > 32 || info->inst_rank_bits < 1 ||
         info->inst_rank_bits > 32 || info->inst_bin_bits + info->inst_rank_bits + bits_for(info->n_instances) > 64))
        return MGS_ERR_INVALID_ARG;
    const int64_t Pv = info->n_visible, M = info->n_instances;
    Layout L = make_layout(S, Pv, M, true);
    if (ws_bytes < L.total) return MGS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageTimer timer(opts, s);
    timer.mark();  // 0
    uint32_t *counters = at<uint32_t>(ws, L.counters);
    k_init<<<1, 64, 0, s>>>(counters);
    const ViewDev *views = at<ViewDev>(ws, L.views);
    const mgs_render_opts defaults{};
    const mgs_render_opts &o = opts ? *opts : defaults;
    BlendBwdArgs bb;
    bb.views = views;
    bb.n_views = n_views;
    bb.n_items = S.B_total;
    bb.range = at<uint2>(ws, L.tile_range);
    bb.order = at<uint32_t>(ws, L.bin_order);
    bb.inst = instances_of(ws, *info);
    bb.rxy = at<float2>(ws, L.rank_xy);
    bb.rconic = at<float4>(ws, L.rank_conic);
    bb.rrgbd = at<float4>(ws, L.rank_rgbd);
    bb.rrect = at<ushort4>(ws, L.rank_rect);
    bb.bg0 = o.bg_rgb[0]; bb.bg1 = o.bg_rgb[1]; bb.bg2 = o.bg_rgb[2]; bb.bgd = o.bg_depth;
    bb.queues = counters + CNT_Q;
    bb.out_T = out_T;
    bb.dL_rgb = dL_drgb;
    bb.dL_depth = dL_ddepth;
    bb.n_contrib = at<uint32_t>(ws, L.n_contrib);
    bb.records = at<float>(ws, L.records);
    bb.box_cull = box_cull();
    bb.inst_qm = !split_blend(S.btx, S.bty, S.B_total) && S.btx * S.bty > 1 ? at<uint16_t>(ws, L.inst_qm) : nullptr;
    // tracking: no map asks for any Gaussian gradient or statistic
    bool pose_only = true;
    for (int m = 0; m < n_maps; ++m) {
        const mgs_gaussian_grads &gr = grads[m];
        if (gr.d_means || gr.d_scales || gr.d_quats || gr.d_opac || gr.d_sh || gr.grad_norm_sum) pose_only = false;
    }
    // where also no map's colour depends on the view (SH degree 0), the blend
    // forms only the sums the pose reads
    bool pose_blend = pose_only;
    for (int m = 0; m < n_maps; ++m)
        if (S.maps[m].sh_degree != 0) pose_blend = false;
    // few bins: four-wave blocks, one per bin, five to a CU (their LDS)
    const bool split = split_blend(S.btx, S.bty, S.B_total);
    const int64_t grid = split ? std::max<int64_t>(1, std::min<int64_t>(S.B_total, (int64_t)num_cus() * 5))
                               : blend_grid(S.B_total);
    launch_blend_bwd(split, S.btx, S.bty, (unsigned)grid, s, bb, pose_blend);
    MGS_LAUNCHED();
    timer.mark();  // 1
    // per-pair chain rule, then per-Gaussian sums over views, then the poses
    float *grad2d = at<float>(ws, L.grad2d);
    if (Pv > 0) k_rank_reduce<<<grid_of(16 * Pv, 256), 256, 0, s>>>(bb.records, at<uint32_t>(ws, L.rank_off), Pv, grad2d);
    MGS_LAUNCHED();
    float *partial = at<float>(ws, L.pose_partial);
    float *pair_grad = at<float>(ws, L.pair_grad);
    const unsigned nbp = (unsigned)L.pose_blocks;
    for (int m = 0; m < n_maps; ++m) {
        const int nv = S.map_view_off[m + 1] - S.map_view_off[m];
        PairBwdArgs pa;
        pa.views = views;
        pa.maps = at<MapDev>(ws, L.maps);
        pa.n_views = n_views;
        pa.map = m;
        pa.Pv = Pv;
        pa.rank_pair = at<uint32_t>(ws, info->off_rank_pair);
        pa.grad2d = grad2d;
        pa.pair_grad = pair_grad;
        pa.stride = L.grad_stride;
        pa.pose_partial = partial + (int64_t)m * L.pose_blocks * n_views * 9;
        pa.view_list = at<int32_t>(ws, L.vlist) + S.map_view_off[m];
        pa.n_map_views = nv;
        if (pose_only) {
            switch (S.maps[m].sh_degree) {
                case 0: k_pair_bwd<0, true><<<nbp, 256, 0, s>>>(pa); break;
                case 1: k_pair_bwd<1, true><<<nbp, 256, 0, s>>>(pa); break;
                case 2: k_pair_bwd<2, true><<<nbp, 256, 0, s>>>(pa); break;
                default: k_pair_bwd<3, true><<<nbp, 256, 0, s>>>(pa); break;
            }
        } else {
            switch (S.maps[m].sh_degree) {
                case 0: k_pair_bwd<0, false><<<nbp, 256, 0, s>>>(pa); break;
                case 1: k_pair_bwd<1, false><<<nbp, 256, 0, s>>>(pa); break;
                case 2: k_pair_bwd<2, false><<<nbp, 256, 0, s>>>(pa); break;
                default: k_pair_bwd<3, false><<<nbp, 256, 0, s>>>(pa); break;
            }
        }
        MGS_LAUNCHED();
        if (S.maps[m].n == 0 || pose_only) continue;
        GaussBwdArgs ga;
        ga.views = views;
        ga.maps = pa.maps;
        ga.map = m;
        ga.view_list = pa.view_list;
        ga.n_map_views = nv;
        ga.pair_rank = at<uint32_t>(ws, L.pair_rank);
        ga.pair_count = at<uint32_t>(ws, L.pair_count);
        ga.pair_depth = at<uint32_t>(ws, info->off_pair_depth);
        ga.pair_grad = pair_grad;
        ga.stride = L.grad_stride;
        ga.gr = grads[m];
        const unsigned nbg = grid_of(S.maps[m].n, 256);
        switch (S.maps[m].sh_degree) {
            case 0: k_gauss_bwd<0><<<nbg, 256, 0, s>>>(ga); break;
            case 1: k_gauss_bwd<1><<<nbg, 256, 0, s>>>(ga); break;
            case 2: k_gauss_bwd<2><<<nbg, 256, 0, s>>>(ga); break;
            default: k_gauss_bwd<3><<<nbg, 256, 0, s>>>(ga); break;
        }
        MGS_LAUNCHED();
    }
    if (d_pose) {
        PoseFinalArgs pf;
        pf.views = views;
        pf.n_views = n_views;
        pf.pose_partial = partial;
        pf.nb = L.pose_blocks;
        pf.d_pose = d_pose;
        k_pose_final<<<(unsigned)n_views, 256, 0, s>>>(pf);
        MGS_LAUNCHED();
    }
    timer.mark();  // 2
    static const int spans[3][3] = {{0, 0, 1}, {1, 1, 2}, {3, 0, 2}};
    timer.finish(spans, 3);
    return MGS_OK;
}
