// Mapping loss of MemGS (Sec. II-E, Eq. (12)) for gfx950: colour L1, SSIM,
// masked depth L1 and the isotropy term L_iso, value and gradient.
//
//   k_ssim_fwd    one 32x32 output tile of one colour channel per block: the
//                 tile and a 5-pixel halo of both images staged in LDS; the five
//                 window moments E[x], E[y], E[x^2], E[y^2], E[xy] by a
//                 separable 11-tap pass (rows, then columns); per pixel SSIM and
//                 its partial derivatives with respect to E[x], E[x^2] and E[xy]
//                 (written for the second pass); block sums of SSIM and |x - y|.
//                 Channel-0 blocks also form the depth residual and its gradient.
//   k_ssim_bwd    the same tiling over the three derivative maps: their window
//                 sums give d sum(SSIM) / d x, combined with the L1 subgradient.
//   k_iso         one Gaussian per thread in fp64, so that the sign of each
//                 scale's deviation from the mean scale is decided exactly.
//   k_loss_views  one block per view (and one for L_iso): fixed-order fp64 sums
//                 of the block partials; k_loss_total adds the views in order, so
//                 the loss values are deterministic.
//
// The SSIM work is a fixed 11-tap stencil, not a contraction: each pixel is
// read once per pass and the moments stay in LDS.  Memory traffic per pixel and
// channel: 8 bytes in and 12 out (first pass), 20 in and 4 out (second pass).
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "api_range.hpp"
#include "common.hpp"

namespace mgs {
namespace {

constexpr int kLT = 32;             // output tile edge (pixels)
constexpr int kLR = 5;              // window radius
constexpr int kLW = 2 * kLR + 1;    // window taps
constexpr int kLE = kLT + 2 * kLR;  // staged edge, 42
constexpr int kLP = kLE + 1;        // padded LDS row of a staged map
constexpr int kLH = kLT + 1;        // padded LDS row of a row-filtered map
constexpr int kStageRows = 256 / kLE;            // staged rows per pass of the block (6)
constexpr int kStageThreads = kStageRows * kLE;  // threads that stage (252)
constexpr int kStageIt = (kLE + kStageRows - 1) / kStageRows;  // staged rows per thread (7)
constexpr float kC1 = 1e-4f;        // (0.01)^2
constexpr float kC2 = 9e-4f;        // (0.03)^2

struct LossView {
    int32_t W, H, TXn, pad;
    int64_t tile_base;  // first tile of the view (tiles of one channel)
    int64_t pix_base;   // first pixel in the packed one-channel layout
    float inv_n3;       // 1 / (3 W H)
    float inv_n1;       // 1 / (W H)
};

struct SsimArgs {
    const LossView *views;
    int n_views;
    int64_t n_tiles;  // per channel
    int64_t P;        // pixels of all views
    const float *rgb, *gt, *depth, *gtd;
    float *maps;      // three planes of 3P floats, packed like rgb
    float *partial;   // [3][n_tiles][4]: SSIM sum, |x - y| sum, depth sum
    float *d_rgb, *d_depth;
    float lam, w_depth;
    float w[kLW];     // normalised window weights
};

__device__ __forceinline__ int view_of_tile(const LossView *views, int V, int64_t t) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float sgnf(float d) { return d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f); }

// block sums of three values (256 threads); thread 0 gets the result
__device__ __forceinline__ void block_sum3(float &a, float &b, float &c, float (*red)[4]) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
        red[2][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        b = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        c = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    }
}

// Tile origin and channel base of this block.  Workgroups are dealt to the
// eight XCDs round robin (block b on XCD b % 8); each XCD gets a contiguous run
// of tiles, so the halo a tile shares with its neighbours is read through the
// same L2.  The grid has 8 ceil(n / 8) blocks; those past the last tile exit.
struct TileAt {
    LossView V;
    int64_t tile;
    bool valid;
    int ox, oy;
    int64_t cbase;  // offset of this view's channel plane in the packed colour layout
};
__device__ __forceinline__ TileAt tile_at(const SsimArgs &a) {
    TileAt t;
    const int64_t per = (a.n_tiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    t.tile = tile;
    t.valid = tile < a.n_tiles;
    if (!t.valid) return t;
    t.V = a.views[view_of_tile(a.views, a.n_views, tile)];
    const int lt = (int)(tile - t.V.tile_base), ty = lt / t.V.TXn, tx = lt - ty * t.V.TXn;
    t.ox = tx * kLT;
    t.oy = ty * kLT;
    t.cbase = 3 * t.V.pix_base + (int64_t)blockIdx.y * t.V.W * t.V.H;
    return t;
}

__global__ __launch_bounds__(256) void k_ssim_fwd(SsimArgs a) {
    // the staged images and the row-filtered moments share the LDS: the rows
    // pass keeps its results in registers until every thread has read the images
    __shared__ float lds[5 * kLE * kLH];
    __shared__ float red[3][4];
    float(*sx)[kLP] = reinterpret_cast<float(*)[kLP]>(lds);
    float(*sy)[kLP] = reinterpret_cast<float(*)[kLP]>(lds + kLE * kLP);
    float(*hm)[kLE][kLH] = reinterpret_cast<float(*)[kLE][kLH]>(lds);
    static_assert(2 * kLE * kLP <= 5 * kLE * kLH, "staged images fit in the moments' space");
    const TileAt T = tile_at(a);
    if (!T.valid) return;  // the whole block
    const LossView &V = T.V;
    const int c = blockIdx.y, tid = threadIdx.x;
    const float *X = a.rgb + T.cbase, *Y = a.gt + T.cbase;
    float sL = 0.0f;  // |x - y| over this tile's pixels
    {
        // staging: thread t owns staged column t % 42 of rows t / 42 + 6 k; every
        // load is issued before the first wait
        const int q = tid % kLE, r0 = tid / kLE;
        const int gx = T.ox - kLR + q;
        const bool stager = tid < kStageThreads;
        const bool colok = stager && gx >= 0 && gx < V.W;
        const bool inner_col = q >= kLR && q < kLR + kLT;
        float xv[kStageIt], yv[kStageIt];
#pragma unroll
        for (int k = 0; k < kStageIt; ++k) {
            const int r = r0 + k * kStageRows, gy = T.oy - kLR + r;
            xv[k] = yv[k] = 0.0f;
            if (colok && r < kLE && gy >= 0 && gy < V.H) {
                const int64_t o = (int64_t)gy * V.W + gx;
                xv[k] = X[o];
                yv[k] = Y[o];
            }
        }
#pragma unroll
        for (int k = 0; k < kStageIt; ++k) {
            const int r = r0 + k * kStageRows;
            if (!stager || r >= kLE) continue;
            sx[r][q] = xv[k];
            sy[r][q] = yv[k];
            if (inner_col && r >= kLR && r < kLR + kLT) sL += fabsf(xv[k] - yv[k]);
        }
    }
    __syncthreads();
    // rows: the five moments filtered along x for every staged row
    constexpr int kRowIt = (kLE * kLT + 255) / 256;
    float hv[kRowIt][5];
#pragma unroll
    for (int it = 0; it < kRowIt; ++it) {
        const int i = tid + 256 * it;
        const int r = i >> 5, q = i & 31;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
        if (i < kLE * kLT) {
#pragma unroll
            for (int o = 0; o < kLW; ++o) {
                const float xv = sx[r][q + o], yv = sy[r][q + o], w = a.w[o];
                const float wx = w * xv, wy = w * yv;
                m0 += wx;
                m1 += wy;
                m2 = __builtin_fmaf(wx, xv, m2);
                m3 = __builtin_fmaf(wy, yv, m3);
                m4 = __builtin_fmaf(wx, yv, m4);
            }
        }
        hv[it][0] = m0;
        hv[it][1] = m1;
        hv[it][2] = m2;
        hv[it][3] = m3;
        hv[it][4] = m4;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRowIt; ++it) {
        const int i = tid + 256 * it;
        if (i < kLE * kLT)
#pragma unroll
            for (int k = 0; k < 5; ++k) hm[k][i >> 5][i & 31] = hv[it][k];
    }
    __syncthreads();
    // columns: thread (q, g) finishes rows 4g .. 4g+3 of column q
    const int q = tid & 31, g4 = (tid >> 5) * 4;
    float acc[4][5];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[j][k] = 0.0f;
#pragma unroll
    for (int o = 0; o < kLW + 3; ++o) {
        float h[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) h[k] = hm[k][g4 + o][q];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int tap = o - j;
            if (tap < 0 || tap >= kLW) continue;
#pragma unroll
            for (int k = 0; k < 5; ++k) acc[j][k] = __builtin_fmaf(a.w[tap], h[k], acc[j][k]);
        }
    }
    float sS = 0.0f, sD = 0.0f;
    const int64_t P3 = 3 * a.P;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = g4 + j, gx = T.ox + q, gy = T.oy + r;
        if (gx >= V.W || gy >= V.H) continue;
        const float mx = acc[j][0], my = acc[j][1];
        const float vx = acc[j][2] - mx * mx, vy = acc[j][3] - my * my, cxy = acc[j][4] - mx * my;
        const float A = 2.0f * mx * my + kC1, B = 2.0f * cxy + kC2;
        const float C = mx * mx + my * my + kC1, D = vx + vy + kC2;
        const float iA = __builtin_amdgcn_rcpf(A), iB = __builtin_amdgcn_rcpf(B);
        const float iC = __builtin_amdgcn_rcpf(C), iD = __builtin_amdgcn_rcpf(D);
        const float S = A * B * iC * iD;
        const int64_t o = (int64_t)gy * V.W + gx;
        float *M = a.maps + T.cbase + o;
        M[0] = 2.0f * S * (my * iA - mx * iC + mx * iD - my * iB);
        M[P3] = -S * iD;
        M[2 * P3] = 2.0f * S * iB;
        sS += S;
        if (c == 0 && a.depth) {
            const int64_t pix = V.pix_base + o;
            const float gd = a.gtd[pix];
            const float dd = gd > 0.0f ? a.depth[pix] - gd : 0.0f;
            sD += fabsf(dd);
            a.d_depth[pix] = a.w_depth * V.inv_n1 * sgnf(dd);
        }
    }
    block_sum3(sS, sL, sD, red);
    if (tid == 0) {
        float *p = a.partial + ((int64_t)c * a.n_tiles + T.tile) * 4;
        p[0] = sS;
        p[1] = sL;
        p[2] = sD;
        p[3] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(SsimArgs a) {
    // staged maps and their row-filtered sums share the LDS (as in k_ssim_fwd)
    __shared__ float lds[3 * kLE * kLP];
    float(*sm)[kLE][kLP] = reinterpret_cast<float(*)[kLE][kLP]>(lds);
    float(*hm)[kLE][kLH] = reinterpret_cast<float(*)[kLE][kLH]>(lds);
    const TileAt T = tile_at(a);
    if (!T.valid) return;  // the whole block
    const LossView &V = T.V;
    const int tid = threadIdx.x;
    const int64_t P3 = 3 * a.P;
    const float *M = a.maps + T.cbase;
    {
        const int q = tid % kLE, r0 = tid / kLE;
        const int gx = T.ox - kLR + q;
        const bool stager = tid < kStageThreads;
        const bool colok = stager && gx >= 0 && gx < V.W;
        float mv[kStageIt][3];
#pragma unroll
        for (int k = 0; k < kStageIt; ++k) {
            const int r = r0 + k * kStageRows, gy = T.oy - kLR + r;
            mv[k][0] = mv[k][1] = mv[k][2] = 0.0f;
            if (colok && r < kLE && gy >= 0 && gy < V.H) {
                const int64_t o = (int64_t)gy * V.W + gx;
                mv[k][0] = M[o];
                mv[k][1] = M[P3 + o];
                mv[k][2] = M[2 * P3 + o];
            }
        }
#pragma unroll
        for (int k = 0; k < kStageIt; ++k) {
            const int r = r0 + k * kStageRows;
            if (!stager || r >= kLE) continue;
            sm[0][r][q] = mv[k][0];
            sm[1][r][q] = mv[k][1];
            sm[2][r][q] = mv[k][2];
        }
    }
    __syncthreads();
    constexpr int kRowIt = (kLE * kLT + 255) / 256;
    float hv[kRowIt][3];
#pragma unroll
    for (int it = 0; it < kRowIt; ++it) {
        const int i = tid + 256 * it;
        const int r = i >> 5, q = i & 31;
        float h0 = 0.f, h1 = 0.f, h2 = 0.f;
        if (i < kLE * kLT) {
#pragma unroll
            for (int o = 0; o < kLW; ++o) {
                const float w = a.w[o];
                h0 = __builtin_fmaf(w, sm[0][r][q + o], h0);
                h1 = __builtin_fmaf(w, sm[1][r][q + o], h1);
                h2 = __builtin_fmaf(w, sm[2][r][q + o], h2);
            }
        }
        hv[it][0] = h0;
        hv[it][1] = h1;
        hv[it][2] = h2;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRowIt; ++it) {
        const int i = tid + 256 * it;
        if (i < kLE * kLT)
#pragma unroll
            for (int k = 0; k < 3; ++k) hm[k][i >> 5][i & 31] = hv[it][k];
    }
    __syncthreads();
    const int q = tid & 31, g4 = (tid >> 5) * 4;
    float acc[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0f;
#pragma unroll
    for (int o = 0; o < kLW + 3; ++o) {
        const float h0 = hm[0][g4 + o][q], h1 = hm[1][g4 + o][q], h2 = hm[2][g4 + o][q];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int tap = o - j;
            if (tap < 0 || tap >= kLW) continue;
            acc[j][0] = __builtin_fmaf(a.w[tap], h0, acc[j][0]);
            acc[j][1] = __builtin_fmaf(a.w[tap], h1, acc[j][1]);
            acc[j][2] = __builtin_fmaf(a.w[tap], h2, acc[j][2]);
        }
    }
    const float kl1 = (1.0f - a.lam) * V.inv_n3, ks = a.lam * V.inv_n3;
    const float *X = a.rgb + T.cbase, *Y = a.gt + T.cbase;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int gx = T.ox + q, gy = T.oy + g4 + j;
        if (gx >= V.W || gy >= V.H) continue;
        const int64_t o = (int64_t)gy * V.W + gx;
        const float x = X[o], y = Y[o];
        const float gs = acc[j][0] + 2.0f * x * acc[j][1] + y * acc[j][2];
        a.d_rgb[T.cbase + o] = kl1 * sgnf(x - y) - ks * gs;
    }
}

__device__ __forceinline__ double sgnd(double d) { return d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0); }

__device__ __forceinline__ double wave_sum_f64(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// L_iso per Gaussian: deviations of the three scales from their mean
__global__ __launch_bounds__(256) void k_iso(const float *scales, int64_t n, float w_iso, float *d_scales,
                                             double *partial) {
    __shared__ double red[4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (g < n) {
        const double s0 = scales[3 * g], s1 = scales[3 * g + 1], s2 = scales[3 * g + 2];
        const double m = (s0 + s1 + s2) / 3.0;
        const double e0 = s0 - m, e1 = s1 - m, e2 = s2 - m;
        acc = fabs(e0) + fabs(e1) + fabs(e2);
        const double g0 = sgnd(e0), g1 = sgnd(e1), g2 = sgnd(e2);
        const double mg = (g0 + g1 + g2) / 3.0;
        const double k = (double)w_iso / (3.0 * (double)n);
        d_scales[3 * g] = (float)(k * (g0 - mg));
        d_scales[3 * g + 1] = (float)(k * (g1 - mg));
        d_scales[3 * g + 2] = (float)(k * (g2 - mg));
    }
    acc = wave_sum_f64(acc);
    if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

struct FinalArgs {
    const LossView *views;
    int n_views;
    int64_t n_tiles;
    const float *partial;
    const double *iso_partial;
    int64_t n_iso_blocks;
    int64_t n_gauss;
    float lam, w_depth, w_iso;
    int has_depth;
    double *terms;  // [n_views + 1]: L_view of each view, then L_iso
    float *loss;    // [4 n_views + 2]
};

__device__ __forceinline__ double block_sum_f64(double x, double *red) {
    x = wave_sum_f64(x);
    if (lane_id() == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    const double r = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return r;
}

// block v < n_views: the terms of view v; block n_views: L_iso
__global__ __launch_bounds__(256) void k_loss_views(FinalArgs a) {
    __shared__ double red[4];
    const int tid = threadIdx.x, v = blockIdx.x;
    if (v == a.n_views) {
        double si = 0.0;
        for (int64_t b = tid; b < a.n_iso_blocks; b += 256) si += a.iso_partial[b];
        si = block_sum_f64(si, red);
        const double liso = a.n_gauss > 0 ? (double)a.w_iso * si / (3.0 * (double)a.n_gauss) : 0.0;
        if (tid == 0) {
            a.terms[v] = liso;
            a.loss[4 * v] = (float)liso;
        }
        return;
    }
    const LossView V = a.views[v];
    const int64_t t1 = v + 1 < a.n_views ? a.views[v + 1].tile_base : a.n_tiles;
    const int64_t nt = t1 - V.tile_base;
    double sS = 0.0, sL = 0.0, sD = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int64_t t = tid; t < nt; t += 256) {
            const float4 p = *reinterpret_cast<const float4 *>(a.partial + ((int64_t)c * a.n_tiles + V.tile_base + t) * 4);
            sS += p.x;
            sL += p.y;
            sD += p.z;
        }
    sS = block_sum_f64(sS, red);
    sL = block_sum_f64(sL, red);
    sD = block_sum_f64(sD, red);
    if (tid == 0) {
        const double npx = (double)V.W * (double)V.H;
        const double l1 = sL / (3.0 * npx), ssim = sS / (3.0 * npx), ld = a.has_depth ? sD / npx : 0.0;
        const double lv = (1.0 - a.lam) * l1 + a.lam * (1.0 - ssim) + (a.has_depth ? a.w_depth * ld : 0.0);
        a.terms[v] = lv;
        a.loss[4 * v] = (float)l1;
        a.loss[4 * v + 1] = (float)ssim;
        a.loss[4 * v + 2] = (float)ld;
        a.loss[4 * v + 3] = (float)lv;
    }
}

// the total, summed in view order
__global__ void k_loss_total(const double *terms, int n_views, float *loss) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int v = 0; v <= n_views; ++v) t += terms[v];
    loss[4 * n_views + 1] = (float)t;
}

}  // namespace
}  // namespace mgs

using namespace mgs;

namespace {

mgs_status loss_check(const int32_t *sizes, int32_t n_views, const float *rgb, const float *gt_rgb,
                      const float *depth, const float *gt_depth, const float *scales, int64_t n_gauss,
                      const mgs_loss_opts *opts, const float *loss, const float *dL_drgb, const float *dL_ddepth,
                      const float *dL_dscales) {
    if (!sizes || !opts || !rgb || !gt_rgb || !loss || !dL_drgb) return MGS_ERR_INVALID_ARG;
    if (n_views <= 0 || n_views > 4096 || n_gauss < 0) return MGS_ERR_INVALID_ARG;
    if ((depth == nullptr) != (gt_depth == nullptr) || (depth && !dL_ddepth)) return MGS_ERR_INVALID_ARG;
    if (scales && n_gauss > 0 && !dL_dscales) return MGS_ERR_INVALID_ARG;
    if (!std::isfinite(opts->lambda_ssim) || !std::isfinite(opts->w_depth) || !std::isfinite(opts->w_iso))
        return MGS_ERR_INVALID_ARG;
    if (n_gauss >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    for (int v = 0; v < n_views; ++v) {
        const int32_t W = sizes[2 * v], H = sizes[2 * v + 1];
        if (W < 1 || H < 1 || W > 16384 || H > 16384) return MGS_ERR_INVALID_ARG;
    }
    return MGS_OK;
}

// The loss after the argument checks.  views: host room for n_views entries.
// ws == nullptr with ws_bytes == 0 only sizes the call (*ws_required).
mgs_status loss_run(const int32_t *sizes, int32_t n_views, const float *rgb, const float *gt_rgb,
                    const float *depth, const float *gt_depth, const float *scales, int64_t n_gauss,
                    const mgs_loss_opts *opts, LossView *views, void *ws, size_t ws_bytes, size_t *ws_required,
                    float *loss, float *dL_drgb, float *dL_ddepth, float *dL_dscales, void *stream) {
    int64_t tiles = 0, P = 0;
    for (int v = 0; v < n_views; ++v) {
        const int32_t W = sizes[2 * v], H = sizes[2 * v + 1];
        LossView &L = views[v];
        L.W = W;
        L.H = H;
        L.TXn = (int32_t)ceil_div(W, kLT);
        L.pad = 0;
        L.tile_base = tiles;
        L.pix_base = P;
        L.inv_n3 = (float)(1.0 / (3.0 * (double)W * (double)H));
        L.inv_n1 = (float)(1.0 / ((double)W * (double)H));
        tiles += (int64_t)L.TXn * ceil_div(H, kLT);
        P += (int64_t)W * H;
    }
    if (tiles >= (int64_t(1) << 31) - 8) return MGS_ERR_TOO_LARGE;
    const bool iso = scales != nullptr && n_gauss > 0;
    const int64_t n_iso = iso ? ceil_div(n_gauss, 256) : 0;
    Bump b;
    const size_t off_views = b.take(sizeof(LossView) * (size_t)n_views);
    const size_t off_maps = b.take(4 * (size_t)9 * (size_t)P);
    const size_t off_part = b.take(4 * (size_t)12 * (size_t)tiles);
    const size_t off_iso = b.take(8 * (size_t)std::max<int64_t>(n_iso, 1));
    const size_t off_terms = b.take(8 * (size_t)(n_views + 1));
    *ws_required = b.size();
    if (ws_bytes < b.size() || !ws) return MGS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    static_assert(sizeof(LossView) % 4 == 0, "views are copied as words");
    const size_t view_bytes = sizeof(LossView) * (size_t)n_views;
    if (view_bytes <= 4 * (size_t)kArgCopyWords) {
        ArgWords aw;
        memcpy(aw.w, views, view_bytes);
        aw.n = (int32_t)(view_bytes / 4);
        k_arg_copy<<<1, 256, 0, s>>>(aw, at<uint32_t>(ws, off_views));
        MGS_LAUNCHED();
    } else {
        MGS_HIP(hipMemcpyAsync(at<void>(ws, off_views), views, view_bytes, hipMemcpyHostToDevice, s));
    }
    SsimArgs a;
    a.views = at<LossView>(ws, off_views);
    a.n_views = n_views;
    a.n_tiles = tiles;
    a.P = P;
    a.rgb = rgb;
    a.gt = gt_rgb;
    a.depth = depth;
    a.gtd = gt_depth;
    a.maps = at<float>(ws, off_maps);
    a.partial = at<float>(ws, off_part);
    a.d_rgb = dL_drgb;
    a.d_depth = dL_ddepth;
    a.lam = opts->lambda_ssim;
    a.w_depth = opts->w_depth;
    {
        double w[kLW], sum = 0.0;
        for (int o = 0; o < kLW; ++o) {
            const double d = (double)(o - kLR);
            w[o] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
            sum += w[o];
        }
        for (int o = 0; o < kLW; ++o) a.w[o] = (float)(w[o] / sum);
    }
    const dim3 grid((unsigned)(8 * ceil_div(tiles, 8)), 3);
    k_ssim_fwd<<<grid, 256, 0, s>>>(a);
    MGS_LAUNCHED();
    k_ssim_bwd<<<grid, 256, 0, s>>>(a);
    MGS_LAUNCHED();
    double *iso_part = at<double>(ws, off_iso);
    if (iso) {
        k_iso<<<(unsigned)n_iso, 256, 0, s>>>(scales, n_gauss, opts->w_iso, dL_dscales, iso_part);
        MGS_LAUNCHED();
    }
    FinalArgs f;
    f.views = a.views;
    f.n_views = n_views;
    f.n_tiles = tiles;
    f.partial = a.partial;
    f.iso_partial = iso_part;
    f.n_iso_blocks = n_iso;
    f.n_gauss = iso ? n_gauss : 0;
    f.lam = opts->lambda_ssim;
    f.w_depth = opts->w_depth;
    f.w_iso = opts->w_iso;
    f.has_depth = depth != nullptr;
    f.terms = at<double>(ws, off_terms);
    f.loss = loss;
    k_loss_views<<<(unsigned)n_views + 1, 256, 0, s>>>(f);
    MGS_LAUNCHED();
    k_loss_total<<<1, 64, 0, s>>>(f.terms, n_views, loss);
    MGS_LAUNCHED();
    return MGS_OK;
}

}  // namespace

extern "C" mgs_status mgs_mapping_loss(const int32_t *sizes, int32_t n_views, const float *rgb, const float *gt_rgb,
                                       const float *depth, const float *gt_depth, const float *scales,
                                       int64_t n_gauss, const mgs_loss_opts *opts, void *ws, size_t ws_bytes,
                                       size_t *ws_required, float *loss, float *dL_drgb, float *dL_ddepth,
                                       float *dL_dscales, void *stream) {
    ApiRange api_range("mgs_mapping_loss");
    if (!ws_required) return MGS_ERR_INVALID_ARG;
    const mgs_status st = loss_check(sizes, n_views, rgb, gt_rgb, depth, gt_depth, scales, n_gauss, opts, loss,
                                     dL_drgb, dL_ddepth, dL_dscales);
    if (st != MGS_OK) return st;
    std::vector<LossView> views((size_t)n_views);
    return loss_run(sizes, n_views, rgb, gt_rgb, depth, gt_depth, scales, n_gauss, opts, views.data(), ws,
                    ws_bytes, ws_required, loss, dL_drgb, dL_ddepth, dL_dscales, stream);
}

// ------------------------------------------------------- allocation-free entry
// The scratch of mgs_mapping_loss_noalloc: a fixed device array, one copy per
// GPU, held from the module's load until the process ends.  Host code never
// passes its name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device on the entry point's first call
// there.  Every call on one GPU shares the array: calls that overlap on one GPU
// (on different streams or host threads without ordering) race.  Nothing in it
// needs to start at zero: every kernel of the loss writes the scratch it later
// reads in the same call.
static __device__ __align__(256) unsigned char scratch[MGS_LOSS_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
std::atomic<void *> g_scratch_ptr[kScratchDevices];

// Device address of `scratch` on device `dev` (the current device).
mgs_status scratch_on(int dev, void **ptr) {
    if (dev < 0 || dev >= kScratchDevices) return MGS_ERR_INVALID_ARG;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            MGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) return MGS_ERR_HIP;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *ptr = p;
    return MGS_OK;
}
}  // namespace

extern "C" mgs_status mgs_mapping_loss_noalloc(const int32_t *sizes, int32_t n_views, const float *rgb,
                                               const float *gt_rgb, const float *depth, const float *gt_depth,
                                               const float *scales, int64_t n_gauss, const mgs_loss_opts *opts,
                                               size_t *scratch_required, float *loss, float *dL_drgb,
                                               float *dL_ddepth, float *dL_dscales, void *stream) {
    ApiRange api_range("mgs_mapping_loss_noalloc");
    const mgs_status st = loss_check(sizes, n_views, rgb, gt_rgb, depth, gt_depth, scales, n_gauss, opts, loss,
                                     dL_drgb, dL_ddepth, dL_dscales);
    if (st != MGS_OK) return st;
    if (n_views > MGS_LOSS_NOALLOC_MAX_VIEWS) return MGS_ERR_SCRATCH;
    // few enough views for the view table to travel in kernel arguments: no
    // host-to-device copy
    static_assert(sizeof(LossView) * MGS_LOSS_NOALLOC_MAX_VIEWS <= 4 * (size_t)kArgCopyWords, "view table");
    LossView views[MGS_LOSS_NOALLOC_MAX_VIEWS];
    // size the call first: nothing is launched when it does not fit
    size_t need = 0;
    mgs_status r = loss_run(sizes, n_views, rgb, gt_rgb, depth, gt_depth, scales, n_gauss, opts, views, nullptr, 0,
                            &need, loss, dL_drgb, dL_ddepth, dL_dscales, stream);
    if (r != MGS_ERR_WORKSPACE) return r == MGS_OK ? MGS_ERR_HIP : r;
    if (scratch_required) *scratch_required = need;
    if (need > (size_t)MGS_LOSS_SCRATCH_BYTES) return MGS_ERR_SCRATCH;
    int dev = -1;
    MGS_HIP(hipGetDevice(&dev));
    if (stream) {
        int sdev = -1;
        MGS_HIP(hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev));
        if (sdev != dev) return MGS_ERR_INVALID_ARG;
    }
    void *ws = nullptr;
    r = scratch_on(dev, &ws);
    if (r != MGS_OK) return r;
    return loss_run(sizes, n_views, rgb, gt_rgb, depth, gt_depth, scales, n_gauss, opts, views, ws,
                    (size_t)MGS_LOSS_SCRATCH_BYTES, &need, loss, dL_drgb, dL_ddepth, dL_dscales, stream);
}
