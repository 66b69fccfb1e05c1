// Patch-Grid sampling of MemGS (Sec. II-B) for gfx950: new Gaussians from a
// keyframe's keypoints and from uniform samples in the patches where
// keypoints are sparse.
//
//   k_pg_count    one thread per keypoint: its pixel (floor(u + 1/2)) and
//                 patch; integer atomics count the keypoints of each patch
//                 (exact, so the counts do not depend on the order)
//   k_pg_resolve  one thread per candidate (the keypoints, then the s x s
//                 lattice of every patch): whether it is kept, and its depth
//                 when it has its own or the depth map gives one
//   k_pg_nearest  one wave per kept candidate still without a depth: the
//                 nearest keypoint with depth by a brute-force scan split over
//                 the lanes (fp32 squared distances, ties to the lower index)
//   scan          order-preserving compaction of the kept candidates
//   k_pg_write    back-projection through the pose and the new Gaussians'
//                 attributes (colour from the image, isotropic scale from the
//                 depth and the sample spacing)
// The nearest-keypoint search costs (candidates needing it) x (keypoints)
// fp32 distance evaluations, 64 lanes per candidate; keyframes hold a few
// thousand keypoints.
#include <cmath>

#include "api_range.hpp"
#include "common.hpp"
#include "scan.hpp"

namespace mgs {
namespace {

constexpr float kShC0 = 0.28209479177387814f;

struct PgArgs {
    int W, H, P, s, PX, PY, min_kp;
    int64_t n_kp, n_cand;
    const float *kp;        // [n_kp][2]
    const float *kp_depth;  // [n_kp]
    const float *depth_map; // [H][W] or null
    const float *image;     // [3][H][W]
    uint32_t *counts;       // [PX * PY]
    float *cand_z;          // [n_cand]: depth, 0 when dropped
};

// pixel of a keypoint, and whether it lies on the image
__device__ __forceinline__ bool kp_pixel(const PgArgs &a, int64_t i, int &x, int &y) {
    const float fx = floorf(a.kp[2 * i] + 0.5f), fy = floorf(a.kp[2 * i + 1] + 0.5f);
    if (!(fx >= 0.0f && fx < (float)a.W && fy >= 0.0f && fy < (float)a.H)) return false;  // NaN: false
    x = (int)fx;
    y = (int)fy;
    return true;
}

// pixel of lattice sample `lat` of patch `p` (over the patch's part of the image)
__device__ __forceinline__ void sample_pixel(const PgArgs &a, int64_t p, int lat, int &x, int &y) {
    const int py = (int)(p / a.PX), px = (int)(p - (int64_t)py * a.PX);
    const int l = lat / a.s, k = lat - l * a.s;
    const int w = min(a.P, a.W - a.P * px), h = min(a.P, a.H - a.P * py);
    x = a.P * px + ((2 * k + 1) * w) / (2 * a.s);
    y = a.P * py + ((2 * l + 1) * h) / (2 * a.s);
}

__global__ __launch_bounds__(256) void k_pg_fill(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_pg_count(PgArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_kp) return;
    int x, y;
    if (kp_pixel(a, i, x, y)) atomicAdd(a.counts + (int64_t)(y / a.P) * a.PX + x / a.P, 1u);
}

// candidate depth still to be found by the nearest-keypoint search
constexpr float kNeedSearch = -1.0f;

__global__ __launch_bounds__(256) void k_pg_resolve(PgArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cand) return;
    bool keep = false;
    float z = 0.0f;
    int x = 0, y = 0;
    if (c < a.n_kp) {
        keep = kp_pixel(a, c, x, y);
        if (keep) {
            const float own = a.kp_depth[c];
            z = own > 0.0f ? own : 0.0f;
        }
    } else {
        const int64_t j = c - a.n_kp, ss = (int64_t)a.s * a.s;
        const int64_t p = j / ss;
        keep = a.counts[p] < (uint32_t)a.min_kp;
        if (keep) sample_pixel(a, p, (int)(j - p * ss), x, y);
    }
    if (keep && z <= 0.0f && a.depth_map) {
        const float dm = a.depth_map[(int64_t)y * a.W + x];
        z = dm > 0.0f ? dm : 0.0f;
    }
    a.cand_z[c] = !keep ? 0.0f : (z > 0.0f ? z : kNeedSearch);
}

// One wave per candidate still without a depth: the lanes split the keypoints
// (lane l takes l, l + 64, ...), keep their nearest with depth (fp32 squared
// distance, the first of equal ones), and a lexicographic (distance, index)
// minimum over the wave gives the nearest, ties to the lower index.
__global__ __launch_bounds__(256) void k_pg_nearest(PgArgs a) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (c >= a.n_cand) return;
    if (a.cand_z[c] != kNeedSearch) return;  // wave-uniform
    float qx, qy;
    if (c < a.n_kp) {
        qx = a.kp[2 * c];
        qy = a.kp[2 * c + 1];
    } else {
        const int64_t j = c - a.n_kp, ss = (int64_t)a.s * a.s;
        const int64_t p = j / ss;
        int x, y;
        sample_pixel(a, p, (int)(j - p * ss), x, y);
        qx = (float)x;
        qy = (float)y;
    }
    float best = INFINITY;
    int arg = (int)a.n_kp;  // none (n_kp < 2^31)
    for (int i = lane_id(); i < (int)a.n_kp; i += 64) {
        if (!(a.kp_depth[i] > 0.0f)) continue;
        const float dx = qx - a.kp[2 * i], dy = qy - a.kp[2 * i + 1];
        const float d2 = dx * dx + dy * dy;
        if (d2 < best) {
            best = d2;
            arg = i;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int oa = __shfl_xor(arg, off, 64);
        if (ob < best || (ob == best && oa < arg)) {
            best = ob;
            arg = oa;
        }
    }
    if (lane_id() == 0) a.cand_z[c] = arg < a.n_kp ? a.kp_depth[arg] : 0.0f;
}

struct LoadKept {
    const float *z;
    __device__ uint32_t operator()(int64_t i) const { return z[i] > 0.0f ? 1u : 0u; }
};

struct PgWrite {
    PgArgs a;
    float R[9], t[3];
    float fx, fy, cx, cy;
    float opacity, scale_mul;  // scale = scale_mul * depth, scale_mul = factor * (P / s) / fx
    mgs_gaussians_out out;
    int32_t *source;
    __device__ void operator()(int64_t c, uint32_t o, uint32_t kept) const {
        if (!kept) return;
        int x, y;
        float qx, qy;
        if (c < a.n_kp) {
            kp_pixel(a, c, x, y);
            qx = a.kp[2 * c];
            qy = a.kp[2 * c + 1];
        } else {
            const int64_t j = c - a.n_kp, ss = (int64_t)a.s * a.s;
            const int64_t p = j / ss;
            sample_pixel(a, p, (int)(j - p * ss), x, y);
            qx = (float)x;
            qy = (float)y;
        }
        const float z = a.cand_z[c];
        const float pc[3] = {z * (qx - cx) / fx - t[0], z * (qy - cy) / fy - t[1], z - t[2]};
        for (int k = 0; k < 3; ++k) out.means[3 * o + k] = R[k] * pc[0] + R[3 + k] * pc[1] + R[6 + k] * pc[2];
        const float sig = scale_mul * z;
        for (int k = 0; k < 3; ++k) out.scales[3 * o + k] = sig;
        out.quats[4 * o] = 1.0f;
        out.quats[4 * o + 1] = out.quats[4 * o + 2] = out.quats[4 * o + 3] = 0.0f;
        out.opac[o] = opacity;
        const int64_t plane = (int64_t)a.W * a.H, pix = (int64_t)y * a.W + x;
        for (int k = 0; k < 3; ++k) out.sh[3 * o + k] = (a.image[k * plane + pix] - 0.5f) / kShC0;
        if (source) source[o] = (int32_t)c;
    }
};

}  // namespace
}  // namespace mgs

using namespace mgs;

extern "C" mgs_status mgs_patch_grid_sample(const mgs_camera *cam, const float *keypoints, const float *kp_depth,
                                            int64_t n_kp, const float *depth_map, const float *image,
                                            const mgs_pg_opts *opts, mgs_gaussians_out *out, int32_t *source,
                                            void *ws, size_t ws_bytes, size_t *ws_required, int64_t *n_out,
                                            void *stream) {
    ApiRange api_range("mgs_patch_grid_sample");
    if (!cam || !opts || !out || !ws_required || !n_out || !image) return MGS_ERR_INVALID_ARG;
    if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384) return MGS_ERR_INVALID_ARG;
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
        return MGS_ERR_INVALID_ARG;
    if (opts->patch < 1 || opts->samples < 1 || opts->samples > 64 || opts->min_keypoints < 0)
        return MGS_ERR_INVALID_ARG;
    if (!std::isfinite(opts->opacity) || !std::isfinite(opts->scale_factor)) return MGS_ERR_INVALID_ARG;
    if (n_kp < 0 || (n_kp > 0 && (!keypoints || !kp_depth))) return MGS_ERR_INVALID_ARG;
    if (!out->means || !out->scales || !out->quats || !out->opac || !out->sh) return MGS_ERR_INVALID_ARG;
    PgArgs a;
    a.W = cam->width;
    a.H = cam->height;
    a.P = opts->patch;
    a.s = opts->samples;
    a.PX = (int)ceil_div(a.W, a.P);
    a.PY = (int)ceil_div(a.H, a.P);
    a.min_kp = opts->min_keypoints;
    a.n_kp = n_kp;
    const int64_t n_patch = (int64_t)a.PX * a.PY;
    a.n_cand = n_kp + n_patch * a.s * a.s;
    if (a.n_cand >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    Bump b;
    const size_t off_counts = b.take(4 * (size_t)n_patch);
    const size_t off_z = b.take(4 * (size_t)a.n_cand);
    const size_t off_tmp = b.take(4 * (size_t)scan_tmp_words(a.n_cand));
    const size_t off_total = b.take(4);
    *ws_required = b.size();
    *n_out = 0;
    if (ws_bytes < b.size() || !ws) return MGS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    a.kp = keypoints;
    a.kp_depth = kp_depth;
    a.depth_map = depth_map;
    a.image = image;
    a.counts = at<uint32_t>(ws, off_counts);
    a.cand_z = at<float>(ws, off_z);
    k_pg_fill<<<(unsigned)ceil_div(n_patch, 256), 256, 0, s>>>(a.counts, n_patch);
    if (n_kp > 0) k_pg_count<<<(unsigned)ceil_div(n_kp, 256), 256, 0, s>>>(a);
    k_pg_resolve<<<(unsigned)ceil_div(a.n_cand, 256), 256, 0, s>>>(a);
    if (n_kp > 0) k_pg_nearest<<<(unsigned)ceil_div(a.n_cand, 4), 256, 0, s>>>(a);
    MGS_LAUNCHED();
    PgWrite w;
    w.a = a;
    for (int k = 0; k < 9; ++k) w.R[k] = cam->Tcw[4 * (k / 3) + k % 3];
    for (int k = 0; k < 3; ++k) w.t[k] = cam->Tcw[4 * k + 3];
    w.fx = cam->fx;
    w.fy = cam->fy;
    w.cx = cam->cx;
    w.cy = cam->cy;
    w.opacity = opts->opacity;
    w.scale_mul = (float)((double)opts->scale_factor * ((double)a.P / a.s) / (double)cam->fx);
    w.out = *out;
    w.source = source;
    // the kept count: to the host's mailbox word 9 when there is one
    const Mailbox mail = host_mailbox();
    uint32_t *total = mail.dev ? mail.dev + 9 : at<uint32_t>(ws, off_total);
    MGS_HIP(scan_exclusive(LoadKept{a.cand_z}, w, a.n_cand, at<uint32_t>(ws, off_tmp), total, s));
    uint32_t hn = 0;
    if (mail.host) {
        const uint32_t ticket = mailbox_ticket();
        k_mail_done<<<1, 1, 0, s>>>(mail.dev, ticket);
        MGS_LAUNCHED();
        MGS_HIP(mailbox_wait(mail, ticket, s));
        hn = static_cast<const volatile uint32_t *>(mail.host)[9];
    } else {
        MGS_HIP(hipMemcpyAsync(&hn, total, 4, hipMemcpyDeviceToHost, s));
        MGS_HIP(hipStreamSynchronize(s));
    }
    *n_out = hn;
    return MGS_OK;
}
