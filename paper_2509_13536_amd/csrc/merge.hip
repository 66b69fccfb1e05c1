// Voxel-space merging of similar Gaussians (MemGS Sec. II-D) for gfx950.
//
//   k_vcells      per Gaussian: eligibility (mask, finite mean, cell range),
//                 voxel cell floor(mean / v) in fp32, per-axis min/max
//   -- one device-to-host copy: eligible count, cell bounds --
//   k_vpack       packed compact key (cell - min, x most significant) of the
//                 eligible Gaussians, compacted by a scan
//   voxel sort    stable radix sort by key => voxels contiguous, members in
//                 index (insertion) order
//   k_voxels      one thread per voxel: sequential insertion with the squared
//                 Mahalanobis test of Eq. (4) against chi2, merged mean of
//                 Eq. (6), merged covariance minimising Eq. (9) (closed-form
//                 W2 barycenter), (q, s) by a Jacobi eigen-decomposition
//                 canonicalised towards slerp(q_i, q_j, 1/2) of Eq. (10);
//                 opacity and colour stay those of the older Gaussian
//   compaction    scan of survivors and a gather of every attribute
//   -- one device-to-host copy: survivor count --
#include <algorithm>
#include <cmath>

#include "api_range.hpp"
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace mgs {

constexpr int kCellBias = 1 << 20;

struct CellArgs {
    const float *means;
    const uint8_t *mask;
    int64_t n;
    float voxel;
    int32_t *cells;     // [n][3]
    uint32_t *elig;     // [n]
    int32_t *partial;   // [blocks][8]: min xyz, max xyz, eligible count
    uint64_t *voxel_key;
};

__global__ void k_mfill(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_vcells(CellArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = false;
    int c[3] = {0, 0, 0};
    if (g < a.n) {
        ok = a.mask ? a.mask[g] != 0 : true;
        for (int k = 0; k < 3; ++k) {
            const float q = floorf(a.means[3 * g + k] / a.voxel);  // correctly rounded division
            if (!(q >= -(float)kCellBias && q < (float)kCellBias)) ok = false;  // also rejects NaN / inf
            c[k] = ok ? (int)q : 0;
        }
        if (!ok) c[0] = c[1] = c[2] = 0;
        a.cells[3 * g] = c[0];
        a.cells[3 * g + 1] = c[1];
        a.cells[3 * g + 2] = c[2];
        a.elig[g] = ok ? 1u : 0u;
        if (a.voxel_key) {
            a.voxel_key[g] = ok ? (((uint64_t)(c[0] + kCellBias) << 42) | ((uint64_t)(c[1] + kCellBias) << 21) |
                                   (uint64_t)(c[2] + kCellBias))
                                : ~0ull;
        }
    }
    // block min/max of eligible cells and eligible count
    __shared__ int smin[3][4], smax[3][4];
    __shared__ uint32_t scnt[4];
    int mn[3], mx[3];
    for (int k = 0; k < 3; ++k) {
        mn[k] = ok ? c[k] : INT32_MAX;
        mx[k] = ok ? c[k] : INT32_MIN;
    }
    uint32_t cnt = ok ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) {
        for (int k = 0; k < 3; ++k) {
            mn[k] = min(mn[k], __shfl_xor(mn[k], off, 64));
            mx[k] = max(mx[k], __shfl_xor(mx[k], off, 64));
        }
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        for (int k = 0; k < 3; ++k) { smin[k][w] = mn[k]; smax[k][w] = mx[k]; }
        scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int ww = 0; ww < 4; ++ww) t += scnt[ww];
        int32_t *out = a.partial + 8 * (int64_t)blockIdx.x;
        for (int k = 0; k < 3; ++k) {
            int lo = smin[k][0], hi = smax[k][0];
            for (int ww = 1; ww < 4; ++ww) { lo = min(lo, smin[k][ww]); hi = max(hi, smax[k][ww]); }
            out[k] = lo;
            out[3 + k] = hi;
        }
        out[6] = (int32_t)t;
    }
}

// Voxels ordered by member count (k_vcount, k_vplace below): classes of
// 2 .. kLongVoxel members, their sizes and cursors after the counters.
constexpr int kLongVoxel = 16;
constexpr int kVoxClasses = 16;  // kLongVoxel - 1 used (2 .. kLongVoxel members)
// bookkeeping words after the counters: class sizes, then class cursors
constexpr int kVoxBookWords = 2 * kVoxClasses;
// at most this many long voxels get a wave of their own
constexpr int64_t kLongWavesMax = 1024;

// One block folds the per-block partials into bounds[0..5] and count[0].
__global__ __launch_bounds__(256) void k_bounds(const int32_t *partial, int64_t nb, int32_t *bounds, uint32_t *count,
                                                uint32_t *mail, uint32_t ticket) {
    __shared__ int32_t s[7][256];
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    uint32_t c = 0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) {
        const int32_t *p = partial + 8 * b;
        for (int k = 0; k < 3; ++k) { lo[k] = min(lo[k], p[k]); hi[k] = max(hi[k], p[3 + k]); }
        c += (uint32_t)p[6];
    }
    for (int k = 0; k < 3; ++k) { s[k][threadIdx.x] = lo[k]; s[3 + k][threadIdx.x] = hi[k]; }
    s[6][threadIdx.x] = (int32_t)c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = min(s[k][threadIdx.x], s[k][threadIdx.x + st]);
                s[3 + k][threadIdx.x] = max(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + st]);
            }
            s[6][threadIdx.x] += s[6][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < kVoxBookWords) count[8 + threadIdx.x] = 0;  // the voxel order's bookkeeping
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) bounds[k] = s[k][0];
        count[0] = (uint32_t)s[6][0];
        count[1] = 0;
        if (mail) {  // the host's copy: the bounds at words 0-5, the count at word 8
            for (int k = 0; k < 6; ++k) mail[k] = (uint32_t)s[k][0];
            mail[8] = (uint32_t)s[6][0];
            mail_flag(mail, ticket);
        }
    }
}

struct LoadElig {
    const uint32_t *e;
    __device__ uint32_t operator()(int64_t i) const { return e[i]; }
};
// K: uint32_t when the packed key fits 32 bits (a room at 5 cm: about 21), else uint64_t
template <class K>
struct StorePacked {
    const int32_t *cells;
    int32_t mnx, mny, mnz;
    int by, bz;
    K *keys;
    uint32_t *vals;
    __device__ void operator()(int64_t g, uint32_t ex, uint32_t v) const {
        if (!v) return;
        const uint64_t x = (uint64_t)(cells[3 * g] - mnx), y = (uint64_t)(cells[3 * g + 1] - mny),
                       z = (uint64_t)(cells[3 * g + 2] - mnz);
        keys[ex] = (K)((x << (by + bz)) | (y << bz) | z);
        vals[ex] = (uint32_t)g;
    }
};

// ---------------------------------------------------------------- 3x3 helpers (fp32)
// Values here decide no integer (the Eq. (4) test compares against chi2 with a
// margin far above fp32 rounding), so the native 1-ulp reciprocal and square
// root are used, and multiply-adds contract to FMAs (the library is built with
// contraction off for the rasteriser's key path; the merge's algebra turns it
// back on, function by function, which also shortens its dependent chains).
#define MGS_CONTRACT _Pragma("clang fp contract(fast)")
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct M3 {
    float a[9];
};

__device__ __forceinline__ M3 mul(const M3 &A, const M3 &B) {
    MGS_CONTRACT
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.a[3 * i + j] = A.a[3 * i] * B.a[j] + A.a[3 * i + 1] * B.a[3 + j] + A.a[3 * i + 2] * B.a[6 + j];
    return C;
}

// A^T B
__device__ __forceinline__ M3 mul_tn(const M3 &A, const M3 &B) {
    MGS_CONTRACT
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.a[3 * i + j] = A.a[i] * B.a[j] + A.a[3 + i] * B.a[3 + j] + A.a[6 + i] * B.a[6 + j];
    return C;
}

// R diag(d) R^T
__device__ __forceinline__ M3 rdrt(const M3 &R, const float *d) {
    MGS_CONTRACT
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.a[3 * i + j] = R.a[3 * i] * d[0] * R.a[3 * j] + R.a[3 * i + 1] * d[1] * R.a[3 * j + 1] +
                             R.a[3 * i + 2] * d[2] * R.a[3 * j + 2];
    return C;
}

__device__ __forceinline__ M3 rot_of(const float *q) {  // unit (w, x, y, z)
    MGS_CONTRACT
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    M3 R;
    R.a[0] = 1 - 2 * (y * y + z * z); R.a[1] = 2 * (x * y - w * z);     R.a[2] = 2 * (x * z + w * y);
    R.a[3] = 2 * (x * y + w * z);     R.a[4] = 1 - 2 * (x * x + z * z); R.a[5] = 2 * (y * z - w * x);
    R.a[6] = 2 * (x * z - w * y);     R.a[7] = 2 * (y * z + w * x);     R.a[8] = 1 - 2 * (x * x + y * y);
    return R;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3: A = V diag(lam) V^T.
// The matrix is kept as its six distinct entries: a rotation in the (p, q)
// plane with t = tan of its angle (the root of t^2 + 2 theta t - 1 of smaller
// magnitude, theta = (a_qq - a_pp) / (2 a_pq)) sets a_pq to zero and moves the
// diagonal by -+ t a_pq; only the third row's two entries turn.
__device__ void jacobi3(M3 A, float *lam, M3 &V) {
    MGS_CONTRACT
    float a00 = A.a[0], a01 = A.a[1], a02 = A.a[2], a11 = A.a[4], a12 = A.a[5], a22 = A.a[8];
#pragma unroll
    for (int i = 0; i < 9; ++i) V.a[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    // rotation in the (p, q) plane; r is the third index
    auto rot = [&](float &app, float &aqq, float &apq, float &arp, float &arq, int p, int q) {
        if (apq == 0.0f) return;
        const float theta = (aqq - app) * frcp(2.0f * apq);
        const float t = copysignf(1.0f, theta) * frcp(fabsf(theta) + fsqrt(theta * theta + 1.0f));
        const float c = frsq(t * t + 1.0f), s = t * c;
        const float tapq = t * apq;
        app -= tapq;
        aqq += tapq;
        apq = 0.0f;
        const float rp = arp, rq = arq;
        arp = c * rp - s * rq;
        arq = s * rp + c * rq;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float vkp = V.a[3 * k + p], vkq = V.a[3 * k + q];
            V.a[3 * k + p] = c * vkp - s * vkq;
            V.a[3 * k + q] = s * vkp + c * vkq;
        }
    };
    for (int sweep = 0; sweep < 8; ++sweep) {
        const float off = fabsf(a01) + fabsf(a02) + fabsf(a12);
        const float dia = fabsf(a00) + fabsf(a11) + fabsf(a22);
        if (!(off > 1e-6f * dia)) break;  // converged to fp32 level (quadratic convergence)
        rot(a00, a11, a01, a02, a12, 0, 1);  // r = 2: (a20, a21)
        rot(a00, a22, a02, a01, a12, 0, 2);  // r = 1: (a10, a12)
        rot(a11, a22, a12, a01, a02, 1, 2);  // r = 0: (a01, a02)
    }
    lam[0] = a00;
    lam[1] = a11;
    lam[2] = a22;
}

__device__ __forceinline__ void quat_of_rot(const M3 &R, float *q) {
    MGS_CONTRACT
    const float *r = R.a;
    const float tr = r[0] + r[4] + r[8];
    float w, x, y, z;
    if (tr > 0.0f) {
        const float s = fsqrt(tr + 1.0f) * 2.0f, is = frcp(s);
        w = 0.25f * s; x = (r[7] - r[5]) * is; y = (r[2] - r[6]) * is; z = (r[3] - r[1]) * is;
    } else if (r[0] > r[4] && r[0] > r[8]) {
        const float s = fsqrt(1.0f + r[0] - r[4] - r[8]) * 2.0f, is = frcp(s);
        w = (r[7] - r[5]) * is; x = 0.25f * s; y = (r[1] + r[3]) * is; z = (r[2] + r[6]) * is;
    } else if (r[4] > r[8]) {
        const float s = fsqrt(1.0f + r[4] - r[0] - r[8]) * 2.0f, is = frcp(s);
        w = (r[2] - r[6]) * is; x = (r[1] + r[3]) * is; y = 0.25f * s; z = (r[5] + r[7]) * is;
    } else {
        const float s = fsqrt(1.0f + r[8] - r[0] - r[4]) * 2.0f, is = frcp(s);
        w = (r[3] - r[1]) * is; x = (r[2] + r[6]) * is; y = (r[5] + r[7]) * is; z = 0.25f * s;
    }
    const float inv = frsq(w * w + x * x + y * y + z * z);
    q[0] = w * inv; q[1] = x * inv; q[2] = y * inv; q[3] = z * inv;
}

// Hamilton product a * b, (w, x, y, z)
__device__ __forceinline__ void qmul(const float *a, const float *b, float *o) {
    MGS_CONTRACT
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// The 24 rotations that map the coordinate axes onto themselves (up to sign),
// as unit quaternions g, fall into three families: the identity and the half
// turns about the axes (g = a unit vector e_k), the third turns about the cube
// diagonals (g = (+-1/2, +-1/2, +-1/2, +-1/2)) and the quarter turns about the
// axes with the half turns about the face diagonals (g = (+-e_k +- e_l) / sqrt2).
// For a unit quaternion r, max |<g, r>| over each family is, with a_k = |r_k|:
// max_k a_k; (a_0 + a_1 + a_2 + a_3) / 2; and (the two largest a_k) / sqrt2,
// reached by the member whose signs follow r's.  nearest_axis_frame returns
// the member of the group with the largest |<g, r>| (ties to the first family,
// then the lower index), in about forty instructions instead of a scan of the
// 24 candidates.
constexpr float kHalfSqrt2 = 0.70710678118654752f;
__device__ __forceinline__ void nearest_axis_frame(const float *r, float *g) {
    MGS_CONTRACT
    const float a[4] = {fabsf(r[0]), fabsf(r[1]), fabsf(r[2]), fabsf(r[3])};
    const float sg[4] = {r[0] < 0.0f ? -1.0f : 1.0f, r[1] < 0.0f ? -1.0f : 1.0f, r[2] < 0.0f ? -1.0f : 1.0f,
                         r[3] < 0.0f ? -1.0f : 1.0f};
    // the largest and second largest |r_k| (lower index first among equals)
    int k1 = 0, k2 = -1;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        if (a[k] > a[k1]) { k2 = k1; k1 = k; }
        else if (k2 < 0 || a[k] > a[k2]) k2 = k;
    }
    const float dA = a[k1];
    const float dB = 0.5f * ((a[0] + a[1]) + (a[2] + a[3]));
    const float dC = kHalfSqrt2 * (a[k1] + a[k2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = 0.0f;
    if (dA >= dB && dA >= dC) {
        g[k1] = 1.0f;
    } else if (dB >= dC) {
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = 0.5f * sg[k];
    } else {
        g[k1] = kHalfSqrt2 * sg[k1];
        g[k2] = kHalfSqrt2 * sg[k2];
    }
}

// Resident state of a Gaussian inside its voxel.
struct Gs {
    float mu[3];
    float q[4];   // unit
    float s[3];
    float P[6];   // Sigma^-1: 00 01 02 11 12 22
    bool merged;
};

__device__ __forceinline__ void precision_of(Gs &g) {
    MGS_CONTRACT
    const M3 R = rot_of(g.q);
    const float d[3] = {frcp(g.s[0] * g.s[0]), frcp(g.s[1] * g.s[1]), frcp(g.s[2] * g.s[2])};
    const M3 P = rdrt(R, d);
    g.P[0] = P.a[0]; g.P[1] = P.a[1]; g.P[2] = P.a[2]; g.P[3] = P.a[4]; g.P[4] = P.a[5]; g.P[5] = P.a[8];
}

// Eq. (4): (mu_j - mu_i)^T Sigma_i^-1 (mu_j - mu_i)
__device__ __forceinline__ float md2(const Gs &i, const float *mu_j) {
    MGS_CONTRACT
    const float d0 = mu_j[0] - i.mu[0], d1 = mu_j[1] - i.mu[1], d2 = mu_j[2] - i.mu[2];
    const float *P = i.P;
    return d0 * (P[0] * d0 + P[1] * d1 + P[2] * d2) + d1 * (P[1] * d0 + P[3] * d1 + P[4] * d2) +
           d2 * (P[2] * d0 + P[4] * d1 + P[5] * d2);
}

// raw attributes of one Gaussian: mean, scale, quaternion
struct RawG {
    float m[3], s[3], q[4];
};

__device__ __forceinline__ void load_raw(const float *means, const float *scales, const float *quats, int64_t g,
                                         RawG &r) {
    for (int k = 0; k < 3; ++k) { r.m[k] = means[3 * g + k]; r.s[k] = scales[3 * g + k]; }
    for (int k = 0; k < 4; ++k) r.q[k] = quats[4 * g + k];
}

__device__ __forceinline__ void gs_of(const RawG &r, Gs &o) {
    MGS_CONTRACT
    for (int k = 0; k < 3; ++k) { o.mu[k] = r.m[k]; o.s[k] = r.s[k]; }
    const float inv = frsq(r.q[0] * r.q[0] + r.q[1] * r.q[1] + r.q[2] * r.q[2] + r.q[3] * r.q[3]);
    for (int k = 0; k < 4; ++k) o.q[k] = r.q[k] * inv;
    o.merged = false;
    precision_of(o);
}

__device__ __forceinline__ void load_gs(const float *means, const float *scales, const float *quats, int64_t g,
                                        Gs &o) {
    RawG r;
    load_raw(means, scales, quats, g, r);
    gs_of(r, o);
}

__device__ void w2_lbfgs(const float *qi, const float *si, const float *qj, const float *sj, float *q_out,
                         float *s_out);

// G_k from G_i (older) and G_j (Eqs. (6), (9), (10)); result replaces i.
// LBFGS: Eq. (9) by the paper's iterative solver instead of its closed form.
template <bool LBFGS>
__device__ void merge_pair(Gs &i, const Gs &j) {
    MGS_CONTRACT
    // Eq. (6), written around mu_i: mu_k = mu_i + (P_i + P_j)^-1 P_j (mu_j - mu_i)
    const float *Pi = i.P, *Pj = j.P;
    const float S[6] = {Pi[0] + Pj[0], Pi[1] + Pj[1], Pi[2] + Pj[2], Pi[3] + Pj[3], Pi[4] + Pj[4], Pi[5] + Pj[5]};
    const float d[3] = {j.mu[0] - i.mu[0], j.mu[1] - i.mu[1], j.mu[2] - i.mu[2]};
    const float b[3] = {Pj[0] * d[0] + Pj[1] * d[1] + Pj[2] * d[2], Pj[1] * d[0] + Pj[3] * d[1] + Pj[4] * d[2],
                        Pj[2] * d[0] + Pj[4] * d[1] + Pj[5] * d[2]};
    // symmetric 3x3 solve by the adjugate
    const float c00 = S[3] * S[5] - S[4] * S[4], c01 = S[2] * S[4] - S[1] * S[5], c02 = S[1] * S[4] - S[2] * S[3];
    const float c11 = S[0] * S[5] - S[2] * S[2], c12 = S[1] * S[2] - S[0] * S[4], c22 = S[0] * S[3] - S[1] * S[1];
    const float det = S[0] * c00 + S[1] * c01 + S[2] * c02;
    const float id = frcp(det);
    const float x0 = (c00 * b[0] + c01 * b[1] + c02 * b[2]) * id;
    const float x1 = (c01 * b[0] + c11 * b[1] + c12 * b[2]) * id;
    const float x2 = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * id;
    if constexpr (LBFGS) {
        float qk[4], sk[3];
        w2_lbfgs(i.q, i.s, j.q, j.s, qk, sk);
        i.mu[0] += x0; i.mu[1] += x1; i.mu[2] += x2;
        for (int k = 0; k < 4; ++k) i.q[k] = qk[k];
        for (int k = 0; k < 3; ++k) i.s[k] = sk[k];
        i.merged = true;
        precision_of(i);
        return;
    }
    // Eq. (9) minimiser: Sigma_k = 1/4 (I + T) Sigma_i (I + T),
    // T = Sigma_i^-1/2 (Sigma_i^1/2 Sigma_j Sigma_i^1/2)^1/2 Sigma_i^-1/2.
    // Everything is formed in G_i's own frame (coordinates R_i^T x), where
    // Sigma_i = diag(s_i^2) and its square roots are diagonal; there the two
    // matrices to decompose are close to diagonal when the pair's axes agree
    // (near-duplicates), so the Jacobi sweeps converge in one or two rounds.
    // An orthogonal change of frame leaves every result unchanged.
    const M3 Ri = rot_of(i.q), Rj = rot_of(j.q);
    const float si[3] = {i.s[0], i.s[1], i.s[2]};
    const float isi[3] = {frcp(i.s[0]), frcp(i.s[1]), frcp(i.s[2])};
    const float si2[3] = {si[0] * si[0], si[1] * si[1], si[2] * si[2]};
    const float sj2[3] = {j.s[0] * j.s[0], j.s[1] * j.s[1], j.s[2] * j.s[2]};
    const M3 Sjl = rdrt(mul_tn(Ri, Rj), sj2);  // Sigma_j in G_i's frame
    M3 Mid;  // diag(s_i) Sjl diag(s_i), symmetric by construction
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Mid.a[3 * r + c] = si[r] * Sjl.a[3 * r + c] * si[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r + 1; c < 3; ++c) {
            const float avg = 0.5f * (Mid.a[3 * r + c] + Mid.a[3 * c + r]);
            Mid.a[3 * r + c] = Mid.a[3 * c + r] = avg;
        }
    float lam[3];
    M3 V;
    jacobi3(Mid, lam, V);
    const float rl[3] = {fsqrt(fmaxf(lam[0], 0.0f)), fsqrt(fmaxf(lam[1], 0.0f)), fsqrt(fmaxf(lam[2], 0.0f))};
    const M3 Root = rdrt(V, rl);
    M3 IT;  // I + diag(1/s_i) Root diag(1/s_i)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) IT.a[3 * r + c] = isi[r] * Root.a[3 * r + c] * isi[c] + (r == c ? 1.0f : 0.0f);
    M3 Sk;  // 1/4 (I + T) diag(s_i^2) (I + T), symmetrised
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Sk.a[3 * r + c] = 0.25f * (IT.a[3 * r] * si2[0] * IT.a[c] + IT.a[3 * r + 1] * si2[1] * IT.a[3 + c] +
                                       IT.a[3 * r + 2] * si2[2] * IT.a[6 + c]);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r + 1; c < 3; ++c) {
            const float avg = 0.5f * (Sk.a[3 * r + c] + Sk.a[3 * c + r]);
            Sk.a[3 * r + c] = Sk.a[3 * c + r] = avg;
        }
    // (q_k, s_k): eigen-decomposition; of the 24 equivalent axis frames E P_g
    // take the one whose quaternion q_E q_g is closest to slerp(q_i, q_j, 1/2):
    // |<q_E q_g, q_ref>| = |<q_g, conj(q_E) q_ref>|.
    float qr[4];
    {
        const float sgn = (i.q[0] * j.q[0] + i.q[1] * j.q[1] + i.q[2] * j.q[2] + i.q[3] * j.q[3]) < 0.0f ? -1.0f : 1.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) qr[k] = i.q[k] + sgn * j.q[k];
        const float inv = frsq(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) qr[k] *= inv;
    }
    float ev[3];
    M3 E;
    {
        M3 El;
        jacobi3(Sk, ev, El);
        E = mul(Ri, El);  // eigenvectors back in world coordinates
    }
    const float dE = E.a[0] * (E.a[4] * E.a[8] - E.a[5] * E.a[7]) - E.a[1] * (E.a[3] * E.a[8] - E.a[5] * E.a[6]) +
                     E.a[2] * (E.a[3] * E.a[7] - E.a[4] * E.a[6]);
    if (dE < 0.0f) { E.a[0] = -E.a[0]; E.a[3] = -E.a[3]; E.a[6] = -E.a[6]; }
    float qE[4];
    quat_of_rot(E, qE);
    const float qEc[4] = {qE[0], -qE[1], -qE[2], -qE[3]};
    float rq[4];
    qmul(qEc, qr, rq);
    float qg[4];
    nearest_axis_frame(rq, qg);
    float qk[4];
    qmul(qE, qg, qk);
    if (qk[0] < 0.0f) for (int k = 0; k < 4; ++k) qk[k] = -qk[k];
    {
        const float inv = frsq(qk[0] * qk[0] + qk[1] * qk[1] + qk[2] * qk[2] + qk[3] * qk[3]);
        for (int k = 0; k < 4; ++k) qk[k] *= inv;
    }
    // column c of R(q_g) is +-e_pi(c): scale c of G_k is sqrt(ev[pi(c)])
    const M3 Pg = rot_of(qg);
    for (int c = 0; c < 3; ++c) {
        int row = 0;
        float mag = fabsf(Pg.a[c]);
        if (fabsf(Pg.a[3 + c]) > mag) { row = 1; mag = fabsf(Pg.a[3 + c]); }
        if (fabsf(Pg.a[6 + c]) > mag) row = 2;
        i.s[c] = fmaxf(fsqrt(fmaxf(ev[row], 0.0f)), 1e-12f);
    }
    i.mu[0] += x0; i.mu[1] += x1; i.mu[2] += x2;
    for (int k = 0; k < 4; ++k) i.q[k] = qk[k];
    i.merged = true;
    precision_of(i);
}

// ---------------------------------------------------------------- Eq. (9) by L-BFGS (alternative)
// The paper minimises Eq. (9), W2^2(Sigma_k, Sigma_i) + W2^2(Sigma_k, Sigma_j),
// over (q_k, s_k) with L-BFGS from the Eq. (10) start q = slerp(q_i, q_j, 1/2),
// s = (s_i + s_j) / 2 + (0.001, 0.002, 0.003).  This path does the same in
// fp64 (the objective is a small difference of traces): s in units of the
// pair's mean scale, W2^2(Sigma_k, S) = tr Sigma_k + tr S - 2 tr (Sigma_k^1/2 S
// Sigma_k^1/2)^1/2 evaluated in G_k's frame (where Sigma_k^1/2 = diag(s)), and
// its gradient d/dSigma_k = I - T_k->S (T the optimal map, diag(1/s) (diag(s)
// S diag(s))^1/2 diag(1/s) in that frame), chained to s and to the normalised
// quaternion.  Memory 4, Armijo backtracking, stop at a largest gradient entry
// of 1e-6 (about 1e-6 relative in Sigma_k) or after kLbfgsIters iterations
// (about 7 on the test room; up to 91 where the pair's frames differ most).
constexpr int kLbfgsMem = 4;
constexpr int kLbfgsIters = 128;

struct D3 {
    double a[9];
};

__device__ void jacobi3_d(D3 A, double *lam, D3 &V) {
    double a00 = A.a[0], a01 = A.a[1], a02 = A.a[2], a11 = A.a[4], a12 = A.a[5], a22 = A.a[8];
#pragma unroll
    for (int i = 0; i < 9; ++i) V.a[i] = (i % 4 == 0) ? 1.0 : 0.0;
    auto rot = [&](double &app, double &aqq, double &apq, double &arp, double &arq, int p, int q) {
        if (apq == 0.0) return;
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        const double tapq = t * apq;
        app -= tapq;
        aqq += tapq;
        apq = 0.0;
        const double rp = arp, rq = arq;
        arp = c * rp - s * rq;
        arq = s * rp + c * rq;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double vkp = V.a[3 * k + p], vkq = V.a[3 * k + q];
            V.a[3 * k + p] = c * vkp - s * vkq;
            V.a[3 * k + q] = s * vkp + c * vkq;
        }
    };
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = fabs(a01) + fabs(a02) + fabs(a12);
        const double dia = fabs(a00) + fabs(a11) + fabs(a22);
        if (!(off > 1e-15 * dia)) break;
        rot(a00, a11, a01, a02, a12, 0, 1);
        rot(a00, a22, a02, a01, a12, 0, 2);
        rot(a11, a22, a12, a01, a02, 1, 2);
    }
    lam[0] = a00;
    lam[1] = a11;
    lam[2] = a22;
}

__device__ __forceinline__ D3 rot_of_d(const double *q) {  // unit (w, x, y, z)
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    D3 R;
    R.a[0] = 1 - 2 * (y * y + z * z); R.a[1] = 2 * (x * y - w * z);     R.a[2] = 2 * (x * z + w * y);
    R.a[3] = 2 * (x * y + w * z);     R.a[4] = 1 - 2 * (x * x + z * z); R.a[5] = 2 * (y * z - w * x);
    R.a[6] = 2 * (x * z - w * y);     R.a[7] = 2 * (y * z + w * x);     R.a[8] = 1 - 2 * (x * x + y * y);
    return R;
}

// Eq. (9) objective at x = (q[4], s[3]) and its gradient g[7]; Si, Sj are the
// pair's covariances in the scaled units, world frame.
__device__ double w2_objective(const double *x, const D3 &Si, const D3 &Sj, double *g) {
    const double nq = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    const double qh[4] = {x[0] / nq, x[1] / nq, x[2] / nq, x[3] / nq};
    const double sk[3] = {x[4], x[5], x[6]};
    const D3 R = rot_of_d(qh);
    double f = 2.0 * (sk[0] * sk[0] + sk[1] * sk[1] + sk[2] * sk[2]);
    double G[9] = {2, 0, 0, 0, 2, 0, 0, 0, 2};  // d f / d Sigma_k in G_k's frame
    for (int w = 0; w < 2; ++w) {
        const D3 &S = w ? Sj : Si;
        double RS[9];  // R^T S
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                RS[3 * i + j] = R.a[i] * S.a[j] + R.a[3 + i] * S.a[3 + j] + R.a[6 + i] * S.a[6 + j];
        D3 inner;  // diag(s) R^T S R diag(s)
        double trA = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double A = RS[3 * i] * R.a[j] + RS[3 * i + 1] * R.a[3 + j] + RS[3 * i + 2] * R.a[6 + j];
                if (i == j) trA += A;
                inner.a[3 * i + j] = sk[i] * A * sk[j];
            }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i + 1; j < 3; ++j) inner.a[3 * i + j] = inner.a[3 * j + i] = 0.5 * (inner.a[3 * i + j] + inner.a[3 * j + i]);
        double lam[3];
        D3 V;
        jacobi3_d(inner, lam, V);
        const double r[3] = {sqrt(fmax(lam[0], 0.0)), sqrt(fmax(lam[1], 0.0)), sqrt(fmax(lam[2], 0.0))};
        f += trA - 2.0 * (r[0] + r[1] + r[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double root = V.a[3 * i] * r[0] * V.a[3 * j] + V.a[3 * i + 1] * r[1] * V.a[3 * j + 1] +
                                    V.a[3 * i + 2] * r[2] * V.a[3 * j + 2];
                G[3 * i + j] -= root / (sk[i] * sk[j]);
            }
    }
    // d f / d s_c = 2 s_c G_cc; d f / d R = 2 R G diag(s^2)
    for (int c = 0; c < 3; ++c) g[4 + c] = 2.0 * sk[c] * G[4 * c];
    double F[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            F[3 * i + j] = 2.0 * (R.a[3 * i] * G[j] + R.a[3 * i + 1] * G[3 + j] + R.a[3 * i + 2] * G[6 + j]) * sk[j] * sk[j];
    // through R(q) of the unit quaternion (w, x, y, z), then its normalisation
    const double w = qh[0], xq = qh[1], y = qh[2], z = qh[3];
    double gq[4];
    gq[0] = 2.0 * (F[1] * -z + F[2] * y + F[3] * z + F[5] * -xq + F[6] * -y + F[7] * xq);
    gq[1] = 2.0 * (F[1] * y + F[2] * z + F[3] * y + F[4] * -2.0 * xq + F[5] * -w + F[6] * z + F[7] * w +
                   F[8] * -2.0 * xq);
    gq[2] = 2.0 * (F[0] * -2.0 * y + F[1] * xq + F[2] * w + F[3] * xq + F[5] * z + F[6] * -w + F[7] * z +
                   F[8] * -2.0 * y);
    gq[3] = 2.0 * (F[0] * -2.0 * z + F[1] * -w + F[2] * xq + F[3] * w + F[4] * -2.0 * z + F[5] * y + F[6] * xq +
                   F[7] * y);
    const double dq = qh[0] * gq[0] + qh[1] * gq[1] + qh[2] * gq[2] + qh[3] * gq[3];
    for (int k = 0; k < 4; ++k) g[k] = (gq[k] - qh[k] * dq) / nq;
    return f;
}

// (q_k, s_k) minimising Eq. (9) for the pair (qi, si), (qj, sj) (unit quaternions,
// world frame), from the Eq. (10) start.
__device__ void w2_lbfgs(const float *qi, const float *si, const float *qj, const float *sj, float *q_out,
                         float *s_out) {
    const double sigma = (si[0] + si[1] + si[2] + sj[0] + sj[1] + sj[2]) / 6.0;
    D3 Si, Sj;
    {
        const double qa[4] = {qi[0], qi[1], qi[2], qi[3]}, qb[4] = {qj[0], qj[1], qj[2], qj[3]};
        const D3 Ra = rot_of_d(qa), Rb = rot_of_d(qb);
        const double da[3] = {si[0] / sigma, si[1] / sigma, si[2] / sigma};
        const double db[3] = {sj[0] / sigma, sj[1] / sigma, sj[2] / sigma};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Si.a[3 * i + j] = Ra.a[3 * i] * da[0] * da[0] * Ra.a[3 * j] + Ra.a[3 * i + 1] * da[1] * da[1] * Ra.a[3 * j + 1] +
                                  Ra.a[3 * i + 2] * da[2] * da[2] * Ra.a[3 * j + 2];
                Sj.a[3 * i + j] = Rb.a[3 * i] * db[0] * db[0] * Rb.a[3 * j] + Rb.a[3 * i + 1] * db[1] * db[1] * Rb.a[3 * j + 1] +
                                  Rb.a[3 * i + 2] * db[2] * db[2] * Rb.a[3 * j + 2];
            }
    }
    // Eq. (10) averages the scales axis by axis, which presumes corresponding
    // axes: of G_j's 24 equivalent (q, s) take the one whose frame is nearest
    // q_i (the same covariance), then slerp(q_i, q_j, 1/2) on the shortest
    // path and the mean scale plus the offsets (metres).
    float qa[4], sa[3];
    {
        const float qjc[4] = {qj[0], -qj[1], -qj[2], -qj[3]};
        float r[4], g[4];
        qmul(qjc, qi, r);
        nearest_axis_frame(r, g);
        qmul(qj, g, qa);
        const M3 Pg = rot_of(g);  // column c is +-e_pi(c)
        for (int c = 0; c < 3; ++c) {
            int row = 0;
            float mag = fabsf(Pg.a[c]);
            if (fabsf(Pg.a[3 + c]) > mag) { row = 1; mag = fabsf(Pg.a[3 + c]); }
            if (fabsf(Pg.a[6 + c]) > mag) row = 2;
            sa[c] = sj[row];
        }
    }
    double x[7];
    {
        const double sg = (qi[0] * qa[0] + qi[1] * qa[1] + qi[2] * qa[2] + qi[3] * qa[3]) < 0.0 ? -1.0 : 1.0;
        double m[4], nm = 0.0;
        for (int k = 0; k < 4; ++k) { m[k] = (double)qi[k] + sg * (double)qa[k]; nm += m[k] * m[k]; }
        nm = sqrt(nm);
        for (int k = 0; k < 4; ++k) x[k] = m[k] / nm;
        const double delta[3] = {0.001, 0.002, 0.003};
        for (int c = 0; c < 3; ++c) x[4 + c] = (0.5 * ((double)si[c] + (double)sa[c]) + delta[c]) / sigma;
    }
    double g[7];
    double f = w2_objective(x, Si, Sj, g);
    double S[kLbfgsMem][7], Y[kLbfgsMem][7], rho[kLbfgsMem];
    int nmem = 0, head = 0;
    for (int it = 0; it < kLbfgsIters; ++it) {
        double gmax = 0.0;
        for (int k = 0; k < 7; ++k) gmax = fmax(gmax, fabs(g[k]));
        if (gmax <= 1e-6) break;
        // two-loop recursion: d = -H g
        double qv[7], al[kLbfgsMem];
        for (int k = 0; k < 7; ++k) qv[k] = g[k];
        for (int u = 0; u < nmem; ++u) {
            const int b = (head - 1 - u + kLbfgsMem) % kLbfgsMem;
            double a = 0.0;
            for (int k = 0; k < 7; ++k) a += S[b][k] * qv[k];
            a *= rho[b];
            al[u] = a;
            for (int k = 0; k < 7; ++k) qv[k] -= a * Y[b][k];
        }
        double gam;
        if (nmem > 0) {
            const int b = (head - 1 + kLbfgsMem) % kLbfgsMem;
            double sy = 0.0, yy = 0.0;
            for (int k = 0; k < 7; ++k) { sy += S[b][k] * Y[b][k]; yy += Y[b][k] * Y[b][k]; }
            gam = sy / yy;
        } else {
            gam = 1e-2 / gmax;
        }
        for (int k = 0; k < 7; ++k) qv[k] *= gam;
        for (int u = nmem - 1; u >= 0; --u) {
            const int b = (head - 1 - u + kLbfgsMem) % kLbfgsMem;
            double bb = 0.0;
            for (int k = 0; k < 7; ++k) bb += Y[b][k] * qv[k];
            bb *= rho[b];
            for (int k = 0; k < 7; ++k) qv[k] += S[b][k] * (al[u] - bb);
        }
        double d[7], gd = 0.0;
        for (int k = 0; k < 7; ++k) { d[k] = -qv[k]; gd += g[k] * d[k]; }
        if (!(gd < 0.0)) {  // not a descent direction: restart from the gradient
            nmem = 0;
            gd = 0.0;
            for (int k = 0; k < 7; ++k) { d[k] = -g[k] * (1e-2 / gmax); gd += g[k] * d[k]; }
        }
        // Armijo backtracking
        double t = 1.0, xn[7], gn[7], fn = f;
        bool ok = false;
        for (int ls = 0; ls < 30; ++ls) {
            for (int k = 0; k < 7; ++k) xn[k] = x[k] + t * d[k];
            fn = w2_objective(xn, Si, Sj, gn);
            if (fn <= f + 1e-4 * t * gd) { ok = true; break; }
            t *= 0.5;
        }
        if (!ok) break;  // no decrease left at fp64 resolution
        double sy = 0.0;
        for (int k = 0; k < 7; ++k) {
            S[head][k] = xn[k] - x[k];
            Y[head][k] = gn[k] - g[k];
            sy += S[head][k] * Y[head][k];
        }
        if (sy > 1e-300) {
            rho[head] = 1.0 / sy;
            head = (head + 1) % kLbfgsMem;
            nmem = nmem < kLbfgsMem ? nmem + 1 : kLbfgsMem;
        }
        for (int k = 0; k < 7; ++k) { x[k] = xn[k]; g[k] = gn[k]; }
        f = fn;
    }
    const double nq = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
    const double sgn = x[0] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 4; ++k) q_out[k] = (float)(sgn * x[k] / nq);
    for (int c = 0; c < 3; ++c) s_out[c] = fmaxf((float)(fabs(x[4 + c]) * sigma), 1e-12f);
}

// first sorted position of a voxel that holds at least two Gaussians
template <class K>
struct LoadMultiHead {
    const K *keys;
    int64_t ne;
    __device__ uint32_t operator()(int64_t i) const {
        const K k = keys[i];
        return (i == 0 || keys[i - 1] != k) && i + 1 < ne && keys[i + 1] == k ? 1u : 0u;
    }
};
struct StoreHead {
    uint32_t *vlist;
    __device__ void operator()(int64_t i, uint32_t ex, uint32_t v) const {
        if (v) vlist[ex] = (uint32_t)i;
    }
};

// A voxel's members merge one after another (a sequential chain), so a wave
// of 64 voxels takes as long as its longest chain, and the longest chains
// (kLongVoxel or more members) set the end of the merge.  The voxels are
// therefore ordered by member count, longest first: k_vcount adds up the
// class sizes (class 0: kLongVoxel or more members, then one class per count,
// fewer members later), k_vplace gives each block a slice of every class (one
// global atomic per class and block) and scatters the voxel heads.  A wave
// then holds voxels of one length, and the long chains start first.  The
// order within a class is unspecified, which changes no result: voxels are
// independent.

template <class K>
__device__ __forceinline__ uint32_t voxel_class(const K *keys, int64_t ne, uint32_t head) {
    const K key = keys[head];
    uint32_t len = 1;
    while (len < (uint32_t)kLongVoxel && (int64_t)head + len < ne && keys[head + len] == key) ++len;
    return (uint32_t)kLongVoxel - len;
}

template <class K>
__global__ __launch_bounds__(256) void k_vcount(const K *keys, int64_t ne, const uint32_t *vlist,
                                                const uint32_t *nvox, uint32_t *book) {
    __shared__ uint32_t h[kVoxClasses];
    if (threadIdx.x < kVoxClasses) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)*nvox) atomicAdd(&h[voxel_class(keys, ne, vlist[t])], 1u);
    __syncthreads();
    if (threadIdx.x < kVoxClasses && h[threadIdx.x]) atomicAdd(book + threadIdx.x, h[threadIdx.x]);
}

// Same grid and items as k_vcount.
template <class K>
__global__ __launch_bounds__(256) void k_vplace(const K *keys, int64_t ne, const uint32_t *vlist,
                                                const uint32_t *nvox, uint32_t *book, uint32_t *order) {
    __shared__ uint32_t h[kVoxClasses], base[kVoxClasses];
    if (threadIdx.x < kVoxClasses) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = t < (int64_t)*nvox;
    uint32_t head = 0, c = 0;
    if (in) {
        head = vlist[t];
        c = voxel_class(keys, ne, head);
        atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kVoxClasses) {
        const int k = threadIdx.x;
        uint32_t ex = 0;
        for (int j = 0; j < k; ++j) ex += book[j];
        base[k] = ex + (h[k] ? atomicAdd(book + kVoxClasses + k, h[k]) : 0u);
        h[k] = 0;
    }
    __syncthreads();
    if (in) order[base[c] + atomicAdd(&h[c], 1u)] = head;
}

template <class K>
struct VoxelArgs {
    const float *means, *scales, *quats;
    const K *keys;          // sorted
    const uint32_t *gids;   // sorted (ascending within a voxel)
    int64_t ne;
    const uint32_t *order;  // first positions of the voxels with >= 2 members, longest first
    const uint32_t *nvox;   // their number (device)
    const uint32_t *nlong;  // the number with >= kLongVoxel members (device): order's first entries
    int64_t long_waves;     // blocks given to them, one voxel each (more long voxels join the rest)
    float chi2;
    int policy;
    Gs *res;                // scratch, one slot per sorted position
    uint32_t *alive;        // [n]
    uint32_t *merged;       // [n]
    float *new_mu, *new_q, *new_s;  // [n][3], [n][4], [n][3]
};

// One thread per voxel with at least two members, in the order of k_vplace.
// The first long_waves blocks take one long voxel each, on lane 0 at raised
// issue priority: a wave lasts as long as its longest chain, and 64 long
// chains in one wave cost the diverging lanes' work and their extra
// residents on every step of it.  The other voxels follow 64 to a wave (dense,
// so the lanes all merge, along chains of one length).
template <class K, bool LBFGS>
__global__ __launch_bounds__(64) void k_voxels(VoxelArgs<K> a) {
    const int64_t nlong = min((int64_t)*a.nlong, a.long_waves);
    int64_t t;
    if ((int64_t)blockIdx.x < a.long_waves) {
        if (threadIdx.x != 0 || (int64_t)blockIdx.x >= nlong) return;
        t = blockIdx.x;
        __builtin_amdgcn_s_setprio(3);
    } else {
        t = nlong + ((int64_t)blockIdx.x - a.long_waves) * 64 + threadIdx.x;
        if (t >= (int64_t)*a.nvox) return;
    }
    const int64_t i = a.order[t];
    const K key = a.keys[i];
    int64_t end = i + 1;
    while (end < a.ne && a.keys[end] == key) ++end;
    Gs *R = a.res + i;
    if ((a.policy & 1) == 0) {
        // the merge chain of a voxel is sequential: the next member's
        // attributes are fetched while the current one merges
        // Resident 0, which absorbs most members, stays in registers (copied to
        // its scratch slot at the end); the others live in the scratch slots.
        int64_t nres = 0;
        Gs R0;
        uint32_t gn = a.gids[i];
        RawG next;
        load_raw(a.means, a.scales, a.quats, gn, next);
        for (int64_t m = i; m < end; ++m) {
            const uint32_t gj = gn;
            const RawG cur = next;
            if (m + 1 < end) {
                gn = a.gids[m + 1];
                load_raw(a.means, a.scales, a.quats, gn, next);
            }
            Gs J;
            gs_of(cur, J);
            int64_t best = -1;
            float bd = 0.0f;
            if (nres > 0) {
                best = 0;
                bd = md2(R0, J.mu);
            }
            for (int64_t r = 1; r < nres; ++r) {
                const float d = md2(R[r], J.mu);
                if (d < bd) { best = r; bd = d; }
            }
            if (best >= 0 && bd < a.chi2) {
                Gs B;
                if (best == 0) B = R0;
                else B = R[best];
                merge_pair<LBFGS>(B, J);  // one merge site: the merge is long code
                if (best == 0) R0 = B;
                else R[best] = B;
                a.alive[gj] = 0u;
            } else {
                if (nres == 0) R0 = J;
                else R[nres] = J;
                ++nres;
            }
        }
        if (nres > 0) R[0] = R0;
        // write back merged residents: resident r is the r-th Gaussian that stayed
        int64_t r = 0;
        for (int64_t m = i; m < end && r < nres; ++m) {
            const uint32_t g = a.gids[m];
            if (!a.alive[g]) continue;
            if (R[r].merged) {
                a.merged[g] = 1u;
                for (int k = 0; k < 3; ++k) { a.new_mu[3 * g + k] = R[r].mu[k]; a.new_s[3 * g + k] = R[r].s[k]; }
                for (int k = 0; k < 4; ++k) a.new_q[4 * g + k] = R[r].q[k];
            }
            ++r;
        }
    } else {
        const int64_t n = end - i;
        for (int64_t m = 0; m < n; ++m) load_gs(a.means, a.scales, a.quats, a.gids[i + m], R[m]);
        int64_t bi = -1, bj = -1;
        float bd = 0.0f;
        for (int64_t x = 0; x < n; ++x)
            for (int64_t y = x + 1; y < n; ++y) {
                const float d = md2(R[x], R[y].mu);
                if (bi < 0 || d < bd) { bi = x; bj = y; bd = d; }
            }
        if (bi >= 0 && bd < a.chi2) {
            Gs B = R[bi];
            const Gs J = R[bj];
            merge_pair<LBFGS>(B, J);
            const uint32_t gi = a.gids[i + bi], gj = a.gids[i + bj];
            a.alive[gj] = 0u;
            a.merged[gi] = 1u;
            for (int k = 0; k < 3; ++k) { a.new_mu[3 * gi + k] = B.mu[k]; a.new_s[3 * gi + k] = B.s[k]; }
            for (int k = 0; k < 4; ++k) a.new_q[4 * gi + k] = B.q[k];
        }
    }
}

struct StoreNewIndex {
    uint32_t *newidx;
    __device__ void operator()(int64_t i, uint32_t ex, uint32_t) const { newidx[i] = ex; }
};

struct CompactArgs {
    mgs_gaussians in;
    mgs_gaussians_out out;
    int K3;
    const uint32_t *alive, *merged, *newidx;
    const float *new_mu, *new_q, *new_s;
    int32_t *old_to_new;
};

__global__ __launch_bounds__(256) void k_compact(CompactArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.in.n) return;
    const bool keep = a.alive[g] != 0;
    if (a.old_to_new) a.old_to_new[g] = keep ? (int32_t)a.newidx[g] : -1;
    if (!keep) return;
    const int64_t o = a.newidx[g];
    const bool mg = a.merged[g] != 0;
    for (int k = 0; k < 3; ++k) {
        a.out.means[3 * o + k] = mg ? a.new_mu[3 * g + k] : a.in.means[3 * g + k];
        a.out.scales[3 * o + k] = mg ? a.new_s[3 * g + k] : a.in.scales[3 * g + k];
    }
    for (int k = 0; k < 4; ++k) a.out.quats[4 * o + k] = mg ? a.new_q[4 * g + k] : a.in.quats[4 * g + k];
    a.out.opac[o] = a.in.opac[g];
    for (int k = 0; k < a.K3; ++k) a.out.sh[(int64_t)a.K3 * o + k] = a.in.sh[(int64_t)a.K3 * g + k];
}

namespace {
struct MergeLayout {
    size_t cells, elig, bounds, partial, keys0, keys1, vals0, vals1, hist, tmp, res, alive, merged, newidx, new_mu, new_q,
        new_s, vlist, total;
};
MergeLayout merge_layout(int64_t n) {
    MergeLayout L{};
    Bump b;
    L.cells = b.take(12 * n);
    L.elig = b.take(4 * n);
    L.bounds = b.take(64 + 4 * kVoxBookWords);  // bounds, counters, the voxel order's bookkeeping
    L.partial = b.take(32 * std::max<int64_t>(ceil_div(n, 256), 1));
    L.keys0 = b.take(8 * n);
    L.keys1 = b.take(8 * n);
    L.vals0 = b.take(4 * n);
    L.vals1 = b.take(4 * n);
    const int64_t nn = std::max<int64_t>(n, 1);
    L.hist = b.take(4 * radix_hist_words(nn));
    L.tmp = b.take(4 * scan_tmp_words(std::max<int64_t>(radix_hist_words(nn), nn)));
    L.res = b.take(sizeof(Gs) * n);
    L.alive = b.take(4 * n);
    L.merged = b.take(4 * n);
    L.newidx = b.take(4 * n);
    L.new_mu = b.take(12 * n);
    L.new_q = b.take(16 * n);
    L.new_s = b.take(12 * n);
    L.vlist = b.take(4 * n);
    L.total = b.size();
    return L;
}
int bits_of(int64_t span) {  // bits to hold values 0..span
    int b = 0;
    while ((int64_t(1) << b) <= span) ++b;
    return b;
}

// Packed voxel keys of the eligible Gaussians, the stable sort, the list of
// multi-member voxels and the merge itself, with keys of type K.
template <class K>
hipError_t sort_and_merge(void *ws, const MergeLayout &L, const int32_t *hb, int by, int bz, int bits,
                          const CellArgs &ca, int64_t ne, const mgs_gaussians *in, float chi2, int32_t policy,
                          uint32_t *alive, uint32_t *merged, uint32_t *count, hipStream_t s) {
    const int64_t n = in->n;
    K *keys[2] = {at<K>(ws, L.keys0), at<K>(ws, L.keys1)};
    uint32_t *vals[2] = {at<uint32_t>(ws, L.vals0), at<uint32_t>(ws, L.vals1)};
    hipError_t e = scan_exclusive(LoadElig{ca.elig}, StorePacked<K>{ca.cells, hb[0], hb[1], hb[2], by, bz, keys[0], vals[0]},
                                  n, at<uint32_t>(ws, L.tmp), nullptr, s);
    if (e != hipSuccess) return e;
    int cur = 0;
    for (int sh = 0; sh < bits; sh += 8) {
        e = radix_pass<K>(keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], ne, DigitOfKey<K>{sh},
                          at<uint32_t>(ws, L.hist), s);
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    uint32_t *vlist = at<uint32_t>(ws, L.vlist);
    e = scan_exclusive(LoadMultiHead<K>{keys[cur], ne}, StoreHead{vlist}, ne, at<uint32_t>(ws, L.tmp), count + 2, s);
    if (e != hipSuccess) return e;
    // the voxel heads by member count, longest first, go to vals[cur ^ 1], free
    // after the sort; book (zeroed by k_bounds) holds the class sizes and cursors
    uint32_t *order = vals[cur ^ 1];
    uint32_t *book = count + 8;
    const unsigned cgrid = (unsigned)ceil_div(ne, 256);  // ne bounds the number of voxels
    k_vcount<K><<<cgrid, 256, 0, s>>>(keys[cur], ne, vlist, count + 2, book);
    k_vplace<K><<<cgrid, 256, 0, s>>>(keys[cur], ne, vlist, count + 2, book, order);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t long_waves = std::min<int64_t>(ne / kLongVoxel, kLongWavesMax);
    VoxelArgs<K> va{in->means, in->scales, in->quats, keys[cur], vals[cur], ne, order, count + 2, book,
                    long_waves, chi2, policy, at<Gs>(ws, L.res), alive, merged, at<float>(ws, L.new_mu),
                    at<float>(ws, L.new_q), at<float>(ws, L.new_s)};
    const unsigned vgrid = (unsigned)(long_waves + ceil_div(ne, 64));
    if (policy & MGS_MERGE_LBFGS) k_voxels<K, true><<<vgrid, 64, 0, s>>>(va);
    else k_voxels<K, false><<<vgrid, 64, 0, s>>>(va);
    return hipGetLastError();
}
}  // namespace

// M(G) of Eq. (3), one Gaussian per thread: the average gradient (sum over
// count, a correctly rounded fp32 division) below tau, inside the keyframe
// window; unseen Gaussians (count 0) are not eligible
__global__ __launch_bounds__(256) void k_merge_mask(const float *gsum, const uint32_t *count, const int32_t *kf,
                                                    int64_t n, float tau, int32_t kf_min, int32_t kf_max,
                                                    uint8_t *mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = count[i];
    bool ok = c > 0 && gsum[i] / (float)c < tau;
    if (kf) {
        const int32_t k = kf[i];
        ok = ok && k >= kf_min && k <= kf_max;
    }
    mask[i] = ok ? 1 : 0;
}
}  // namespace mgs

using namespace mgs;

extern "C" mgs_status mgs_merge_mask(const float *grad_norm_sum, const uint32_t *visible_count,
                                     const int32_t *kf_index, int64_t n, float tau, int32_t kf_min, int32_t kf_max,
                                     uint8_t *mask, void *stream) {
    ApiRange api_range("mgs_merge_mask");
    if (n < 0 || std::isnan(tau)) return MGS_ERR_INVALID_ARG;
    if (n == 0) return MGS_OK;
    if (!grad_norm_sum || !visible_count || !mask) return MGS_ERR_INVALID_ARG;
    if (n >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_merge_mask<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(grad_norm_sum, visible_count, kf_index, n, tau, kf_min,
                                                           kf_max, mask);
    MGS_LAUNCHED();
    return MGS_OK;
}

extern "C" mgs_status mgs_voxel_merge(const mgs_gaussians *in, const uint8_t *mask, float voxel_size, float chi2,
                                      int32_t policy, mgs_gaussians_out *out, int32_t *old_to_new,
                                      uint64_t *voxel_key, void *ws, size_t ws_bytes, size_t *ws_required,
                                      int64_t *n_out, void *stream) {
    ApiRange api_range("mgs_voxel_merge");
    if (!in || !out || !n_out || !ws_required) return MGS_ERR_INVALID_ARG;
    if (in->n < 0 || in->sh_degree < 0 || in->sh_degree > 3) return MGS_ERR_INVALID_ARG;
    if (!(voxel_size > 0.0f) || !std::isfinite(voxel_size) || !(chi2 >= 0.0f) ||
        (policy & ~(MGS_MERGE_BEST_PAIR | MGS_MERGE_LBFGS)) != 0)
        return MGS_ERR_INVALID_ARG;
    const int64_t n = in->n;
    if (n >= (int64_t(1) << 31)) return MGS_ERR_TOO_LARGE;
    if (n > 0 && (!in->means || !in->scales || !in->quats || !in->opac || !in->sh || !out->means ||
                  !out->scales || !out->quats || !out->opac || !out->sh))
        return MGS_ERR_INVALID_ARG;
    *n_out = 0;
    if (n == 0) {  // nothing to merge: no workspace, no device work
        *ws_required = 0;
        return MGS_OK;
    }
    const MergeLayout L = merge_layout(n);
    *ws_required = L.total;
    if (ws_bytes < L.total || (L.total > 0 && !ws)) return MGS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *bounds = at<int32_t>(ws, L.bounds);
    uint32_t *count = reinterpret_cast<uint32_t *>(bounds + 8);
    const int64_t ncb = ceil_div(n, 256);
    CellArgs ca{in->means, mask, n, voxel_size, at<int32_t>(ws, L.cells), at<uint32_t>(ws, L.elig),
                at<int32_t>(ws, L.partial), voxel_key};
    k_vcells<<<(unsigned)ncb, 256, 0, s>>>(ca);
    const Mailbox mail = host_mailbox();
    const uint32_t ticket = mailbox_ticket();
    k_bounds<<<1, 256, 0, s>>>(ca.partial, ncb, bounds, count, mail.dev, ticket);
    MGS_LAUNCHED();
    // the flags do not depend on the read-back: queued before it
    uint32_t *alive = at<uint32_t>(ws, L.alive);
    uint32_t *merged = at<uint32_t>(ws, L.merged);
    const unsigned g256 = (unsigned)ceil_div(n, 256);
    k_mfill<<<g256, 256, 0, s>>>(alive, n, 1u);
    k_mfill<<<g256, 256, 0, s>>>(merged, n, 0u);
    MGS_LAUNCHED();
    int32_t hb[10];
    if (mail.host) {
        MGS_HIP(mailbox_wait(mail, ticket, s));
        const volatile uint32_t *vm = mail.host;
        for (int k = 0; k < 9; ++k) hb[k] = (int32_t)vm[k];
    } else {
        MGS_HIP(hipMemcpyAsync(hb, bounds, 40, hipMemcpyDeviceToHost, s));
        MGS_HIP(hipStreamSynchronize(s));
    }
    const int64_t ne = (int64_t)(uint32_t)hb[8];
    if (ne >= 2) {
        const int bx = bits_of(hb[3] - hb[0]), by = bits_of(hb[4] - hb[1]), bz = bits_of(hb[5] - hb[2]);
        const int bits = bx + by + bz;
        if (bits <= 32)
            MGS_HIP(sort_and_merge<uint32_t>(ws, L, hb, by, bz, bits, ca, ne, in, chi2, policy, alive, merged, count, s));
        else
            MGS_HIP(sort_and_merge<uint64_t>(ws, L, hb, by, bz, bits, ca, ne, in, chi2, policy, alive, merged, count, s));
        MGS_LAUNCHED();
    }
    uint32_t *newidx = at<uint32_t>(ws, L.newidx);
    uint32_t *tmp = at<uint32_t>(ws, L.tmp);
    // the number kept goes to the host's word 9 (or to count[1], then copied)
    MGS_HIP(scan_exclusive(LoadElig{alive}, StoreNewIndex{newidx}, n, tmp, mail.dev ? mail.dev + 9 : count + 1, s));
    CompactArgs cp{*in, *out, 3 * (in->sh_degree + 1) * (in->sh_degree + 1), alive, merged, newidx,
                   at<float>(ws, L.new_mu), at<float>(ws, L.new_q), at<float>(ws, L.new_s), old_to_new};
    k_compact<<<g256, 256, 0, s>>>(cp);
    MGS_LAUNCHED();
    uint32_t hn = 0;
    if (mail.host) {
        const uint32_t done = mailbox_ticket();
        k_mail_done<<<1, 1, 0, s>>>(mail.dev, done);
        MGS_LAUNCHED();
        MGS_HIP(mailbox_wait(mail, done, s));
        hn = static_cast<const volatile uint32_t *>(mail.host)[9];
    } else {
        MGS_HIP(hipMemcpyAsync(&hn, count + 1, 4, hipMemcpyDeviceToHost, s));
        MGS_HIP(hipStreamSynchronize(s));
    }
    *n_out = hn;
    return MGS_OK;
}
