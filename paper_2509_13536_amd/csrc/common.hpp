// Shared device/host definitions of the gfx950 MemGS path.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "memgs.h"

namespace mgs {

// Compositing constants of the 3DGS lineage that the paper builds on (Sec. II-E):
// alpha clamp, alpha skip threshold, transmittance stop threshold, 2D dilation,
// Jacobian frustum clamp.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kDilation = 0.3f;
constexpr float kFrustum = 1.3f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr int kTile = 16;
constexpr int kRecord = 10;  // per-instance gradient record (see blend backward)

// One view as the kernels see it.
struct ViewDev {
    float R[9];
    float t[3];
    float cam_center[3];  // -R^T t
    float fx, fy, cx, cy, near_z;
    float limx, limy;  // frustum clamp of the normalised coordinates: 1.3 (W/2) / fx, 1.3 (H/2) / fy
    int32_t W, H, TX, TY;  // image size; 16x16 tiles per row and column
    int32_t map;
    int32_t BTX, BTY;      // tiles per list bin along x and y (the same for every view of a call)
    int32_t BX, BY;        // bins per row and column
    int32_t bin_base;      // first global bin id of this view
    int64_t pair_base;  // first (Gaussian, view) pair index
    int64_t pix_base;   // first pixel in the packed one-channel outputs
};

struct MapDev {
    const float *means, *scales, *quats, *opac, *sh;
    int64_t n;
    int32_t sh_degree, K;
    int64_t pair_first_view;  // unused placeholder for alignment
};

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ float dpp_f32(float x) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, BANK_MASK, true));
}

// Sum over the 64 lanes; the total is returned in every lane.  Inactive lanes
// must hold 0.  Rows of 16 are reduced with DPP quad permutes and rotates,
// then rows are combined with row broadcasts; lane 63 ends with the total.
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp_f32<0xB1>(x);        // quad_perm [1,0,3,2]
    x += dpp_f32<0x4E>(x);        // quad_perm [2,3,0,1]
    x += dpp_f32<0x124>(x);       // row_ror 4
    x += dpp_f32<0x128>(x);       // row_ror 8 : every lane holds its row sum
    x += dpp_f32<0x142, 0xA>(x);  // row_bcast 15 into rows 1, 3
    x += dpp_f32<0x143, 0xC>(x);  // row_bcast 31 into rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

// Sum over each row of 16 lanes; every lane of the row receives its row's sum.
__device__ __forceinline__ float row16_sum(float x) {
    x += dpp_f32<0xB1>(x);
    x += dpp_f32<0x4E>(x);
    x += dpp_f32<0x124>(x);
    x += dpp_f32<0x128>(x);
    return x;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t y = __shfl_xor(x, off, 64);
        x = x > y ? x : y;
    }
    return x;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// inclusive prefix sum over the lanes
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    const int lane = __lane_id();
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// value of lane l (l wave-uniform) in every lane
__device__ __forceinline__ int readlane_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ float readlane_f(float x, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}

__device__ __forceinline__ uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }

// ---------------------------------------------------------------- host helpers
struct Bump {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return o;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};

template <class T>
__host__ __device__ inline T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Error tracking for mgs_last_hip_error().
void set_hip_error(hipError_t e);

// kMailWords pinned, coherent host words per host thread that kernels write
// the counts a call reads back into (the call then only waits for its stream):
// `dev` is the address kernels write, `host` the one the call reads.  Both null
// if the pinned allocation failed, and the caller copies instead.  Allocated
// on the thread's first such call and freed when the thread ends.
constexpr int kMailWords = 64;
struct Mailbox {
    uint32_t *host = nullptr, *dev = nullptr;
};
Mailbox host_mailbox();
// Word kMailFlag of the mailbox carries a per-call ticket that a kernel writes
// after its values (behind a system-scope fence): the host spins on it instead
// of waiting for the stream.
constexpr int kMailFlag = kMailWords - 1;
uint32_t mailbox_ticket();
// Waits until the flag holds `ticket`; after 2 s without it, waits for the
// stream instead (and returns what that returns, e.g. a kernel's error).
hipError_t mailbox_wait(const Mailbox &m, uint32_t ticket, hipStream_t s);
__device__ __forceinline__ void mail_flag(uint32_t *mail, uint32_t ticket) {
    __threadfence_system();
    __hip_atomic_store(mail + kMailFlag, ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Raises the flag once every earlier kernel on the stream is done.
static __global__ void k_mail_done(uint32_t *mail, uint32_t ticket) { mail_flag(mail, ticket); }

// A small per-call table carried in a kernel's arguments and written to device
// memory by that kernel: no host-to-device copy from pageable memory (a staging
// copy on the host and a copy kernel).  Kernel arguments hold at most 4 KB.
constexpr int kArgCopyWords = 896;  // with the hidden arguments, under 4 KB
struct ArgWords {
    uint32_t w[kArgCopyWords];
    int32_t n;
};
static __global__ void k_arg_copy(ArgWords a, uint32_t *dst) {
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.w[i];
}
#define MGS_HIP(call)                      \
    do {                                   \
        hipError_t e_ = (call);            \
        if (e_ != hipSuccess) {            \
            ::mgs::set_hip_error(e_);      \
            return MGS_ERR_HIP;            \
        }                                  \
    } while (0)
#define MGS_LAUNCHED()                                       \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) {                              \
            ::mgs::set_hip_error(e_);                        \
            return MGS_ERR_HIP;                              \
        }                                                    \
    } while (0)

}  // namespace mgs
