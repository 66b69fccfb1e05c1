/*
 * memgs.h - C ABI of the MI355X (gfx950) MemGS hot path.
 *
 * Operations, after MemGS (Bai et al., "MemGS: Memory-Efficient Gaussian
 * Splatting for Real-Time SLAM"):
 *
 *   mgs_render_forward   tile-based rasterisation of colour and depth
 *                        (Sec. II-C Eq. (1)-(2), Sec. II-E Eq. (11));
 *   mgs_render_backward  its gradient w.r.t. means, scales, rotations,
 *                        opacities, SH colour and the SE(3) camera pose
 *                        (what the mapping loss of Eq. (12) back-propagates);
 *   mgs_voxel_merge      voxel-space merging of similar Gaussians
 *                        (Sec. II-D, Eqs. (3)-(10));
 *   mgs_merge_mask       the merge-eligibility mask of Eq. (3);
 *   mgs_mapping_loss     the mapping loss of Eq. (12) and its gradient;
 *   mgs_patch_grid_sample  new Gaussians by Patch-Grid sampling (Sec. II-B);
 *   mgs_adam_step        one optimiser step of the mapping loop (Sec. II-E).
 *
 * Memory.  Every array argument marked "device" lives in device memory owned by
 * the caller; the library never allocates or frees device memory, and retains
 * none of the caller's.  Scratch space is a caller-provided workspace `ws` of
 * `ws_bytes` bytes (256-byte aligned).  The library keeps three pieces of state
 * of its own: (1) per host thread, 64 words of pinned host memory into which
 * kernels write the counts that mgs_render_forward, mgs_voxel_merge and
 * mgs_patch_grid_sample read back, allocated on the thread's first such call
 * and freed when the thread ends; (2) the fixed device scratch of
 * mgs_mapping_loss_noalloc (MGS_LOSS_SCRATCH_BYTES per GPU, held until the
 * process ends); (3) with MGS_ROCTX=1 in the environment, the two roctx entry
 * points, looked up once per process, through which every call opens a roctx
 * range named after itself (rocprofv3 --marker-trace).  Calls are asynchronous on `stream` (a hipStream_t, NULL =
 * default stream) except where stated.  Calls on distinct streams with distinct
 * workspaces may run concurrently (mgs_mapping_loss_noalloc excepted, see there).
 *
 * Errors.  Functions return MGS_OK (0) or a negative mgs_status; no C++
 * exception crosses the ABI.  On MGS_ERR_INVALID_ARG nothing was launched.  On
 * MGS_ERR_WORKSPACE nothing was written to the outputs and *ws_required (or
 * info->ws_required) holds the size to retry with.  On MGS_ERR_HIP the last HIP
 * error is available from mgs_last_hip_error().
 *
 * Conventions.  Quaternions are (w, x, y, z) of any positive norm.  Scales are
 * linear standard deviations (> 0).  Cameras look along +z, x right, y down;
 * pixel (u, v) of a W x H image is evaluated at the integer point (u, v).
 * Images are packed view after view: view v occupies 3*H_v*W_v floats of the
 * colour buffer as [3][H_v][W_v] and H_v*W_v floats of each one-channel buffer.
 */
#ifndef MEMGS_H
#define MEMGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mgs_status;
#define MGS_OK 0
#define MGS_ERR_INVALID_ARG (-1)
#define MGS_ERR_WORKSPACE (-2)
#define MGS_ERR_HIP (-3)
#define MGS_ERR_TOO_LARGE (-4) /* an internal count would exceed 2^31 - 1 */
#define MGS_ERR_SCRATCH (-5)   /* the input needs more than an allocation-free entry point's fixed scratch */

/* A Gaussian map G = {mu_i, Sigma_i(q_i, s_i), o_i, c_i(SH)} (Sec. II-C), as
 * device arrays (structure of arrays). */
typedef struct mgs_gaussians {
    int64_t n;            /* number of Gaussians, >= 0 */
    const float *means;   /* device [n][3] world positions */
    const float *scales;  /* device [n][3] standard deviations along the local axes */
    const float *quats;   /* device [n][4] rotation (w, x, y, z), any norm > 0 */
    const float *opac;    /* device [n] opacity in [0, 1] */
    const float *sh;      /* device [n][K][3], K = (sh_degree + 1)^2, coefficient-major */
    int32_t sh_degree;    /* 0..3 */
    int32_t reserved;
} mgs_gaussians;

/* Gradient outputs for one map (device, nullable each).  The five gradients
 * are overwritten, not accumulated; Gaussians invisible in every view get 0.
 *
 * The two statistics behind the average gradient of Eq. (3) (Sec. II-D) are
 * ACCUMULATED (+=) over calls, so that a mapping loop can gather them over
 * many iterations; the caller zeroes them when a statistics window starts.
 * For every view of the call in which Gaussian i survives culling (its
 * 3-sigma tile rectangle is not empty), grad_norm_sum[i] grows by the
 * Euclidean norm of that view's loss gradient with respect to mean i and
 * visible_count[i] by one.  The views are added in view order in fp32.
 * mgs_merge_mask turns the pair into M(G).  Set both or neither. */
typedef struct mgs_gaussian_grads {
    float *d_means;   /* [n][3] */
    float *d_scales;  /* [n][3] */
    float *d_quats;   /* [n][4] w.r.t. the raw (unnormalised) quaternion */
    float *d_opac;    /* [n] */
    float *d_sh;      /* [n][K][3] */
    float *grad_norm_sum;     /* [n] accumulated, see above */
    uint32_t *visible_count;  /* [n] accumulated, see above */
} mgs_gaussian_grads;

/* A pinhole camera with pose T_CW (Eq. (1)). */
typedef struct mgs_camera {
    int32_t width, height; /* pixels, 1..16384 */
    float fx, fy, cx, cy;  /* intrinsics, fx, fy > 0 */
    float Tcw[12];         /* row-major [R | t], world -> camera */
    float near_z;          /* Gaussians with camera-frame z <= near_z are culled */
    int32_t map;           /* index of the rendered map in the `maps` array */
} mgs_camera;

typedef struct mgs_render_opts {
    float bg_rgb[3];       /* background colour composited behind the last Gaussian */
    float bg_depth;        /* background depth (0: D is the plain Eq. (11) sum) */
    int32_t need_backward; /* non-zero: reserve workspace for mgs_render_backward */
    int32_t count_blended; /* non-zero: the forward also counts, per pixel, the Gaussians it
                              blends (uint32 at info->off_n_blend; a slower instrumented blend) */
    /* host float[4] (nullable): device time of the call's stages in ms, taken
     * with HIP events on `stream`; the call then waits for its stream before
     * returning.  Forward: [0] projection, [1] binning and sorting (includes the
     * count read-back), [2] blend, [3] whole call.  Backward: [0] blend
     * backward, [1] per-Gaussian backward and pose reduction, [2] unused,
     * [3] whole call. */
    float *stage_ms;
    /* host void*[4] (nullable): caller-created hipEvent_t handles.  The call
     * records stage boundary b (the ends of the stages listed for stage_ms,
     * preceded by the call's start) into stage_events[b] on `stream` and does
     * not wait: forward boundaries 0..3 (start, projection, binning, blend),
     * backward 0..2 (start, blend backward, end).  Elapsed times are the
     * caller's to read once the stream has reached them. */
    void **stage_events;
} mgs_render_opts;

/* Sizes and the layout of the forward state kept in the workspace.  Filled by
 * mgs_render_forward (also when it returns MGS_ERR_WORKSPACE after counting);
 * passed unchanged to mgs_render_backward. */
typedef struct mgs_forward_info {
    int64_t n_pairs;      /* sum over views of the rendered map's size */
    int64_t n_visible;    /* (Gaussian, view) pairs that survive culling and reach a tile */
    int64_t n_instances;  /* (pair, bin) instances = entries of all bin lists */
    int64_t n_bins;       /* list bins: sum over views of ceil(TX/bin_tx) * ceil(TY/bin_ty),
                             TX = ceil(W/16), TY = ceil(H/16) */
    int64_t n_pixels;     /* sum over views of W * H */
    size_t ws_required;   /* bytes needed for this call (and its backward when requested) */
    /* byte offsets of the forward state inside ws (inspection and tests) */
    size_t off_pair_depth;  /* uint32 [n_pairs] float bits of camera z; 0xFFFFFFFF when culled */
    size_t off_pair_rect;   /* uint16 [n_pairs][4] tile rectangle x0, y0, x1, y1 (half open);
                               only for pairs whose depth key is not 0xFFFFFFFF */
    size_t off_pair_uvr;    /* float [n_pairs][4] image mean u, v, radius r, camera z (same) */
    size_t off_rank_pair;   /* uint32 [n_visible] pair index of each depth rank */
    /* the sorted bin lists (by bin, then depth rank), in one of two formats:
     * packed (inst_bin_bits > 0): off_inst_key: uint64 [n_instances]
     *   bin | rank << inst_bin_bits | slot << (inst_bin_bits + inst_rank_bits),
     *   slot = the backward record slot; off_inst_rec: unused (0);
     * wide (inst_bin_bits = 0): off_inst_key: uint64 [n_instances]
     *   (global bin id << 32) | depth rank; off_inst_rec: uint32 [n_instances]
     *   backward record slot of each sorted instance. */
    size_t off_inst_key;
    size_t off_inst_rec;
    size_t off_bin_range;   /* uint32 [n_bins][2] [first, last) instance of each bin */
    size_t off_n_contrib;   /* uint32 [n_pixels] 1 + position, in the pixel's bin list, of the
                               last blended Gaussian (0: none) */
    size_t off_n_blend;     /* uint32 [n_pixels] blended Gaussians (written when count_blended) */
    int32_t n_views;
    int32_t n_maps;
    int32_t need_backward;
    int32_t bin_tx;  /* 16x16 tiles per list bin along x (1 or 2) */
    int32_t bin_ty;  /* and along y (1 or 2) */
    int32_t inst_bin_bits;   /* packed instance keys when > 0: bits of the bin field, enough for
                                n_bins + 1 values; used when bin, rank and slot fit 64 bits (the
                                environment variable MGS_WIDE_INSTANCES=1 forces the wide format) */
    int32_t inst_rank_bits;  /* packed: bits of the depth-rank field (enough for n_visible values) */
} mgs_forward_info;

/*
 * mgs_render_forward - rasterise n_views views (Sec. II-E, Eq. (11)).
 *
 * maps [n_maps] (host array of map descriptors), cams [n_views] (host).
 * For every view: project every Gaussian of its map (Eq. (1)-(2) with a
 * +0.3 px^2 low-pass dilation), cull (non-finite or non-positive inputs,
 * z <= near_z, non-positive 2D determinant, empty tile rectangle), bin into
 * 16x16 tiles over a 3-sigma rectangle, sort each tile's list by camera depth
 * (ties by Gaussian index), and composite front to back per pixel.  Lists are
 * kept per bin of bin_tx x bin_ty tiles (one tile by default; the
 * environment variable MGS_BIN_TILES = "2x1" or "2x2" selects bins of 32 x 16
 * or 32 x 32 pixels, one wavefront each); within a bin each Gaussian reaches
 * only the pixels of its own tile rectangle.  Bins of the rectangle
 * where no pixel can reach alpha >= 1/255 (a conservative ellipse test per
 * bin row) are left out of the lists: every image is the one the full
 * rectangle gives, the list positions are those of the shorter lists, and a
 * Gaussian with no such bin is not visible.  Per pixel:
 * alpha = min(0.99, o * exp(-d^T Sigma_I^-1 d / 2)); Gaussians with alpha < 1/255
 * are skipped; the walk stops before a Gaussian that would take the
 * transmittance below 1e-4.  C = sum c_i alpha_i T_i + T bg_rgb,
 * D = sum z_i alpha_i T_i + T bg_depth.
 *
 * out_rgb   device float [sum_v 3 H_v W_v]   (packed per view, see above)
 * out_depth device float [sum_v H_v W_v]
 * out_T     device float [sum_v H_v W_v]     final transmittance (kept for backward)
 * ws, ws_bytes  workspace; info (host, required) receives counts and layout.
 *
 * Synchronisation: the call waits on `stream` once, for a 16-byte device-to-
 * host copy of the visible-pair and instance counts, before it can size the
 * sort; everything else is asynchronous.  If ws_bytes < info->ws_required the
 * call returns MGS_ERR_WORKSPACE after that wait (outputs untouched); retry with
 * a workspace of at least info->ws_required bytes.  When this error (or
 * MGS_ERR_TOO_LARGE) comes after work was queued on the workspace, the call
 * first waits for its stream, so the workspace may be freed or regrown at once.
 */
mgs_status mgs_render_forward(const mgs_gaussians *maps, int32_t n_maps, const mgs_camera *cams,
                              int32_t n_views, const mgs_render_opts *opts, void *ws,
                              size_t ws_bytes, mgs_forward_info *info, float *out_rgb,
                              float *out_depth, float *out_T, void *stream);

/*
 * mgs_render_backward - gradient of a loss L through the forward pass above.
 *
 * Same maps, cams and opts as the forward; ws and info exactly as the forward
 * left them (the forward must have been called with opts->need_backward != 0);
 * out_T is the forward's out_T.  Per-pixel transmittance along each list is
 * recomputed from the final transmittance, not stored.
 *
 * dL_drgb   device float, packed like out_rgb (required)
 * dL_ddepth device float, packed like out_depth (nullable: no depth loss)
 * grads     host array [n_maps]; each map's device outputs, nullable each
 * d_pose    device float [n_views][6] (nullable): dL/dxi for the left
 *           perturbation T_CW <- Exp(xi) T_CW, xi = (rho, theta)
 * Tracking: when no map asks for any Gaussian gradient or statistic (every
 * pointer of every grads entry null), only the pose gradient is formed and the
 * per-Gaussian passes are skipped; d_pose is bit-identical to a full call's.
 * Asynchronous on `stream`.
 */
mgs_status mgs_render_backward(const mgs_gaussians *maps, int32_t n_maps, const mgs_camera *cams,
                               int32_t n_views, const mgs_render_opts *opts,
                               const mgs_forward_info *info, void *ws, size_t ws_bytes,
                               const float *out_T, const float *dL_drgb, const float *dL_ddepth,
                               const mgs_gaussian_grads *grads, float *d_pose, void *stream);

/* mgs_voxel_merge policy flags */
#define MGS_MERGE_SEQUENTIAL 0
#define MGS_MERGE_BEST_PAIR 1
#define MGS_MERGE_LBFGS 2

/* Writable map for the merge output (device, capacity n each; all required). */
typedef struct mgs_gaussians_out {
    float *means, *scales, *quats, *opac, *sh;
} mgs_gaussians_out;

/*
 * mgs_voxel_merge - merge geometrically similar Gaussians that share a voxel
 * (Sec. II-D).
 *
 * in        the map; mask device uint8 [n] (nullable = all eligible) is the
 *           merge-eligibility mask M(G) of Eq. (3), computed by the caller.
 * Eligible Gaussians with finite means are grouped by the voxel
 * floor(mean / voxel_size) (per axis, fp32, cells within [-2^20, 2^20)).
 * Within a voxel Gaussians are visited in index (insertion) order; a visited
 * G_j is compared with the Gaussians G_i already present by the squared
 * Mahalanobis distance of Eq. (4) under Sigma_i; if the smallest one is below
 * `chi2` (the paper uses 7.815) the pair merges: mean by Eq. (6), covariance
 * by the minimiser of Eq. (9) (the equal-weight 2-Wasserstein barycenter,
 * computed in closed form), rotation and scale by its eigen-decomposition
 * canonicalised towards slerp(q_i, q_j, 1/2) (Eq. (10)), opacity and colour
 * from G_i.  policy, OR-ed flags: 0 (MGS_MERGE_SEQUENTIAL): every visited
 * Gaussian merges into its nearest present Gaussian when similar, else it
 * stays (sequential insertion); MGS_MERGE_BEST_PAIR: only the single closest
 * pair of the voxel merges; MGS_MERGE_LBFGS: the merged covariance comes from
 * the paper's own solver instead of the closed form, L-BFGS over (q_k, s_k)
 * from the Eq. (10) start slerp(q_i, q_j, 1/2), (s_i + s_j)/2 + (1, 2, 3) mm
 * (with G_j's axes first matched to G_i's: of its 24 equivalent (q, s), the
 * one nearest q_i), in fp64 until the largest gradient entry (scales in units
 * of the pair's mean scale) is 1e-6 or 128 iterations; (q_k, s_k) are then the
 * solver's (the quaternion with w >= 0), not the canonical frame.  It is
 * slower (a few tens of objective evaluations per merge).
 *
 * out        compacted map (survivors in their original order, merged values
 *            in the surviving slot); must not alias `in`.
 * old_to_new device int32 [n] (nullable): new index, or -1 for removed Gaussians.
 * voxel_key  device uint64 [n] (nullable): packed cell of each Gaussian, 21 bits
 *            per axis biased by 2^20, x most significant; ~0 when not eligible.
 * n_out      host: number of Gaussians written to out.
 * ws, ws_bytes, ws_required (host): workspace protocol as in the forward, but
 *            the size is known before any work: ws_required is set on return
 *            in every case (0 for an empty map, which needs no workspace).
 * Synchronisation: waits on `stream` twice: for the cell bounds and the
 * eligible count (40 bytes, to size the key sort) and for the survivor count.
 */
mgs_status mgs_voxel_merge(const mgs_gaussians *in, const uint8_t *mask, float voxel_size,
                           float chi2, int32_t policy, mgs_gaussians_out *out, int32_t *old_to_new,
                           uint64_t *voxel_key, void *ws, size_t ws_bytes, size_t *ws_required,
                           int64_t *n_out, void *stream);

/*
 * mgs_merge_mask - the merge-eligibility mask M(G) of Eq. (3) (Sec. II-D):
 * M(G) = [grad G < tau  and  K_min <= K <= K_max].
 *
 * grad G is the average gradient of each Gaussian over the statistics window,
 * grad_norm_sum[i] / visible_count[i] as accumulated by mgs_render_backward,
 * divided in fp32 (correctly rounded); a Gaussian with visible_count 0 has no
 * average and is not eligible.  K is the index, in the keyframe list, of the
 * keyframe at which the Gaussian entered the map.
 *
 * grad_norm_sum  device float [n]
 * visible_count  device uint32 [n]
 * kf_index       device int32 [n] (nullable: every Gaussian is inside the window)
 * tau            gradient threshold (the paper uses 0.001); NaN is rejected
 * kf_min, kf_max keyframe window, inclusive at both ends
 * mask           device uint8 [n] out: 1 eligible, 0 not; the mask argument of
 *                mgs_voxel_merge
 * Errors: MGS_ERR_INVALID_ARG for n < 0, a NaN tau or a null array with n > 0
 * (nothing launched).  Asynchronous on `stream`; n = 0 launches nothing.
 */
mgs_status mgs_merge_mask(const float *grad_norm_sum, const uint32_t *visible_count, const int32_t *kf_index,
                          int64_t n, float tau, int32_t kf_min, int32_t kf_max, uint8_t *mask, void *stream);

/* Weights of the mapping loss (Eq. (12)). */
typedef struct mgs_loss_opts {
    float lambda_ssim; /* lambda of Eq. (12): weight of 1 - SSIM against the colour L1 (0.2 is usual) */
    float w_depth;     /* weight of the depth residual (used when depth and gt_depth are given) */
    float w_iso;       /* weight of L_iso (used when scales are given) */
    int32_t reserved;
} mgs_loss_opts;

/*
 * mgs_mapping_loss - value and gradient of the mapping loss of Eq. (12)
 * (Sec. II-E) over n_views rendered views, packed as mgs_render_forward
 * writes them, so that its gradients feed mgs_render_backward directly.
 *
 * Per view (W x H pixels, means over every pixel and colour channel):
 *   L_view = (1 - lambda) mean |I_r - I_gt| + lambda (1 - mean SSIM(I_r, I_gt))
 *            + w_depth mean(valid |D - D_gt|),  valid = D_gt > 0,
 * and for the map  L_iso = w_iso mean_{i,k} |s_ik - (s_i0 + s_i1 + s_i2) / 3|.
 * The total is the sum of L_view over the views plus L_iso.  SSIM uses an
 * 11 x 11 Gaussian window (sigma 1.5, weights summing to 1) with zero padding
 * at the border and C1 = 0.01^2, C2 = 0.03^2, per channel; the L1 terms take
 * sign(0) = 0.
 *
 * sizes       host int32 [n_views][2]: width, height of each view (1..16384)
 * rgb, gt_rgb device float, packed colour: view v holds 3*H_v*W_v floats [3][H][W]
 * depth, gt_depth device float, packed one-channel (nullable: no depth term;
 *             give both or neither)
 * scales      device float [n_gauss][3] linear scales (nullable: no L_iso)
 * loss        device float [4 * n_views + 2], written: per view (mean |I_r - I_gt|,
 *             mean SSIM, mean(valid |D - D_gt|), L_view), then L_iso, then the total
 * dL_drgb     device float packed like rgb, written
 * dL_ddepth   device float packed like depth, written (required with depth)
 * dL_dscales  device float [n_gauss][3], written (required with scales)
 * ws, ws_bytes, ws_required (host): workspace; *ws_required is set on return in
 *             every case; MGS_ERR_WORKSPACE when ws_bytes is smaller (nothing
 *             launched).  About 36 bytes per pixel.
 * Errors: MGS_ERR_INVALID_ARG (nothing launched) for n_views <= 0 or > 4096, a
 * size out of range, a null required pointer, n_gauss < 0, a non-finite weight.
 * Asynchronous on `stream`; the values are deterministic (fixed reduction order).
 */
mgs_status mgs_mapping_loss(const int32_t *sizes, int32_t n_views, const float *rgb, const float *gt_rgb,
                            const float *depth, const float *gt_depth, const float *scales, int64_t n_gauss,
                            const mgs_loss_opts *opts, void *ws, size_t ws_bytes, size_t *ws_required,
                            float *loss, float *dL_drgb, float *dL_ddepth, float *dL_dscales, void *stream);

/*
 * mgs_mapping_loss_noalloc - mgs_mapping_loss without a workspace, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid hipMalloc.
 *
 * The same loss, gradients and argument meanings as mgs_mapping_loss, bit for
 * bit (the same kernels); in place of ws / ws_bytes / ws_required the call uses
 * a scratch array compiled into the library: MGS_LOSS_SCRATCH_BYTES (64 MiB) of
 * device memory per GPU, held from the library's first use on that GPU until
 * the process ends.  The call allocates and frees nothing.
 *
 * scratch_required host (nullable): the scratch the input needs, about 36 bytes
 *             per pixel (a 1200 x 680 view takes 29.4 MB, so two such views fit)
 * Limits: at most MGS_LOSS_NOALLOC_MAX_VIEWS views and MGS_LOSS_SCRATCH_BYTES of
 * scratch; beyond either the call returns MGS_ERR_SCRATCH and launches nothing
 * (use mgs_mapping_loss with a workspace instead).
 * The stream must belong to the current device (else MGS_ERR_INVALID_ARG).
 * Concurrency: every call on one GPU shares that GPU's scratch, which keeps the
 * last call's contents; calls that overlap on one GPU (different streams, or
 * host threads without ordering between them) race and must be serialised by
 * the caller.  Asynchronous on `stream`.
 */
#define MGS_LOSS_SCRATCH_BYTES ((size_t)64 << 20)
#define MGS_LOSS_NOALLOC_MAX_VIEWS 64
mgs_status mgs_mapping_loss_noalloc(const int32_t *sizes, int32_t n_views, const float *rgb, const float *gt_rgb,
                                    const float *depth, const float *gt_depth, const float *scales, int64_t n_gauss,
                                    const mgs_loss_opts *opts, size_t *scratch_required, float *loss,
                                    float *dL_drgb, float *dL_ddepth, float *dL_dscales, void *stream);

/* Controls of Patch-Grid sampling (Sec. II-B). */
typedef struct mgs_pg_opts {
    int32_t patch;          /* patch edge P in pixels, >= 1 */
    int32_t min_keypoints;  /* a patch holding fewer keypoints than this is sampled, >= 0 */
    int32_t samples;        /* s: an s x s lattice of samples per sampled patch, 1..64 */
    float opacity;          /* opacity of the new Gaussians */
    float scale_factor;     /* their isotropic scale: scale_factor * depth * (P / s) / fx */
    int32_t reserved;
} mgs_pg_opts;

/*
 * mgs_patch_grid_sample - new Gaussians from a keyframe by Patch-Grid sampling
 * (Sec. II-B): the image is cut into P x P patches; a patch holding fewer than
 * min_keypoints keypoints is sampled uniformly; every keypoint and every sample
 * becomes a Gaussian centred on its back-projection.
 *
 * cam        host: image size, intrinsics and pose T_CW (near_z and map unused)
 * keypoints  device float [n_kp][2] pixel coordinates (u, v), pixel centres at
 *            integers; keypoint i lies on pixel (floor(u + 1/2), floor(v + 1/2));
 *            keypoints off the image are ignored
 * kp_depth   device float [n_kp]: measured depth of each keypoint, <= 0 (or NaN)
 *            when it has none (inactive or monocular keypoints)
 * depth_map  device float [H][W] (nullable: monocular); <= 0 marks no depth
 * image      device float [3][H][W] colour in [0, 1]
 * Sampling: pixel (x, y) lies in patch (x / P, y / P); a sampled patch gets an
 *   s x s lattice over its part of the image (w x h pixels): sample (k, l) on
 *   pixel (P px + ((2k+1) w) / (2s), P py + ((2l+1) h) / (2s)) (integer division).
 * Depth of a point: a keypoint's own depth; else the depth map at its pixel;
 *   else the depth of the nearest keypoint that has its own depth (fp32 squared
 *   pixel distance, ties to the lower index).  A point without any is dropped.
 * Output, in order: the kept keypoints (input order), then the kept samples by
 *   patch (row-major) and lattice position (row-major).  Gaussian: mean
 *   R_CW^T (z ((x - cx)/fx, (y - cy)/fy, 1) - t_CW) with (x, y) the keypoint's
 *   coordinates or the sample's pixel; isotropic scale; identity rotation;
 *   opacity; SH degree 0 colour (rgb - 1/2) / C0 from the image at its pixel.
 * out        device arrays with room for n_kp + ceil(W/P) ceil(H/P) s^2
 *            Gaussians (sh: [n][1][3]); must not alias the inputs
 * source     device int32 [same capacity] (nullable): the candidate of each
 *            output, i < n_kp a keypoint, else n_kp + patch s^2 + l s + k
 * n_out      host: Gaussians written
 * ws, ws_bytes, ws_required (host): workspace; *ws_required is set in every
 *            case, MGS_ERR_WORKSPACE when ws_bytes is smaller (nothing launched)
 * Errors: MGS_ERR_INVALID_ARG (nothing launched) for bad sizes, intrinsics or
 * options, null required pointers.  Waits on `stream` once, for the count.
 */
mgs_status mgs_patch_grid_sample(const mgs_camera *cam, const float *keypoints, const float *kp_depth,
                                 int64_t n_kp, const float *depth_map, const float *image,
                                 const mgs_pg_opts *opts, mgs_gaussians_out *out, int32_t *source, void *ws,
                                 size_t ws_bytes, size_t *ws_required, int64_t *n_out, void *stream);

/* Adam hyper-parameters (one learning rate per parameter group). */
typedef struct mgs_adam_opts {
    float lr[5];     /* means, scales, quats, opac, sh */
    float beta1;     /* in [0, 1) */
    float beta2;     /* in [0, 1) */
    float eps;       /* >= 0 */
    int32_t step;    /* t >= 1, for the bias corrections 1 - beta^t */
} mgs_adam_opts;

/*
 * mgs_adam_step - one Adam step over a map's parameters for the mapping loop
 * that minimises the loss of Eq. (12) (Sec. II-E; the paper does not name its
 * optimiser, the Gaussian-splatting lineage it follows uses Adam).  Per element,
 * with g the gradient:  m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 * p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)  (fp32).
 *
 * params      device, updated in place: the map's arrays, [n] Gaussians
 * grads       device gradients (as mgs_render_backward writes them, plus any
 *             other terms the caller adds); a null gradient leaves its group
 *             untouched (its params and moments may then be null too)
 * exp_avg, exp_avg_sq  device first and second moments, laid out like params,
 *             updated in place (zero before the first step)
 * One launch for all groups; asynchronous on `stream`.  Errors:
 * MGS_ERR_INVALID_ARG for n < 0, sh_degree outside 0..3, step < 1, betas
 * outside [0, 1), a negative or non-finite eps, a non-finite learning rate, or
 * a null array of a group whose gradient is given.
 */
mgs_status mgs_adam_step(const mgs_gaussians_out *params, int64_t n, int32_t sh_degree,
                         const mgs_gaussian_grads *grads, const mgs_gaussians_out *exp_avg,
                         const mgs_gaussians_out *exp_avg_sq, const mgs_adam_opts *opts, void *stream);

/* Static description of a status code. */
const char *mgs_status_string(mgs_status status);

/* Text of the last HIP error seen by this thread inside the library ("" if none). */
const char *mgs_last_hip_error(void);

/* ABI version, (major << 16) | minor. */
int32_t mgs_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MEMGS_H */
