/* Drives the host side of the C ABI (include/memgs.h) on the paths that end
 * before any device work: argument validation, workspace sizing (the query
 * with no workspace), the fixed-scratch limits, status strings.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (test
 * infrastructure, CPU only, no GPU needed).  Device pointers are never
 * dereferenced on these paths, so placeholders stand in for them.  Exits 0
 * when every call returns the expected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "memgs.h"

static int failures = 0;
#define EXPECT(call, want)                                                                    \
    do {                                                                                      \
        const mgs_status got_ = (call);                                                       \
        if (got_ != (want)) {                                                                 \
            fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, got_, \
                    (int)(want));                                                             \
            ++failures;                                                                       \
        }                                                                                     \
    } while (0)

static float dev_placeholder[64];
#define DP ((void *)dev_placeholder)

static mgs_camera camera(int W, int H, int map) {
    mgs_camera c;
    memset(&c, 0, sizeof(c));
    c.width = W;
    c.height = H;
    c.fx = c.fy = 600.0f;
    c.cx = 0.5f * (float)W;
    c.cy = 0.5f * (float)H;
    c.Tcw[0] = c.Tcw[5] = c.Tcw[10] = 1.0f;
    c.near_z = 0.2f;
    c.map = map;
    return c;
}

int main(void) {
    for (int s = 1; s >= -6; --s) (void)strlen(mgs_status_string(s));
    (void)strlen(mgs_last_hip_error());
    if (mgs_abi_version() <= 0) ++failures;

    /* ---- forward: validation and the workspace query */
    mgs_gaussians maps[3];
    for (int m = 0; m < 3; ++m) {
        maps[m].n = 1000 * (m + 1);
        maps[m].means = maps[m].scales = maps[m].quats = maps[m].opac = maps[m].sh = (const float *)DP;
        maps[m].sh_degree = m;
        maps[m].reserved = 0;
    }
    mgs_camera cams[40];
    for (int v = 0; v < 40; ++v) cams[v] = camera(v % 3 == 0 ? 1200 : 97 + v, v % 3 == 0 ? 680 : 33 + 2 * v, v % 3);
    mgs_render_opts opts;
    memset(&opts, 0, sizeof(opts));
    opts.need_backward = 1;
    mgs_forward_info info;
    float *o = (float *)DP;
    EXPECT(mgs_render_forward(maps, 3, cams, 40, &opts, NULL, 0, NULL, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    EXPECT(mgs_render_forward(maps, 0, cams, 4, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    EXPECT(mgs_render_forward(maps, 3, cams, 0, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    EXPECT(mgs_render_forward(maps, 3, cams, 40, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_WORKSPACE);
    if (!(info.ws_required > 0 && info.n_views == 40 && info.n_pairs > 0)) ++failures;
    EXPECT(mgs_render_forward(maps, 3, cams, 5, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_WORKSPACE);
    mgs_camera bad = cams[1];
    bad.width = 0;
    EXPECT(mgs_render_forward(maps, 3, &bad, 1, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    bad = cams[1];
    bad.map = 3;
    EXPECT(mgs_render_forward(maps, 3, &bad, 1, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    bad = cams[1];
    bad.fx = -1.0f;
    EXPECT(mgs_render_forward(maps, 3, &bad, 1, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    mgs_gaussians deg4 = maps[0];
    deg4.sh_degree = 4;
    EXPECT(mgs_render_forward(&deg4, 1, cams, 1, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_INVALID_ARG);
    mgs_gaussians huge = maps[0];
    huge.n = (int64_t)1 << 40;
    EXPECT(mgs_render_forward(&huge, 1, cams, 1, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_TOO_LARGE);

    /* ---- backward: validation against the forward's info */
    mgs_gaussian_grads grads[3];
    memset(grads, 0, sizeof(grads));
    EXPECT(mgs_render_backward(maps, 3, cams, 40, &opts, NULL, DP, 0, o, o, NULL, grads, NULL, NULL),
           MGS_ERR_INVALID_ARG);
    EXPECT(mgs_render_forward(maps, 3, cams, 40, &opts, NULL, 0, &info, o, o, o, NULL), MGS_ERR_WORKSPACE);
    mgs_forward_info wrong = info;
    wrong.n_views = 39;
    EXPECT(mgs_render_backward(maps, 3, cams, 40, &opts, &wrong, DP, 1 << 20, o, o, NULL, grads, NULL, NULL),
           MGS_ERR_INVALID_ARG);
    grads[1].grad_norm_sum = o;  /* a statistic without its pair */
    EXPECT(mgs_render_backward(maps, 3, cams, 40, &opts, &info, DP, 1 << 20, o, o, NULL, grads, NULL, NULL),
           MGS_ERR_INVALID_ARG);
    grads[1].grad_norm_sum = NULL;
    EXPECT(mgs_render_backward(maps, 3, cams, 40, &opts, &info, DP, 16, o, o, NULL, grads, NULL, NULL),
           MGS_ERR_WORKSPACE);

    /* ---- voxel merge */
    mgs_gaussians_out out = {o, o, o, o, o};
    size_t req = 0;
    int64_t n_out = -1;
    EXPECT(mgs_voxel_merge(&maps[1], NULL, 0.05f, 7.815f, 0, &out, NULL, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_WORKSPACE);
    if (req == 0) ++failures;
    EXPECT(mgs_voxel_merge(&maps[1], NULL, 0.0f, 7.815f, 0, &out, NULL, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_INVALID_ARG);
    EXPECT(mgs_voxel_merge(&maps[1], NULL, 0.05f, NAN, 0, &out, NULL, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_INVALID_ARG);
    EXPECT(mgs_voxel_merge(&maps[1], NULL, 0.05f, 7.815f, 4, &out, NULL, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_INVALID_ARG);
    mgs_gaussians empty = maps[0];
    empty.n = 0;
    EXPECT(mgs_voxel_merge(&empty, NULL, 0.05f, 7.815f, 0, &out, NULL, NULL, NULL, 0, &req, &n_out, NULL), MGS_OK);
    if (req != 0 || n_out != 0) ++failures;

    /* ---- merge mask */
    EXPECT(mgs_merge_mask(o, (const uint32_t *)DP, NULL, -1, 1e-3f, 0, 10, (uint8_t *)DP, NULL), MGS_ERR_INVALID_ARG);
    EXPECT(mgs_merge_mask(o, (const uint32_t *)DP, NULL, 10, NAN, 0, 10, (uint8_t *)DP, NULL), MGS_ERR_INVALID_ARG);
    EXPECT(mgs_merge_mask(NULL, NULL, NULL, 0, 1e-3f, 0, 10, NULL, NULL), MGS_OK);

    /* ---- mapping loss and its allocation-free form */
    int32_t sizes[2 * 70];
    for (int v = 0; v < 70; ++v) { sizes[2 * v] = 1200; sizes[2 * v + 1] = 680; }
    mgs_loss_opts lo = {0.2f, 1.0f, 0.1f, 0};
    EXPECT(mgs_mapping_loss(sizes, 2, o, o, o, o, o, 1000, &lo, NULL, 0, &req, o, o, o, o, NULL), MGS_ERR_WORKSPACE);
    if (req < (size_t)2 * 1200 * 680 * 36) ++failures;
    EXPECT(mgs_mapping_loss(sizes, 0, o, o, NULL, NULL, NULL, 0, &lo, NULL, 0, &req, o, o, NULL, NULL, NULL),
           MGS_ERR_INVALID_ARG);
    lo.w_depth = INFINITY;
    EXPECT(mgs_mapping_loss(sizes, 1, o, o, o, o, NULL, 0, &lo, NULL, 0, &req, o, o, o, NULL, NULL),
           MGS_ERR_INVALID_ARG);
    lo.w_depth = 1.0f;
    EXPECT(mgs_mapping_loss(sizes, 1, o, o, o, NULL, NULL, 0, &lo, NULL, 0, &req, o, o, o, NULL, NULL),
           MGS_ERR_INVALID_ARG);  /* depth without a target */
    size_t need = 0;
    EXPECT(mgs_mapping_loss_noalloc(sizes, 3, o, o, NULL, NULL, NULL, 0, &lo, &need, o, o, NULL, NULL, NULL),
           MGS_ERR_SCRATCH);
    if (need <= MGS_LOSS_SCRATCH_BYTES) ++failures;
    EXPECT(mgs_mapping_loss_noalloc(sizes, MGS_LOSS_NOALLOC_MAX_VIEWS + 1, o, o, NULL, NULL, NULL, 0, &lo, &need, o,
                                    o, NULL, NULL, NULL),
           MGS_ERR_SCRATCH);
    sizes[0] = 0;
    EXPECT(mgs_mapping_loss_noalloc(sizes, 1, o, o, NULL, NULL, NULL, 0, &lo, &need, o, o, NULL, NULL, NULL),
           MGS_ERR_INVALID_ARG);

    /* ---- Patch-Grid sampling */
    mgs_camera kf = camera(1200, 680, 0);
    mgs_pg_opts pg = {32, 4, 2, 0.5f, 0.5f, 0};
    EXPECT(mgs_patch_grid_sample(&kf, o, o, 2000, NULL, o, &pg, &out, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_WORKSPACE);
    pg.samples = 0;
    EXPECT(mgs_patch_grid_sample(&kf, o, o, 2000, NULL, o, &pg, &out, NULL, NULL, 0, &req, &n_out, NULL),
           MGS_ERR_INVALID_ARG);

    /* ---- Adam */
    mgs_gaussian_grads g;
    memset(&g, 0, sizeof(g));
    g.d_means = o;
    mgs_adam_opts ao = {{1e-3f, 1e-3f, 1e-3f, 1e-3f, 1e-3f}, 0.9f, 0.999f, 1e-8f, 0};
    EXPECT(mgs_adam_step(&out, 100, 0, &g, &out, &out, &ao, NULL), MGS_ERR_INVALID_ARG);  /* step 0 */
    ao.step = 1;
    ao.beta1 = 1.0f;
    EXPECT(mgs_adam_step(&out, 100, 0, &g, &out, &out, &ao, NULL), MGS_ERR_INVALID_ARG);
    ao.beta1 = 0.9f;
    EXPECT(mgs_adam_step(&out, -1, 0, &g, &out, &out, &ao, NULL), MGS_ERR_INVALID_ARG);

    printf("abi host checks: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
