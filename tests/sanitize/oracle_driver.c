/* Drives every entry point of the C render oracle on a small scene with
 * degenerate members, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure, CPU only).  Inputs come
 * from a 64-bit linear congruential generator; nothing here computes the
 * method.  Prints a checksum of the outputs and exits 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_keys(int64_t n, const float *means, const float *scales, const float *quats, const float *opac,
                 const float *cam32, uint8_t *valid, uint32_t *depth_bits, int32_t *rect, float *uvr,
                 int64_t *tile_off, int32_t *tile_gid);
int64_t orc_forward(int64_t n, const float *means, const float *scales, const float *quats, const float *opac,
                    const float *sh, int deg, const float *cam32, const double *cam64, const double *bg,
                    double *out_rgb, double *out_depth, double *out_T, int32_t *out_nc, uint8_t *out_amb,
                    const double *bd3);
void orc_forward_alternatives(int64_t n, const float *means, const float *scales, const float *quats,
                              const float *opac, const float *sh, int deg, const float *cam32, const double *cam64,
                              const double *bg, const double *bd2, int64_t n_pix, const int32_t *pxs,
                              const int32_t *pys, int max_leaves, double *leaves, int32_t *leaf_gid,
                              int32_t *n_leaves);
int64_t orc_contributors(int64_t n, const float *means, const float *scales, const float *quats, const float *opac,
                         const float *sh, int deg, const float *cam32, const double *cam64, int64_t *counts,
                         int32_t *gids, uint8_t *clamped);
void orc_backward(int64_t n, const float *means, const float *scales, const float *quats, const float *opac,
                  const float *sh, int deg, const float *cam32, const double *cam64, const double *bg,
                  const double *dL_rgb, const double *dL_depth, double *d_means, double *d_scales, double *d_quats,
                  double *d_opac, double *d_sh, double *d_pose, double *grad2d);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double unif(void) { /* [0, 1) */
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    const int n = 300, deg = 2, K = (deg + 1) * (deg + 1), W = 45, H = 33;
    float *means = malloc(sizeof(float) * 3 * n), *scales = malloc(sizeof(float) * 3 * n);
    float *quats = malloc(sizeof(float) * 4 * n), *opac = malloc(sizeof(float) * n);
    float *sh = malloc(sizeof(float) * 3 * K * n);
    for (int g = 0; g < n; ++g) {
        means[3 * g] = (float)(unif() * 2 - 1);
        means[3 * g + 1] = (float)(unif() * 2 - 1);
        means[3 * g + 2] = (float)(unif() * 2 + 0.5);
        for (int k = 0; k < 3; ++k) scales[3 * g + k] = (float)exp(-3.0 + 0.7 * (unif() - 0.5));
        for (int k = 0; k < 4; ++k) quats[4 * g + k] = (float)(unif() - 0.5);
        opac[g] = (float)(0.05 + 0.94 * unif());
        for (int k = 0; k < 3 * K; ++k) sh[3 * K * g + k] = (float)(unif() - 0.5);
    }
    /* degenerate members: zero scale, zero quaternion, NaN mean, behind the camera, huge */
    scales[0] = 0.0f;
    for (int k = 0; k < 4; ++k) quats[4 + k] = 0.0f;
    means[6] = NAN;
    means[11] = -1.0f;
    for (int k = 0; k < 3; ++k) scales[12 + k] = 3.0f;
    opac[5] = 1.0f;
    float cam32[19] = {(float)W, (float)H, 40.0f, 42.0f, 22.0f, 16.0f, 0.2f, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.01f, -0.02f, 0.0f};
    double cam64[19];
    for (int k = 0; k < 19; ++k) cam64[k] = (double)cam32[k];
    const double bg[4] = {0.1, 0.2, 0.3, 0.5}, bands[2] = {2e-6, 1.5e-6};
    const int TX = (W + 15) / 16, TY = (H + 15) / 16, P = W * H;
    uint8_t *valid = malloc(n);
    uint32_t *depth_bits = malloc(sizeof(uint32_t) * n);
    int32_t *rect = malloc(sizeof(int32_t) * 4 * n);
    float *uvr = malloc(sizeof(float) * 3 * n);
    int64_t *tile_off = malloc(sizeof(int64_t) * (TX * TY + 1));
    const int64_t M = orc_keys(n, means, scales, quats, opac, cam32, valid, depth_bits, rect, uvr, tile_off, NULL);
    int32_t *tile_gid = malloc(sizeof(int32_t) * (M > 0 ? M : 1));
    orc_keys(n, means, scales, quats, opac, cam32, NULL, NULL, NULL, NULL, NULL, tile_gid);
    double *rgb = malloc(sizeof(double) * 3 * P), *depth = malloc(sizeof(double) * P), *T = malloc(sizeof(double) * P);
    int32_t *nc = malloc(sizeof(int32_t) * P);
    uint8_t *amb = malloc(P);
    orc_forward(n, means, scales, quats, opac, sh, deg, cam32, cam64, bg, rgb, depth, T, nc, amb, bands);
    int32_t *px = malloc(sizeof(int32_t) * P), *py = malloc(sizeof(int32_t) * P);
    for (int i = 0; i < P; ++i) { px[i] = i % W; py[i] = i / W; }
    const int L = 16;
    double *leaves = malloc(sizeof(double) * (size_t)P * L * 5);
    int32_t *lgid = malloc(sizeof(int32_t) * (size_t)P * L), *nl = malloc(sizeof(int32_t) * P);
    orc_forward_alternatives(n, means, scales, quats, opac, sh, deg, cam32, cam64, bg, bands, P, px, py, L, leaves,
                             lgid, nl);
    int64_t *counts = malloc(sizeof(int64_t) * P);
    const int64_t tot = orc_contributors(n, means, scales, quats, opac, sh, deg, cam32, cam64, counts, NULL, NULL);
    int32_t *gids = malloc(sizeof(int32_t) * (tot > 0 ? tot : 1));
    uint8_t *cl = malloc(tot > 0 ? tot : 1);
    orc_contributors(n, means, scales, quats, opac, sh, deg, cam32, cam64, counts, gids, cl);
    double *g_rgb = malloc(sizeof(double) * 3 * P), *g_d = malloc(sizeof(double) * P);
    for (int i = 0; i < 3 * P; ++i) g_rgb[i] = unif() - 0.5;
    for (int i = 0; i < P; ++i) g_d[i] = unif() - 0.5;
    double *dm = calloc(3 * n, sizeof(double)), *ds = calloc(3 * n, sizeof(double)), *dq = calloc(4 * n, sizeof(double));
    double *dop = calloc(n, sizeof(double)), *dsh = calloc(3 * K * n, sizeof(double)), *dpose = calloc(6, sizeof(double));
    double *g2 = calloc(10 * (size_t)n, sizeof(double)); /* [n][10] per-Gaussian 2D gradient sums */
    orc_backward(n, means, scales, quats, opac, sh, deg, cam32, cam64, bg, g_rgb, g_d, dm, ds, dq, dop, dsh, dpose, g2);
    double sum = 0.0;
    for (int i = 0; i < 3 * P; ++i) sum += rgb[i];
    for (int i = 0; i < P; ++i) sum += depth[i] + T[i] + nc[i] + amb[i] + (nl[i] > 0 ? leaves[(size_t)i * L * 5] : 0);
    for (int i = 0; i < 3 * n; ++i) sum += dm[i] + ds[i];
    for (int i = 0; i < 6; ++i) sum += dpose[i];
    printf("instances %lld contributors %lld checksum %.9g\n", (long long)M, (long long)tot, sum);
    free(means); free(scales); free(quats); free(opac); free(sh); free(valid); free(depth_bits); free(rect);
    free(uvr); free(tile_off); free(tile_gid); free(rgb); free(depth); free(T); free(nc); free(amb); free(px);
    free(py); free(leaves); free(lgid); free(nl); free(counts); free(gids); free(cl); free(g_rgb); free(g_d);
    free(dm); free(ds); free(dq); free(dop); free(dsh); free(dpose); free(g2);
    return isfinite(sum) ? 0 : 1;
}
