/*
 * CPU oracle for the MemGS rasterizer: forward and backward.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code, header, table or constant generator with the
 * HIP path.
 *
 * What it computes (one camera at a time):
 *   - Sec. II-C, Eq. (1)-(2): covariance from rotation and scale, mean and
 *     covariance projected to the image with the linearised (EWA) projection.
 *   - Sec. II-C: colour from spherical harmonics (degree <= 3).
 *   - Sec. II-E, Eq. (11): front-to-back alpha compositing of colour and of
 *     camera-frame depth over the depth-sorted Gaussians of the pixel's 16x16
 *     tile ("tile-based rendering").
 *   - the exact derivative of that forward pass w.r.t. means, scales,
 *     quaternions, opacities, SH coefficients and the SE(3) camera pose
 *     (left perturbation T <- Exp(xi) T, xi = (rho, theta)).
 *
 * Two numeric paths:
 *   1. the fp32 "key path" decides culling, the tile rectangle and the depth
 *      sort key; it is written as a fixed sequence of IEEE fp32 operations
 *      (this file is compiled with -ffp-contract=off) because those decisions
 *      are integers that the GPU must reproduce bit for bit;
 *   2. the fp64 "value path" computes every value (image, depth, gradients)
 *      from the same fp32 inputs widened to double.
 *
 * Readings of the paper taken here where it is silent are listed in the
 * design notes: alpha clamp 0.99, skip alpha < 1/255, stop before a Gaussian
 * that would take transmittance below 1e-4 (that Gaussian is not blended),
 * +0.3 px^2 low-pass dilation, 3-sigma radius from the larger eigenvalue with a
 * 0.1 floor, near plane, 1.3x frustum clamp of the Jacobian, pixel (u,v)
 * evaluated at integer coordinates, ties in depth broken by Gaussian index.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16

static const float kAlphaMax = 0.99f;
static const float kAlphaMin = 1.0f / 255.0f;
static const float kTMin = 1e-4f;
static const float kDilation = 0.3f;
static const float kFrustum = 1.3f;

/* Real spherical-harmonic basis, degree 0..3, index l*l + l + m: sqrt(2) Re Y_l^m
 * for m > 0 and sqrt(2) Im Y_l^|m| for m < 0 of the complex harmonics carrying
 * the Condon-Shortley phase (the 3DGS convention).  The tests check
 * orthonormality by quadrature and the match with scipy's harmonics. */
static const double SH_C0 = 0.28209479177387814;
static const double SH_C1 = 0.4886025119029199;
static const double SH_C2[5] = {1.0925484305920792, -1.0925484305920792, 0.31539156525252005,
                                -1.0925484305920792, 0.5462742152960396};
static const double SH_C3[7] = {-0.5900435899266435, 2.890611442640554, -0.4570457994644658,
                                0.3731763325901154, -0.4570457994644658, 1.445305721320277,
                                -0.5900435899266435};

/* camera layout (float32 for the key path, float64 for the value path):
 * [W, H, fx, fy, cx, cy, near, R00, R01, R02, R10, R11, R12, R20, R21, R22, t0, t1, t2] */
enum { CW = 0, CH, CFX, CFY, CCX, CCY, CNEAR, CR, CT = 16, CAM_LEN = 19 };

/* ------------------------------------------------------------------ key path */
typedef struct {
    int valid;
    uint32_t depth_bits;
    float u, v, r;
    int32_t rect[4]; /* x0, y0, x1, y1 (tile units, half open) */
} keyproj;

static uint32_t f32_bits(float x) {
    uint32_t b;
    memcpy(&b, &x, 4);
    return b;
}

static float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

/* The pinned fp32 sequence K1..K12. */
static void key_path(const float *m, const float *s, const float *q, float o, const float *cam,
                     int TX, int TY, keyproj *out) {
    out->valid = 0;
    const float Wf = cam[CW], Hf = cam[CH], fx = cam[CFX], fy = cam[CFY], cx = cam[CCX],
                cy = cam[CCY], nearz = cam[CNEAR];
    const float *Rc = cam + CR, *t = cam + CT;
    /* K1 inputs finite, scales and opacity positive */
    for (int k = 0; k < 3; ++k) {
        if (!isfinite(m[k])) return;
        if (!(s[k] > 0.0f) || !isfinite(s[k])) return;
    }
    if (!(o > 0.0f) || !isfinite(o)) return;
    /* K2 rotation of q/|q| written with 2/|q|^2 (no square root) */
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    const float nq = ((w * w + x * x) + y * y) + z * z;
    if (!(nq > 0.0f) || !isfinite(nq)) return;
    const float k2 = 2.0f / nq;
    float R[9];
    R[0] = 1.0f - k2 * (y * y + z * z);
    R[1] = k2 * (x * y - w * z);
    R[2] = k2 * (x * z + w * y);
    R[3] = k2 * (x * y + w * z);
    R[4] = 1.0f - k2 * (x * x + z * z);
    R[5] = k2 * (y * z - w * x);
    R[6] = k2 * (x * z - w * y);
    R[7] = k2 * (y * z + w * x);
    R[8] = 1.0f - k2 * (x * x + y * y);
    /* K3 Sigma_W = M M^T with M = R diag(s) */
    float M[9];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) M[3 * a + k] = R[3 * a + k] * s[k];
    float S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S[3 * a + b] = (M[3 * a + 0] * M[3 * b + 0] + M[3 * a + 1] * M[3 * b + 1]) +
                           M[3 * a + 2] * M[3 * b + 2];
    /* K4 camera-frame mean, near-plane cull */
    float p[3];
    for (int a = 0; a < 3; ++a)
        p[a] = ((Rc[3 * a + 0] * m[0] + Rc[3 * a + 1] * m[1]) + Rc[3 * a + 2] * m[2]) + t[a];
    if (!(p[2] > nearz)) return;
    /* K5 Jacobian with the frustum clamp */
    const float xn = p[0] / p[2], yn = p[1] / p[2];
    const float limx = kFrustum * ((0.5f * Wf) / fx);
    const float limy = kFrustum * ((0.5f * Hf) / fy);
    const float xc = clampf(xn, -limx, limx) * p[2];
    const float yc = clampf(yn, -limy, limy) * p[2];
    const float pz2 = p[2] * p[2];
    const float J00 = fx / p[2], J02 = -(fx * xc) / pz2;
    const float J11 = fy / p[2], J12 = -(fy * yc) / pz2;
    /* K6 T = J W */
    float T[6];
    for (int b = 0; b < 3; ++b) {
        T[b] = J00 * Rc[b] + J02 * Rc[6 + b];
        T[3 + b] = J11 * Rc[3 + b] + J12 * Rc[6 + b];
    }
    /* K7 Sigma_I = T Sigma_W T^T, dilated */
    float U[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            U[3 * a + b] = (T[3 * a + 0] * S[b] + T[3 * a + 1] * S[3 + b]) + T[3 * a + 2] * S[6 + b];
    const float s00 = (U[0] * T[0] + U[1] * T[1]) + U[2] * T[2];
    const float s01 = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
    const float s11 = (U[3] * T[3] + U[4] * T[4]) + U[5] * T[5];
    const float a = s00 + kDilation, b = s01, c = s11 + kDilation;
    /* K8 */
    const float det = a * c - b * b;
    if (!(det > 0.0f)) return;
    /* K9 radius */
    const float mid = 0.5f * (a + c);
    const float disc = mid * mid - det;
    const float lam = mid + sqrtf(fmaxf(0.1f, disc));
    const float r = ceilf(3.0f * sqrtf(lam));
    /* K10 image-plane mean */
    const float u = fx * xn + cx, v = fy * yn + cy;
    if (!(fabsf(u) < 1e6f) || !(fabsf(v) < 1e6f) || !(r < 1e6f)) return;
    /* K11 tile rectangle */
    const float TXf = (float)TX, TYf = (float)TY;
    const int x0 = (int)clampf(floorf((u - r) * 0.0625f), 0.0f, TXf);
    const int x1 = (int)clampf(floorf((u + r) * 0.0625f) + 1.0f, 0.0f, TXf);
    const int y0 = (int)clampf(floorf((v - r) * 0.0625f), 0.0f, TYf);
    const int y1 = (int)clampf(floorf((v + r) * 0.0625f) + 1.0f, 0.0f, TYf);
    if (x0 >= x1 || y0 >= y1) return;
    /* K12 */
    out->valid = 1;
    out->depth_bits = f32_bits(p[2]);
    out->u = u;
    out->v = v;
    out->r = r;
    out->rect[0] = x0;
    out->rect[1] = y0;
    out->rect[2] = x1;
    out->rect[3] = y1;
}

/* ---------------------------------------------------------------- value path */
typedef struct {
    double qn[4], nq;       /* unit quaternion, |q| */
    double R[9];            /* R(qn) */
    double s[3];
    double SigW[9], Sigc[9];
    double p[3];
    int xclamp, yclamp;     /* 0 inside, -1 / +1 clamped at the lower / upper limit */
    double lim[2];
    double J[6];            /* rows (J00 J01 J02), (J10 J11 J12) */
    double cov[3];          /* dilated a, b, c */
    double conic[3];        /* A, B, C */
    double uv[2];
    double depth;
    double dir[3], dirn;    /* mean - camera centre, and its norm */
    double basis[16];
    double raw[3], rgb[3];
    double opac;
} vproj;

static void sh_basis(int deg, const double d[3], double *Y) {
    const double x = d[0], y = d[1], z = d[2];
    Y[0] = SH_C0;
    if (deg < 1) return;
    Y[1] = -SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = -SH_C1 * x;
    if (deg < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
    Y[4] = SH_C2[0] * xy;
    Y[5] = SH_C2[1] * yz;
    Y[6] = SH_C2[2] * (2.0 * zz - xx - yy);
    Y[7] = SH_C2[3] * xz;
    Y[8] = SH_C2[4] * (xx - yy);
    if (deg < 3) return;
    Y[9] = SH_C3[0] * y * (3.0 * xx - yy);
    Y[10] = SH_C3[1] * xy * z;
    Y[11] = SH_C3[2] * y * (4.0 * zz - xx - yy);
    Y[12] = SH_C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = SH_C3[4] * x * (4.0 * zz - xx - yy);
    Y[14] = SH_C3[5] * z * (xx - yy);
    Y[15] = SH_C3[6] * x * (xx - 3.0 * yy);
}

/* Partial derivatives dY_k/d(x,y,z) of the basis above (before normalisation of d). */
static void sh_basis_grad(int deg, const double d[3], double dY[16][3]) {
    const double x = d[0], y = d[1], z = d[2];
    memset(dY, 0, sizeof(double) * 16 * 3);
    if (deg < 1) return;
    dY[1][1] = -SH_C1;
    dY[2][2] = SH_C1;
    dY[3][0] = -SH_C1;
    if (deg < 2) return;
    dY[4][0] = SH_C2[0] * y;  dY[4][1] = SH_C2[0] * x;
    dY[5][1] = SH_C2[1] * z;  dY[5][2] = SH_C2[1] * y;
    dY[6][0] = SH_C2[2] * (-2.0 * x); dY[6][1] = SH_C2[2] * (-2.0 * y); dY[6][2] = SH_C2[2] * (4.0 * z);
    dY[7][0] = SH_C2[3] * z;  dY[7][2] = SH_C2[3] * x;
    dY[8][0] = SH_C2[4] * 2.0 * x; dY[8][1] = SH_C2[4] * (-2.0 * y);
    if (deg < 3) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    dY[9][0] = SH_C3[0] * y * 6.0 * x;
    dY[9][1] = SH_C3[0] * (3.0 * xx - 3.0 * yy);
    dY[10][0] = SH_C3[1] * y * z; dY[10][1] = SH_C3[1] * x * z; dY[10][2] = SH_C3[1] * x * y;
    dY[11][0] = SH_C3[2] * y * (-2.0 * x);
    dY[11][1] = SH_C3[2] * (4.0 * zz - xx - 3.0 * yy);
    dY[11][2] = SH_C3[2] * y * 8.0 * z;
    dY[12][0] = SH_C3[3] * z * (-6.0 * x);
    dY[12][1] = SH_C3[3] * z * (-6.0 * y);
    dY[12][2] = SH_C3[3] * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    dY[13][0] = SH_C3[4] * (4.0 * zz - 3.0 * xx - yy);
    dY[13][1] = SH_C3[4] * x * (-2.0 * y);
    dY[13][2] = SH_C3[4] * x * 8.0 * z;
    dY[14][0] = SH_C3[5] * z * 2.0 * x;
    dY[14][1] = SH_C3[5] * z * (-2.0 * y);
    dY[14][2] = SH_C3[5] * (xx - yy);
    dY[15][0] = SH_C3[6] * (3.0 * xx - 3.0 * yy);
    dY[15][1] = SH_C3[6] * x * (-6.0 * y);
}

static void quat_to_R(const double *q, double *R) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = acc;
        }
}

static void matmul3_bt(const double *A, const double *B, double *C) { /* A B^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += A[3 * i + k] * B[3 * j + k];
            C[3 * i + j] = acc;
        }
}

static void matmul3_at(const double *A, const double *B, double *C) { /* A^T B */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += A[3 * k + i] * B[3 * k + j];
            C[3 * i + j] = acc;
        }
}

/* Value-path projection of one Gaussian (Eq. (1), Eq. (2)) and its SH colour. */
static void value_project(const double *m, const double *s, const double *q, double o,
                          const double *sh, int deg, const double *cam, vproj *P) {
    const double *Rc = cam + CR, *t = cam + CT;
    const double fx = cam[CFX], fy = cam[CFY];
    P->nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) P->qn[k] = q[k] / P->nq;
    quat_to_R(P->qn, P->R);
    for (int k = 0; k < 3; ++k) P->s[k] = s[k];
    double M[9];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) M[3 * a + k] = P->R[3 * a + k] * s[k];
    matmul3_bt(M, M, P->SigW);                 /* R S S^T R^T */
    double tmp[9];
    matmul3(Rc, P->SigW, tmp);
    matmul3_bt(tmp, Rc, P->Sigc);              /* W Sigma_W W^T */
    for (int a = 0; a < 3; ++a)
        P->p[a] = Rc[3 * a] * m[0] + Rc[3 * a + 1] * m[1] + Rc[3 * a + 2] * m[2] + t[a];
    const double pz = P->p[2];
    const double xn = P->p[0] / pz, yn = P->p[1] / pz;
    P->lim[0] = (double)kFrustum * 0.5 * cam[CW] / fx;
    P->lim[1] = (double)kFrustum * 0.5 * cam[CH] / fy;
    double xc = xn, yc = yn;
    P->xclamp = 0;
    P->yclamp = 0;
    if (xn < -P->lim[0]) { xc = -P->lim[0]; P->xclamp = -1; }
    if (xn > P->lim[0]) { xc = P->lim[0]; P->xclamp = 1; }
    if (yn < -P->lim[1]) { yc = -P->lim[1]; P->yclamp = -1; }
    if (yn > P->lim[1]) { yc = P->lim[1]; P->yclamp = 1; }
    xc *= pz;
    yc *= pz;
    P->J[0] = fx / pz; P->J[1] = 0; P->J[2] = -fx * xc / (pz * pz);
    P->J[3] = 0; P->J[4] = fy / pz; P->J[5] = -fy * yc / (pz * pz);
    /* Sigma_I = J Sigma_c J^T */
    double JS[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += P->J[3 * a + k] * P->Sigc[3 * k + b];
            JS[3 * a + b] = acc;
        }
    double S2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += JS[3 * a + k] * P->J[3 * b + k];
            S2[2 * a + b] = acc;
        }
    P->cov[0] = S2[0] + (double)kDilation;
    P->cov[1] = S2[1];
    P->cov[2] = S2[3] + (double)kDilation;
    const double det = P->cov[0] * P->cov[2] - P->cov[1] * P->cov[1];
    P->conic[0] = P->cov[2] / det;
    P->conic[1] = -P->cov[1] / det;
    P->conic[2] = P->cov[0] / det;
    P->uv[0] = fx * xn + cam[CCX];
    P->uv[1] = fy * yn + cam[CCY];
    P->depth = pz;
    /* colour: direction from the camera centre c = -W^T t to the mean */
    double cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = -(Rc[a] * t[0] + Rc[3 + a] * t[1] + Rc[6 + a] * t[2]);
    for (int a = 0; a < 3; ++a) P->dir[a] = m[a] - cc[a];
    P->dirn = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
    double d[3] = {P->dir[0] / P->dirn, P->dir[1] / P->dirn, P->dir[2] / P->dirn};
    sh_basis(deg, d, P->basis);
    const int K = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < K; ++k) acc += P->basis[k] * sh[3 * k + ch];
        P->raw[ch] = acc;
        P->rgb[ch] = acc > 0 ? acc : 0;
    }
    P->opac = o;
}

/* ---------------------------------------------------------------- common input block */
typedef struct {
    int64_t n;
    const float *means, *scales, *quats, *opac, *sh;
    int deg;
} gauss32;

static void widen(const gauss32 *G, int64_t g, double m[3], double s[3], double q[4], double *o,
                  double *sh) {
    const int K = (G->deg + 1) * (G->deg + 1);
    for (int k = 0; k < 3; ++k) { m[k] = G->means[3 * g + k]; s[k] = G->scales[3 * g + k]; }
    for (int k = 0; k < 4; ++k) q[k] = G->quats[4 * g + k];
    *o = G->opac[g];
    for (int k = 0; k < 3 * K; ++k) sh[k] = G->sh[3 * K * g + k];
}

/* ---------------------------------------------------------------- tile lists */
typedef struct {
    int TX, TY;
    keyproj *kp;         /* [n] */
    int64_t *tile_off;   /* [TX*TY+1] */
    int32_t *tile_gid;   /* [M], per tile sorted by (depth_bits, gid) */
    int64_t M;
} tiling;

static int cmp_depth_gid(const void *pa, const void *pb, void *ctx) {
    const keyproj *kp = (const keyproj *)ctx;
    const int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    const uint32_t da = kp[a].depth_bits, db = kp[b].depth_bits;
    if (da != db) return da < db ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static void build_tiling(const gauss32 *G, const float *cam32, tiling *tl) {
    const int W = (int)cam32[CW], H = (int)cam32[CH];
    tl->TX = (W + TILE - 1) / TILE;
    tl->TY = (H + TILE - 1) / TILE;
    const int ntiles = tl->TX * tl->TY;
    tl->kp = (keyproj *)calloc((size_t)(G->n > 0 ? G->n : 1), sizeof(keyproj));
    tl->tile_off = (int64_t *)calloc((size_t)ntiles + 1, sizeof(int64_t));
    for (int64_t g = 0; g < G->n; ++g)
        key_path(G->means + 3 * g, G->scales + 3 * g, G->quats + 4 * g, G->opac[g], cam32, tl->TX,
                 tl->TY, &tl->kp[g]);
    for (int64_t g = 0; g < G->n; ++g) {
        const keyproj *k = &tl->kp[g];
        if (!k->valid) continue;
        for (int ty = k->rect[1]; ty < k->rect[3]; ++ty)
            for (int tx = k->rect[0]; tx < k->rect[2]; ++tx) tl->tile_off[ty * tl->TX + tx + 1]++;
    }
    for (int i = 0; i < ntiles; ++i) tl->tile_off[i + 1] += tl->tile_off[i];
    tl->M = tl->tile_off[ntiles];
    tl->tile_gid = (int32_t *)malloc((size_t)(tl->M > 0 ? tl->M : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)ntiles, sizeof(int64_t));
    for (int64_t g = 0; g < G->n; ++g) {
        const keyproj *k = &tl->kp[g];
        if (!k->valid) continue;
        for (int ty = k->rect[1]; ty < k->rect[3]; ++ty)
            for (int tx = k->rect[0]; tx < k->rect[2]; ++tx) {
                const int t = ty * tl->TX + tx;
                tl->tile_gid[tl->tile_off[t] + fill[t]++] = (int32_t)g;
            }
    }
    free(fill);
    for (int t = 0; t < ntiles; ++t)
        qsort_r(tl->tile_gid + tl->tile_off[t], (size_t)(tl->tile_off[t + 1] - tl->tile_off[t]),
                sizeof(int32_t), cmp_depth_gid, tl->kp);
}

static void free_tiling(tiling *tl) {
    free(tl->kp);
    free(tl->tile_off);
    free(tl->tile_gid);
}

/* value projections of all key-path-visible Gaussians */
static vproj *project_all(const gauss32 *G, const tiling *tl, const double *cam64) {
    vproj *vp = (vproj *)calloc((size_t)(G->n > 0 ? G->n : 1), sizeof(vproj));
    const int K = (G->deg + 1) * (G->deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < G->n; ++g) {
        if (!tl->kp[g].valid) continue;
        double m[3], s[3], q[4], o, sh[48];
        widen(G, g, m, s, q, &o, sh);
        value_project(m, s, q, o, sh, G->deg, cam64, &vp[g]);
    }
    (void)K;
    return vp;
}

/* ---------------------------------------------------------------- one pixel, forward */
typedef struct {
    int32_t gid;
    int32_t pos;      /* position in the tile list */
    int clamped;
    double alpha, G, T, dx, dy;
} contrib;

/* Ambiguity bands: decisions that a fp32 implementation may take differently.
 * The image means of the fp32 key path are known exactly (they are pinned), so
 * for every evaluated Gaussian the log-alpha error of a fp32 renderer is
 * bounded by the change of the exponent between the fp64 and the fp32 means,
 * plus conic_rel times the sum of the absolute terms of the quadratic form
 * (rounding of a fp32 conic), plus exp_abs (rounding of a fp32 exponential,
 * and of a fp32 log of the opacity where the renderer folds it into the
 * exponent).
 * A skip or clamp decision is ambiguous when alpha lies within that error of
 * its threshold; the stop decision when log T' lies within the error
 * accumulated along the walk: alpha/(1-alpha) times each blended log-alpha
 * error plus the rounding of each fp32 product T (1 - alpha), taken as
 * 6e-8 (2 + 1/(1-alpha)). */
typedef struct { double conic_rel, exp_abs; } bands;

static double power_at(const vproj *P, double u, double v, double px, double py, double *dx, double *dy) {
    *dx = u - px;
    *dy = v - py;
    return -0.5 * (P->conic[0] * (*dx) * (*dx) + P->conic[2] * (*dy) * (*dy)) - P->conic[1] * (*dx) * (*dy);
}

/* Front-to-back walk of Eq. (11) for pixel (px, py).  Returns the number of
 * contributors written to `cs` (if not NULL); sets *flag when a decision lies
 * within the ambiguity band (needs kp, the key-path results, when bd != NULL). */
static int walk_pixel(const int32_t *list, int64_t len, const vproj *vp, const keyproj *kp, double px,
                      double py, const double *bg, double out[5], int32_t *n_contrib, contrib *cs,
                      const bands *bd, int *flag) {
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
    int nc = 0;
    int32_t last = 0;
    int amb = 0;
    double err_lnT = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        const int32_t g = list[i];
        const vproj *P = &vp[g];
        double dx, dy;
        const double power = power_at(P, P->uv[0], P->uv[1], px, py, &dx, &dy);
        double e = 0.0;
        if (bd) {
            double dx32, dy32;
            const double p32 = power_at(P, (double)kp[g].u, (double)kp[g].v, px, py, &dx32, &dy32);
            const double absq = 0.5 * (fabs(P->conic[0]) * dx * dx + fabs(P->conic[2]) * dy * dy) +
                                fabs(P->conic[1] * dx * dy);
            e = fabs(power - p32) + bd->conic_rel * absq + bd->exp_abs;
        }
        const double Gv = exp(power);
        const double a_un = P->opac * Gv;
        const int clamped = a_un > (double)kAlphaMax;
        const double alpha = clamped ? (double)kAlphaMax : a_un;
        if (bd) {
            if (fabs(log(a_un / (double)kAlphaMin)) < e) amb = 1;
            if (fabs(log(a_un / (double)kAlphaMax)) < e) amb = 1;
        }
        if (alpha < (double)kAlphaMin) continue;
        const double Tn = T * (1.0 - alpha);
        if (bd) {
            const double step = (clamped ? 0.0 : alpha / (1.0 - alpha) * e) + 6e-8 * (2.0 + 1.0 / (1.0 - alpha));
            if (fabs(log(Tn / (double)kTMin)) < err_lnT + step) amb = 1;
            err_lnT += step;
        }
        if (Tn < (double)kTMin) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += P->rgb[ch] * alpha * T;
        D += P->depth * alpha * T;
        if (cs) {
            cs[nc].gid = g;
            cs[nc].pos = (int32_t)i;
            cs[nc].clamped = clamped;
            cs[nc].alpha = alpha;
            cs[nc].G = Gv;
            cs[nc].T = T;
            cs[nc].dx = dx;
            cs[nc].dy = dy;
        }
        ++nc;
        T = Tn;
        last = (int32_t)i + 1;
    }
    for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * bg[ch];
    out[3] = D + T * bg[3];
    out[4] = T;
    if (n_contrib) *n_contrib = last;
    if (flag) *flag = amb;
    return nc;
}

/* ---------------------------------------------------------------- flagged pixels: every allowed outcome
 * A pixel whose walk has a decision inside the ambiguity band can be rendered
 * correctly in more than one way by a fp32 renderer.  The outcomes are the
 * walks in which any subset of those decisions goes the other way: the skip of
 * alpha < 1/255 (blended anyway with its unclamped alpha, or skipped) and the
 * stop before T' < 1e-4 (blended and continued, or stopped).  The clamp at
 * 0.99 is taken as computed: flipping it moves alpha by less than the band
 * itself, far below the image tolerance.  Decisions flipped are listed in walk
 * order; a walk reports the flagged decisions that follow its last flip, and
 * each of them opens one more walk, so every subset is visited once. */
typedef struct { int64_t i; int kind; } flip; /* kind 0: skip decision at entry i, 1: stop decision */

static int flipped(const flip *fl, int nfl, int64_t i, int kind) {
    for (int k = 0; k < nfl; ++k)
        if (fl[k].i == i && fl[k].kind == kind) return 1;
    return 0;
}

/* One walk with the decisions in fl reversed.  out[5] = rgb, depth, T;
 * *n_contrib = 1 + the position of the last blended entry (0: none),
 * *last_gid = its Gaussian (-1: none).  Flagged decisions after the last flip
 * go to found (at most max_found; the count is returned, or -1 past it). */
static int walk_flipped(const int32_t *list, int64_t len, const vproj *vp, const keyproj *kp, double px, double py,
                        const double *bg, const bands *bd, const flip *fl, int nfl, double out[5],
                        int32_t *n_contrib, int32_t *last_gid, flip *found, int max_found) {
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0, err_lnT = 0.0;
    int32_t last = 0, lgid = -1;
    int nf = 0;
    const int64_t after_i = nfl ? fl[nfl - 1].i : -1;
    const int after_k = nfl ? fl[nfl - 1].kind : 1;
#define MGS_LATER(ii, kk) ((ii) > after_i || ((ii) == after_i && (kk) > after_k))
    for (int64_t i = 0; i < len; ++i) {
        const int32_t g = list[i];
        const vproj *P = &vp[g];
        double dx, dy, dx32, dy32;
        const double power = power_at(P, P->uv[0], P->uv[1], px, py, &dx, &dy);
        const double p32 = power_at(P, (double)kp[g].u, (double)kp[g].v, px, py, &dx32, &dy32);
        const double absq = 0.5 * (fabs(P->conic[0]) * dx * dx + fabs(P->conic[2]) * dy * dy) +
                            fabs(P->conic[1] * dx * dy);
        const double e = fabs(power - p32) + bd->conic_rel * absq + bd->exp_abs;
        const double a_un = P->opac * exp(power);
        const int clamped = a_un > (double)kAlphaMax;
        const double alpha = clamped ? (double)kAlphaMax : a_un;
        int skip = alpha < (double)kAlphaMin;
        if (fabs(log(a_un / (double)kAlphaMin)) < e) {
            if (flipped(fl, nfl, i, 0)) skip = !skip;
            else if (MGS_LATER(i, 0)) {
                if (nf >= max_found) return -1;
                found[nf].i = i; found[nf].kind = 0; ++nf;
            }
        }
        if (skip) continue;
        const double Tn = T * (1.0 - alpha);
        const double step = (clamped ? 0.0 : alpha / (1.0 - alpha) * e) + 6e-8 * (2.0 + 1.0 / (1.0 - alpha));
        int stop = Tn < (double)kTMin;
        if (fabs(log(Tn / (double)kTMin)) < err_lnT + step) {
            if (flipped(fl, nfl, i, 1)) stop = !stop;
            else if (MGS_LATER(i, 1)) {
                if (nf >= max_found) return -1;
                found[nf].i = i; found[nf].kind = 1; ++nf;
            }
        }
        err_lnT += step;
        if (stop) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += P->rgb[ch] * alpha * T;
        D += P->depth * alpha * T;
        T = Tn;
        last = (int32_t)i + 1;
        lgid = g;
    }
#undef MGS_LATER
    for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * bg[ch];
    out[3] = D + T * bg[3];
    out[4] = T;
    *n_contrib = last;
    *last_gid = lgid;
    return nf;
}

#define ALT_MAX_FLIPS 12
typedef struct {
    const int32_t *list; int64_t len; const vproj *vp; const keyproj *kp; double px, py;
    const double *bg; const bands *bd;
    int max_leaves, n_leaves, overflow;
    double *leaf;        /* [max_leaves][5] */
    int32_t *leaf_gid;   /* [max_leaves] */
} altctx;

static void alt_enum(altctx *c, flip *fl, int nfl) {
    if (c->overflow) return;
    if (c->n_leaves >= c->max_leaves) { c->overflow = 1; return; }
    flip found[ALT_MAX_FLIPS];
    int32_t nc, gid;
    const int nf = walk_flipped(c->list, c->len, c->vp, c->kp, c->px, c->py, c->bg, c->bd, fl, nfl,
                                c->leaf + 5 * c->n_leaves, &nc, &gid, found, ALT_MAX_FLIPS);
    if (nf < 0) { c->overflow = 1; return; }
    c->leaf_gid[c->n_leaves++] = gid;
    if (nfl + 1 > ALT_MAX_FLIPS && nf > 0) { c->overflow = 1; return; }
    for (int k = 0; k < nf; ++k) {
        fl[nfl] = found[k];
        alt_enum(c, fl, nfl + 1);
        if (c->overflow) return;
    }
}

/* Every outcome that the ambiguity bands allow at n_pix pixels (px[k], py[k])
 * of one view: leaves [n_pix][max_leaves][5] (rgb, depth, T), leaf_gid
 * [n_pix][max_leaves] (Gaussian of the last blended entry, -1: none),
 * n_leaves [n_pix] (-1 when a pixel has more than max_leaves outcomes). */
void orc_forward_alternatives(int64_t n, const float *means, const float *scales, const float *quats,
                              const float *opac, const float *sh, int deg, const float *cam32,
                              const double *cam64, const double *bg, const double *bd2, int64_t n_pix,
                              const int32_t *pxs, const int32_t *pys, int max_leaves, double *leaves,
                              int32_t *leaf_gid, int32_t *n_leaves) {
    gauss32 G = {n, means, scales, quats, opac, sh, deg};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    vproj *vp = project_all(&G, &tl, cam64);
    bands bd;
    bd.conic_rel = bd2[0];
    bd.exp_abs = bd2[1];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_pix; ++k) {
        const int x = pxs[k], y = pys[k];
        const int t = (y / TILE) * tl.TX + x / TILE;
        altctx c;
        c.list = tl.tile_gid + tl.tile_off[t];
        c.len = tl.tile_off[t + 1] - tl.tile_off[t];
        c.vp = vp;
        c.kp = tl.kp;
        c.px = (double)x;
        c.py = (double)y;
        c.bg = bg;
        c.bd = &bd;
        c.max_leaves = max_leaves;
        c.n_leaves = 0;
        c.overflow = 0;
        c.leaf = leaves + (size_t)k * max_leaves * 5;
        c.leaf_gid = leaf_gid + (size_t)k * max_leaves;
        flip fl[ALT_MAX_FLIPS + 1];
        alt_enum(&c, fl, 0);
        n_leaves[k] = c.overflow ? -1 : c.n_leaves;
    }
    free(vp);
    free_tiling(&tl);
}

/* ================================================================ exported API */

/* Key path only: per-Gaussian cull flag, depth key, rect, u, v, r, and the tile
 * lists.  tile_off [TX*TY+1] (int64) and tile_gid [M] are filled when non-NULL;
 * returns M (the instance count). */
int64_t orc_keys(int64_t n, const float *means, const float *scales, const float *quats,
                 const float *opac, const float *cam32, uint8_t *valid, uint32_t *depth_bits,
                 int32_t *rect, float *uvr, int64_t *tile_off, int32_t *tile_gid) {
    gauss32 G = {n, means, scales, quats, opac, NULL, 0};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    for (int64_t g = 0; g < n; ++g) {
        const keyproj *k = &tl.kp[g];
        if (valid) valid[g] = (uint8_t)k->valid;
        if (depth_bits) depth_bits[g] = k->valid ? k->depth_bits : 0xFFFFFFFFu;
        if (rect)
            for (int j = 0; j < 4; ++j) rect[4 * g + j] = k->valid ? k->rect[j] : 0;
        if (uvr) {
            uvr[3 * g] = k->valid ? k->u : 0.f;
            uvr[3 * g + 1] = k->valid ? k->v : 0.f;
            uvr[3 * g + 2] = k->valid ? k->r : 0.f;
        }
    }
    const int ntiles = tl.TX * tl.TY;
    if (tile_off) memcpy(tile_off, tl.tile_off, sizeof(int64_t) * (size_t)(ntiles + 1));
    if (tile_gid) memcpy(tile_gid, tl.tile_gid, sizeof(int32_t) * (size_t)tl.M);
    const int64_t M = tl.M;
    free_tiling(&tl);
    return M;
}

/* Value-path projection of every Gaussian (for pins): uv[2], conic[3], cov[3],
 * depth, rgb[3] per Gaussian; Gaussians culled by the key path are left 0. */
void orc_project_values(int64_t n, const float *means, const float *scales, const float *quats,
                        const float *opac, const float *sh, int deg, const float *cam32,
                        const double *cam64, double *out12) {
    gauss32 G = {n, means, scales, quats, opac, sh, deg};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    vproj *vp = project_all(&G, &tl, cam64);
    for (int64_t g = 0; g < n; ++g) {
        double *o = out12 + 12 * g;
        memset(o, 0, 12 * sizeof(double));
        if (!tl.kp[g].valid) continue;
        o[0] = vp[g].uv[0]; o[1] = vp[g].uv[1];
        o[2] = vp[g].conic[0]; o[3] = vp[g].conic[1]; o[4] = vp[g].conic[2];
        o[5] = vp[g].cov[0]; o[6] = vp[g].cov[1]; o[7] = vp[g].cov[2];
        o[8] = vp[g].depth;
        o[9] = vp[g].rgb[0]; o[10] = vp[g].rgb[1]; o[11] = vp[g].rgb[2];
    }
    free(vp);
    free_tiling(&tl);
}

/* Forward render of one view.
 * out_rgb [3,H,W], out_depth [H,W], out_T [H,W] (double); out_nc [H,W] (int32);
 * out_amb [H,W] (uint8, nullable): pixel has a decision within the ambiguity
 * bands bd2 = {conic_rel, exp_abs} (nullable: no flags).  Returns M. */
int64_t orc_forward(int64_t n, const float *means, const float *scales, const float *quats,
                    const float *opac, const float *sh, int deg, const float *cam32,
                    const double *cam64, const double *bg, double *out_rgb, double *out_depth,
                    double *out_T, int32_t *out_nc, uint8_t *out_amb, const double *bd3) {
    /* bd3: {conic_rel, exp_abs} */
    gauss32 G = {n, means, scales, quats, opac, sh, deg};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    vproj *vp = project_all(&G, &tl, cam64);
    const int W = (int)cam32[CW], H = (int)cam32[CH];
    bands bd;
    if (bd3) { bd.conic_rel = bd3[0]; bd.exp_abs = bd3[1]; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int t = (y / TILE) * tl.TX + x / TILE;
            double out[5];
            int32_t nc;
            int flag = 0;
            walk_pixel(tl.tile_gid + tl.tile_off[t], tl.tile_off[t + 1] - tl.tile_off[t], vp, tl.kp,
                       (double)x, (double)y, bg, out, &nc, NULL, bd3 ? &bd : NULL, &flag);
            const int64_t pix = (int64_t)y * W + x;
            for (int ch = 0; ch < 3; ++ch) out_rgb[(int64_t)ch * H * W + pix] = out[ch];
            out_depth[pix] = out[3];
            out_T[pix] = out[4];
            if (out_nc) out_nc[pix] = nc;
            if (out_amb) out_amb[pix] = (uint8_t)flag;
        }
    }
    const int64_t M = tl.M;
    free(vp);
    free_tiling(&tl);
    return M;
}

/* Contributor lists of every pixel (for frozen-decision finite differences).
 * First call with gids == NULL returns the total count and fills counts[H*W];
 * the second call fills gids and clamped in pixel order. */
int64_t orc_contributors(int64_t n, const float *means, const float *scales, const float *quats,
                         const float *opac, const float *sh, int deg, const float *cam32,
                         const double *cam64, int64_t *counts, int32_t *gids, uint8_t *clamped) {
    gauss32 G = {n, means, scales, quats, opac, sh, deg};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    vproj *vp = project_all(&G, &tl, cam64);
    const int W = (int)cam32[CW], H = (int)cam32[CH];
    const double bg[4] = {0, 0, 0, 0};
    int64_t maxlen = 1;
    for (int t = 0; t < tl.TX * tl.TY; ++t)
        if (tl.tile_off[t + 1] - tl.tile_off[t] > maxlen) maxlen = tl.tile_off[t + 1] - tl.tile_off[t];
    contrib *cs = (contrib *)malloc(sizeof(contrib) * (size_t)maxlen);
    int64_t total = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int t = (y / TILE) * tl.TX + x / TILE;
            double out[5];
            const int nc = walk_pixel(tl.tile_gid + tl.tile_off[t], tl.tile_off[t + 1] - tl.tile_off[t],
                                      vp, tl.kp, (double)x, (double)y, bg, out, NULL, cs, NULL, NULL);
            if (gids == NULL) {
                counts[(int64_t)y * W + x] = nc;
            } else {
                for (int i = 0; i < nc; ++i) {
                    gids[total + i] = cs[i].gid;
                    clamped[total + i] = (uint8_t)cs[i].clamped;
                }
            }
            total += nc;
        }
    free(cs);
    free(vp);
    free_tiling(&tl);
    return total;
}

/* Forward with frozen decisions: pixel p composites exactly the listed
 * contributors (in order), alpha = 0.99 where `clamped`, else o * exp(power),
 * with no skip or stop tests.  All parameters and the camera are double so that
 * finite differences can perturb them. */
void orc_forward_frozen(int64_t n, const double *means, const double *scales, const double *quats,
                        const double *opac, const double *sh, int deg, const double *cam64,
                        const double *bg, const int64_t *counts, const int32_t *gids,
                        const uint8_t *clamped, double *out_rgb, double *out_depth) {
    const int W = (int)cam64[CW], H = (int)cam64[CH];
    const int K = (deg + 1) * (deg + 1);
    vproj *vp = (vproj *)calloc((size_t)(n > 0 ? n : 1), sizeof(vproj));
    char *need = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t total = 0;
    for (int64_t p = 0; p < (int64_t)W * H; ++p) total += counts[p];
    for (int64_t i = 0; i < total; ++i) need[gids[i]] = 1;
    for (int64_t g = 0; g < n; ++g)
        if (need[g])
            value_project(means + 3 * g, scales + 3 * g, quats + 4 * g, opac[g], sh + 3 * K * g, deg,
                          cam64, &vp[g]);
    int64_t off = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int64_t pix = (int64_t)y * W + x;
            double T = 1, C[3] = {0, 0, 0}, D = 0;
            for (int64_t i = 0; i < counts[pix]; ++i) {
                const vproj *P = &vp[gids[off + i]];
                const double dx = P->uv[0] - x, dy = P->uv[1] - y;
                const double power = -0.5 * (P->conic[0] * dx * dx + P->conic[2] * dy * dy) -
                                     P->conic[1] * dx * dy;
                const double alpha = clamped[off + i] ? (double)kAlphaMax : P->opac * exp(power);
                for (int ch = 0; ch < 3; ++ch) C[ch] += P->rgb[ch] * alpha * T;
                D += P->depth * alpha * T;
                T *= 1 - alpha;
            }
            off += counts[pix];
            for (int ch = 0; ch < 3; ++ch) out_rgb[(int64_t)ch * H * W + pix] = C[ch] + T * bg[ch];
            out_depth[pix] = D + T * bg[3];
        }
    free(need);
    free(vp);
}

/* ---------------------------------------------------------------- backward */
/* 2D gradient record per Gaussian: u, v, A, B, C, opacity, r, g, b, depth */
enum { G2_U = 0, G2_V, G2_A, G2_B, G2_C, G2_O, G2_R, G2_G, G2_BL, G2_D, G2_N };

/* Chain the 2D gradient of one Gaussian to its parameters and the pose. */
static void chain_gaussian(const vproj *P, const double *g2, int deg, const double *sh,
                           const double *cam, double *d_mean, double *d_scale, double *d_quat,
                           double *d_opac, double *d_sh, double pose_p[3], double pose_th[3],
                           double gdir_sum[3]) {
    const double *Rc = cam + CR;
    const double fx = cam[CFX], fy = cam[CFY];
    const int K = (deg + 1) * (deg + 1);
    /* colour: clamp mask, SH coefficients, direction */
    double graw[3];
    for (int ch = 0; ch < 3; ++ch) graw[ch] = P->raw[ch] > 0 ? g2[G2_R + ch] : 0.0;
    for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) d_sh[3 * k + ch] += P->basis[k] * graw[ch];
    double gv[3] = {0, 0, 0};
    if (deg > 0) {
        const double d[3] = {P->dir[0] / P->dirn, P->dir[1] / P->dirn, P->dir[2] / P->dirn};
        double dY[16][3];
        sh_basis_grad(deg, d, dY);
        double gd[3] = {0, 0, 0};
        for (int k = 1; k < K; ++k) {
            double gY = 0;
            for (int ch = 0; ch < 3; ++ch) gY += sh[3 * k + ch] * graw[ch];
            for (int a = 0; a < 3; ++a) gd[a] += gY * dY[k][a];
        }
        const double dot = gd[0] * d[0] + gd[1] * d[1] + gd[2] * d[2];
        for (int a = 0; a < 3; ++a) gv[a] = (gd[a] - d[a] * dot) / P->dirn;
    }
    /* opacity */
    *d_opac += g2[G2_O];
    /* conic -> dilated covariance: G = -Q Ghat Q with Ghat = [[gA, gB/2], [gB/2, gC]] */
    const double Q[4] = {P->conic[0], P->conic[1], P->conic[1], P->conic[2]};
    const double Gh[4] = {g2[G2_A], 0.5 * g2[G2_B], 0.5 * g2[G2_B], g2[G2_C]};
    double QG[4], GI[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * Gh[j] + Q[2 * i + 1] * Gh[2 + j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) GI[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
    /* Sigma_I = J Sigma_c J^T: G_c = J^T G_I J ; dL/dJ = 2 G_I J Sigma_c */
    double Gc[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) acc += P->J[3 * i + a] * GI[2 * i + j] * P->J[3 * j + b];
            Gc[3 * a + b] = acc;
        }
    double GJ[6];
    for (int i = 0; i < 2; ++i)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 3; ++k) acc += GI[2 * i + j] * P->J[3 * j + k] * P->Sigc[3 * k + b];
            GJ[3 * i + b] = 2.0 * acc;
        }
    /* Sigma_c = W Sigma_W W^T: G_W = W^T G_c W */
    double tmp[9], GW[9];
    matmul3_at(Rc, Gc, tmp);
    matmul3(tmp, Rc, GW);
    /* Sigma_W = M M^T, M = R diag(s): dL/dM = 2 G_W M */
    double M[9], GM[9];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) M[3 * a + k] = P->R[3 * a + k] * P->s[k];
    matmul3(GW, M, GM);
    for (int i = 0; i < 9; ++i) GM[i] *= 2.0;
    double GR[9];
    for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int a = 0; a < 3; ++a) {
            acc += GM[3 * a + k] * P->R[3 * a + k];
            GR[3 * a + k] = GM[3 * a + k] * P->s[k];
        }
        d_scale[k] += acc;
    }
    /* R(q) for unit q = (w,x,y,z) */
    const double w = P->qn[0], x = P->qn[1], y = P->qn[2], z = P->qn[3];
    double gq[4];
    gq[0] = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    gq[1] = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] +
                 w * GR[7] - 2 * x * GR[8]);
    gq[2] = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] +
                 z * GR[7] - 2 * y * GR[8]);
    gq[3] = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] +
                 x * GR[6] + y * GR[7]);
    const double qd = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
    d_quat[0] += (gq[0] - w * qd) / P->nq;
    d_quat[1] += (gq[1] - x * qd) / P->nq;
    d_quat[2] += (gq[2] - y * qd) / P->nq;
    d_quat[3] += (gq[3] - z * qd) / P->nq;
    /* camera-frame mean p: image mean, depth, Jacobian */
    const double px = P->p[0], py = P->p[1], pz = P->p[2];
    double gp[3] = {0, 0, 0};
    gp[0] += g2[G2_U] * fx / pz;
    gp[1] += g2[G2_V] * fy / pz;
    gp[2] += -(g2[G2_U] * fx * px + g2[G2_V] * fy * py) / (pz * pz);
    gp[2] += g2[G2_D];
    gp[2] += -GJ[0] * fx / (pz * pz) - GJ[4] * fy / (pz * pz);
    if (P->xclamp == 0) {
        gp[0] += -GJ[2] * fx / (pz * pz);
        gp[2] += GJ[2] * 2.0 * fx * px / (pz * pz * pz);
    } else {
        gp[2] += GJ[2] * (-P->J[2] / pz);
    }
    if (P->yclamp == 0) {
        gp[1] += -GJ[5] * fy / (pz * pz);
        gp[2] += GJ[5] * 2.0 * fy * py / (pz * pz * pz);
    } else {
        gp[2] += GJ[5] * (-P->J[5] / pz);
    }
    /* world mean: p = W m + t */
    for (int a = 0; a < 3; ++a)
        d_mean[a] += Rc[a] * gp[0] + Rc[3 + a] * gp[1] + Rc[6 + a] * gp[2] + gv[a];
    /* pose (left perturbation): d/drho += gp ; d/dtheta += p x gp + 2 vee(Gc Sc - Sc Gc) */
    for (int a = 0; a < 3; ++a) pose_p[a] += gp[a];
    pose_th[0] += py * gp[2] - pz * gp[1];
    pose_th[1] += pz * gp[0] - px * gp[2];
    pose_th[2] += px * gp[1] - py * gp[0];
    double A1[9], A2[9], Acomm[9];
    matmul3(Gc, P->Sigc, A1);
    matmul3(P->Sigc, Gc, A2);
    for (int i = 0; i < 9; ++i) Acomm[i] = A1[i] - A2[i];
    /* vee of the antisymmetric matrix K: (K21, K02, K10) */
    pose_th[0] += 2.0 * Acomm[7];
    pose_th[1] += 2.0 * Acomm[2];
    pose_th[2] += 2.0 * Acomm[3];
    for (int a = 0; a < 3; ++a) gdir_sum[a] += gv[a];
}

/* Backward of one view.  dL_rgb [3,H,W], dL_depth [H,W] (nullable) in double.
 * Gradients are ACCUMULATED into the double outputs (the caller zeroes them):
 * d_means [n,3], d_scales [n,3], d_quats [n,4], d_opac [n], d_sh [n,K,3],
 * d_pose [6] = (rho, theta); grad2d [n,10] (nullable) receives the per-Gaussian
 * image-space gradient record (u, v, A, B, C, o, r, g, b, depth). */
void orc_backward(int64_t n, const float *means, const float *scales, const float *quats,
                  const float *opac, const float *sh, int deg, const float *cam32,
                  const double *cam64, const double *bg, const double *dL_rgb,
                  const double *dL_depth, double *d_means, double *d_scales, double *d_quats,
                  double *d_opac, double *d_sh, double *d_pose, double *grad2d) {
    gauss32 G = {n, means, scales, quats, opac, sh, deg};
    tiling tl;
    build_tiling(&G, cam32, &tl);
    vproj *vp = project_all(&G, &tl, cam64);
    const int W = (int)cam32[CW], H = (int)cam32[CH];
    const int K = (deg + 1) * (deg + 1);
    double *g2 = (double *)calloc((size_t)(n > 0 ? n : 1) * G2_N, sizeof(double));
    int64_t maxlen = 1;
    for (int t = 0; t < tl.TX * tl.TY; ++t)
        if (tl.tile_off[t + 1] - tl.tile_off[t] > maxlen) maxlen = tl.tile_off[t + 1] - tl.tile_off[t];
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double **priv = (double **)calloc((size_t)nthreads, sizeof(double *));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = (double *)calloc((size_t)(n > 0 ? n : 1) * G2_N, sizeof(double));
        priv[tid] = acc;
        contrib *cs = (contrib *)malloc(sizeof(contrib) * (size_t)maxlen);
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                const int t = (y / TILE) * tl.TX + x / TILE;
                double out[5];
                const int nc = walk_pixel(tl.tile_gid + tl.tile_off[t],
                                          tl.tile_off[t + 1] - tl.tile_off[t], vp, tl.kp, (double)x,
                                          (double)y, bg, out, NULL, cs, NULL, NULL);
                const int64_t pix = (int64_t)y * W + x;
                double gC[3], gD = dL_depth ? dL_depth[pix] : 0.0;
                for (int ch = 0; ch < 3; ++ch) gC[ch] = dL_rgb[(int64_t)ch * H * W + pix];
                /* back to front: S = colour (and depth) of everything behind, bg last */
                double S[3] = {bg[0], bg[1], bg[2]}, SD = bg[3];
                for (int i = nc - 1; i >= 0; --i) {
                    const contrib *c = &cs[i];
                    const vproj *P = &vp[c->gid];
                    double *r = acc + (int64_t)c->gid * G2_N;
                    const double wgt = c->alpha * c->T;
                    double galpha = 0;
                    for (int ch = 0; ch < 3; ++ch) {
                        r[G2_R + ch] += wgt * gC[ch];
                        galpha += (P->rgb[ch] - S[ch]) * gC[ch];
                    }
                    r[G2_D] += wgt * gD;
                    galpha += (P->depth - SD) * gD;
                    galpha *= c->T;
                    if (!c->clamped) {
                        const double gpow = galpha * c->alpha; /* dalpha/dpower = alpha */
                        r[G2_O] += galpha * c->G;
                        r[G2_U] += gpow * -(P->conic[0] * c->dx + P->conic[1] * c->dy);
                        r[G2_V] += gpow * -(P->conic[1] * c->dx + P->conic[2] * c->dy);
                        r[G2_A] += gpow * -0.5 * c->dx * c->dx;
                        r[G2_B] += gpow * -c->dx * c->dy;
                        r[G2_C] += gpow * -0.5 * c->dy * c->dy;
                    }
                    for (int ch = 0; ch < 3; ++ch) S[ch] = c->alpha * P->rgb[ch] + (1 - c->alpha) * S[ch];
                    SD = c->alpha * P->depth + (1 - c->alpha) * SD;
                }
            }
        }
        free(cs);
    }
    for (int th = 0; th < nthreads; ++th) {
        if (!priv[th]) continue;
        for (int64_t i = 0; i < n * G2_N; ++i) g2[i] += priv[th][i];
        free(priv[th]);
    }
    free(priv);
    double pose_p[3] = {0, 0, 0}, pose_th[3] = {0, 0, 0}, gdir[3] = {0, 0, 0};
    for (int64_t g = 0; g < n; ++g) {
        if (!tl.kp[g].valid) continue;
        double m[3], s[3], q[4], o, shd[48];
        widen(&G, g, m, s, q, &o, shd);
        chain_gaussian(&vp[g], g2 + g * G2_N, deg, shd, cam64, d_means + 3 * g, d_scales + 3 * g,
                       d_quats + 4 * g, d_opac + g, d_sh + 3 * K * g, pose_p, pose_th, gdir);
        if (grad2d)
            for (int k = 0; k < G2_N; ++k) grad2d[G2_N * g + k] += g2[G2_N * g + k];
    }
    /* camera centre c = -W^T t moves by -W^T rho: d/drho += W * sum(dL/d(mean - c)) */
    const double *Rc = cam64 + CR;
    for (int a = 0; a < 3; ++a)
        pose_p[a] += Rc[3 * a] * gdir[0] + Rc[3 * a + 1] * gdir[1] + Rc[3 * a + 2] * gdir[2];
    for (int a = 0; a < 3; ++a) {
        d_pose[a] += pose_p[a];
        d_pose[3 + a] += pose_th[a];
    }
    free(g2);
    free(vp);
    free_tiling(&tl);
}

/* SH basis values for `n` unit directions (for the orthonormality pins). */
void orc_sh_basis(int deg, int64_t n, const double *dirs, double *out16) {
    for (int64_t i = 0; i < n; ++i) sh_basis(deg, dirs + 3 * i, out16 + 16 * i);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
