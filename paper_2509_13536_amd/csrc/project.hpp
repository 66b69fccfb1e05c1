// Per-(Gaussian, view) projection: the fp32 key path that decides culling,
// the tile rectangle and the depth key (a fixed IEEE operation sequence, built
// with FMA contraction off and correctly rounded division and square root, so
// those integer decisions are reproducible), the values the blend needs
// (conic, colour, depth), and the chain rule of the backward pass.
//
// Eq. (1): mu_I = pi(T_CW mu_W), Sigma_I = J W Sigma_W W^T J^T
// Eq. (2): Sigma_W = R S S^T R^T, R from the quaternion, S = diag(scale)
// Colour from real spherical harmonics of degree <= 3 (Sec. II-C).
#pragma once
#include "common.hpp"

namespace mgs {

struct Proj {
    float R[9];   // rotation of q/|q|
    float S[6];   // Sigma_W: 00 01 02 11 12 22
    float p[3];   // camera-frame mean
    float xn, yn;
    float J00, J02, J11, J12;
    bool xclamp, yclamp;
    float T[6];   // J W (2x3)
    float U[6];   // T Sigma_W (2x3)
    float a, b, c;  // dilated image covariance
    float u, v, r;
    int x0, y0, x1, y1;
};

__device__ __forceinline__ float sclamp(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// Key path.  Every product and sum below is a separately rounded IEEE fp32
// operation (the library is compiled with -ffp-contract=off); `/` and sqrtf
// are correctly rounded.  Returns false when the Gaussian is culled.
__device__ __forceinline__ bool key_path(const float *m, const float *s, const float *q, float o,
                                         const ViewDev &V, Proj &P) {
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        if (!isfinite(m[k])) return false;
        if (!(s[k] > 0.0f) || !isfinite(s[k])) return false;
    }
    if (!(o > 0.0f) || !isfinite(o)) return false;
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    const float nq = ((w * w + x * x) + y * y) + z * z;
    if (!(nq > 0.0f) || !isfinite(nq)) return false;
    const float k2 = 2.0f / nq;
    float *R = P.R;
    R[0] = 1.0f - k2 * (y * y + z * z);
    R[1] = k2 * (x * y - w * z);
    R[2] = k2 * (x * z + w * y);
    R[3] = k2 * (x * y + w * z);
    R[4] = 1.0f - k2 * (x * x + z * z);
    R[5] = k2 * (y * z - w * x);
    R[6] = k2 * (x * z - w * y);
    R[7] = k2 * (y * z + w * x);
    R[8] = 1.0f - k2 * (x * x + y * y);
    float M[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) M[3 * a + k] = R[3 * a + k] * s[k];
    float Sf[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            Sf[3 * a + b] = (M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1]) + M[3 * a + 2] * M[3 * b + 2];
    P.S[0] = Sf[0]; P.S[1] = Sf[1]; P.S[2] = Sf[2]; P.S[3] = Sf[4]; P.S[4] = Sf[5]; P.S[5] = Sf[8];
    const float *Rc = V.R;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        P.p[a] = ((Rc[3 * a] * m[0] + Rc[3 * a + 1] * m[1]) + Rc[3 * a + 2] * m[2]) + V.t[a];
    const float pz = P.p[2];
    if (!(pz > V.near_z)) return false;
    P.xn = P.p[0] / pz;
    P.yn = P.p[1] / pz;
    const float limx = V.limx, limy = V.limy;  // per view, the same fp32 operations on the host
    P.xclamp = (P.xn < -limx) || (P.xn > limx);
    P.yclamp = (P.yn < -limy) || (P.yn > limy);
    const float xc = sclamp(P.xn, -limx, limx) * pz;
    const float yc = sclamp(P.yn, -limy, limy) * pz;
    const float pz2 = pz * pz;
    P.J00 = V.fx / pz;
    P.J02 = -(V.fx * xc) / pz2;
    P.J11 = V.fy / pz;
    P.J12 = -(V.fy * yc) / pz2;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        P.T[b] = P.J00 * Rc[b] + P.J02 * Rc[6 + b];
        P.T[3 + b] = P.J11 * Rc[3 + b] + P.J12 * Rc[6 + b];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            P.U[3 * a + b] = (P.T[3 * a] * Sf[b] + P.T[3 * a + 1] * Sf[3 + b]) + P.T[3 * a + 2] * Sf[6 + b];
    const float s00 = (P.U[0] * P.T[0] + P.U[1] * P.T[1]) + P.U[2] * P.T[2];
    const float s01 = (P.U[0] * P.T[3] + P.U[1] * P.T[4]) + P.U[2] * P.T[5];
    const float s11 = (P.U[3] * P.T[3] + P.U[4] * P.T[4]) + P.U[5] * P.T[5];
    P.a = s00 + kDilation;
    P.b = s01;
    P.c = s11 + kDilation;
    const float det = P.a * P.c - P.b * P.b;
    if (!(det > 0.0f)) return false;
    const float mid = 0.5f * (P.a + P.c);
    const float disc = mid * mid - det;
    const float lam = mid + __builtin_sqrtf(fmaxf(0.1f, disc));
    P.r = ceilf(3.0f * __builtin_sqrtf(lam));
    P.u = V.fx * P.xn + V.cx;
    P.v = V.fy * P.yn + V.cy;
    if (!(fabsf(P.u) < 1e6f) || !(fabsf(P.v) < 1e6f) || !(P.r < 1e6f)) return false;
    const float TXf = (float)V.TX, TYf = (float)V.TY;
    P.x0 = (int)sclamp(floorf((P.u - P.r) * 0.0625f), 0.0f, TXf);
    P.x1 = (int)sclamp(floorf((P.u + P.r) * 0.0625f) + 1.0f, 0.0f, TXf);
    P.y0 = (int)sclamp(floorf((P.v - P.r) * 0.0625f), 0.0f, TYf);
    P.y1 = (int)sclamp(floorf((P.v + P.r) * 0.0625f) + 1.0f, 0.0f, TYf);
    return P.x0 < P.x1 && P.y0 < P.y1;
}

// Conic (inverse of the dilated image covariance); the determinant uses an
// error-compensated difference of products.
__device__ __forceinline__ void conic_of(const Proj &P, float &A, float &B, float &C) {
    const float bb = P.b * P.b;
    const float eb = __builtin_fmaf(P.b, P.b, -bb);
    const float det = __builtin_fmaf(P.a, P.c, -bb) - eb;
    const float inv = 1.0f / det;
    A = P.c * inv;
    B = -P.b * inv;
    C = P.a * inv;
}

// ---------------------------------------------------------------- SH
// Real spherical harmonics of degree <= 3 (3DGS sign convention), index
// l*l + l + m.  Constants: sqrt(1/(4 pi)), sqrt(3/(4 pi)), sqrt(15/(4 pi)),
// sqrt(5/(16 pi)), sqrt(15/(16 pi)), sqrt(35/(32 pi)), sqrt(105/(4 pi)),
// sqrt(21/(32 pi)), sqrt(7/(16 pi)), sqrt(105/(16 pi)).
struct SHc {
    static constexpr float c0 = 0.28209479177387814f;
    static constexpr float c1 = 0.4886025119029199f;
    static constexpr float c2a = 1.0925484305920792f;
    static constexpr float c2b = 0.31539156525252005f;
    static constexpr float c2c = 0.5462742152960396f;
    static constexpr float c3a = 0.5900435899266435f;
    static constexpr float c3b = 2.890611442640554f;
    static constexpr float c3c = 0.4570457994644658f;
    static constexpr float c3d = 0.3731763325901154f;
    static constexpr float c3e = 1.445305721320277f;
};

__device__ __forceinline__ void sh_values(int deg, float x, float y, float z, float *Y) {
    Y[0] = SHc::c0;
    if (deg < 1) return;
    Y[1] = -SHc::c1 * y;
    Y[2] = SHc::c1 * z;
    Y[3] = -SHc::c1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SHc::c2a * x * y;
    Y[5] = -SHc::c2a * y * z;
    Y[6] = SHc::c2b * (2.0f * zz - xx - yy);
    Y[7] = -SHc::c2a * x * z;
    Y[8] = SHc::c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -SHc::c3a * y * (3.0f * xx - yy);
    Y[10] = SHc::c3b * x * y * z;
    Y[11] = -SHc::c3c * y * (4.0f * zz - xx - yy);
    Y[12] = SHc::c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -SHc::c3c * x * (4.0f * zz - xx - yy);
    Y[14] = SHc::c3e * z * (xx - yy);
    Y[15] = -SHc::c3a * x * (xx - 3.0f * yy);
}

// g_dir += sum_k gY[k] * dY_k/d(x,y,z) for k >= 1
__device__ __forceinline__ void sh_backprop_dir(int deg, float x, float y, float z, const float *gY, float *g) {
    if (deg < 1) return;
    g[0] += -SHc::c1 * gY[3];
    g[1] += -SHc::c1 * gY[1];
    g[2] += SHc::c1 * gY[2];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += SHc::c2a * y * gY[4] - SHc::c2b * 2.0f * x * gY[6] - SHc::c2a * z * gY[7] + SHc::c2c * 2.0f * x * gY[8];
    g[1] += SHc::c2a * x * gY[4] - SHc::c2a * z * gY[5] - SHc::c2b * 2.0f * y * gY[6] - SHc::c2c * 2.0f * y * gY[8];
    g[2] += -SHc::c2a * y * gY[5] + SHc::c2b * 4.0f * z * gY[6] - SHc::c2a * x * gY[7];
    if (deg < 3) return;
    g[0] += -SHc::c3a * 6.0f * x * y * gY[9] + SHc::c3b * y * z * gY[10] + SHc::c3c * 2.0f * x * y * gY[11] -
            SHc::c3d * 6.0f * x * z * gY[12] - SHc::c3c * (4.0f * zz - 3.0f * xx - yy) * gY[13] +
            SHc::c3e * 2.0f * x * z * gY[14] - SHc::c3a * 3.0f * (xx - yy) * gY[15];
    g[1] += -SHc::c3a * 3.0f * (xx - yy) * gY[9] + SHc::c3b * x * z * gY[10] -
            SHc::c3c * (4.0f * zz - xx - 3.0f * yy) * gY[11] - SHc::c3d * 6.0f * y * z * gY[12] +
            SHc::c3c * 2.0f * x * y * gY[13] - SHc::c3e * 2.0f * y * z * gY[14] + SHc::c3a * 6.0f * x * y * gY[15];
    g[2] += SHc::c3b * x * y * gY[10] - SHc::c3c * 8.0f * y * z * gY[11] +
            SHc::c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * gY[12] - SHc::c3c * 8.0f * x * z * gY[13] +
            SHc::c3e * (xx - yy) * gY[14];
}

// Colour of a Gaussian seen from the camera centre: 0.5 + sum_k Y_k(dir) sh_k,
// clamped below at 0.  Returns the unclamped values in raw[3].
template <int DEG>
__device__ __forceinline__ void sh_colour(const MapDev &Mp, int64_t g, const float *m, const ViewDev &V,
                                          float *rgb, float *raw, float *dir_unit, float *dir_len) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    float d0 = m[0] - V.cam_center[0], d1 = m[1] - V.cam_center[1], d2 = m[2] - V.cam_center[2];
    const float len = __builtin_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    const float inv = 1.0f / len;
    d0 *= inv; d1 *= inv; d2 *= inv;
    float Y[16];
    sh_values(DEG, d0, d1, d2, Y);
    const float *sh = Mp.sh + (int64_t)g * K * 3;
    float acc0 = 0.5f, acc1 = 0.5f, acc2 = 0.5f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc0 = __builtin_fmaf(Y[k], sh[3 * k + 0], acc0);
        acc1 = __builtin_fmaf(Y[k], sh[3 * k + 1], acc1);
        acc2 = __builtin_fmaf(Y[k], sh[3 * k + 2], acc2);
    }
    raw[0] = acc0; raw[1] = acc1; raw[2] = acc2;
    rgb[0] = fmaxf(acc0, 0.0f); rgb[1] = fmaxf(acc1, 0.0f); rgb[2] = fmaxf(acc2, 0.0f);
    if (dir_unit) { dir_unit[0] = d0; dir_unit[1] = d1; dir_unit[2] = d2; *dir_len = len; }
}

// Per-pair gradient sums accumulated by the blend backward over every pixel the
// pair touches (power is -1/2 d^T Q d with d = mu_I - pixel, gp = dL/dpower):
//   [0] sum gp, [1] sum gp dx, [2] sum gp dy, [3] sum gp dx^2, [4] sum gp dx dy,
//   [5] sum gp dy^2, [6..8] dL/dcolour, [9] dL/ddepth.
struct PairGrad {
    float g[kRecord];
};

// Chain of one pair's sums to the Gaussian parameters and the pose (fp32).
// Adds into gm[3], gsc[3], gq[4], *go, gsh[K*3]; pose_acc[9] = (dL/dp,
// p x dL/dp + 2 vee(Gc Sc - Sc Gc), dL/d(mean - camera centre)).
template <int DEG>
__device__ __forceinline__ void chain_pair(const Proj &P, const float *q, const float *s, float o,
                                           const MapDev &Mp, int64_t g, const float *m, const ViewDev &V,
                                           const PairGrad &rg, float *gm, float *gsc, float *gq, float *go,
                                           float *gsh, float *pose_acc) {
    float A, B, C;
    conic_of(P, A, B, C);
    const float *r = rg.g;
    const float gu = -(A * r[1] + B * r[2]);
    const float gv = -(B * r[1] + C * r[2]);
    const float gA = -0.5f * r[3], gB = -r[4], gC = -0.5f * r[5];
    *go += r[0] / o;
    // colour
    constexpr int K = (DEG + 1) * (DEG + 1);
    float rgb[3], raw[3], du[3], dl;
    sh_colour<DEG>(Mp, g, m, V, rgb, raw, du, &dl);
    const float graw[3] = {raw[0] > 0.0f ? r[6] : 0.0f, raw[1] > 0.0f ? r[7] : 0.0f, raw[2] > 0.0f ? r[8] : 0.0f};
    float Y[16];
    sh_values(DEG, du[0], du[1], du[2], Y);
    const float *sh = Mp.sh + (int64_t)g * K * 3;
    float gY[16];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gsh[3 * k + 0] += Y[k] * graw[0];
        gsh[3 * k + 1] += Y[k] * graw[1];
        gsh[3 * k + 2] += Y[k] * graw[2];
        gY[k] = sh[3 * k] * graw[0] + sh[3 * k + 1] * graw[1] + sh[3 * k + 2] * graw[2];
    }
    float gdir[3] = {0.0f, 0.0f, 0.0f};
    if (DEG > 0) {
        float gd[3] = {0.0f, 0.0f, 0.0f};
        sh_backprop_dir(DEG, du[0], du[1], du[2], gY, gd);
        const float dot = gd[0] * du[0] + gd[1] * du[1] + gd[2] * du[2];
        const float il = 1.0f / dl;
        for (int a = 0; a < 3; ++a) gdir[a] = (gd[a] - du[a] * dot) * il;
    }
    // conic -> dilated covariance: GI = -Q Ghat Q, Ghat = [[gA, gB/2], [gB/2, gC]]
    const float h = 0.5f * gB;
    const float QG00 = A * gA + B * h, QG01 = A * h + B * gC;
    const float QG10 = B * gA + C * h, QG11 = B * h + C * gC;
    const float GI00 = -(QG00 * A + QG01 * B);
    const float GI01 = -(QG00 * B + QG01 * C);
    const float GI11 = -(QG10 * B + QG11 * C);
    // dL/dSigma_W = T^T GI T
    const float *T = P.T;
    float GIT[6];  // GI T (2x3)
    for (int b = 0; b < 3; ++b) {
        GIT[b] = GI00 * T[b] + GI01 * T[3 + b];
        GIT[3 + b] = GI01 * T[b] + GI11 * T[3 + b];
    }
    float GW[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GW[3 * a + b] = T[a] * GIT[b] + T[3 + a] * GIT[3 + b];
    // dL/dJ = 2 GI (T Sigma_W) W^T = 2 GI U W^T
    const float *Rc = V.R;
    float UWt[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b)
            UWt[3 * a + b] = P.U[3 * a] * Rc[3 * b] + P.U[3 * a + 1] * Rc[3 * b + 1] + P.U[3 * a + 2] * Rc[3 * b + 2];
    const float GJ00 = 2.0f * (GI00 * UWt[0] + GI01 * UWt[3]);
    const float GJ02 = 2.0f * (GI00 * UWt[2] + GI01 * UWt[5]);
    const float GJ11 = 2.0f * (GI01 * UWt[1] + GI11 * UWt[4]);
    const float GJ12 = 2.0f * (GI01 * UWt[2] + GI11 * UWt[5]);
    // Sigma_W = M M^T, M = R diag(s)
    const float *R = P.R;
    float GR[9];
    for (int k = 0; k < 3; ++k) {
        float acc = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const float gmak = 2.0f * (GW[3 * a] * R[k] * s[k] + GW[3 * a + 1] * R[3 + k] * s[k] +
                                       GW[3 * a + 2] * R[6 + k] * s[k]);
            acc += gmak * R[3 * a + k];
            GR[3 * a + k] = gmak * s[k];
        }
        gsc[k] += acc;
    }
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
    const float gw_ = 2.0f * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    const float gx_ = 2.0f * (y * GR[1] + z * GR[2] + y * GR[3] - 2.0f * x * GR[4] - w * GR[5] + z * GR[6] +
                              w * GR[7] - 2.0f * x * GR[8]);
    const float gy_ = 2.0f * (-2.0f * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] +
                              z * GR[7] - 2.0f * y * GR[8]);
    const float gz_ = 2.0f * (-2.0f * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.0f * z * GR[4] +
                              y * GR[5] + x * GR[6] + y * GR[7]);
    const float dq = gw_ * w + gx_ * x + gy_ * y + gz_ * z;
    gq[0] += (gw_ - w * dq) * qn;
    gq[1] += (gx_ - x * dq) * qn;
    gq[2] += (gy_ - y * dq) * qn;
    gq[3] += (gz_ - z * dq) * qn;
    // camera-frame mean
    const float px = P.p[0], py = P.p[1], pz = P.p[2];
    const float iz = 1.0f / pz, iz2 = iz * iz;
    float gp0 = gu * V.fx * iz, gp1 = gv * V.fy * iz;
    float gp2 = -(gu * V.fx * px + gv * V.fy * py) * iz2 + r[9];
    gp2 += -(GJ00 * V.fx + GJ11 * V.fy) * iz2;
    if (!P.xclamp) {
        gp0 += -GJ02 * V.fx * iz2;
        gp2 += GJ02 * 2.0f * V.fx * px * iz2 * iz;
    } else {
        gp2 += -GJ02 * P.J02 * iz;
    }
    if (!P.yclamp) {
        gp1 += -GJ12 * V.fy * iz2;
        gp2 += GJ12 * 2.0f * V.fy * py * iz2 * iz;
    } else {
        gp2 += -GJ12 * P.J12 * iz;
    }
    for (int a = 0; a < 3; ++a) gm[a] += Rc[a] * gp0 + Rc[3 + a] * gp1 + Rc[6 + a] * gp2 + gdir[a];
    // pose
    pose_acc[0] += gp0;
    pose_acc[1] += gp1;
    pose_acc[2] += gp2;
    pose_acc[3] += py * gp2 - pz * gp1;
    pose_acc[4] += pz * gp0 - px * gp2;
    pose_acc[5] += px * gp1 - py * gp0;
    // Gc = J^T GI J (J sparse), Sc = W Sigma_W W^T; X = Gc Sc; theta += 2 (X21-X12, X02-X20, X10-X01)
    float Gc[9];
    {
        const float j0[3] = {P.J00, 0.0f, P.J02};
        const float j1[3] = {0.0f, P.J11, P.J12};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Gc[3 * a + b] = j0[a] * (GI00 * j0[b] + GI01 * j1[b]) + j1[a] * (GI01 * j0[b] + GI11 * j1[b]);
    }
    float Sc[9];
    {
        const float Sw[9] = {P.S[0], P.S[1], P.S[2], P.S[1], P.S[3], P.S[4], P.S[2], P.S[4], P.S[5]};
        float RS[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                RS[3 * a + b] = Rc[3 * a] * Sw[b] + Rc[3 * a + 1] * Sw[3 + b] + Rc[3 * a + 2] * Sw[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Sc[3 * a + b] = RS[3 * a] * Rc[3 * b] + RS[3 * a + 1] * Rc[3 * b + 1] + RS[3 * a + 2] * Rc[3 * b + 2];
    }
    float X[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            X[3 * a + b] = Gc[3 * a] * Sc[b] + Gc[3 * a + 1] * Sc[3 + b] + Gc[3 * a + 2] * Sc[6 + b];
    pose_acc[3] += 2.0f * (X[7] - X[5]);
    pose_acc[4] += 2.0f * (X[2] - X[6]);
    pose_acc[5] += 2.0f * (X[3] - X[1]);
    pose_acc[6] += gdir[0];
    pose_acc[7] += gdir[1];
    pose_acc[8] += gdir[2];
}

}  // namespace mgs
