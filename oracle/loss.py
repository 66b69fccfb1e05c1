"""Mapping loss of Eq. (12) (Sec. II-E), numpy float64.  TEST INFRASTRUCTURE ONLY:
imported by tests, the smoke check and the benchmark's CPU-baseline leg, never
by the product path.

For one view with rendered colour I_r [3,H,W], target I_gt, rendered depth D and
target depth D_gt [H,W]:

  L_view = (1 - lambda) mean|I_r - I_gt| + lambda (1 - mean SSIM(I_r, I_gt))
           + w_depth mean(valid |D - D_gt|),   valid = D_gt > 0,

means over every pixel (and channel); and for the map's linear scales s [N,3]

  L_iso = w_iso mean_{i,k} |s_ik - mean_m s_im|.

The total is the sum of L_view over the views plus L_iso.

SSIM follows its usual definition: local statistics under an 11x11 Gaussian
window (sigma 1.5, weights normalised to sum 1) with zero padding at the image
border, C1 = 0.01^2, C2 = 0.03^2, per channel and pixel
  S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)).

Readings where the paper is silent (the design notes list them): lambda = 0.2,
the depth residual as the masked L1 above with its weight a parameter, L_iso as
the mean absolute deviation of each Gaussian's scales from their mean (the
isotropic term of the cited Gaussian-splatting SLAM), sign(0) = 0 for the L1
subgradient.

Gradients are the exact derivatives, written out:
  d mean S / d x(q) = 1/N [ (G * dS/dmu_x)(q) + 2 x(q) (G * dS/dE[x^2])(q) + y(q) (G * dS/dE[xy])(q) ]
with, per pixel p, A = 2 mu_x mu_y + C1, B = 2 sigma_xy + C2, C = mu_x^2 + mu_y^2 + C1,
D = sigma_x^2 + sigma_y^2 + C2:
  dS/dE[x^2] = -S / D,   dS/dE[xy] = 2 S / B,
  dS/dmu_x   = 2 S (mu_y / A - mu_x / C + mu_x / D - mu_y / B),
and G * f the same zero-padded window sum (the window is symmetric).
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5
LAMBDA_SSIM = 0.2


def window() -> np.ndarray:
    """[11,11] Gaussian window, sigma 1.5, normalised to sum 1 (outer product of the 1D weights)."""
    r = np.arange(WIN) - WIN // 2
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def window_sum(f: np.ndarray) -> np.ndarray:
    """(G * f)(p) = sum over the 11x11 offsets o of G(o) f(p + o), f zero outside the image."""
    H, W = f.shape
    h = WIN // 2
    fp = np.zeros((H + 2 * h, W + 2 * h))
    fp[h:h + H, h:h + W] = f
    Gw = window()
    out = np.zeros((H, W))
    for dy in range(WIN):
        for dx in range(WIN):
            out += Gw[dy, dx] * fp[dy:dy + H, dx:dx + W]
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray):
    """Per-pixel SSIM of two [H,W] images and its partial derivatives."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = window_sum(x), window_sum(y)
    sxx = window_sum(x * x) - mx * mx
    syy = window_sum(y * y) - my * my
    sxy = window_sum(x * y) - mx * my
    A = 2 * mx * my + C1
    B = 2 * sxy + C2
    C = mx * mx + my * my + C1
    D = sxx + syy + C2
    S = A * B / (C * D)
    d_mu = 2 * S * (my / A - mx / C + mx / D - my / B)
    d_xx = -S / D
    d_xy = 2 * S / B
    return S, d_mu, d_xx, d_xy


def ssim_grad_sum(x, y):
    """Gradient of sum_p S(p) with respect to every pixel of x."""
    _, d_mu, d_xx, d_xy = ssim_terms(x, y)
    return window_sum(d_mu) + 2 * np.asarray(x, np.float64) * window_sum(d_xx) + \
        np.asarray(y, np.float64) * window_sum(d_xy)


def view_loss(rgb, gt, depth=None, gt_depth=None, lam=LAMBDA_SSIM, w_depth=0.0):
    """(terms, d_rgb, d_depth) of one view.  terms = (mean|I_r - I_gt|, mean SSIM,
    mean(valid |D - D_gt|), L_view)."""
    rgb = np.asarray(rgb, np.float64)
    gt = np.asarray(gt, np.float64)
    _, H, W = rgb.shape
    n = 3 * H * W
    diff = rgb - gt
    l1 = np.abs(diff).sum() / n
    ssum = 0.0
    d_rgb = (1 - lam) / n * np.sign(diff)
    for c in range(3):
        S, _, _, _ = ssim_terms(rgb[c], gt[c])
        ssum += S.sum()
        d_rgb[c] -= lam / n * ssim_grad_sum(rgb[c], gt[c])
    ssim = ssum / n
    ld = 0.0
    d_depth = None
    if depth is not None and gt_depth is not None:
        depth = np.asarray(depth, np.float64)
        gd = np.asarray(gt_depth, np.float64)
        valid = gd > 0
        dd = np.where(valid, depth - gd, 0.0)
        ld = np.abs(dd).sum() / (H * W)
        d_depth = w_depth / (H * W) * np.sign(dd)
    total = (1 - lam) * l1 + lam * (1 - ssim) + w_depth * ld
    return (l1, ssim, ld, total), d_rgb, d_depth


def iso_loss(scales, w_iso):
    """(L_iso, d L_iso / d scales) for linear scales [N,3]."""
    s = np.asarray(scales, np.float64)
    if s.shape[0] == 0:
        return 0.0, np.zeros_like(s)
    dev = s - s.mean(axis=1, keepdims=True)
    m = s.size
    L = w_iso * np.abs(dev).sum() / m
    sg = np.sign(dev)
    d = w_iso / m * (sg - sg.mean(axis=1, keepdims=True))
    return L, d
