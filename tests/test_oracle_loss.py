"""Pins of the Eq. (12) mapping-loss oracle (oracle/loss.py).

* SSIM against an independent construction from scipy.ndimage.gaussian_filter
  (normalised 11-tap Gaussian, sigma 1.5, zero padding): a library routine in
  place of the explicit window sum.
* SSIM(x, x) = 1 at every pixel, and the SSIM gradient vanishes there.
* Constant images: away from the border SSIM = (2ab + C1) / (a^2 + b^2 + C1).
* The whole loss (colour L1, SSIM, masked depth L1, L_iso) against central
  finite differences in fp64, on points away from the L1 kinks.
* L_iso of isotropic Gaussians is 0.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

from oracle import loss as L


def _blur(f):
    return gaussian_filter(np.asarray(f, np.float64), sigma=1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)


def test_ssim_matches_scipy_gaussian_filter():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(23, 31))
    y = np.clip(x + rng.normal(0, 0.2, size=x.shape), 0, 1)
    mx, my = _blur(x), _blur(y)
    vx, vy, cxy = _blur(x * x) - mx ** 2, _blur(y * y) - my ** 2, _blur(x * y) - mx * my
    ref = (2 * mx * my + L.C1) * (2 * cxy + L.C2) / ((mx ** 2 + my ** 2 + L.C1) * (vx + vy + L.C2))
    S, _, _, _ = L.ssim_terms(x, y)
    np.testing.assert_allclose(S, ref, rtol=1e-12, atol=1e-13)
    assert abs(L.window().sum() - 1.0) < 1e-15


def test_ssim_of_identical_images_is_one_with_zero_gradient():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(17, 12))
    S, _, _, _ = L.ssim_terms(x, x)
    np.testing.assert_allclose(S, 1.0, rtol=0, atol=1e-13)
    assert np.abs(L.ssim_grad_sum(x, x)).max() < 1e-10


def test_ssim_constant_images_closed_form():
    a, b = 0.7, 0.3
    x = np.full((20, 24), a)
    y = np.full((20, 24), b)
    S, _, _, _ = L.ssim_terms(x, y)
    inner = S[5:-5, 5:-5]
    np.testing.assert_allclose(inner, (2 * a * b + L.C1) / (a * a + b * b + L.C1), rtol=1e-12)


def _away_from_kinks(rng, shape, gap=0.05):
    a = rng.uniform(0.1, 0.9, size=shape)
    s = rng.choice([-1.0, 1.0], size=shape)
    return a, np.clip(a + s * rng.uniform(gap, 0.3, size=shape), 0.0, 1.0)


def test_view_loss_matches_finite_differences():
    rng = np.random.default_rng(3)
    H, W = 9, 13
    rgb, gt = _away_from_kinks(rng, (3, H, W))
    depth = rng.uniform(1.0, 3.0, size=(H, W))
    gt_d = depth + rng.choice([-1.0, 1.0], size=(H, W)) * rng.uniform(0.05, 0.3, size=(H, W))
    gt_d[rng.uniform(size=(H, W)) < 0.2] = 0.0  # no target depth there
    lam, wd = 0.2, 0.3
    _, d_rgb, d_depth = L.view_loss(rgb, gt, depth, gt_d, lam, wd)

    def total(r, d):
        return L.view_loss(r, gt, d, gt_d, lam, wd)[0][3]

    eps = 1e-6
    fd = np.zeros_like(rgb)
    for i in range(rgb.size):
        p, m = rgb.copy(), rgb.copy()
        p.reshape(-1)[i] += eps
        m.reshape(-1)[i] -= eps
        fd.reshape(-1)[i] = (total(p, depth) - total(m, depth)) / (2 * eps)
    np.testing.assert_allclose(d_rgb, fd, rtol=1e-6, atol=1e-9)
    fdd = np.zeros_like(depth)
    for i in range(depth.size):
        p, m = depth.copy(), depth.copy()
        p.reshape(-1)[i] += eps
        m.reshape(-1)[i] -= eps
        fdd.reshape(-1)[i] = (total(rgb, p) - total(rgb, m)) / (2 * eps)
    np.testing.assert_allclose(d_depth, fdd, rtol=1e-6, atol=1e-9)
    assert np.all(d_depth[gt_d == 0] == 0)
    # the SSIM part alone is not zero: the test covers it
    _, d_l1, _ = L.view_loss(rgb, gt, None, None, 0.0, 0.0)
    assert np.abs(d_rgb - (1 - lam) * d_l1).max() > 1e-4


def test_iso_loss_gradient_and_isotropic_zero():
    rng = np.random.default_rng(4)
    s = rng.uniform(0.01, 0.1, size=(7, 3))
    w = 2.5
    Lv, d = L.iso_loss(s, w)
    eps = 1e-8
    fd = np.zeros_like(s)
    for i in range(s.size):
        p, m = s.copy(), s.copy()
        p.reshape(-1)[i] += eps
        m.reshape(-1)[i] -= eps
        fd.reshape(-1)[i] = (L.iso_loss(p, w)[0] - L.iso_loss(m, w)[0]) / (2 * eps)
    np.testing.assert_allclose(d, fd, rtol=1e-6, atol=1e-9)
    iso = np.repeat(rng.uniform(0.01, 0.1, size=(5, 1)), 3, axis=1)
    assert L.iso_loss(iso, w)[0] == 0.0
    assert Lv > 0
