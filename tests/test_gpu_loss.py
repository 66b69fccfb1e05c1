"""GPU parity of the Eq. (12) mapping loss (mgs_mapping_loss) against the oracle.

Bars: loss values within 1e-5 relative (fp32 stencil sums against fp64); the
colour gradient within 1e-4 relative L2 and element-wise 1e-4 |g*| + 1e-4 max|g*|;
the depth and L_iso gradients (sign decisions taken on the same inputs, the L_iso
ones in fp64 on both sides) within 1e-6 relative; repeated calls bit-identical.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import loss as OL
from paper_2509_13536_amd import autograd as AG
from paper_2509_13536_amd import GaussianMap, View, mapping_loss, render_backward, render_forward

from gpu_helpers import grad_parity

pytestmark = pytest.mark.gpu


def _images(rng, sizes):
    rgb, gt, d, gd = [], [], [], []
    for W, H in sizes:
        x = rng.uniform(size=(3, H, W))
        y = np.clip(x + rng.normal(0, 0.15, size=x.shape), 0, 1)
        y[:, : H // 3, : W // 4] = 0.5       # a flat patch: SSIM with near-zero variance
        x[1, -3:, :] = y[1, -3:, :]           # equal values: L1 subgradient 0
        z = rng.uniform(1.0, 3.0, size=(H, W))
        zg = z + rng.normal(0, 0.1, size=(H, W))
        zg[rng.uniform(size=(H, W)) < 0.2] = 0.0
        rgb.append(x.astype(np.float32))
        gt.append(y.astype(np.float32))
        d.append(z.astype(np.float32))
        gd.append(zg.astype(np.float32))
    return rgb, gt, d, gd


def _flat(arrs):
    return torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs])).cuda()


def _check(sizes, rgb, gt, d, gd, scales, lam, wd, wi, res, views_checked=None):
    loss = res.loss.cpu().numpy()
    d_rgb = res.d_rgb.cpu().numpy()
    d_dep = res.d_depth.cpu().numpy()
    off1 = np.concatenate([[0], np.cumsum([W * H for W, H in sizes])])
    total = 0.0
    for v, (W, H) in enumerate(sizes):
        if views_checked is not None and v not in views_checked:
            total = None
            continue
        terms, g_rgb, g_d = OL.view_loss(rgb[v], gt[v], d[v], gd[v], lam, wd)
        print(f"view {v} {W}x{H}: gpu {loss[4 * v:4 * v + 4]} oracle {np.array(terms)}", flush=True)
        np.testing.assert_allclose(loss[4 * v:4 * v + 4], terms, rtol=1e-5, atol=1e-7)
        o = off1[v]
        grad_parity(d_rgb[3 * o:3 * (o + W * H)], g_rgb, f"d_rgb view {v}", rel_l2=1e-4, elem=1e-4)
        np.testing.assert_allclose(d_dep[o:o + W * H], g_d.reshape(-1), rtol=1e-6, atol=0)
        if total is not None:
            total += terms[3]
    if scales is not None:
        li, g_s = OL.iso_loss(scales, wi)
        np.testing.assert_allclose(loss[-2], li, rtol=1e-6)
        np.testing.assert_allclose(res.d_scales.cpu().numpy(), g_s, rtol=1e-6, atol=0)
        if total is not None:
            total += li
    if total is not None:
        np.testing.assert_allclose(loss[-1], total, rtol=1e-5)


def test_loss_ragged_views_match_oracle():
    rng = np.random.default_rng(11)
    sizes = [(50, 37), (129, 70), (33, 32), (1, 1)]
    rgb, gt, d, gd = _images(rng, sizes)
    scales = rng.uniform(0.01, 0.1, size=(300, 3)).astype(np.float32)
    scales[:7] = scales[:7, :1]  # isotropic ones: zero deviation
    lam, wd, wi = 0.2, 0.7, 3.0
    print("case loss ragged 4 views", flush=True)
    res = mapping_loss(sizes, _flat(rgb), _flat(gt), _flat(d), _flat(gd), torch.from_numpy(scales).cuda(),
                       lam, wd, wi)
    torch.cuda.synchronize()
    _check(sizes, rgb, gt, d, gd, scales, lam, wd, wi, res)
    again = mapping_loss(sizes, _flat(rgb), _flat(gt), _flat(d), _flat(gd), torch.from_numpy(scales).cuda(),
                         lam, wd, wi)
    torch.cuda.synchronize()
    assert torch.equal(res.loss, again.loss) and torch.equal(res.d_rgb, again.d_rgb)
    # no depth, no scales: those terms vanish
    r2 = mapping_loss(sizes, _flat(rgb), _flat(gt), lambda_ssim=lam)
    l2 = r2.loss.cpu().numpy()
    assert l2[-2] == 0.0 and np.all(l2[2:-2:4] == 0.0)
    np.testing.assert_allclose(l2[3:-2:4], res.loss.cpu().numpy()[3:-2:4] - wd * res.loss.cpu().numpy()[2:-2:4],
                               rtol=1e-5)


def test_loss_full_window_size():
    """The window's 8 views of 1200x680 in one call: view 0 against the whole
    oracle; view 7 on three bands of rows (top, middle, bottom), each from the
    oracle on a crop reaching 10 rows beyond the band (the gradient at a pixel
    depends only on pixels within 10 of it), at the full image's normalisation."""
    rng = np.random.default_rng(12)
    sizes = [(1200, 680)] * 8
    rgb, gt, d, gd = _images(rng, sizes)
    lam = 0.2
    print("case loss 8 x 1200x680", flush=True)
    res = mapping_loss(sizes, _flat(rgb), _flat(gt), _flat(d), _flat(gd), lambda_ssim=lam, w_depth=1.0)
    torch.cuda.synchronize()
    _check(sizes, rgb, gt, d, gd, None, lam, 1.0, 0.0, res, views_checked={0})
    W, H = sizes[7]
    n = 3 * W * H
    o = 7 * W * H
    g7 = res.d_rgb.cpu().numpy()[3 * o:3 * (o + W * H)].reshape(3, H, W)
    for r0, r1 in ((0, 40), (320, 360), (640, 680)):
        c0, c1 = max(r0 - 10, 0), min(r1 + 10, H)
        x, y = rgb[7][:, c0:c1].astype(np.float64), gt[7][:, c0:c1].astype(np.float64)
        exp = np.stack([(1 - lam) / n * np.sign(x[c] - y[c]) - lam / n * OL.ssim_grad_sum(x[c], y[c])
                        for c in range(3)])[:, r0 - c0:r1 - c0]
        grad_parity(g7[:, r0:r1], exp, f"d_rgb view 7 rows {r0}-{r1}", rel_l2=1e-4, elem=1e-4)


def test_loss_autograd_feeds_the_renderer():
    sc = synth.tiny_scene(1500, 96, 72, 21, sh_degree=1, pose=True)
    views = [View.from_camera(sc.cams[0])]
    t = lambda a, g=False: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(g)
    means, scales, quats, opac, sh = (t(sc.means, True), t(sc.scales, True), t(sc.quats, True), t(sc.opac, True),
                                      t(sc.sh, True))
    rng = np.random.default_rng(3)
    gt = t(rng.uniform(size=3 * 96 * 72))
    gtd = t(rng.uniform(1.5, 3.0, size=96 * 72))
    rgb, depth = AG.render(means, scales, quats, opac, sh, views, sc.sh_degree)
    total, terms = AG.loss(rgb, gt, views, depth, gtd, scales, w_depth=0.5, w_iso=2.0)
    total.backward()
    # the same chain by hand through the C ABI
    m = GaussianMap.from_numpy(sc)
    st = render_forward([m], views, need_backward=True)
    res = mapping_loss([(96, 72)], st.rgb, gt.detach(), st.depth, gtd.detach(), m.scales, w_depth=0.5, w_iso=2.0)
    grads, _ = render_backward(st, res.d_rgb, res.d_depth)
    torch.cuda.synchronize()
    assert torch.equal(total.detach(), res.loss[-1])
    assert torch.equal(means.grad, grads[0]["means"])
    assert torch.equal(opac.grad, grads[0]["opac"])
    assert torch.equal(scales.grad, grads[0]["scales"] + res.d_scales)
