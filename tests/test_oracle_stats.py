"""Pins of the Eq. (3) merge-eligibility oracle: the gradient statistics that
the renderer's backward accumulates, and the mask M(G) formed from them.

* The per-view gradient norms are checked against central finite differences
  of the frozen-decision forward loss, view by view, in fp64 (an independent
  route to d L_v / d mu that does not go through the analytic backward).
* The view count is checked on Gaussians placed where the answer is known:
  behind the camera, outside the image, on the optical axis.
* The mask is checked on a hand-built table, including the strict inequality
  at tau, an unseen Gaussian and both ends of the keyframe window.
"""
import numpy as np

import oracle
import synth
from oracle import merge as M


def _two_view_scene():
    sc = synth.tiny_scene(10, 32, 24, seed=31, sh_degree=1, log_scale_mu=-2.6)
    cam0 = sc.cams[0]
    # a second view: the first one turned by 0.12 rad about y and shifted
    a = 0.12
    R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    T1 = np.concatenate([R, np.array([[0.08], [-0.03], [0.05]])], axis=1).astype(np.float32)
    cam1 = synth.Camera(cam0.W, cam0.H, cam0.fx, cam0.fy, cam0.cx, cam0.cy, T1)
    return sc, [cam0, cam1]


def test_grad_norms_match_finite_differences_per_view():
    sc, cams = _two_view_scene()
    rng = np.random.default_rng(5)
    w_rgb = [rng.normal(size=(3, c.H, c.W)) for c in cams]
    w_d = [rng.normal(size=(c.H, c.W)) for c in cams]
    total, count = oracle.grad_stats(sc, cams, w_rgb, w_d)
    base = [sc.means.astype(np.float64), sc.scales.astype(np.float64), sc.quats.astype(np.float64),
            sc.opac.astype(np.float64), sc.sh.astype(np.float64)]
    eps = 1e-6
    expect = np.zeros(sc.n)
    per_view = []
    for v, cam in enumerate(cams):
        frozen = oracle.contributors(sc, cam)
        _, c64 = oracle.cam_arrays(cam)

        def loss(means):
            rgb, d = oracle.forward_frozen([means] + base[1:], sc.sh_degree, c64, frozen)
            return float((w_rgb[v] * rgb).sum() + (w_d[v] * d).sum())

        fd = np.zeros((sc.n, 3))
        for i in range(sc.n):
            for c in range(3):
                p, m = base[0].copy(), base[0].copy()
                p[i, c] += eps
                m[i, c] -= eps
                fd[i, c] = (loss(p) - loss(m)) / (2 * eps)
        per_view.append(fd)
        expect += np.linalg.norm(fd, axis=1)
    assert (count == 2).sum() >= 5, "most Gaussians must be seen by both views"
    np.testing.assert_allclose(total, expect, rtol=1e-5, atol=1e-7 * expect.max())
    # a statistic of the summed gradient would differ: the norms are taken per view
    summed = np.linalg.norm(per_view[0] + per_view[1], axis=1)
    assert np.abs(summed - expect).max() > 1e-3 * expect.max()


def test_view_count_closed_cases():
    sc = synth.tiny_scene(3, 32, 24, seed=4, log_scale_mu=-3.0)
    cam = sc.cams[0]
    sc.means[0] = [0.0, 0.0, -2.0]          # behind the camera
    sc.means[1] = [40.0, 0.0, 2.0]          # far outside the image
    sc.means[2] = [0.0, 0.0, 2.0]           # on the optical axis
    sc.opac[:] = 0.8
    g = [np.ones((3, cam.H, cam.W))] * 3
    _, count = oracle.grad_stats(sc, [cam, cam, cam], g, None)
    assert count.tolist() == [0, 0, 3]


def test_merge_mask_table():
    tau = np.float32(1e-3)
    # average exactly tau (4 tau / 4 is exact in binary): not below tau
    grad_sum = np.array([4 * tau, 0.0039, 0.0, 0.0, 2.5e-4, 1.0, 5e-4, 5e-4, 5e-4], np.float32)
    count = np.array([4, 4, 0, 3, 1, 1, 1, 1, 1])
    kf = np.array([3, 3, 3, 3, 3, 3, 2, 7, 8])
    expect = np.array([0, 1, 0, 1, 1, 0, 1, 1, 0], np.uint8)
    got = M.merge_mask(grad_sum, count, tau, kf_index=kf, kf_min=2, kf_max=7)
    assert np.array_equal(got, expect)
    # without keyframe indices the window test is skipped
    assert np.array_equal(M.merge_mask(grad_sum, count, tau), np.array([0, 1, 0, 1, 1, 0, 1, 1, 1], np.uint8))
    # the paper's tau
    assert M.GRAD_TAU == 1e-3
