"""GPU parity of Patch-Grid sampling (mgs_patch_grid_sample, Sec. II-B) against
the oracle.

Bars: the kept candidates and their order (the source of every new Gaussian,
which carries every integer decision: pixels, patch counts, lattice, nearest
keypoint) bit-exact; means within 1e-5 relative to the scene extent (fp32
back-projection against fp64), scales and colours within 1e-6 relative,
rotations and opacities exact.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import patch_grid as PG
from paper_2509_13536_amd import View, patch_grid_sample, render_forward

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _compare(kf, res, exp, n_kp):
    assert res.n_out == len(exp["source"]), (res.n_out, len(exp["source"]))
    assert np.array_equal(res.source.cpu().numpy(), exp["source"])
    m = res.map
    ext = max(1.0, float(np.abs(exp["means"]).max(initial=1.0)))
    np.testing.assert_allclose(m.means.cpu().numpy(), exp["means"], rtol=0, atol=1e-5 * ext)
    np.testing.assert_allclose(m.scales.cpu().numpy(), exp["scales"], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(m.sh.cpu().numpy(), exp["sh"], rtol=1e-6, atol=1e-6)
    assert np.all(m.quats.cpu().numpy() == np.array([1, 0, 0, 0], np.float32))
    assert np.all(m.opac.cpu().numpy() == np.float32(exp["opac"][0] if len(exp["opac"]) else 0))
    src = exp["source"]
    print(f"kept {res.n_out}: {int((src < n_kp).sum())} keypoints, {int((src >= n_kp).sum())} samples", flush=True)


@pytest.mark.parametrize("rgbd", [False, True])
def test_keyframe_matches_oracle(rgbd):
    kf = synth.keyframe_features(60)
    print(f"case patch grid 1200x680 rgbd={rgbd}", flush=True)
    view = View.from_camera(kf.cam)
    dm = kf.depth_map if rgbd else None
    res = patch_grid_sample(view, _t(kf.keypoints), _t(kf.kp_depth), _t(kf.image), None if dm is None else _t(dm),
                            patch=32, min_keypoints=4, samples=2, opacity=0.5, scale_factor=0.5)
    torch.cuda.synchronize()
    exp = PG.patch_grid_sample(kf.cam, kf.keypoints, kf.kp_depth, kf.image, dm, P=32, min_kp=4, s=2, opacity=0.5,
                               scale_factor=0.5)
    _compare(kf, res, exp, len(kf.keypoints))
    # the new Gaussians render through the same library
    st = render_forward([res.map], [view])
    torch.cuda.synchronize()
    assert int(st.info.n_visible) > 0.9 * res.n_out


def test_ragged_and_edge_cases():
    rng = np.random.default_rng(5)
    W, H = 70, 45
    T = np.concatenate([np.eye(3), [[0.1], [0.0], [0.2]]], axis=1).astype(np.float32)
    cam = synth.Camera(W, H, 60.0, 60.0, 35.0, 22.0, T)
    view = View.from_camera(cam)
    kp = np.concatenate([rng.uniform(-3, [73, 48], size=(40, 2)),
                         [[15.5, 3.0], [15.49, 3.0], [-0.6, 2.0], [np.nan, 4.0], [69.4, 44.4], [20.0, 20.0],
                          [22.0, 20.0]]]).astype(np.float32)
    kd = np.where(rng.uniform(size=len(kp)) < 0.3, rng.uniform(1, 3, len(kp)), 0).astype(np.float32)
    kd[-2:] = 2.0  # two keypoints at equal distance from sample (21, y): the lower index wins
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    dm = rng.uniform(1, 3, size=(H, W)).astype(np.float32)
    dm[rng.uniform(size=(H, W)) < 0.5] = 0
    for depth_map, P, s, mk in ((None, 16, 3, 3), (dm, 16, 3, 3), (None, 7, 1, 100), (dm, 45, 5, 1)):
        print(f"case ragged P={P} s={s} min_kp={mk} rgbd={depth_map is not None}", flush=True)
        res = patch_grid_sample(view, _t(kp), _t(kd), _t(img), None if depth_map is None else _t(depth_map),
                                patch=P, min_keypoints=mk, samples=s, opacity=0.3, scale_factor=0.7)
        torch.cuda.synchronize()
        exp = PG.patch_grid_sample(cam, kp, kd, img, depth_map, P=P, min_kp=mk, s=s, opacity=0.3, scale_factor=0.7)
        _compare(None, res, exp, len(kp))
    # no keypoints: samples only; monocular and no keypoints: nothing has a depth
    e = np.zeros((0, 2), np.float32)
    r0 = patch_grid_sample(view, _t(e), _t(np.zeros(0)), _t(img), _t(dm), patch=16, min_keypoints=1, samples=2)
    x0 = PG.patch_grid_sample(cam, e, np.zeros(0, np.float32), img, dm, P=16, min_kp=1, s=2)
    torch.cuda.synchronize()
    _compare(None, r0, x0, 0)
    r1 = patch_grid_sample(view, _t(e), _t(np.zeros(0)), _t(img), None, patch=16, min_keypoints=1, samples=2)
    assert r1.n_out == 0


def test_many_keypoints():
    kf = synth.keyframe_features(61, n_kp=20000, clusters=40)
    print("case patch grid 20k keypoints P=16", flush=True)
    view = View.from_camera(kf.cam)
    res = patch_grid_sample(view, _t(kf.keypoints), _t(kf.kp_depth), _t(kf.image), None, patch=16,
                            min_keypoints=6, samples=2)
    torch.cuda.synchronize()
    exp = PG.patch_grid_sample(kf.cam, kf.keypoints, kf.kp_depth, kf.image, None, P=16, min_kp=6, s=2)
    _compare(kf, res, exp, len(kf.keypoints))
