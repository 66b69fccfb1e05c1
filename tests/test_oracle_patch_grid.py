"""Pins of the Patch-Grid sampling oracle (oracle/patch_grid.py, Sec. II-B).

* Keypoint counts per patch against numpy's 2D histogram.
* The nearest keypoint with depth against scipy's k-d tree (on queries whose
  nearest neighbour is unique by a margin), and the tie rule on a hand case.
* A hand-built 64 x 64 image: which patches are sampled and where the samples lie.
* Depth precedence (own depth, then the depth map, then the nearest keypoint;
  dropped without any) on a hand case.
* Back-projection: every new mean, projected with the camera, lands on its
  keypoint or sample pixel at its depth; the colour reproduces the image.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import synth
from oracle import patch_grid as PG


def _cam(W, H, pose=None):
    T = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1) if pose is None else pose
    return synth.Camera(W, H, 0.9 * W, 0.9 * W, (W - 1) / 2.0, (H - 1) / 2.0, np.asarray(T, np.float32))


def test_counts_match_histogram():
    rng = np.random.default_rng(1)
    W, H, P = 200, 130, 32
    kp = rng.uniform(-5, [205, 135], size=(500, 2)).astype(np.float32)
    px, on = PG.keypoint_pixels(kp, W, H)
    PX, PY = -(-W // P), -(-H // P)
    h, _, _ = np.histogram2d(px[on, 1], px[on, 0], bins=[np.arange(0, P * PY + 1, P), np.arange(0, P * PX + 1, P)])
    assert np.array_equal(PG.patch_counts(kp, W, H, P), h.reshape(-1).astype(np.int64))
    assert (~on).sum() > 0


def test_nearest_keypoint_with_depth():
    rng = np.random.default_rng(2)
    kp = rng.uniform(0, 300, size=(400, 2)).astype(np.float32)
    kd = np.where(rng.uniform(size=400) < 0.3, 2.0, 0.0).astype(np.float32)
    q = rng.uniform(0, 300, size=(300, 2)).astype(np.float32)
    got = PG.nearest_with_depth(q, kp, kd)
    idx = np.nonzero(kd > 0)[0]
    tree = cKDTree(kp[idx].astype(np.float64))
    d, j = tree.query(q.astype(np.float64), k=2)
    clear = d[:, 1] - d[:, 0] > 1e-3
    assert clear.sum() > 250
    assert np.array_equal(got[clear], idx[j[clear, 0]])
    # equal distances: the lower index wins; no keypoint with depth: -1
    kp2 = np.array([[0, 0], [2, 0], [1, 5]], np.float32)
    assert PG.nearest_with_depth([[1, 0]], kp2, [1.0, 1.0, 1.0])[0] == 0
    assert PG.nearest_with_depth([[1, 0]], kp2, [0.0, 1.0, 1.0])[0] == 1
    assert PG.nearest_with_depth([[1, 0]], kp2, [0.0, 0.0, 0.0])[0] == -1


def test_hand_built_grid():
    W = H = 64
    kp = np.array([[3, 3], [10, 4], [20, 20], [30, 1], [15, 25], [40, 9]], np.float32)  # 5 in patch 0, 1 in patch 1
    counts = PG.patch_counts(kp, W, H, 32)
    assert counts.tolist() == [5, 1, 0, 0]
    spx = PG.sample_pixels(W, H, 32, 2, counts, 4)
    assert spx.tolist() == [[40, 8], [56, 8], [40, 24], [56, 24], [8, 40], [24, 40], [8, 56], [24, 56],
                            [40, 40], [56, 40], [40, 56], [56, 56]]
    # a clipped border patch: 70 wide, patch 2 covers x in [64, 70)
    c2 = PG.patch_counts(np.zeros((0, 2)), 70, 32, 32)
    assert PG.sample_pixels(70, 32, 32, 2, c2, 1).tolist() == [[8, 8], [24, 8], [8, 24], [24, 24],
                                                             [40, 8], [56, 8], [40, 24], [56, 24],
                                                             [65, 8], [68, 8], [65, 24], [68, 24]]


def test_depth_precedence():
    W = H = 64
    cam = _cam(W, H)
    kp = np.array([[5, 5], [50, 5], [5, 50], [60, 60]], np.float32)
    kd = np.array([2.0, 0.0, 0.0, 0.0], np.float32)
    img = np.zeros((3, H, W), np.float32)
    dm = np.zeros((H, W), np.float32)
    dm[5, 50] = 3.0  # map depth for keypoint 1 only
    o = PG.patch_grid_sample(cam, kp, kd, img, dm, P=32, min_kp=0, s=1)
    assert o["source"].tolist() == [0, 1, 2, 3] and o["point"].tolist() == [0, 1, 2, 3]
    assert o["depth"].tolist() == [2.0, 3.0, 2.0, 2.0]  # own, map, nearest (kp 0), nearest (kp 0)
    none = PG.patch_grid_sample(cam, kp, np.zeros(4, np.float32), img, None, P=32, min_kp=0, s=1)
    assert len(none["source"]) == 0


@pytest.mark.parametrize("exact", [True, False])
def test_back_projection_round_trip_and_colour(exact):
    """exact: a signed-permutation rotation (every entry exact in fp32, R^T R = I
    exactly), so the round trip closes to rounding; otherwise a random rotation
    stored in fp32, whose transpose inverts it to about 1e-7."""
    rng = np.random.default_rng(3)
    W, H = 160, 96
    R = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], float) if exact else Rotation.random(random_state=4).as_matrix()
    pose = np.concatenate([R, np.array([[0.25], [-0.5], [0.75]])], axis=1)
    cam = _cam(W, H, pose)
    kp = np.concatenate([rng.normal([40, 30], 6, size=(60, 2)), rng.uniform(0, [W, H], size=(10, 2))]).astype(np.float32)
    kd = np.where(rng.uniform(size=70) < 0.4, rng.uniform(1, 4, 70), 0).astype(np.float32)
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    dm = rng.uniform(1, 4, size=(H, W)).astype(np.float32)
    dm[rng.uniform(size=(H, W)) < 0.3] = 0
    o = PG.patch_grid_sample(cam, kp, kd, img, dm, P=32, min_kp=3, s=2, opacity=0.4, scale_factor=0.5)
    n_kp = len(kp)
    src = o["point"]  # index into keypoints, then into the sample list
    assert (src >= n_kp).sum() > 10 and (src < n_kp).sum() > 30
    # lattice slots of the kept samples: patch * s^2 + l * s + k, increasing
    slots = o["source"][o["source"] >= n_kp] - n_kp
    assert np.all(np.diff(slots) > 0)
    PX = -(-W // 32)
    spx = o["sample_pixels"][src[src >= n_kp] - n_kp]
    assert np.array_equal((spx[:, 1] // 32) * PX + spx[:, 0] // 32, slots // 4)
    T = np.asarray(cam.Tcw, np.float64)
    pc = o["means"] @ T[:, :3].T + T[:, 3]
    uv = np.stack([cam.fx * pc[:, 0] / pc[:, 2] + cam.cx, cam.fy * pc[:, 1] / pc[:, 2] + cam.cy], axis=1)
    spx = o["sample_pixels"]
    want = np.where((src < n_kp)[:, None], kp[np.minimum(src, n_kp - 1)].astype(np.float64),
                    spx[np.maximum(src - n_kp, 0)].astype(np.float64))
    np.testing.assert_allclose(uv, want, atol=1e-9 if exact else 1e-4)
    np.testing.assert_allclose(pc[:, 2], o["depth"], rtol=1e-12 if exact else 1e-6)
    pix = np.where((src < n_kp)[:, None], PG.keypoint_pixels(kp, W, H)[0][np.minimum(src, n_kp - 1)],
                   spx[np.maximum(src - n_kp, 0)])
    rgb = 0.5 + PG.SH_C0 * o["sh"][:, 0, :]
    np.testing.assert_allclose(rgb, img[:, pix[:, 1], pix[:, 0]].T, atol=1e-12)
    np.testing.assert_allclose(o["scales"][:, 0], 0.5 * o["depth"] * 16 / cam.fx, rtol=1e-12)
    assert np.all(o["opac"] == 0.4) and np.all(o["quats"] == [1, 0, 0, 0])
