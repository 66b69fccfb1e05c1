"""Analytic fp64 gradients of the render oracle against central finite differences.

The forward used for the differences composites the contributor lists taken at
the base point (frozen decisions: the same Gaussians, the same alpha clamps),
so the function is smooth and its derivative is what the backward computes.
Pose perturbations use the exact SE(3) exponential (scipy expm of the twist),
applied on the left: T <- Exp(xi) T, xi = (rho, theta).
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth


def _skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def _se3_exp(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = _skew(xi[3:])
    X[:3, 3] = xi[:3]
    return expm(X)


def _scene_with_special_cases(seed, deg):
    sc = synth.tiny_scene(14, 32, 24, seed, sh_degree=deg, pose=True, log_scale_mu=-2.6)
    cam = sc.cams[0]
    R_cw = cam.Tcw[:, :3].astype(np.float64)
    t_cw = cam.Tcw[:, 3].astype(np.float64)

    def to_world(pc):
        return R_cw.T @ (np.asarray(pc, np.float64) - t_cw)

    extra_means = [
        to_world([1.15 * 2.0 * (1.3 * 0.5 * cam.W / cam.fx), 0.05, 2.0]),    # beyond the x frustum clamp
        to_world([0.0, -1.15 * 2.2 * (1.3 * 0.5 * cam.H / cam.fy), 2.2]),    # beyond the y clamp
        to_world([(3.0 - cam.cx) * 1.8 / cam.fx, (4.0 - cam.cy) * 1.8 / cam.fy, 1.8]),    # near pixel (3,4)
    ]
    K = (deg + 1) ** 2
    rng = np.random.default_rng(seed)
    add = len(extra_means)
    sc.means = np.concatenate([sc.means, np.asarray(extra_means, np.float32)])
    sc.scales = np.concatenate([sc.scales, np.array([[0.45, 0.3, 0.2], [0.25, 0.5, 0.3], [0.05, 0.04, 0.06]], np.float32)])
    q = rng.normal(size=(add, 4))
    sc.quats = np.concatenate([sc.quats, q.astype(np.float32)])
    sc.opac = np.concatenate([sc.opac, np.array([0.6, 0.5, 0.9999], np.float32)])   # last one clamps at 0.99
    extra_sh = rng.normal(0, 0.2, size=(add, K, 3)).astype(np.float32)
    extra_sh[0, 0, 0] = -3.0                                                          # red clamped to 0
    sc.sh = np.concatenate([sc.sh, extra_sh])
    return sc


@pytest.mark.parametrize("seed,deg", [(21, 0), (22, 3), (23, 1)])
def test_gradients_match_central_differences(seed, deg):
    sc = _scene_with_special_cases(seed, deg)
    cam = sc.cams[0]
    frozen = oracle.contributors(sc, cam)
    counts, gids, clamped = frozen
    assert clamped.any(), "scene must exercise the alpha clamp"
    k = oracle.keys(sc, cam)
    assert k["valid"][-3:].all()
    n = sc.n
    assert {n - 3, n - 2, n - 1} <= set(gids.tolist()), "special cases must contribute"
    rng = np.random.default_rng(seed + 1)
    w_rgb = rng.normal(size=(3, cam.H, cam.W))
    w_d = rng.normal(size=(cam.H, cam.W))
    an = oracle.backward(sc, cam, w_rgb, w_d)
    _, c64 = oracle.cam_arrays(cam)
    base = [sc.means.astype(np.float64), sc.scales.astype(np.float64), sc.quats.astype(np.float64),
            sc.opac.astype(np.float64), sc.sh.astype(np.float64)]

    def loss(params, cam64):
        rgb, d = oracle.forward_frozen(params, sc.sh_degree, cam64, frozen)
        return float((w_rgb * rgb).sum() + (w_d * d).sum())

    eps = 1e-6
    names = ["means", "scales", "quats", "opac", "sh"]
    for pi, name in enumerate(names):
        fd = np.zeros_like(base[pi])
        flat = fd.reshape(-1)
        for i in range(flat.size):
            plus = [b.copy() for b in base]
            minus = [b.copy() for b in base]
            plus[pi].reshape(-1)[i] += eps
            minus[pi].reshape(-1)[i] -= eps
            flat[i] = (loss(plus, c64) - loss(minus, c64)) / (2 * eps)
        a = an[name].reshape(fd.shape)
        scale = np.abs(a).max()
        assert scale > 0
        np.testing.assert_allclose(a, fd, rtol=1e-5, atol=1e-6 * scale, err_msg=name)
    # pose: T <- Exp(xi) T
    T4 = np.eye(4)
    T4[:3, :3] = c64[7:16].reshape(3, 3)
    T4[:3, 3] = c64[16:19]
    fd_pose = np.zeros(6)
    for kk in range(6):
        out = []
        for sgn in (1, -1):
            xi = np.zeros(6)
            xi[kk] = sgn * eps
            Tn = _se3_exp(xi) @ T4
            cn = c64.copy()
            cn[7:16] = Tn[:3, :3].reshape(-1)
            cn[16:19] = Tn[:3, 3]
            out.append(loss(base, cn))
        fd_pose[kk] = (out[0] - out[1]) / (2 * eps)
    np.testing.assert_allclose(an["pose"], fd_pose, rtol=1e-5, atol=1e-6 * np.abs(fd_pose).max())
