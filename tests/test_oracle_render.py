"""Pins of the render oracle against things other than itself (CPU only).

* a single isotropic Gaussian on the optical axis: closed-form footprint;
* brute-force per-pixel compositing (no tiles, Python) on tiny scenes, and
  unculled compositing over every Gaussian when opacity <= 0.3 (then 3-sigma
  culling provably drops nothing);
* the projection of Eq. (1) rebuilt from scipy's rotation and a numerical
  Jacobian of the pinhole map;
* spherical-harmonic basis: orthonormality by quadrature, scipy's harmonics;
* compositing invariants of Eq. (11);
* fp32 key path against the fp64 value path; culling of degenerate inputs.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from synth.scenes import Camera, Scene

A_MAX, A_MIN, T_MIN = float(np.float32(0.99)), float(np.float32(1 / 255)), float(np.float32(1e-4))


def _single(z=2.0, s=0.02, o=0.7, W=64, H=48, f=100.0, cx=31.0, cy=22.0):
    means = np.array([[0.0, 0.0, z]], np.float32)
    scales = np.full((1, 3), s, np.float32)
    quats = np.array([[1.0, 0.0, 0.0, 0.0]], np.float32)
    opac = np.array([o], np.float32)
    sh = np.zeros((1, 1, 3), np.float32)  # colour 0.5
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    return Scene(means, scales, quats, opac, sh, 0, [Camera(W, H, f, f, cx, cy, Tcw)])


def test_single_isotropic_gaussian_closed_form():
    sc = _single()
    cam = sc.cams[0]
    z, s, o, f = 2.0, float(np.float32(0.02)), float(np.float32(0.7)), 100.0
    var = (f * s / z) ** 2 + 0.3                 # J W (s^2 I) W^T J^T + 0.3 I at the axis
    lam = var + math.sqrt(0.1)                   # radius rule with the 0.1 floor (isotropic: disc = 0)
    r = math.ceil(3 * math.sqrt(lam))
    out = oracle.forward(sc, cam, bands=None)
    yy, xx = np.mgrid[0:cam.H, 0:cam.W].astype(np.float64)
    d2 = (xx - cam.cx) ** 2 + (yy - cam.cy) ** 2
    alpha = np.minimum(A_MAX, o * np.exp(-0.5 * d2 / var))
    alpha[alpha < A_MIN] = 0.0
    tx0, tx1 = math.floor((cam.cx - r) / 16), math.floor((cam.cx + r) / 16) + 1
    ty0, ty1 = math.floor((cam.cy - r) / 16), math.floor((cam.cy + r) / 16) + 1
    inside = ((xx // 16 >= max(tx0, 0)) & (xx // 16 < tx1) & (yy // 16 >= max(ty0, 0)) & (yy // 16 < ty1))
    alpha[~inside] = 0.0
    np.testing.assert_allclose(out["rgb"][0], 0.5 * alpha, atol=1e-12)
    np.testing.assert_allclose(out["depth"], z * alpha, atol=1e-12)
    np.testing.assert_allclose(out["T"], 1 - alpha, atol=1e-12)
    k = oracle.keys(sc, cam)
    assert k["valid"][0] and k["uvr"][0, 2] == r
    assert tuple(k["rect"][0]) == (max(tx0, 0), max(ty0, 0), min(tx1, k["TX"]), min(ty1, k["TY"]))


def _brute_force(scene, cam, use_rect=True, bg=(0, 0, 0, 0)):
    """Per pixel: every key-visible Gaussian (optionally only those whose rect
    covers the pixel's tile), sorted by (depth key, index), composited front to back."""
    k = oracle.keys(scene, cam)
    vals = oracle.project_values(scene, cam)
    H, W = cam.H, cam.W
    rgb = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    T_out = np.zeros((H, W))
    vis = [g for g in range(scene.n) if k["valid"][g]]
    vis.sort(key=lambda g: (int(k["depth_bits"][g]), g))
    for y in range(H):
        for x in range(W):
            tx, ty = x // 16, y // 16
            T, C, D = 1.0, np.zeros(3), 0.0
            for g in vis:
                x0, y0, x1, y1 = k["rect"][g]
                if use_rect and not (x0 <= tx < x1 and y0 <= ty < y1):
                    continue
                u, v, A, B, Cc = vals[g, :5]
                dx, dy = u - x, v - y
                power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
                a = min(A_MAX, float(scene.opac[g]) * math.exp(power))
                if a < A_MIN:
                    continue
                Tn = T * (1 - a)
                if Tn < T_MIN:
                    break
                C += vals[g, 9:12] * a * T
                D += vals[g, 8] * a * T
                T = Tn
            rgb[:, y, x] = C + T * np.asarray(bg[:3])
            depth[y, x] = D + T * bg[3]
            T_out[y, x] = T
    return rgb, depth, T_out


@pytest.mark.parametrize("seed,deg", [(11, 0), (12, 3)])
def test_tiled_equals_brute_force(seed, deg):
    sc = synth.tiny_scene(60, 50, 37, seed, sh_degree=deg, pose=True, log_scale_mu=-2.8)
    cam = sc.cams[0]
    bg = (0.1, 0.2, 0.3, 0.5)
    out = oracle.forward(sc, cam, bg=bg, bands=None)
    rgb, depth, T = _brute_force(sc, cam, bg=bg)
    np.testing.assert_allclose(out["rgb"], rgb, atol=1e-12)
    np.testing.assert_allclose(out["depth"], depth, atol=1e-12)
    np.testing.assert_allclose(out["T"], T, atol=1e-12)


def test_low_opacity_culling_drops_nothing():
    # With o <= 0.3 every pixel outside the 3-sigma box has alpha < 0.3 e^-4.5 < 1/255.
    sc = synth.tiny_scene(60, 50, 37, 13, opac_max=0.3, pose=True, log_scale_mu=-2.8)
    cam = sc.cams[0]
    out = oracle.forward(sc, cam, bands=None)
    rgb, depth, T = _brute_force(sc, cam, use_rect=False)
    np.testing.assert_allclose(out["rgb"], rgb, atol=1e-12)
    np.testing.assert_allclose(out["depth"], depth, atol=1e-12)


def test_projection_matches_independent_construction():
    sc = synth.tiny_scene(200, 120, 90, 14, pose=True, log_scale_mu=-3.0)
    cam = sc.cams[0]
    vals = oracle.project_values(sc, cam)
    k = oracle.keys(sc, cam)
    R = cam.Tcw[:, :3].astype(np.float64)
    t = cam.Tcw[:, 3].astype(np.float64)

    def pi(p):
        return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    checked = 0
    for g in np.nonzero(k["valid"])[0]:
        m = sc.means[g].astype(np.float64)
        q = sc.quats[g].astype(np.float64)
        Rg = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        SigW = Rg @ np.diag(sc.scales[g].astype(np.float64) ** 2) @ Rg.T
        p = R @ m + t
        lim = 1.3 * 0.5 * cam.W / cam.fx
        if abs(p[0] / p[2]) > lim or abs(p[1] / p[2]) > 1.3 * 0.5 * cam.H / cam.fy:
            continue
        h = 1e-6
        J = np.stack([(pi(p + h * e) - pi(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        S2 = J @ R @ SigW @ R.T @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(vals[g, 0:2], pi(p), rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(vals[g, 5:8], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-9)
        conic = np.linalg.inv(S2)
        np.testing.assert_allclose(vals[g, 2:5], [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=1e-6)
        assert abs(vals[g, 8] - p[2]) < 1e-12
        checked += 1
    assert checked > 50


def _real_sh_scipy(l, m, dirs):
    """Real SH as sqrt(2) Re / sqrt(2) Im of scipy's complex harmonics (which carry
    the Condon-Shortley phase), with no further (-1)^m factor."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * Y.real
    return math.sqrt(2) * Y.imag


def test_sh_basis_orthonormal_and_matches_scipy():
    # Gauss-Legendre in cos(theta) x uniform phi integrates products of degree <= 6 exactly.
    nt, nphi = 12, 24
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_basis(3, dirs)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[:, l * l + l + m], _real_sh_scipy(l, m, dirs), atol=1e-12,
                                       err_msg=f"l={l} m={m}")


def test_compositing_invariants():
    sc = synth.cfg1_plain_forward(n=2000)
    cam = sc.cams[0]
    out = oracle.forward(sc, cam, bands=None)
    assert np.all(out["T"] >= T_MIN) and np.all(out["T"] <= 1.0)
    assert np.all(out["rgb"] >= 0)
    k = oracle.keys(sc, cam)
    tl = np.diff(k["tile_off"])
    yy, xx = np.mgrid[0:cam.H, 0:cam.W]
    tile = (yy // 16) * k["TX"] + xx // 16
    assert np.all(out["n_contrib"] <= tl[tile])
    counts, gids, clamped = oracle.contributors(sc, cam)
    vals = oracle.project_values(sc, cam)
    off = np.concatenate([[0], np.cumsum(counts)])
    rng = np.random.default_rng(0)
    for pix in rng.choice(cam.W * cam.H, 300, replace=False):
        y, x = divmod(int(pix), cam.W)
        T = 1.0
        for i in range(off[pix], off[pix + 1]):
            g = gids[i]
            dx, dy = vals[g, 0] - x, vals[g, 1] - y
            power = -0.5 * (vals[g, 2] * dx * dx + vals[g, 4] * dy * dy) - vals[g, 3] * dx * dy
            a = min(A_MAX, float(sc.opac[g]) * math.exp(power))
            assert A_MIN <= a <= A_MAX
            assert bool(clamped[i]) == (float(sc.opac[g]) * math.exp(power) > A_MAX)
            Tn = T * (1 - a)
            assert Tn <= T
            T = Tn
        assert abs(T - out["T"][y, x]) < 1e-12


def test_uniform_colour_and_depth_closed_forms():
    rng = np.random.default_rng(3)
    sc = synth.tiny_scene(300, 64, 48, 15, log_scale_mu=-2.5)
    sc.sh[:, 0, :] = 0.7                       # every Gaussian the same colour
    sc.means[:, 2] = np.float32(2.25)          # every Gaussian at the same depth
    sc.opac[:] = rng.uniform(0.2, 0.99, sc.n).astype(np.float32)
    cam = sc.cams[0]
    out = oracle.forward(sc, cam, bands=None)
    col = oracle.project_values(sc, cam)[:, 9:12]
    c0 = col[oracle.keys(sc, cam)["valid"]][0]
    np.testing.assert_allclose(out["rgb"], c0[:, None, None] * (1 - out["T"])[None], atol=1e-12)
    np.testing.assert_allclose(out["depth"], 2.25 * (1 - out["T"]), atol=1e-12)


def test_key_path_agrees_with_value_path():
    sc = synth.tiny_scene(500, 160, 120, 16, pose=True)
    cam = sc.cams[0]
    k = oracle.keys(sc, cam)
    vals = oracle.project_values(sc, cam)
    v = k["valid"]
    assert v.sum() > 300
    np.testing.assert_allclose(k["uvr"][v, :2], vals[v, :2], rtol=0, atol=5e-4)
    depth32 = k["depth_bits"][v].view(np.float32).astype(np.float64)
    np.testing.assert_allclose(depth32, vals[v, 8], rtol=1e-6)
    a, b, c = vals[v, 5], vals[v, 6], vals[v, 7]
    det = a * c - b * b
    mid = 0.5 * (a + c)
    lam = mid + np.sqrt(np.maximum(0.1, mid * mid - det))
    r64 = np.ceil(3 * np.sqrt(lam))
    near_int = np.abs(3 * np.sqrt(lam) - np.round(3 * np.sqrt(lam))) < 1e-4
    assert np.all((k["uvr"][v, 2] == r64) | near_int)


def test_degenerate_inputs_are_culled():
    sc = synth.tiny_scene(8, 64, 48, 17)
    sc.quats[0] = 0.0                       # zero quaternion
    sc.means[1, 0] = np.nan                 # NaN mean
    sc.scales[2, 1] = 0.0                   # zero scale
    sc.opac[3] = 0.0                        # zero opacity
    sc.means[4, 2] = 0.1                    # in front of the near plane
    sc.means[5] = [100.0, 0.0, 2.0]         # far outside the image
    k = oracle.keys(sc, sc.cams[0])
    assert not k["valid"][:6].any()
    assert k["valid"][6:].all()


# ---- every outcome a fp32 renderer may take at a flagged pixel

def test_alternatives_skip_decision_on_a_single_gaussian():
    """One isotropic Gaussian whose alpha at a chosen pixel sits just above
    1/255: the oracle flags the pixel, and its two outcomes are 'skipped'
    (colour 0, T 1) and 'blended' (colour 0.5 alpha, T 1 - alpha), in closed form."""
    z, s, f = 2.0, 0.02, 100.0
    var = (f * float(np.float32(s)) / z) ** 2 + 0.3
    d = 3.0
    # opacity that puts alpha at pixel (cx + 3, cy) at 1/255 (1 + 2e-8): well inside the band
    o = float(np.float32(A_MIN * (1 + 2e-8) / math.exp(-0.5 * d * d / var)))
    sc = _single(z=z, s=s, o=o)
    cam = sc.cams[0]
    out = oracle.forward(sc, cam)
    x, y = int(cam.cx + d), int(cam.cy)
    assert out["amb"][y, x]
    alpha = o * math.exp(-0.5 * d * d / var)
    leaves, gid, n = oracle.forward_alternatives(sc, cam, [x], [y])
    assert n[0] == 2
    order = np.argsort(gid[0, :2])  # skipped (gid -1) first
    assert list(gid[0, order]) == [-1, 0]
    np.testing.assert_array_equal(leaves[0, order[0]], [0.0, 0.0, 0.0, 0.0, 1.0])
    # the closed form here rounds s and the dilation differently from the fp32 inputs: 1e-6 relative
    np.testing.assert_allclose(leaves[0, order[1]], [0.5 * alpha] * 3 + [z * alpha, 1 - alpha], rtol=1e-6)
    # an unflagged pixel has exactly its forward value as its only outcome
    x2, y2 = int(cam.cx), int(cam.cy)
    assert not out["amb"][y2, x2]
    leaves, gid, n = oracle.forward_alternatives(sc, cam, [x2], [y2])
    assert n[0] == 1 and gid[0, 0] == 0
    np.testing.assert_array_equal(leaves[0, 0, :3], out["rgb"][:, y2, x2])
    assert leaves[0, 0, 3] == out["depth"][y2, x2] and leaves[0, 0, 4] == out["T"][y2, x2]


def test_alternatives_stop_decision_after_two_clamped_gaussians():
    """Two opaque Gaussians on the axis (alpha clamped at 0.99 at the centre):
    after both, T' = (1 - 0.99f)^2 lies within the band of 1e-4, so the second
    may stop the walk (not blended) or be blended.  Outcomes in closed form."""
    means = np.array([[0.0, 0.0, 2.0], [0.0, 0.0, 2.5]], np.float32)
    scales = np.full((2, 3), 0.05, np.float32)
    quats = np.tile(np.array([1.0, 0, 0, 0], np.float32), (2, 1))
    opac = np.array([1.0, 1.0], np.float32)
    sh = np.zeros((2, 1, 3), np.float32)
    sh[1, 0, :] = 0.5 / 0.28209479177387814  # second Gaussian's colour 1.0
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    sc = Scene(means, scales, quats, opac, sh, 0, [Camera(64, 48, 100.0, 100.0, 31.0, 22.0, Tcw)])
    cam = sc.cams[0]
    out = oracle.forward(sc, cam)
    x, y = 31, 22
    assert out["amb"][y, x]
    leaves, gid, n = oracle.forward_alternatives(sc, cam, [x], [y])
    assert n[0] == 2
    a = A_MAX
    stop = (0.5 * a, 0.5 * a, 0.5 * a, 2.0 * a, 1 - a)
    cont = tuple([0.5 * a + 1.0 * a * (1 - a)] * 3 + [2.0 * a + 2.5 * a * (1 - a), (1 - a) ** 2])
    order = np.argsort(gid[0, :2])
    assert list(gid[0, order]) == [0, 1]
    # colour 1.0 is 0.5 + C0 * fp32((1.0 - 0.5) / C0): 1e-7 relative
    np.testing.assert_allclose(leaves[0, order[0]], stop, rtol=1e-7)
    np.testing.assert_allclose(leaves[0, order[1]], cont, rtol=1e-7)


def test_alternatives_include_the_forward_and_cover_random_scenes():
    """On a random scene, every flagged pixel's first outcome is the forward's
    own walk (no decision reversed), bit for bit, and each pixel has at least
    two outcomes; unflagged pixels have one."""
    sc = synth.tiny_scene(400, 70, 45, seed=11, sh_degree=1, pose=True, log_scale_mu=-2.8)
    cam = sc.cams[0]
    out = oracle.forward(sc, cam)
    yy, xx = np.nonzero(np.ones((cam.H, cam.W), bool))
    leaves, gid, n = oracle.forward_alternatives(sc, cam, xx, yy)
    amb = out["amb"][yy, xx]
    assert amb.sum() > 0 and np.all(n > 0)
    assert np.all(n[~amb] == 1) and np.all(n[amb] >= 2)
    np.testing.assert_array_equal(leaves[:, 0, 0], out["rgb"][0][yy, xx])
    np.testing.assert_array_equal(leaves[:, 0, 3], out["depth"][yy, xx])
    np.testing.assert_array_equal(leaves[:, 0, 4], out["T"][yy, xx])
