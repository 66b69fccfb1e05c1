"""Scene recipes.

Every generator takes an explicit seed and draws from numpy's PCG64, in float64,
casting to float32 at the end.  Conventions of the arrays produced:

* means  [N,3]  world positions (metres)
* scales [N,3]  linear standard deviations along the Gaussian's own axes (> 0)
* quats  [N,4]  rotation as (w, x, y, z); not necessarily unit length
* opac   [N]    opacity in (0, 1)
* sh     [N,K,3] colour coefficients, K = (degree+1)^2, coefficient-major
* Camera.Tcw [3,4] row-major world->camera [R | t]; camera looks along +z, x right, y down.

None of the renderer's or the merge's arithmetic lives here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np
from scipy.spatial.transform import Rotation

# Degree-0 coefficient range: the DC term times the order-0 basis constant plus
# 0.5 spans colours in [0, 1] when the coefficient spans [-sqrt(pi), sqrt(pi)].
SH_DC_RANGE = math.sqrt(math.pi)


@dataclass
class Camera:
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    Tcw: np.ndarray  # float32 [3,4]
    near: float = 0.2

    def as_array32(self) -> np.ndarray:
        """[W, H, fx, fy, cx, cy, near, R00..R22, t0..t2] as float32 (19 entries)."""
        return np.concatenate([
            np.array([self.W, self.H, self.fx, self.fy, self.cx, self.cy, self.near], np.float32),
            self.Tcw[:, :3].reshape(-1).astype(np.float32),
            self.Tcw[:, 3].astype(np.float32),
        ])


@dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opac: np.ndarray
    sh: np.ndarray
    sh_degree: int
    cams: List[Camera] = field(default_factory=list)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.scales[idx].copy(), self.quats[idx].copy(),
                     self.opac[idx].copy(), self.sh[idx].copy(), self.sh_degree, list(self.cams),
                     self.name + "[subset]")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _attributes(rng, n, sh_degree, log_scale_mu=-3.5, log_scale_sigma=0.5, rest_sigma=0.2):
    scales = np.exp(rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3)))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = rng.uniform(0.05, 0.95, size=n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.uniform(-SH_DC_RANGE, SH_DC_RANGE, size=(n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_sigma, size=(n, K - 1, 3))
    return scales, q, opac, sh


def _pack(means, scales, quats, opac, sh, deg, cams, name):
    f = np.float32
    return Scene(np.ascontiguousarray(means, f), np.ascontiguousarray(scales, f),
                 np.ascontiguousarray(quats, f), np.ascontiguousarray(opac, f),
                 np.ascontiguousarray(sh, f), deg, cams, name)


def look_at(position, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera [R|t] (float64) for a camera at `position` looking at `target`."""
    position = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - position
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R_wc = np.stack([right, down, fwd], axis=1)
    R_cw = R_wc.T
    t_cw = -R_cw @ position
    return np.concatenate([R_cw, t_cw[:, None]], axis=1)


# ---------------------------------------------------------------- cfg1
def cfg1_plain_forward(seed: int = 1, n: int = 10_000) -> Scene:
    """10k Gaussians in a 2x2x2 m box 1-3 m in front of an identity-pose 320x240 camera."""
    rng = _rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(1, 3, n)], axis=1)
    scales, q, opac, sh = _attributes(rng, n, 0)
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    cam = Camera(320, 240, 300.0, 300.0, 160.0, 120.0, Tcw)
    return _pack(means, scales, q, opac, sh, 0, [cam], "cfg1")


# ---------------------------------------------------------------- cfg2
def _depth_surface(rng, W, H):
    z0 = rng.uniform(1.5, 2.5)
    g = rng.uniform(-1.5e-3, 1.5e-3, size=2)
    amp = rng.uniform(0.05, 0.3, size=3)
    ang = rng.uniform(0, 2 * math.pi, size=3)
    mag = rng.uniform(1 / 400, 1 / 80, size=3)
    freq = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=1)
    phase = rng.uniform(0, 2 * math.pi, size=3)

    def z(u, v):
        out = z0 + g[0] * u + g[1] * v
        for k in range(3):
            out = out + amp[k] * np.sin(2 * math.pi * (freq[k, 0] * u + freq[k, 1] * v) + phase[k])
        return np.clip(out, 0.5, 4.0)
    return z


def cfg2_keyframe(seed: int = 2, n: int = 200_000):
    """One 640x480 keyframe over a bumpy depth surface; returns (scene, target_rgb, target_depth)."""
    rng = _rng(seed)
    W, H, f, cx, cy = 640, 480, 525.0, 320.0, 240.0
    zf = _depth_surface(rng, W, H)
    u = rng.uniform(0, W, n)
    v = rng.uniform(0, H, n)
    z = zf(u, v)
    pc = np.stack([(u - cx) * z / f, (v - cy) * z / f, z], axis=1)
    pc += rng.uniform(-0.02, 0.02, size=(n, 3))
    R_wc = Rotation.random(random_state=rng).as_matrix()
    t_wc = rng.uniform(-1, 1, size=3)
    means = pc @ R_wc.T + t_wc
    R_cw = R_wc.T
    Tcw = np.concatenate([R_cw, (-R_cw @ t_wc)[:, None]], axis=1).astype(np.float32)
    scales, q, opac, sh = _attributes(rng, n, 0)
    cam = Camera(W, H, f, f, cx, cy, Tcw)
    scene = _pack(means, scales, q, opac, sh, 0, [cam], "cfg2")
    uu, vv = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    target_rgb = rng.uniform(0, 1, size=(3, H, W)).astype(np.float32)
    target_depth = (zf(uu, vv) + rng.normal(0, 0.01, size=(H, W))).astype(np.float32)
    return scene, target_rgb, target_depth


# ---------------------------------------------------------------- room (cfg3/4/5)
ROOM = (8.0, 6.0, 3.0)


def _room_faces(rng, n_boxes=50):
    """Planar rectangles (origin, edge1, edge2) of the 6 walls and 50 floor boxes."""
    X, Y, Z = ROOM
    faces = [
        ((0, 0, 0), (X, 0, 0), (0, Y, 0)),      # floor
        ((0, 0, Z), (X, 0, 0), (0, Y, 0)),      # ceiling
        ((0, 0, 0), (0, Y, 0), (0, 0, Z)),      # x = 0
        ((X, 0, 0), (0, Y, 0), (0, 0, Z)),      # x = X
        ((0, 0, 0), (X, 0, 0), (0, 0, Z)),      # y = 0
        ((0, Y, 0), (X, 0, 0), (0, 0, Z)),      # y = Y
    ]
    faces = [tuple(np.asarray(a, np.float64) for a in f) for f in faces]
    for _ in range(n_boxes):
        sx, sy, sz = rng.uniform(0.2, 1.0, size=3)
        c = np.array([rng.uniform(0.6, X - 0.6), rng.uniform(0.6, Y - 0.6), 0.0])
        yaw = rng.uniform(0, 2 * math.pi)
        ex = np.array([math.cos(yaw), math.sin(yaw), 0.0])
        ey = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
        ez = np.array([0.0, 0.0, 1.0])
        o = c - 0.5 * sx * ex - 0.5 * sy * ey
        faces.append((o + sz * ez, sx * ex, sy * ey))   # top
        faces.append((o, sx * ex, sz * ez))             # side faces
        faces.append((o + sy * ey, sx * ex, sz * ez))
        faces.append((o, sy * ey, sz * ez))
        faces.append((o + sx * ex, sy * ey, sz * ez))
    return faces


def room_gaussians(n_orig: int, n_dup: int, seed: int, sh_degree: int = 0, n_boxes: int = 50):
    """Room surfaces sampled area-uniformly, plus near-duplicates appended last.

    Near-duplicates copy a random original with position jittered by U(+-5 mm)
    per axis and scales by a factor U(1 +- 5%) per axis; everything else copied.
    """
    rng = _rng(seed)
    faces = _room_faces(rng, n_boxes)
    area = np.array([np.linalg.norm(np.cross(e1, e2)) for _, e1, e2 in faces])
    counts = rng.multinomial(n_orig, area / area.sum())
    pts = []
    for (o, e1, e2), c in zip(faces, counts):
        if c == 0:
            continue
        a = rng.uniform(0, 1, size=(c, 1))
        b = rng.uniform(0, 1, size=(c, 1))
        pts.append(o + a * e1 + b * e2)
    means = np.concatenate(pts, axis=0)
    means = means[rng.permutation(n_orig)]
    scales, q, opac, sh = _attributes(rng, n_orig, sh_degree)
    if n_dup > 0:
        src = rng.integers(0, n_orig, size=n_dup)
        means = np.concatenate([means, means[src] + rng.uniform(-0.005, 0.005, size=(n_dup, 3))])
        scales = np.concatenate([scales, scales[src] * (1 + rng.uniform(-0.05, 0.05, size=(n_dup, 3)))])
        q = np.concatenate([q, q[src]])
        opac = np.concatenate([opac, opac[src]])
        sh = np.concatenate([sh, sh[src]])
    return means, scales, q, opac, sh


def _intrinsics(W, H, f):
    return dict(W=W, H=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0)


def trajectory_cams(seed: int, n_views: int, W: int, H: int, f: float) -> List[Camera]:
    """Keyframes on an ellipse (semi-axes 2.5 x 1.5 m, height 1.5 +- 0.2 m) looking roughly along the path."""
    rng = _rng(seed + 1000)
    th0 = rng.uniform(0, 2 * math.pi)
    cams = []
    for k in range(n_views):
        th = th0 + 0.3 * k
        pos = np.array([4.0 + 2.5 * math.cos(th), 3.0 + 1.5 * math.sin(th), 1.5 + 0.2 * math.sin(2 * th)])
        tang = np.array([-2.5 * math.sin(th), 1.5 * math.cos(th)])
        psi = math.atan2(tang[1], tang[0]) + rng.uniform(-0.3, 0.3)
        target = pos + np.array([math.cos(psi), math.sin(psi), -0.15])
        Tcw = look_at(pos, target).astype(np.float32)
        cams.append(Camera(Tcw=Tcw, **_intrinsics(W, H, f)))
    return cams


def random_pose_in_room(rng: np.random.Generator) -> np.ndarray:
    pos = np.array([rng.uniform(1, 7), rng.uniform(1, 5), rng.uniform(1.0, 2.0)])
    yaw = rng.uniform(0, 2 * math.pi)
    pitch = rng.uniform(-0.3, 0.3)
    target = pos + np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    return look_at(pos, target).astype(np.float32)


def cfg3_room_window(seed: int = 3, n: int = 500_000, dup_fraction: float = 0.3, n_views: int = 8,
                     W: int = 1200, H: int = 680, f: float = 600.0) -> Scene:
    n_dup = int(round(n * dup_fraction))
    means, scales, q, opac, sh = room_gaussians(n - n_dup, n_dup, seed, 0)
    cams = trajectory_cams(seed, n_views, W, H, f)
    return _pack(means, scales, q, opac, sh, 0, cams, "cfg3")


SERVE_RESOLUTIONS = ((320, 240, 300.0), (640, 480, 525.0), (1200, 680, 600.0))


def cfg4_serving_maps(sizes=(50_000, 300_000, 1_000_000, 2_000_000), seeds=(41, 42, 43, 44)) -> List[Scene]:
    maps = []
    for n, s in zip(sizes, seeds):
        means, scales, q, opac, sh = room_gaussians(n, 0, s, 0)
        maps.append(_pack(means, scales, q, opac, sh, 0, [], f"cfg4-map{n}"))
    return maps


def serving_camera(rng: np.random.Generator) -> Camera:
    W, H, f = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
    return Camera(Tcw=random_pose_in_room(rng), **_intrinsics(W, H, f))


def cfg5_large_sh3(seed: int = 5, n: int = 3_000_000, W: int = 1200, H: int = 680, f: float = 600.0) -> Scene:
    means, scales, q, opac, sh = room_gaussians(n, 0, seed, 3)
    cams = trajectory_cams(seed, 1, W, H, f)
    return _pack(means, scales, q, opac, sh, 3, cams, "cfg5")


def gradcheck_crop(seed: int = 55, n: int = 1000, sh_degree: int = 3) -> Scene:
    """1k Gaussians in front of a 32x32 camera (f=600, c=(16,16)), for gradient checks."""
    rng = _rng(seed)
    z = rng.uniform(2.0, 4.0, n)
    x = rng.uniform(-22, 22, n) * z / 600.0
    y = rng.uniform(-22, 22, n) * z / 600.0
    means = np.stack([x, y, z], axis=1)
    scales, q, opac, sh = _attributes(rng, n, sh_degree, log_scale_mu=-5.0, log_scale_sigma=0.4)
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    cam = Camera(32, 32, 600.0, 600.0, 16.0, 16.0, Tcw)
    return _pack(means, scales, q, opac, sh, sh_degree, [cam], "gradcheck")


def tiny_scene(n: int, W: int, H: int, seed: int, sh_degree: int = 0, f: float = None,
               opac_max: float = 0.95, log_scale_mu: float = -3.0, pose: bool = False) -> Scene:
    """Small scene for brute-force and finite-difference checks: Gaussians 1.5-3 m ahead."""
    rng = _rng(seed)
    f = f if f is not None else 0.9 * W
    z = rng.uniform(1.5, 3.0, n)
    x = rng.uniform(-0.6, 0.6, n) * z * (W / 2) / f
    y = rng.uniform(-0.6, 0.6, n) * z * (H / 2) / f
    means_c = np.stack([x, y, z], axis=1)
    scales, q, opac, sh = _attributes(rng, n, sh_degree, log_scale_mu=log_scale_mu)
    opac = opac * (opac_max / 0.95)
    if pose:
        R_wc = Rotation.random(random_state=rng).as_matrix()
        t_wc = rng.uniform(-1, 1, 3)
        means = means_c @ R_wc.T + t_wc
        R_cw = R_wc.T
        Tcw = np.concatenate([R_cw, (-R_cw @ t_wc)[:, None]], axis=1).astype(np.float32)
    else:
        means = means_c
        Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    cam = Camera(W, H, f, f, (W - 1) / 2.0 + 0.25, (H - 1) / 2.0 - 0.25, Tcw)
    return _pack(means, scales, q, opac, sh, sh_degree, [cam], f"tiny{n}")


def upstream_grads(cams: List[Camera], seed: int, depth: bool = True):
    """Seeded N(0,1) upstream gradients, one [3,H,W] colour and one [H,W] depth array per view."""
    rng = _rng(seed + 7000)
    g_rgb = [rng.normal(size=(3, c.H, c.W)).astype(np.float32) for c in cams]
    g_d = [rng.normal(size=(c.H, c.W)).astype(np.float32) if depth else None for c in cams]
    return g_rgb, g_d


# ---------------------------------------------------------------- Patch-Grid keyframes
@dataclass
class KeyframeFeatures:
    cam: Camera
    keypoints: np.ndarray   # [n,2] float32 pixel coordinates
    kp_depth: np.ndarray    # [n] float32, 0 where the keypoint has no depth
    image: np.ndarray       # [3,H,W] float32 in [0, 1]
    depth_map: np.ndarray   # [H,W] float32, 0 where invalid


def keyframe_features(seed: int, W: int = 1200, H: int = 680, f: float = 600.0, n_kp: int = 2000,
                      active: float = 0.3, clusters: int = 12, holes: float = 0.05) -> KeyframeFeatures:
    """A keyframe for Patch-Grid sampling: keypoints concentrated in textured
    areas (a mixture of `clusters` blobs, 20-60 px wide, plus 10 % spread
    uniformly), a fraction `active` of them with a depth (the depth surface at
    the keypoint plus 1 cm noise), the bumpy depth surface of the keyframe
    recipe as the depth map with a fraction `holes` of invalid pixels, a random
    colour image and a random pose."""
    rng = _rng(seed)
    zf = _depth_surface(rng, W, H)
    n_uni = n_kp // 10
    centres = rng.uniform([0, 0], [W, H], size=(clusters, 2))
    width = rng.uniform(20, 60, size=clusters)
    which = rng.integers(0, clusters, size=n_kp - n_uni)
    blob = centres[which] + rng.normal(size=(n_kp - n_uni, 2)) * width[which, None]
    kp = np.concatenate([blob, rng.uniform([0, 0], [W, H], size=(n_uni, 2))])
    kp = kp[rng.permutation(n_kp)]
    has = rng.uniform(size=n_kp) < active
    kd = np.where(has, zf(kp[:, 0], kp[:, 1]) + rng.normal(0, 0.01, size=n_kp), 0.0)
    uu, vv = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    dm = zf(uu, vv)
    dm[rng.uniform(size=(H, W)) < holes] = 0.0
    image = rng.uniform(0, 1, size=(3, H, W))
    R_wc = Rotation.random(random_state=rng).as_matrix()
    t_wc = rng.uniform(-1, 1, size=3)
    R_cw = R_wc.T
    Tcw = np.concatenate([R_cw, (-R_cw @ t_wc)[:, None]], axis=1).astype(np.float32)
    cam = Camera(W, H, f, f, W / 2.0, H / 2.0, Tcw)
    return KeyframeFeatures(cam, kp.astype(np.float32), kd.astype(np.float32), image.astype(np.float32),
                            dm.astype(np.float32))
