"""Patch-Grid (PG) sampling of Sec. II-B, numpy.  TEST INFRASTRUCTURE ONLY:
imported by tests, the smoke check and the benchmark's CPU-baseline leg, never
by the product path.

The image is divided into square patches.  A patch that holds fewer keypoints
than a threshold is sampled uniformly.  Every keypoint and every sample then
becomes the centre of a new 3D Gaussian.  A point without a measured depth
takes the depth of its nearest keypoint that has one (the monocular case).

Steps, as the paper states them, with the readings this build takes where it is
silent (listed in the design notes):
  1. a keypoint (u, v) (pixel centres at integer coordinates) lies on pixel
     (floor(u + 1/2), floor(v + 1/2)); keypoints off the image are ignored;
     pixel (x, y) lies in patch (x // P, y // P);
  2. count the keypoints of each patch; a patch with fewer than `min_kp` is
     sampled with an s x s lattice over the patch's part of the image (w x h
     pixels, w = min(P, W - P px), h = min(P, H - P py)): sample (k, l) sits on
     pixel (P px + ((2k + 1) w) // (2 s), P py + ((2l + 1) h) // (2 s));
  3. depth: a keypoint's own depth when it has one (> 0); otherwise the depth
     map at the point's pixel when a map is given and valid (> 0); otherwise
     the depth of the nearest keypoint (squared pixel distance in fp32, ties to
     the lower index) with its own depth; a point with none of these is dropped;
  4. back-projection with the pinhole camera and the pose T_CW:
     p_c = z ((x - cx) / fx, (y - cy) / fy, 1), mu = R_CW^T (p_c - t_CW), with
     (x, y) the keypoint's own coordinates or the sample's pixel;
  5. attributes: colour from the image at the point's pixel (SH degree 0,
     DC = (rgb - 1/2) / C0), opacity `opacity`, identity rotation, isotropic
     scale `scale_factor * z * (P / s) / fx`.
Output order: the kept keypoints in input order, then the kept samples by patch
(row-major) and lattice position (row-major).

The integer decisions (pixel, patch, nearest keypoint) are taken in fp32 as
written above; the values are fp64.
"""
from __future__ import annotations

import numpy as np

SH_C0 = 0.28209479177387814


def keypoint_pixels(kp, W, H):
    """Pixel of each keypoint (fp32 floor(u + 1/2)) and whether it is on the image."""
    k32 = np.asarray(kp, np.float32).reshape(-1, 2)
    with np.errstate(invalid="ignore"):
        px = np.floor(k32 + np.float32(0.5))
    on = np.all(np.isfinite(px), axis=1)
    on &= (px[:, 0] >= 0) & (px[:, 0] < W) & (px[:, 1] >= 0) & (px[:, 1] < H)
    return np.where(on[:, None], px, 0).astype(np.int64), on


def patch_counts(kp, W, H, P):
    px, on = keypoint_pixels(kp, W, H)
    PX, PY = -(-W // P), -(-H // P)
    counts = np.zeros(PX * PY, np.int64)
    for i in np.nonzero(on)[0]:
        counts[(px[i, 1] // P) * PX + px[i, 0] // P] += 1
    return counts


def sample_pixels(W, H, P, s, counts, min_kp, with_slot=False):
    """Pixels of the samples of every patch with fewer than min_kp keypoints (and,
    with_slot, each sample's lattice slot patch * s^2 + l * s + k)."""
    PX, PY = -(-W // P), -(-H // P)
    out, slot = [], []
    for py in range(PY):
        for pxi in range(PX):
            if counts[py * PX + pxi] >= min_kp:
                continue
            w, h = min(P, W - P * pxi), min(P, H - P * py)
            for l in range(s):
                for k in range(s):
                    out.append((P * pxi + ((2 * k + 1) * w) // (2 * s), P * py + ((2 * l + 1) * h) // (2 * s)))
                    slot.append((py * PX + pxi) * s * s + l * s + k)
    px = np.asarray(out, np.int64).reshape(-1, 2)
    return (px, np.asarray(slot, np.int64)) if with_slot else px


def nearest_with_depth(q, kp, kp_depth):
    """Index of the nearest keypoint with its own depth (> 0) to each query point
    (fp32 squared distance dx*dx + dy*dy, ties to the lower index), -1 if none."""
    k32 = np.asarray(kp, np.float32).reshape(-1, 2)
    has = np.asarray(kp_depth, np.float32) > 0
    q32 = np.asarray(q, np.float32).reshape(-1, 2)
    best = np.full(len(q32), -1, np.int64)
    idx = np.nonzero(has)[0]
    if len(idx) == 0:
        return best
    for n, (x, y) in enumerate(q32):
        dx = np.float32(x) - k32[idx, 0]
        dy = np.float32(y) - k32[idx, 1]
        d2 = dx * dx + dy * dy  # float32 elementwise, no contraction
        best[n] = idx[int(np.argmin(d2))]  # argmin returns the first of equal minima
    return best


def patch_grid_sample(cam, kp, kp_depth, image, depth_map=None, P=32, min_kp=4, s=2, opacity=0.5,
                      scale_factor=0.5):
    """New Gaussians (means, scales, quats, opac, sh [n,1,3]) from keypoints and
    Patch-Grid samples, and the source of each: i < n_kp keypoint i, else
    n_kp + its lattice slot (patch * s^2 + l * s + k)."""
    W, H = int(cam.W), int(cam.H)
    kp = np.asarray(kp, np.float32).reshape(-1, 2)
    kpd = np.asarray(kp_depth, np.float32).reshape(-1)
    px, on = keypoint_pixels(kp, W, H)
    counts = patch_counts(kp, W, H, P)
    spx, slot = sample_pixels(W, H, P, s, counts, min_kp, with_slot=True)
    # candidates: keypoints on the image, then samples
    pts = np.concatenate([kp.astype(np.float64), spx.astype(np.float64)])
    pix = np.concatenate([px, spx])
    keep = np.concatenate([on, np.ones(len(spx), bool)])
    own = np.concatenate([np.where(kpd > 0, kpd, 0.0), np.zeros(len(spx))]).astype(np.float64)
    z = own.copy()
    need = keep & (z <= 0)
    if depth_map is not None:
        dm = np.asarray(depth_map, np.float32)
        vals = dm[pix[:, 1].clip(0, H - 1), pix[:, 0].clip(0, W - 1)].astype(np.float64)
        use = need & (vals > 0)
        z[use] = vals[use]
        need &= ~use
    nn = nearest_with_depth(pts[need], kp, kpd)
    zi = np.zeros(need.sum())
    zi[nn >= 0] = kpd[nn[nn >= 0]]
    z[np.nonzero(need)[0]] = zi
    keep &= z > 0
    sel = np.nonzero(keep)[0]
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    T = np.asarray(cam.Tcw, np.float64).reshape(3, 4)
    R, t = T[:, :3], T[:, 3]
    pc = np.stack([z * (pts[:, 0] - cx) / fx, z * (pts[:, 1] - cy) / fy, z], axis=1)
    mu = (pc - t) @ R  # R^T (p_c - t) for each row
    img = np.asarray(image, np.float64)
    rgb = img[:, pix[:, 1].clip(0, H - 1), pix[:, 0].clip(0, W - 1)].T
    sig = scale_factor * z * (P / s) / fx
    n = len(sel)
    out = dict(means=mu[sel], scales=np.repeat(sig[sel, None], 3, axis=1),
               quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), opac=np.full(n, float(opacity)),
               sh=((rgb[sel] - 0.5) / SH_C0)[:, None, :],
               source=np.where(sel < len(kp), sel, len(kp) + slot[np.maximum(sel - len(kp), 0)] if len(slot) else sel),
               point=sel, depth=z[sel], counts=counts, sample_pixels=spx)
    return out
