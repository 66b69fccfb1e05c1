"""CPU oracle for the MemGS hot path.  TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package.  It shares no code with the HIP path
(`paper_2509_13536_amd`), and neither imports the other.

* `render_oracle.c` (built to `liboracle.so` by `build.py`): the rasterizer
  forward/backward of Sec. II-C and Eq. (11), fp32 key path + fp64 value path.
* `merge.py`: the voxel merge of Sec. II-D (Eqs. (3)-(10)) in numpy fp64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_keys.restype = i64
        L.orc_keys.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_project_values.restype = None
        L.orc_project_values.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P]
        L.orc_forward.restype = i64
        L.orc_forward.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P, P, P]
        L.orc_forward_alternatives.restype = None
        L.orc_forward_alternatives.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P, P, i64, P, P, C.c_int, P, P,
                                               P]
        L.orc_contributors.restype = i64
        L.orc_contributors.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P, P, P]
        L.orc_forward_frozen.restype = None
        L.orc_forward_frozen.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P]
        L.orc_backward.restype = None
        L.orc_backward.argtypes = [i64, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_sh_basis.restype = None
        L.orc_sh_basis.argtypes = [C.c_int, i64, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def cam_arrays(cam):
    """(float32[19], float64[19]) camera blocks for a synth.Camera."""
    c32 = cam.as_array32()
    return c32, c32.astype(np.float64)


def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    """[n,16] basis values (entries beyond (deg+1)^2 are unspecified)."""
    d = _f64(dirs)
    out = np.zeros((d.shape[0], 16))
    lib().orc_sh_basis(deg, d.shape[0], _p(d), _p(out))
    return out[:, :(deg + 1) ** 2]


def num_threads() -> int:
    return int(lib().orc_num_threads())


def keys(scene, cam):
    """Key path of one view: dict(valid, depth_bits, rect, uvr, tile_off, tile_gid, M)."""
    n = scene.n
    c32, _ = cam_arrays(cam)
    m, s, q, o = (_f32(scene.means), _f32(scene.scales), _f32(scene.quats), _f32(scene.opac))
    TX, TY = (cam.W + 15) // 16, (cam.H + 15) // 16
    valid = np.zeros(n, np.uint8)
    depth_bits = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    uvr = np.zeros((n, 3), np.float32)
    tile_off = np.zeros(TX * TY + 1, np.int64)
    M = lib().orc_keys(n, _p(m), _p(s), _p(q), _p(o), _p(c32), _p(valid), _p(depth_bits), _p(rect),
                       _p(uvr), _p(tile_off), None)
    tile_gid = np.zeros(max(M, 1), np.int32)
    lib().orc_keys(n, _p(m), _p(s), _p(q), _p(o), _p(c32), None, None, None, None, None, _p(tile_gid))
    return dict(valid=valid.astype(bool), depth_bits=depth_bits, rect=rect, uvr=uvr,
                tile_off=tile_off, tile_gid=tile_gid[:M], M=int(M), TX=TX, TY=TY)


def project_values(scene, cam):
    """fp64 value-path projection: [n,12] = uv(2), conic(3), dilated cov(3), depth, rgb(3)."""
    c32, c64 = cam_arrays(cam)
    out = np.zeros((scene.n, 12), np.float64)
    lib().orc_project_values(scene.n, _p(_f32(scene.means)), _p(_f32(scene.scales)), _p(_f32(scene.quats)),
                             _p(_f32(scene.opac)), _p(_f32(scene.sh)), scene.sh_degree, _p(c32), _p(c64),
                             _p(out))
    return out


# Ambiguity bands (see the bands struct in render_oracle.c): relative rounding
# of a fp32 conic; absolute error (natural log) of a fp32 evaluation of alpha
# beyond the quadratic form: the exponential (about one ulp) and a fp32 log2 of
# the opacity added to the exponent (a ulp of |log2 o| <= 8, one more rounding
# of the sum), 1.5e-6 in all.
DEFAULT_BANDS = (2e-6, 1.5e-6)


def forward(scene, cam, bg=(0, 0, 0, 0), bands=DEFAULT_BANDS):
    """Forward render of one view.  Returns dict(rgb[3,H,W], depth, T, n_contrib, amb, M)."""
    c32, c64 = cam_arrays(cam)
    H, W = cam.H, cam.W
    rgb = np.zeros((3, H, W), np.float64)
    depth = np.zeros((H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    nc = np.zeros((H, W), np.int32)
    amb = np.zeros((H, W), np.uint8)
    bgv = _f64(bg)
    bd = None if bands is None else _f64(bands)
    M = lib().orc_forward(scene.n, _p(_f32(scene.means)), _p(_f32(scene.scales)), _p(_f32(scene.quats)),
                          _p(_f32(scene.opac)), _p(_f32(scene.sh)), scene.sh_degree, _p(c32), _p(c64),
                          _p(bgv), _p(rgb), _p(depth), _p(T), _p(nc), _p(amb), _p(bd))
    return dict(rgb=rgb, depth=depth, T=T, n_contrib=nc, amb=amb.astype(bool), M=int(M))


def forward_alternatives(scene, cam, xs, ys, bg=(0, 0, 0, 0), bands=DEFAULT_BANDS, max_leaves=32):
    """Every outcome of the pixels (xs[k], ys[k]) that the ambiguity bands allow
    (see orc_forward_alternatives).  Returns (leaves [P, L, 5] = rgb, depth, T;
    last_gid [P, L]; n_leaves [P], -1 where a pixel has more than max_leaves)."""
    c32, c64 = cam_arrays(cam)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    P = xs.shape[0]
    leaves = np.zeros((P, max_leaves, 5), np.float64)
    gid = np.full((P, max_leaves), -1, np.int32)
    n_leaves = np.zeros(P, np.int32)
    lib().orc_forward_alternatives(scene.n, _p(_f32(scene.means)), _p(_f32(scene.scales)), _p(_f32(scene.quats)),
                                   _p(_f32(scene.opac)), _p(_f32(scene.sh)), scene.sh_degree, _p(c32), _p(c64),
                                   _p(_f64(bg)), _p(_f64(bands)), P, _p(xs), _p(ys), int(max_leaves),
                                   _p(leaves), _p(gid), _p(n_leaves))
    return leaves, gid, n_leaves


def contributors(scene, cam):
    c32, c64 = cam_arrays(cam)
    args = [_p(_f32(scene.means)), _p(_f32(scene.scales)), _p(_f32(scene.quats)), _p(_f32(scene.opac)),
            _p(_f32(scene.sh)), scene.sh_degree, _p(c32), _p(c64)]
    counts = np.zeros(cam.H * cam.W, np.int64)
    total = lib().orc_contributors(scene.n, *args, _p(counts), None, None)
    gids = np.zeros(max(total, 1), np.int32)
    clamped = np.zeros(max(total, 1), np.uint8)
    lib().orc_contributors(scene.n, *args, _p(counts), _p(gids), _p(clamped))
    return counts, gids[:total], clamped[:total]


def forward_frozen(params, sh_degree, cam64, frozen, bg=(0, 0, 0, 0)):
    """Frozen-decision forward on float64 params (means, scales, quats, opac, sh) and camera block."""
    means, scales, quats, opac, sh = (_f64(a) for a in params)
    counts, gids, clamped = frozen
    W, H = int(cam64[0]), int(cam64[1])
    rgb = np.zeros((3, H, W), np.float64)
    depth = np.zeros((H, W), np.float64)
    lib().orc_forward_frozen(means.shape[0], _p(means), _p(scales), _p(quats), _p(opac), _p(sh), sh_degree,
                             _p(_f64(cam64)), _p(_f64(bg)), _p(counts), _p(gids), _p(clamped), _p(rgb),
                             _p(depth))
    return rgb, depth


def backward(scene, cam, dL_rgb, dL_depth=None, bg=(0, 0, 0, 0), want_grad2d=False):
    """Backward of one view in fp64.  Returns dict of gradients (float64)."""
    c32, c64 = cam_arrays(cam)
    n, K = scene.n, (scene.sh_degree + 1) ** 2
    out = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opac=np.zeros(n), sh=np.zeros((n, K, 3)), pose=np.zeros(6))
    g2 = np.zeros((n, 10)) if want_grad2d else None
    lib().orc_backward(n, _p(_f32(scene.means)), _p(_f32(scene.scales)), _p(_f32(scene.quats)),
                       _p(_f32(scene.opac)), _p(_f32(scene.sh)), scene.sh_degree, _p(c32), _p(c64),
                       _p(_f64(bg)), _p(_f64(dL_rgb)), _p(None if dL_depth is None else _f64(dL_depth)),
                       _p(out["means"]), _p(out["scales"]), _p(out["quats"]), _p(out["opac"]),
                       _p(out["sh"]), _p(out["pose"]), _p(g2))
    if want_grad2d:
        out["grad2d"] = g2
    return out


def grad_stats(scene, cams, dL_rgbs, dL_depths=None, bg=(0, 0, 0, 0)):
    """Accumulators behind the average gradient of Eq. (3) for one backward
    call over several views of one map.

    Per Gaussian: the sum, over the views in which it survives culling (its
    3-sigma tile rectangle is not empty, the key path's `valid`), of the norm of
    that view's loss gradient with respect to its 3D mean; and the number of
    those views.  The average gradient of Eq. (3) is sum / count.  Returns
    (sum float64 [n], count int64 [n])."""
    n = scene.n
    total = np.zeros(n)
    count = np.zeros(n, np.int64)
    for v, cam in enumerate(cams):
        g_d = None if dL_depths is None else dL_depths[v]
        g = backward(scene, cam, dL_rgbs[v], g_d, bg=bg)["means"]
        total += np.sqrt((g * g).sum(axis=1))
        count += keys(scene, cam)["valid"].astype(np.int64)
    return total, count
