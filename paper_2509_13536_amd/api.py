"""Python entry points over the C ABI (include/memgs.h), on torch device tensors.

PyTorch supplies device memory and the stream; the computation is the HIP
library's.  Names follow the ABI: render_forward, render_backward, voxel_merge.
"""
from __future__ import annotations

import ctypes as C
import itertools
import struct
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi

CHI2_3DOF_95 = 7.815  # critical value the paper uses for the similarity test (Sec. II-D)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _check_dev(t: torch.Tensor, name: str, dtype=torch.float32):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


@dataclass
class GaussianMap:
    """A Gaussian map on the device (structure of arrays)."""
    means: torch.Tensor   # [n,3]
    scales: torch.Tensor  # [n,3] linear
    quats: torch.Tensor   # [n,4] (w,x,y,z)
    opac: torch.Tensor    # [n]
    sh: torch.Tensor      # [n,K,3]
    sh_degree: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_numpy(scene, device="cuda") -> "GaussianMap":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussianMap(t(scene.means), t(scene.scales), t(scene.quats), t(scene.opac), t(scene.sh),
                           int(scene.sh_degree))

    def c_struct(self) -> _abi.Gaussians:
        for name in ("means", "scales", "quats", "opac", "sh"):
            _check_dev(getattr(self, name), name)
        return _abi.Gaussians(self.n, self.means.data_ptr(), self.scales.data_ptr(), self.quats.data_ptr(),
                              self.opac.data_ptr(), self.sh.data_ptr(), int(self.sh_degree), 0)

    def nbytes(self) -> int:
        return sum(getattr(self, k).numel() * 4 for k in ("means", "scales", "quats", "opac", "sh"))


@dataclass
class View:
    """A pinhole view of map `map` (index into the maps list)."""
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    Tcw: np.ndarray  # [3,4] world->camera
    near: float = 0.2
    map: int = 0

    @staticmethod
    def from_camera(cam, map_index: int = 0) -> "View":
        return View(int(cam.W), int(cam.H), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                    np.asarray(cam.Tcw, np.float32), float(cam.near), map_index)

    def c_struct(self) -> _abi.Camera:
        c = _abi.Camera()
        c.width, c.height = int(self.W), int(self.H)
        c.fx, c.fy, c.cx, c.cy = self.fx, self.fy, self.cx, self.cy
        c.Tcw[:] = np.asarray(self.Tcw, np.float32).reshape(12).tolist()
        c.near_z = float(self.near)
        c.map = int(self.map)
        return c


def _maps_array(maps: Sequence[GaussianMap]):
    arr = (_abi.Gaussians * len(maps))()
    for i, m in enumerate(maps):
        arr[i] = m.c_struct()
    return arr


_CAMERA = struct.Struct("<2i4f12f f i")  # the layout of _abi.Camera


def _views_array(views: Sequence[View]):
    """Packed mgs_camera structs (the same bytes as View.c_struct, built in one
    buffer: per-field ctypes assignment costs several microseconds a view)."""
    n = len(views)
    buf = bytearray(_CAMERA.size * n)
    for i, v in enumerate(views):
        _CAMERA.pack_into(buf, i * _CAMERA.size, int(v.W), int(v.H), v.fx, v.fy, v.cx, v.cy,
                          *np.asarray(v.Tcw, np.float32).reshape(12).tolist(), float(v.near), int(v.map))
    return (_abi.Camera * n).from_buffer(buf)


class Workspace:
    """A growable device byte buffer for the library's scratch space.

    `generation` counts the forward renders that wrote their state into it, so
    that a backward can tell whether a later forward has overwritten the state
    it needs (see ForwardState)."""

    def __init__(self, device="cuda", nbytes: int = 0):
        self.device = device
        self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.generation = 0

    @property
    def nbytes(self) -> int:
        return int(self.buf.numel())

    def ensure(self, nbytes: int, slack: float = 1.25):
        if nbytes > self.nbytes:
            self.buf = torch.empty(int(nbytes * slack) + 256, dtype=torch.uint8, device=self.device)

    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())

    def view(self, offset: int, count: int, dtype) -> torch.Tensor:
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.buf[offset:offset + count * itemsize].view(dtype)


@dataclass
class GradStats:
    """Device accumulators of the average gradient of Eq. (3) for one map,
    filled by render_backward (+= per call) and read by merge_mask."""
    grad_norm_sum: torch.Tensor  # [n] float32
    visible_count: torch.Tensor  # [n] int32 on the torch side, uint32 in the ABI

    @staticmethod
    def zeros(n: int, device="cuda") -> "GradStats":
        return GradStats(torch.zeros(n, dtype=torch.float32, device=device),
                         torch.zeros(n, dtype=torch.int32, device=device))

    def zero_(self) -> "GradStats":
        self.grad_norm_sum.zero_()
        self.visible_count.zero_()
        return self

    def average(self) -> torch.Tensor:
        """sum / count (NaN where the count is 0), for inspection."""
        return self.grad_norm_sum / self.visible_count.to(torch.float32)


@dataclass
class ForwardState:
    maps: List[GaussianMap]
    views: List[View]
    bg: tuple
    info: _abi.ForwardInfo
    ws: Workspace
    rgb: torch.Tensor    # packed
    depth: torch.Tensor  # packed
    T: torch.Tensor      # packed
    pix_off: List[int] = field(default_factory=list)
    fwd_ms: Optional[List[float]] = None  # stage times when timing was requested
    bwd_ms: Optional[List[float]] = None
    ws_generation: int = -1               # ws.generation right after this forward
    ws_buf: Optional[torch.Tensor] = None  # the buffer that holds this forward's state

    def check_workspace(self):
        """Raise if a later forward (or a regrowth) has replaced the state this
        forward left in its workspace: a backward from it would read another
        call's lists."""
        if self.ws.generation != self.ws_generation or self.ws.buf is not self.ws_buf:
            raise RuntimeError("the workspace of this forward was reused by a later render_forward: run the "
                               "backward before reusing the workspace, or give each forward its own")

    def view_images(self, v: int):
        """(rgb [3,H,W], depth [H,W], T [H,W]) of view v (views into the packed buffers)."""
        V = self.views[v]
        o, n = self.pix_off[v], V.W * V.H
        return (self.rgb[3 * o:3 * o + 3 * n].view(3, V.H, V.W), self.depth[o:o + n].view(V.H, V.W),
                self.T[o:o + n].view(V.H, V.W))


def _event_handles(events):
    """Raw handles of torch.cuda.Event objects (recorded once so that they exist)."""
    if events is None:
        return None
    arr = (C.c_void_p * 6)()
    for i, ev in enumerate(events):
        if not ev.cuda_event:
            ev.record()
        arr[i] = ev.cuda_event
    return arr


def _opts(bg, need_backward, stage=None, count_blended=False, events=None) -> _abi.RenderOpts:
    o = _abi.RenderOpts()
    for i in range(3):
        o.bg_rgb[i] = float(bg[i])
    o.bg_depth = float(bg[3])
    o.need_backward = 1 if need_backward else 0
    o.count_blended = 1 if count_blended else 0
    if stage is not None:
        o.stage_ms = C.cast(stage, C.POINTER(C.c_float))
    if events is not None:
        o.stage_events = C.cast(events, C.POINTER(C.c_void_p))
    return o


def render_forward(maps: Sequence[GaussianMap], views: Sequence[View], bg=(0.0, 0.0, 0.0, 0.0),
                   need_backward: bool = False, ws: Optional[Workspace] = None, stream=None,
                   out: Optional[tuple] = None, timing: bool = False, count_blended: bool = False,
                   events: Optional[list] = None) -> ForwardState:
    """mgs_render_forward over `views` (any number, any map, any resolution).
    timing: stage times in ms (the call waits for its stream); events: four
    torch.cuda.Event recorded at the stage boundaries without waiting."""
    lib = _abi.load()
    maps, views = list(maps), list(views)
    dev = maps[0].means.device
    ws = ws if ws is not None else Workspace(dev)
    npix = sum(v.W * v.H for v in views)
    pix_off = [0, *itertools.accumulate(v.W * v.H for v in views)]
    if out is None:
        rgb = torch.empty(3 * npix, dtype=torch.float32, device=dev)
        depth = torch.empty(npix, dtype=torch.float32, device=dev)
        T = torch.empty(npix, dtype=torch.float32, device=dev)
    else:
        rgb, depth, T = out
    m_arr, v_arr = _maps_array(maps), _views_array(views)
    stage = (C.c_float * 4)() if timing else None
    ev = _event_handles(events)
    opts = _opts(bg, need_backward, stage, count_blended, ev)
    info = _abi.ForwardInfo()
    s = _stream(stream)
    for _ in range(4):
        status = lib.mgs_render_forward(m_arr, len(maps), v_arr, len(views), C.byref(opts), ws.ptr(), ws.nbytes,
                                        C.byref(info), _ptr(rgb), _ptr(depth), _ptr(T), s)
        if status == _abi.MGS_ERR_WORKSPACE:
            ws.ensure(int(info.ws_required))
            continue
        if status != _abi.MGS_OK:
            raise _abi.MemgsError("mgs_render_forward", status)
        break
    else:
        raise _abi.MemgsError("mgs_render_forward", _abi.MGS_ERR_WORKSPACE)
    ws.generation += 1
    return ForwardState(maps, views, tuple(bg), info, ws, rgb, depth, T, pix_off,
                        list(stage) if timing else None, ws_generation=ws.generation, ws_buf=ws.buf)


def render_backward(state: ForwardState, dL_rgb: torch.Tensor, dL_depth: Optional[torch.Tensor] = None,
                    stream=None, want=("means", "scales", "quats", "opac", "sh"), pose: bool = True,
                    timing: bool = False, grads_out: Optional[list] = None, d_pose: Optional[torch.Tensor] = None,
                    events: Optional[list] = None, stats: Optional[Sequence[Optional[GradStats]]] = None):
    """mgs_render_backward.  dL_rgb / dL_depth are packed like the forward outputs.
    events: three torch.cuda.Event recorded at the stage boundaries without waiting.
    stats: per map, a GradStats (or None) that the call accumulates into.
    Returns (list of per-map dicts of gradient tensors, d_pose [V,6] or None)."""
    lib = _abi.load()
    state.check_workspace()
    _check_dev(dL_rgb, "dL_rgb")
    if dL_depth is not None:
        _check_dev(dL_depth, "dL_depth")
    if grads_out is None:
        grads_out = []
        for m in state.maps:
            d = {}
            for name, shape in (("means", (m.n, 3)), ("scales", (m.n, 3)), ("quats", (m.n, 4)), ("opac", (m.n,)),
                                ("sh", tuple(m.sh.shape))):
                if name in want:
                    d[name] = torch.empty(shape, dtype=torch.float32, device=m.means.device)
            grads_out.append(d)
    if stats is not None and len(stats) != len(state.maps):
        raise ValueError("stats needs one entry (or None) per map")
    g_arr = (_abi.GaussianGrads * len(state.maps))()
    for i, d in enumerate(grads_out):
        st_i = None if stats is None else stats[i]
        if st_i is not None:
            n = state.maps[i].n
            _check_dev(st_i.grad_norm_sum, "grad_norm_sum")
            _check_dev(st_i.visible_count, "visible_count", torch.int32)
            if st_i.grad_norm_sum.numel() != n or st_i.visible_count.numel() != n:
                raise ValueError("GradStats size differs from the map's")
        g_arr[i] = _abi.GaussianGrads(*(d[k].data_ptr() if k in d else None
                                        for k in ("means", "scales", "quats", "opac", "sh")),
                                      _ptr(None if st_i is None else st_i.grad_norm_sum),
                                      _ptr(None if st_i is None else st_i.visible_count))
    if d_pose is None and pose:
        d_pose = torch.empty((len(state.views), 6), dtype=torch.float32, device=dL_rgb.device)
    stage = (C.c_float * 4)() if timing else None
    ev = _event_handles(events)
    status = lib.mgs_render_backward(_maps_array(state.maps), len(state.maps), _views_array(state.views),
                                     len(state.views), C.byref(_opts(state.bg, True, stage, False, ev)),
                                     C.byref(state.info),
                                     state.ws.ptr(), state.ws.nbytes, _ptr(state.T), _ptr(dL_rgb), _ptr(dL_depth),
                                     g_arr, _ptr(d_pose), _stream(stream))
    if status != _abi.MGS_OK:
        raise _abi.MemgsError("mgs_render_backward", status)
    if timing:
        state.bwd_ms = list(stage)
    return grads_out, d_pose


GRAD_TAU = 1e-3  # gradient threshold of Eq. (3) in the paper


def merge_mask(stats: GradStats, tau: float = GRAD_TAU, kf_index: Optional[torch.Tensor] = None,
               kf_min: int = 0, kf_max: int = 2 ** 31 - 1, stream=None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """mgs_merge_mask: M(G) of Eq. (3) as a uint8 device tensor (the mask of voxel_merge)."""
    lib = _abi.load()
    n = int(stats.grad_norm_sum.numel())
    _check_dev(stats.grad_norm_sum, "grad_norm_sum")
    _check_dev(stats.visible_count, "visible_count", torch.int32)
    if stats.visible_count.numel() != n:
        raise ValueError("visible_count size differs from grad_norm_sum's")
    if kf_index is not None:
        _check_dev(kf_index, "kf_index", torch.int32)
        if kf_index.numel() != n:
            raise ValueError("kf_index size differs")
    mask = out if out is not None else torch.empty(n, dtype=torch.uint8, device=stats.grad_norm_sum.device)
    _check_dev(mask, "mask", torch.uint8)
    status = lib.mgs_merge_mask(_ptr(stats.grad_norm_sum), _ptr(stats.visible_count), _ptr(kf_index), n,
                                float(tau), int(kf_min), int(kf_max), _ptr(mask), _stream(stream))
    if status != _abi.MGS_OK:
        raise _abi.MemgsError("mgs_merge_mask", status)
    return mask


LAMBDA_SSIM = 0.2  # lambda of Eq. (12) (the paper leaves it unstated; the 3DGS lineage's value)


@dataclass
class LossResult:
    loss: torch.Tensor                 # [4 V + 2]: per view (L1, SSIM, depth L1, L_view), L_iso, total
    d_rgb: torch.Tensor                # packed like the colour
    d_depth: Optional[torch.Tensor]    # packed like the depth
    d_scales: Optional[torch.Tensor]   # [n,3]

    @property
    def total(self) -> torch.Tensor:
        return self.loss[-1]


def mapping_loss(sizes: Sequence[tuple], rgb: torch.Tensor, gt_rgb: torch.Tensor,
                 depth: Optional[torch.Tensor] = None, gt_depth: Optional[torch.Tensor] = None,
                 scales: Optional[torch.Tensor] = None, lambda_ssim: float = LAMBDA_SSIM, w_depth: float = 1.0,
                 w_iso: float = 0.0, ws: Optional[Workspace] = None, stream=None,
                 out: Optional[LossResult] = None) -> LossResult:
    """mgs_mapping_loss: Eq. (12) over views of sizes [(W, H), ...], packed as the renderer writes them."""
    lib = _abi.load()
    for t, name in ((rgb, "rgb"), (gt_rgb, "gt_rgb")):
        _check_dev(t, name)
    npix = sum(int(w) * int(h) for w, h in sizes)
    if rgb.numel() != 3 * npix or gt_rgb.numel() != 3 * npix:
        raise ValueError("colour buffers do not match the view sizes")
    if (depth is None) != (gt_depth is None):
        raise ValueError("give depth and gt_depth together")
    if depth is not None:
        _check_dev(depth, "depth")
        _check_dev(gt_depth, "gt_depth")
        if depth.numel() != npix or gt_depth.numel() != npix:
            raise ValueError("depth buffers do not match the view sizes")
    n_g = 0
    if scales is not None:
        _check_dev(scales, "scales")
        n_g = int(scales.shape[0])
    dev = rgb.device
    if out is None:
        out = LossResult(torch.empty(4 * len(sizes) + 2, dtype=torch.float32, device=dev), torch.empty_like(rgb),
                         None if depth is None else torch.empty_like(depth),
                         None if scales is None else torch.empty_like(scales))
    sz = (C.c_int32 * (2 * len(sizes)))(*[int(x) for wh in sizes for x in wh])
    o = _abi.LossOpts(float(lambda_ssim), float(w_depth), float(w_iso), 0)
    ws = ws if ws is not None else Workspace(dev)
    req = C.c_size_t(0)
    for _ in range(2):
        status = lib.mgs_mapping_loss(sz, len(sizes), _ptr(rgb), _ptr(gt_rgb), _ptr(depth), _ptr(gt_depth),
                                      _ptr(scales), n_g, C.byref(o), ws.ptr(), ws.nbytes, C.byref(req),
                                      _ptr(out.loss), _ptr(out.d_rgb), _ptr(out.d_depth), _ptr(out.d_scales),
                                      _stream(stream))
        if status == _abi.MGS_ERR_WORKSPACE:
            ws.ensure(int(req.value))
            continue
        if status != _abi.MGS_OK:
            raise _abi.MemgsError("mgs_mapping_loss", status)
        return out
    raise _abi.MemgsError("mgs_mapping_loss", _abi.MGS_ERR_WORKSPACE)


def mapping_loss_noalloc(sizes: Sequence[tuple], rgb: torch.Tensor, gt_rgb: torch.Tensor,
                         depth: Optional[torch.Tensor] = None, gt_depth: Optional[torch.Tensor] = None,
                         scales: Optional[torch.Tensor] = None, lambda_ssim: float = LAMBDA_SSIM,
                         w_depth: float = 1.0, w_iso: float = 0.0, stream=None,
                         out: Optional[LossResult] = None) -> LossResult:
    """mgs_mapping_loss_noalloc: the same loss as mapping_loss, with the library's
    fixed per-GPU scratch in place of a workspace (the call allocates nothing
    when `out` is given).  Calls that overlap on one GPU race on that scratch."""
    lib = _abi.load()
    for t, name in ((rgb, "rgb"), (gt_rgb, "gt_rgb")):
        _check_dev(t, name)
    npix = sum(int(w) * int(h) for w, h in sizes)
    if rgb.numel() != 3 * npix or gt_rgb.numel() != 3 * npix:
        raise ValueError("colour buffers do not match the view sizes")
    if (depth is None) != (gt_depth is None):
        raise ValueError("give depth and gt_depth together")
    if depth is not None:
        _check_dev(depth, "depth")
        _check_dev(gt_depth, "gt_depth")
        if depth.numel() != npix or gt_depth.numel() != npix:
            raise ValueError("depth buffers do not match the view sizes")
    n_g = 0
    if scales is not None:
        _check_dev(scales, "scales")
        n_g = int(scales.shape[0])
    if out is None:
        dev = rgb.device
        out = LossResult(torch.empty(4 * len(sizes) + 2, dtype=torch.float32, device=dev), torch.empty_like(rgb),
                         None if depth is None else torch.empty_like(depth),
                         None if scales is None else torch.empty_like(scales))
    sz = (C.c_int32 * (2 * len(sizes)))(*[int(x) for wh in sizes for x in wh])
    o = _abi.LossOpts(float(lambda_ssim), float(w_depth), float(w_iso), 0)
    req = C.c_size_t(0)
    status = lib.mgs_mapping_loss_noalloc(sz, len(sizes), _ptr(rgb), _ptr(gt_rgb), _ptr(depth), _ptr(gt_depth),
                                          _ptr(scales), n_g, C.byref(o), C.byref(req), _ptr(out.loss),
                                          _ptr(out.d_rgb), _ptr(out.d_depth), _ptr(out.d_scales), _stream(stream))
    if status != _abi.MGS_OK:
        err = _abi.MemgsError("mgs_mapping_loss_noalloc", status)
        err.scratch_required = int(req.value)
        raise err
    return out


@dataclass
class PatchGridResult:
    map: GaussianMap            # the new Gaussians (SH degree 0), views of capacity-sized buffers
    n_out: int
    source: torch.Tensor        # [n_out] candidate of each: < n_kp a keypoint, else a lattice sample


def patch_grid_sample(view: View, keypoints: torch.Tensor, kp_depth: torch.Tensor, image: torch.Tensor,
                      depth_map: Optional[torch.Tensor] = None, patch: int = 32, min_keypoints: int = 4,
                      samples: int = 2, opacity: float = 0.5, scale_factor: float = 0.5,
                      ws: Optional[Workspace] = None, stream=None) -> PatchGridResult:
    """mgs_patch_grid_sample (Sec. II-B): Gaussians from keypoints [n,2] (with
    depths [n], <= 0 for none) and Patch-Grid samples of a keyframe."""
    lib = _abi.load()
    _check_dev(keypoints, "keypoints")
    _check_dev(kp_depth, "kp_depth")
    _check_dev(image, "image")
    n_kp = int(keypoints.shape[0])
    if keypoints.numel() != 2 * n_kp or kp_depth.numel() != n_kp:
        raise ValueError("keypoints must be [n,2] with one depth each")
    if image.numel() != 3 * view.W * view.H:
        raise ValueError("image must be [3,H,W]")
    if depth_map is not None:
        _check_dev(depth_map, "depth_map")
        if depth_map.numel() != view.W * view.H:
            raise ValueError("depth_map must be [H,W]")
    dev = keypoints.device
    cap = n_kp + (-(-view.W // patch)) * (-(-view.H // patch)) * samples * samples
    m = GaussianMap(torch.empty((cap, 3), device=dev), torch.empty((cap, 3), device=dev),
                    torch.empty((cap, 4), device=dev), torch.empty(cap, device=dev),
                    torch.empty((cap, 1, 3), device=dev), 0)
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    out = _abi.GaussiansOut(m.means.data_ptr(), m.scales.data_ptr(), m.quats.data_ptr(), m.opac.data_ptr(),
                            m.sh.data_ptr())
    o = _abi.PgOpts(int(patch), int(min_keypoints), int(samples), float(opacity), float(scale_factor), 0)
    ws = ws if ws is not None else Workspace(dev)
    cam = view.c_struct()
    req = C.c_size_t(0)
    n_out = C.c_int64(0)
    for _ in range(2):
        status = lib.mgs_patch_grid_sample(C.byref(cam), _ptr(keypoints), _ptr(kp_depth), n_kp, _ptr(depth_map),
                                           _ptr(image), C.byref(o), C.byref(out), _ptr(src), ws.ptr(), ws.nbytes,
                                           C.byref(req), C.byref(n_out), _stream(stream))
        if status == _abi.MGS_ERR_WORKSPACE:
            ws.ensure(int(req.value))
            continue
        if status != _abi.MGS_OK:
            raise _abi.MemgsError("mgs_patch_grid_sample", status)
        break
    k = int(n_out.value)
    res = GaussianMap(m.means[:k], m.scales[:k], m.quats[:k], m.opac[:k], m.sh[:k], 0)
    return PatchGridResult(res, k, src[:k])


ADAM_GROUPS = ("means", "scales", "quats", "opac", "sh")


@dataclass
class AdamState:
    """First and second moments of every parameter array of a map, and the step count."""
    exp_avg: GaussianMap
    exp_avg_sq: GaussianMap
    step: int = 0

    @staticmethod
    def zeros_like(m: GaussianMap) -> "AdamState":
        z = lambda: GaussianMap(*(torch.zeros_like(getattr(m, k)) for k in ADAM_GROUPS), m.sh_degree)
        return AdamState(z(), z(), 0)


def _out_struct(m: GaussianMap) -> _abi.GaussiansOut:
    for k in ADAM_GROUPS:
        _check_dev(getattr(m, k), k)
    return _abi.GaussiansOut(*(getattr(m, k).data_ptr() for k in ADAM_GROUPS))


def adam_step(m: GaussianMap, grads: dict, state: AdamState, lr, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-15, stream=None) -> AdamState:
    """mgs_adam_step: one Adam step of the map's parameters in place.  grads is
    a dict of gradient tensors by group name (a missing group is not updated);
    lr a float or a dict by group name."""
    lib = _abi.load()
    lrs = [float(lr[k]) if isinstance(lr, dict) else float(lr) for k in ADAM_GROUPS]
    for k, g in grads.items():
        _check_dev(g, f"grad {k}")
        if g.numel() != getattr(m, k).numel():
            raise ValueError(f"gradient {k} has the wrong size")
    state.step += 1
    o = _abi.AdamOpts((C.c_float * 5)(*lrs), float(beta1), float(beta2), float(eps), int(state.step))
    gr = _abi.GaussianGrads(*(grads[k].data_ptr() if k in grads else None for k in ADAM_GROUPS))
    p, e1, e2 = _out_struct(m), _out_struct(state.exp_avg), _out_struct(state.exp_avg_sq)
    status = lib.mgs_adam_step(C.byref(p), m.n, int(m.sh_degree), C.byref(gr), C.byref(e1), C.byref(e2),
                               C.byref(o), _stream(stream))
    if status != _abi.MGS_OK:
        state.step -= 1
        raise _abi.MemgsError("mgs_adam_step", status)
    return state


class MergeResult:
    """The compacted map (`map`: views of the first n_out rows of the output
    buffers, made on first use), n_out, old -> new indices, voxel keys."""

    def __init__(self, buffers: GaussianMap, n_out: int, old_to_new: torch.Tensor,
                 voxel_key: Optional[torch.Tensor]):
        self._buffers = buffers
        self._map = None
        self.n_out = n_out
        self.old_to_new = old_to_new
        self.voxel_key = voxel_key

    @property
    def map(self) -> GaussianMap:
        if self._map is None:
            b, k = self._buffers, self.n_out
            self._map = GaussianMap(b.means[:k], b.scales[:k], b.quats[:k], b.opac[:k], b.sh[:k], b.sh_degree)
        return self._map


MERGE_BEST_PAIR = 1  # policy flag: only the closest pair of each voxel merges
MERGE_LBFGS = 2      # policy flag: Eq. (9) by the paper's L-BFGS solver instead of the closed form


def voxel_merge(m: GaussianMap, mask: Optional[torch.Tensor] = None, voxel_size: float = 0.05,
                chi2: float = CHI2_3DOF_95, policy: int = 0, ws: Optional[Workspace] = None,
                want_keys: bool = False, stream=None, out: Optional[GaussianMap] = None,
                solver: str = "closed") -> MergeResult:
    """mgs_voxel_merge; returns the compacted map (views of capacity-n buffers).
    policy: 0 sequential insertion, 1 (MERGE_BEST_PAIR) closest pair per voxel;
    solver: "closed" (the exact minimiser of Eq. (9)) or "lbfgs" (adds MERGE_LBFGS)."""
    if solver not in ("closed", "lbfgs"):
        raise ValueError("solver must be 'closed' or 'lbfgs'")
    if solver == "lbfgs":
        policy = int(policy) | MERGE_LBFGS
    lib = _abi.load()
    dev = m.means.device
    ws = ws if ws is not None else Workspace(dev)
    if out is None:
        out = GaussianMap(torch.empty_like(m.means), torch.empty_like(m.scales), torch.empty_like(m.quats),
                          torch.empty_like(m.opac), torch.empty_like(m.sh), m.sh_degree)
    o2n = torch.empty(m.n, dtype=torch.int32, device=dev)
    keys = torch.empty(m.n, dtype=torch.int64, device=dev) if want_keys else None
    if mask is not None:
        if mask.dtype != torch.uint8 or not mask.is_cuda:
            raise ValueError("mask must be a uint8 CUDA tensor")
    gin = m.c_struct()
    gout = _abi.GaussiansOut(out.means.data_ptr(), out.scales.data_ptr(), out.quats.data_ptr(),
                             out.opac.data_ptr(), out.sh.data_ptr())
    req = C.c_size_t(0)
    n_out = C.c_int64(0)
    for _ in range(2):
        status = lib.mgs_voxel_merge(C.byref(gin), _ptr(mask), float(voxel_size), float(chi2), int(policy),
                                     C.byref(gout), _ptr(o2n), _ptr(keys), ws.ptr(), ws.nbytes, C.byref(req),
                                     C.byref(n_out), _stream(stream))
        if status == _abi.MGS_ERR_WORKSPACE:
            ws.ensure(int(req.value))
            continue
        if status != _abi.MGS_OK:
            raise _abi.MemgsError("mgs_voxel_merge", status)
        break
    return MergeResult(GaussianMap(out.means, out.scales, out.quats, out.opac, out.sh, m.sh_degree),
                       int(n_out.value), o2n, keys)
