"""torch.autograd.Function over mgs_render_forward / mgs_render_backward.

The forward keeps only the forward state the library leaves in its workspace
(sorted tile lists, tile ranges, final transmittance and the index of each
pixel's last contributor); the backward recomputes every per-pixel
transmittance from the final one instead of storing it.

Camera poses enter through a twist xi in se(3) per view (xi = (rho, theta)),
applied on the left: T_CW <- Exp(xi) T_CW.  The gradient returned for xi is the
library's pose gradient, which is d L / d xi at xi = 0, the usual tracking
parameterisation (the twist is folded into the pose and reset after each
update).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from .api import (LAMBDA_SSIM, GaussianMap, GradStats, View, Workspace, mapping_loss, render_backward,
                  render_forward)


def se3_exp(xi: np.ndarray) -> np.ndarray:
    """4x4 exponential of the twist xi = (rho, theta) (float64)."""
    xi = np.asarray(xi, np.float64)
    rho, th = xi[:3], xi[3:]
    a = float(np.linalg.norm(th))
    K = np.array([[0, -th[2], th[1]], [th[2], 0, -th[0]], [-th[1], th[0], 0]])
    if a < 1e-8:
        R = np.eye(3) + K
        Vm = np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + np.sin(a) / a * K + (1 - np.cos(a)) / a ** 2 * K @ K
        Vm = np.eye(3) + (1 - np.cos(a)) / a ** 2 * K + (a - np.sin(a)) / a ** 3 * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = Vm @ rho
    return T


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opac, sh, pose_xi, views, sh_degree, bg, ws, stats):
        xi = pose_xi.detach().cpu().numpy().astype(np.float64)
        posed = []
        for v, x in zip(views, xi):
            if np.any(x != 0):
                T4 = np.eye(4)
                T4[:3, :] = np.asarray(v.Tcw, np.float64)
                T4 = se3_exp(x) @ T4
                v = View(v.W, v.H, v.fx, v.fy, v.cx, v.cy, T4[:3, :].astype(np.float32), v.near, v.map)
            posed.append(v)
        m = GaussianMap(means.detach(), scales.detach(), quats.detach(), opac.detach(), sh.detach(), sh_degree)
        st = render_forward([m], posed, bg=bg, need_backward=True, ws=ws)
        ctx.state = st
        ctx.stats = stats
        ctx.shapes = (means.shape, sh.shape)
        return st.rgb, st.depth

    @staticmethod
    def backward(ctx, g_rgb, g_depth):
        st = ctx.state
        g_rgb = torch.zeros_like(st.rgb) if g_rgb is None else g_rgb.contiguous()
        g_depth = None if g_depth is None else g_depth.contiguous()
        grads, d_pose = render_backward(st, g_rgb, g_depth, stats=None if ctx.stats is None else [ctx.stats])
        g = grads[0]
        return g["means"], g["scales"], g["quats"], g["opac"], g["sh"], d_pose, None, None, None, None, None


def render(means: torch.Tensor, scales: torch.Tensor, quats: torch.Tensor, opac: torch.Tensor, sh: torch.Tensor,
           views: Sequence[View], sh_degree: int, pose_xi: Optional[torch.Tensor] = None, bg=(0.0, 0.0, 0.0, 0.0),
           ws: Optional[Workspace] = None, stats: Optional[GradStats] = None):
    """Differentiable render of one map into `views`.

    Returns (rgb, depth) packed view after view ([3,H,W] then [H,W] per view);
    use `split_views` to get per-view tensors.  Gradients flow to all Gaussian
    parameters and to `pose_xi` ([V,6], default zeros).  `stats`, when given,
    accumulates the Eq. (3) gradient statistics during the backward."""
    views = [View(v.W, v.H, v.fx, v.fy, v.cx, v.cy, v.Tcw, v.near, 0) for v in views]
    if pose_xi is None:
        pose_xi = torch.zeros((len(views), 6), dtype=torch.float32, device=means.device)
    return _Render.apply(means, scales, quats, opac, sh, pose_xi, views, sh_degree, tuple(bg), ws, stats)


def split_views(rgb: torch.Tensor, depth: torch.Tensor, views: Sequence[View]) -> List[tuple]:
    out, o = [], 0
    for v in views:
        n = v.W * v.H
        out.append((rgb[3 * o:3 * o + 3 * n].view(3, v.H, v.W), depth[o:o + n].view(v.H, v.W)))
        o += n
    return out


class _MappingLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgb, depth, scales, gt_rgb, gt_depth, sizes, lambda_ssim, w_depth, w_iso, ws):
        r = mapping_loss(sizes, rgb.detach().contiguous(), gt_rgb.contiguous(),
                         None if depth is None else depth.detach().contiguous(),
                         None if gt_depth is None else gt_depth.contiguous(),
                         None if scales is None else scales.detach().contiguous(), lambda_ssim, w_depth, w_iso, ws)
        ctx.res = r
        ctx.mark_non_differentiable(r.loss)
        return r.total.clone(), r.loss

    @staticmethod
    def backward(ctx, g_total, g_terms):
        r = ctx.res
        scale = g_total.to(torch.float32)
        gd = None if r.d_depth is None else r.d_depth * scale
        gs = None if r.d_scales is None else r.d_scales * scale
        return r.d_rgb * scale, gd, gs, None, None, None, None, None, None, None


def loss(rgb: torch.Tensor, gt_rgb: torch.Tensor, views: Sequence[View], depth: Optional[torch.Tensor] = None,
         gt_depth: Optional[torch.Tensor] = None, scales: Optional[torch.Tensor] = None,
         lambda_ssim: float = LAMBDA_SSIM, w_depth: float = 1.0, w_iso: float = 0.0,
         ws: Optional[Workspace] = None):
    """Differentiable mapping loss of Eq. (12) over the packed output of `render`.
    Returns (total, terms): terms are the per-view (L1, SSIM, depth L1, L_view),
    then L_iso and the total (not differentiable).  The gradient flows to rgb,
    depth and scales (the SSIM window and the weights are fixed)."""
    sizes = [(v.W, v.H) for v in views]
    return _MappingLoss.apply(rgb, depth, scales, gt_rgb, gt_depth, sizes, lambda_ssim, w_depth, w_iso, ws)
