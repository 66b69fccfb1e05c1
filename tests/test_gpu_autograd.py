"""The backward kernels behind torch.autograd.Function, checked against the fp64
oracle's analytic gradient and against central finite differences of the fp64
oracle (frozen decisions), on the 1k-Gaussian 32x32 SH-degree-3 crop."""
import numpy as np
import pytest
import torch
from scipy.linalg import expm

import oracle
import synth
from paper_2509_13536_amd import View
from paper_2509_13536_amd.autograd import render

from gpu_helpers import grad_parity

pytestmark = pytest.mark.gpu


def _params(sc):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(True)
    return [t(sc.means), t(sc.scales), t(sc.quats), t(sc.opac), t(sc.sh)]


def test_autograd_matches_fp64_oracle_and_finite_differences():
    sc = synth.gradcheck_crop()
    cam = sc.cams[0]
    ref = oracle.forward(sc, cam)
    rng = np.random.default_rng(0)
    w_rgb = rng.normal(size=(3, cam.H, cam.W))
    w_d = rng.normal(size=(cam.H, cam.W))
    w_rgb[:, ref["amb"]] = 0
    w_d[ref["amb"]] = 0
    params = _params(sc)
    xi = torch.zeros((1, 6), device="cuda", requires_grad=True)
    rgb, depth = render(*params, [View.from_camera(cam)], sc.sh_degree, pose_xi=xi)
    L = (rgb * torch.from_numpy(w_rgb.reshape(-1)).float().cuda()).sum() + \
        (depth * torch.from_numpy(w_d.reshape(-1)).float().cuda()).sum()
    L.backward()
    gref = oracle.backward(sc, cam, w_rgb, w_d)
    names = ["means", "scales", "quats", "opac", "sh"]
    for name, p in zip(names, params):
        grad_parity(p.grad.cpu().numpy(), gref[name], name)
    grad_parity(xi.grad.cpu().numpy()[0], gref["pose"], "pose")
    # central differences of the fp64 oracle (frozen contributor lists) on a sample
    frozen = oracle.contributors(sc, cam)
    _, c64 = oracle.cam_arrays(cam)
    base = [sc.means.astype(np.float64), sc.scales.astype(np.float64), sc.quats.astype(np.float64),
            sc.opac.astype(np.float64), sc.sh.astype(np.float64)]

    def loss(ps, cam64):
        r, d = oracle.forward_frozen(ps, sc.sh_degree, cam64, frozen)
        return float((w_rgb * r).sum() + (w_d * d).sum())

    eps = 1e-6
    used = np.unique(frozen[1])
    for pi, name in enumerate(names):
        g_gpu = params[pi].grad.cpu().numpy().reshape(len(sc.means), -1)
        for g in rng.choice(used, 12, replace=False):
            for c in range(g_gpu.shape[1]):
                plus = [b.copy() for b in base]
                minus = [b.copy() for b in base]
                plus[pi].reshape(len(sc.means), -1)[g, c] += eps
                minus[pi].reshape(len(sc.means), -1)[g, c] -= eps
                fd = (loss(plus, c64) - loss(minus, c64)) / (2 * eps)
                scale = np.abs(gref[name]).max()
                assert abs(g_gpu[g, c] - fd) <= 1e-3 * abs(fd) + 1e-3 * scale, (name, g, c, g_gpu[g, c], fd)
    T4 = np.eye(4)
    T4[:3, :3] = c64[7:16].reshape(3, 3)
    T4[:3, 3] = c64[16:19]
    for k in range(6):
        vals = []
        for sgn in (1, -1):
            X = np.zeros((4, 4))
            e = np.zeros(6)
            e[k] = sgn * eps
            X[:3, :3] = np.array([[0, -e[5], e[4]], [e[5], 0, -e[3]], [-e[4], e[3], 0]])
            X[:3, 3] = e[:3]
            Tn = expm(X) @ T4
            cn = c64.copy()
            cn[7:16] = Tn[:3, :3].reshape(-1)
            cn[16:19] = Tn[:3, 3]
            vals.append(loss(base, cn))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(xi.grad[0, k].item() - fd) <= 1e-3 * abs(fd) + 1e-3 * np.abs(gref["pose"]).max()


def test_nonzero_twist_moves_the_camera():
    sc = synth.tiny_scene(500, 64, 48, 61, pose=True)
    cam = sc.cams[0]
    params = [p.detach() for p in _params(sc)]
    xi = torch.tensor([[0.01, -0.02, 0.015, 0.02, -0.01, 0.005]], device="cuda")
    rgb, _ = render(*params, [View.from_camera(cam)], sc.sh_degree, pose_xi=xi)
    X = np.zeros((4, 4))
    e = xi.cpu().numpy()[0].astype(np.float64)
    X[:3, :3] = np.array([[0, -e[5], e[4]], [e[5], 0, -e[3]], [-e[4], e[3], 0]])
    X[:3, 3] = e[:3]
    T4 = np.eye(4)
    T4[:3, :] = cam.Tcw
    moved = synth.Camera(cam.W, cam.H, cam.fx, cam.fy, cam.cx, cam.cy, (expm(X) @ T4)[:3].astype(np.float32))
    ref = oracle.forward(sc, moved)
    got = rgb.detach().cpu().numpy().reshape(3, cam.H, cam.W)
    ok = ~ref["amb"]
    assert np.abs(got - ref["rgb"])[:, ok].max() < 1e-4
