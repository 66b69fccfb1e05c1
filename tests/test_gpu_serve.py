"""Render server on the GPU: a request rendered alone equals the same request
rendered in a mixed stream of maps and resolutions (bit for bit), and the
served images match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2509_13536_amd import GaussianMap, View, render_forward
from paper_2509_13536_amd.serve import GpuExecutor, RenderServer

from gpu_helpers import image_parity

pytestmark = pytest.mark.gpu


def test_alone_equals_in_the_mix():
    scenes = [synth.Scene(*synth.room_gaussians(n, 0, s, 0), 0) for n, s in ((20_000, 41), (60_000, 42), (5_000, 43))]
    maps = {i: GaussianMap.from_numpy(sc) for i, sc in enumerate(scenes)}
    ex = GpuExecutor(maps, n_workers=2)
    srv = RenderServer(ex, mem_budget_bytes=4 << 30, max_batch=8)
    rng = np.random.default_rng(0)
    res = [(320, 240, 300.0), (640, 480, 525.0), (200, 120, 150.0)]

    def req(i):
        W, H, f = res[i % 3]
        cam = synth.Camera(W, H, f, f, W / 2, H / 2, synth.random_pose_in_room(rng))
        return i % 3, cam

    probes = [req(i) for i in range(6)]
    alone = []
    for mid, cam in probes:
        r = srv.submit(mid, View.from_camera(cam)).result(timeout=60)
        alone.append((r.rgb.clone(), r.depth.clone(), r.batch_size))
    futs = []
    for k in range(60):
        if k % 10 == 3:
            mid, cam = probes[k // 10]
        else:
            mid, cam = req(100 + k)
        futs.append((k, srv.submit(mid, View.from_camera(cam))))
    results = {k: f.result(timeout=120) for k, f in futs}
    srv.close()
    assert max(r.batch_size for r in results.values()) > 1, "the mix must batch requests together"
    for j in range(6):
        r = results[10 * j + 3]
        assert torch.equal(r.rgb, alone[j][0]) and torch.equal(r.depth, alone[j][1])
    # one served image against the oracle
    mid, cam = probes[1]
    st = srv.stats()
    assert st["completed"] == 66 and st["p99_ms"] >= st["p50_ms"]
    ref = oracle.forward(scenes[mid], cam)
    got = results[13].rgb.cpu().numpy()
    ok = ~ref["amb"]
    assert np.abs(got - ref["rgb"])[:, ok].max() <= 1e-4


def test_nan_pose_view_renders_background_and_spares_the_others():
    """A view whose pose is not finite, inside a multi-view call: every pair of
    it is culled, so it renders the background (T = 1), and the call's other
    views equal their renders alone, bit for bit."""
    sc = synth.Scene(*synth.room_gaussians(30_000, 0, 44, 0), 0)
    m = GaussianMap.from_numpy(sc)
    rng = np.random.default_rng(4)
    cams = [synth.Camera(320, 240, 300.0, 300.0, 160.0, 120.0, synth.random_pose_in_room(rng)) for _ in range(2)]
    bad = View.from_camera(cams[0])
    bad.Tcw = np.full((3, 4), np.nan, np.float32)
    bg = (0.1, 0.2, 0.3, 0.5)
    st = render_forward([m], [View.from_camera(cams[0]), bad, View.from_camera(cams[1])], bg=bg)
    alone = [render_forward([m], [View.from_camera(c)], bg=bg) for c in cams]
    torch.cuda.synchronize()
    for v, a in ((0, alone[0]), (2, alone[1])):
        for x, y in zip(st.view_images(v), a.view_images(0)):
            assert torch.equal(x, y)
    rgb, depth, T = (x.cpu().numpy() for x in st.view_images(1))
    assert np.all(T == 1.0) and np.all(depth == np.float32(bg[3]))
    for c in range(3):
        assert np.all(rgb[c] == np.float32(bg[c]))


def test_poisoned_request_is_refused_alone():
    """A request with a NaN pose in a burst of requests for one map: refused by
    itself (ValueError), while the burst's other requests are served and equal
    their renders alone."""
    sc = synth.Scene(*synth.room_gaussians(30_000, 0, 45, 0), 0)
    ex = GpuExecutor({0: GaussianMap.from_numpy(sc)}, n_workers=2)
    srv = RenderServer(ex, mem_budget_bytes=4 << 30, max_batch=8)
    rng = np.random.default_rng(5)
    cams = [synth.Camera(320, 240, 300.0, 300.0, 160.0, 120.0, synth.random_pose_in_room(rng)) for _ in range(6)]
    alone = [srv.submit(0, View.from_camera(c)).result(timeout=60) for c in cams]
    bad = View.from_camera(cams[0])
    bad.Tcw = np.full((3, 4), np.nan, np.float32)
    futs = [srv.submit(0, View.from_camera(c)) for c in cams[:3]] + [srv.submit(0, bad)] + \
           [srv.submit(0, View.from_camera(c)) for c in cams[3:]]
    with pytest.raises(ValueError):
        futs[3].result(timeout=60)
    got = [f.result(timeout=60) for k, f in enumerate(futs) if k != 3]
    srv.close()
    for g, a in zip(got, alone):
        assert torch.equal(g.rgb, a.rgb) and torch.equal(g.depth, a.depth)
