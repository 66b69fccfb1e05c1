"""GPU parity of the rasteriser (HIP path through the C ABI) against the oracle.

Bars: tile rectangles, depth keys, image means, radii and every tile's sorted
list bit-exact; images within 1e-4 absolute on pixels whose decisions are not
within the ambiguity band of the fp64 oracle (and depth within 1e-4 times the
largest depth); gradients within 1e-3 relative L2 and element-wise
1e-3 |g*| + 1e-3 max|g*|, with the upstream gradient zeroed on ambiguous pixels.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2509_13536_amd import GaussianMap, View, render_backward, render_forward

from gpu_helpers import _inst_lists, assert_keys_and_lists, grad_parity, image_parity, run_forward

pytestmark = pytest.mark.gpu


def _scenes():
    return {
        "tiny_ragged_sh3": synth.tiny_scene(60, 50, 37, 11, sh_degree=3, pose=True, log_scale_mu=-2.8),
        "small_sh1": synth.tiny_scene(2000, 130, 97, 12, sh_degree=1, pose=True, log_scale_mu=-3.0),
        "cfg1_10k_320x240": synth.cfg1_plain_forward(),
    }


@pytest.mark.parametrize("name", ["tiny_ragged_sh3", "small_sh1", "cfg1_10k_320x240"])
def test_forward_keys_and_image(name):
    sc = _scenes()[name]
    bg = (0.1, 0.2, 0.3, 0.5) if name == "tiny_ragged_sh3" else (0, 0, 0, 0)
    print(f"case {name}", flush=True)
    st = run_forward(sc, bg=bg)
    assert_keys_and_lists(sc, sc.cams[0], st)
    image_parity(sc, sc.cams[0], st, bg=bg)


def _edge_scene(seed, n=6000, W=160, H=120, f=150.0):
    """Gaussians around the frustum's sides and the near plane, of scales from
    1 mm to 3 m: pairs just outside the image whose footprint may still reach it,
    and pairs whose Jacobian is clamped."""
    rng = np.random.default_rng(seed)
    z = np.concatenate([rng.uniform(0.2, 0.23, n // 6), rng.uniform(0.23, 6.0, n - n // 6)])
    xr = rng.uniform(-2.5, 2.5, n) * (W / 2) / f
    yr = rng.uniform(-2.5, 2.5, n) * (H / 2) / f
    means = np.stack([xr * z, yr * z, z], axis=1).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(1e-3), np.log(3.0), size=(n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    opac = rng.uniform(0.05, 0.95, n).astype(np.float32)
    sh = rng.uniform(-1, 1, size=(n, 1, 3)).astype(np.float32)
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    cam = synth.Camera(W, H, f, f * 1.1, (W - 1) / 2.0 + 0.25, (H - 1) / 2.0 - 0.25, Tcw)
    return synth.Scene(means, scales, q, opac, sh, 0, [cam], f"edge{seed}")


@pytest.mark.parametrize("seed", [71, 72])
def test_screen_test_keeps_every_visible_pair(seed):
    """The projection's screen test drops only pairs that the key path culls:
    every pair's depth key, rectangle and image mean, and every tile list, equal
    the oracle's on a scene crowded at the frustum's edges and the near plane.
    (Its image is not compared: thousands of metre-sized Gaussians overlap each
    pixel, beyond the scenes the image tolerance is set for; culling shows in
    the keys and lists.)"""
    sc = _edge_scene(seed)
    print(f"case edge scene {seed}", flush=True)
    st = run_forward(sc)
    assert int(st.info.n_visible) > 300
    assert_keys_and_lists(sc, sc.cams[0], st)


def test_forward_is_bit_deterministic():
    sc = synth.cfg1_plain_forward()
    a = run_forward(sc)
    b = run_forward(sc)
    for x, y in zip((a.rgb, a.depth, a.T), (b.rgb, b.depth, b.T)):
        assert torch.equal(x, y)


def test_cfg2_keys_and_image_subset():
    sc, _, _ = synth.cfg2_keyframe()
    sc = sc.subset(np.arange(0, sc.n, 4))  # 50k of the 200k, full 640x480 image
    print("case cfg2 subset", flush=True)
    st = run_forward(sc)
    assert_keys_and_lists(sc, sc.cams[0], st)
    image_parity(sc, sc.cams[0], st)


@pytest.mark.parametrize("seed,deg,n,W,H", [(31, 0, 400, 64, 48), (32, 3, 800, 96, 70), (33, 1, 10_000, 320, 240)])
def test_backward_matches_oracle(seed, deg, n, W, H):
    sc = synth.tiny_scene(n, W, H, seed, sh_degree=deg, pose=True, log_scale_mu=-3.0 if n > 1000 else -2.7)
    cam = sc.cams[0]
    bg = (0.05, 0.1, 0.15, 0.2)
    print(f"case backward seed={seed}", flush=True)
    st = run_forward(sc, bg=bg, need_backward=True)
    ref = oracle.forward(sc, cam, bg=bg)
    g_rgb, g_d = synth.upstream_grads([cam], seed)
    g_rgb, g_d = g_rgb[0], g_d[0]
    g_rgb[:, ref["amb"]] = 0
    g_d[ref["amb"]] = 0
    grads, d_pose = render_backward(st, torch.from_numpy(g_rgb.reshape(-1)).cuda(),
                                    torch.from_numpy(g_d.reshape(-1)).cuda())
    gref = oracle.backward(sc, cam, g_rgb, g_d, bg=bg)
    for name in ("means", "scales", "quats", "opac", "sh"):
        grad_parity(grads[0][name].cpu().numpy(), gref[name], name)
    grad_parity(d_pose.cpu().numpy()[0], gref["pose"], "pose")


@pytest.mark.parametrize("mode", ["all_high", "mixed"])
def test_alpha_clamp_opacities(mode):
    """Opacities at and near 1, where alpha reaches the 0.99 clamp: the kernels
    then take their clamping evaluation (the forward for the whole call, the
    backward per staged batch; "mixed" has batches of both kinds).  Image and
    gradients against the oracle."""
    sc = synth.tiny_scene(3000, 160, 120, 35, sh_degree=1, pose=True, log_scale_mu=-2.7)
    rng = np.random.default_rng(35)
    if mode == "all_high":
        op = rng.uniform(0.97, 1.0, sc.n)
        op[::7] = 1.0
    else:
        op = rng.uniform(0.05, 0.9, sc.n)
        hi = rng.random(sc.n) < 0.2
        op[hi] = rng.uniform(0.985, 1.0, hi.sum())
    sc.opac[:] = op.astype(np.float32)
    cam = sc.cams[0]
    print(f"case alpha clamp {mode}", flush=True)
    st = run_forward(sc, need_backward=True)
    ref, _ = image_parity(sc, cam, st)
    g_rgb, g_d = synth.upstream_grads([cam], 35)
    g_rgb, g_d = g_rgb[0], g_d[0]
    g_rgb[:, ref["amb"]] = 0
    g_d[ref["amb"]] = 0
    grads, d_pose = render_backward(st, torch.from_numpy(g_rgb.reshape(-1)).cuda(),
                                    torch.from_numpy(g_d.reshape(-1)).cuda())
    gref = oracle.backward(sc, cam, g_rgb, g_d)
    for name in ("means", "scales", "quats", "opac", "sh"):
        grad_parity(grads[0][name].cpu().numpy(), gref[name], name)
    grad_parity(d_pose.cpu().numpy()[0], gref["pose"], "pose")


def test_clamp_flag_changes_no_other_pixel():
    """The forward's clamp-free evaluation (no pair can reach the 0.99 clamp in
    its tile rectangle) gives the clamping evaluation's bits: one opaque
    Gaussian confined to the first tile switches the whole call to clamping, and
    every pixel outside that tile keeps its value, bit for bit."""
    sc = synth.tiny_scene(3000, 160, 120, 36, sh_degree=1, pose=True, log_scale_mu=-2.7)
    cam = sc.cams[0]
    a = run_forward(sc)
    # a 1 mm Gaussian of opacity 1 on pixel (4, 4), 1 m ahead of the camera
    z = 1.0
    xc = np.array([(4.0 - cam.cx) / cam.fx * z, (4.0 - cam.cy) / cam.fy * z, z])
    R, t = cam.Tcw[:, :3].astype(np.float64), cam.Tcw[:, 3].astype(np.float64)
    xw = R.T @ (xc - t)
    extra = synth.Scene(np.concatenate([sc.means, xw[None].astype(np.float32)]),
                        np.concatenate([sc.scales, np.full((1, 3), 1e-3, np.float32)]),
                        np.concatenate([sc.quats, np.array([[1, 0, 0, 0]], np.float32)]),
                        np.concatenate([sc.opac, np.ones(1, np.float32)]),
                        np.concatenate([sc.sh, np.ones((1,) + sc.sh.shape[1:], np.float32)]),
                        sc.sh_degree, sc.cams, "tiny_plus_opaque")
    b = run_forward(extra)
    outside = np.ones((cam.H, cam.W), bool)
    outside[:16, :16] = False
    for x, y in zip((a.rgb, a.depth, a.T), (b.rgb, b.depth, b.T)):
        x = x.cpu().numpy().reshape(-1, cam.H, cam.W)
        y = y.cpu().numpy().reshape(-1, cam.H, cam.W)
        assert np.array_equal(x[:, outside], y[:, outside])
        assert not np.array_equal(x[:, ~outside], y[:, ~outside])  # the opaque Gaussian shows


def test_split_forward_equals_unsplit(monkeypatch):
    """The forward's split mode (one wave per 8x8 quadrant, taken automatically
    by calls with few bins) gives the unsplit kernel's bits: images,
    transmittance, depth and last contributors of a multi-view call."""
    sc = synth.cfg3_room_window(n=20_000, n_views=3, W=320, H=180, f=160.0)
    outs = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("MGS_BLEND_SPLIT", mode)
        st = run_forward(sc, need_backward=True)
        nc = st.ws.view(st.info.off_n_contrib, int(st.info.n_pixels), torch.int32)
        outs[mode] = [x.cpu().numpy().copy() for x in (st.rgb, st.depth, st.T, nc)]
    for a, b in zip(outs["0"], outs["1"]):
        assert np.array_equal(a, b)


def _needle_scene(seed, n=4000, W=200, H=150):
    """Gaussians from round to needle-thin (one axis up to 40x longer, another
    up to 10x shorter), opacities up to 0.99, several views in one call."""
    import dataclasses
    sc = synth.tiny_scene(n, W, H, seed, sh_degree=1, log_scale_mu=-3.2, opac_max=0.99)
    rng = np.random.default_rng(seed + 100)
    s = sc.scales.copy()
    idx = np.arange(n)
    s[idx, rng.integers(0, 3, n)] *= np.exp(rng.uniform(0.0, np.log(40.0), n))
    s[idx, rng.integers(0, 3, n)] *= np.exp(-rng.uniform(0.0, np.log(10.0), n))
    cams = [sc.cams[0]]
    for k in range(2):  # two more poses, turned a little about the camera axis
        a = 0.3 * (k + 1)
        R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]], np.float32)
        T = sc.cams[0].Tcw.copy()
        T[:, :3] = R @ T[:, :3]
        T[:, 3] = R @ T[:, 3]
        cams.append(dataclasses.replace(sc.cams[0], Tcw=T))
    return dataclasses.replace(sc, scales=s.astype(np.float32), cams=cams)


@pytest.mark.parametrize("bins,split", [("1x1", "0"), ("2x1", "0"), ("1x1", "1"), ("2x2", "0")])
def test_row_culling_equals_box_culling(bins, split, monkeypatch):
    """Quadrant culling at staging by the ellipse's interval per quadrant row
    gives the bits of the per-quadrant edge test (MGS_QUAD_CULL=box): images,
    depth, transmittance and last contributors, and the gradients, on scenes of
    needle-thin and round Gaussians.  Both tests are conservative, so any
    quadrant the row test dropped wrongly would change a pixel."""
    monkeypatch.setenv("MGS_BIN_TILES", bins)
    monkeypatch.setenv("MGS_BLEND_SPLIT", split)
    for seed in (3, 4):
        sc = _needle_scene(seed)
        print(f"case row culling bins={bins} split={split} seed={seed}", flush=True)
        g_rgb, g_d = synth.upstream_grads(sc.cams, seed)
        G = torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_rgb])).cuda()
        Gd = torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_d])).cuda()
        out = {}
        for cull in ("rows", "box"):
            if cull == "box":
                monkeypatch.setenv("MGS_QUAD_CULL", "box")
            else:
                monkeypatch.delenv("MGS_QUAD_CULL", raising=False)
            st = run_forward(sc, need_backward=True)
            nc = st.ws.view(st.info.off_n_contrib, int(st.info.n_pixels), torch.int32)
            img = [x.cpu().numpy().copy() for x in (st.rgb, st.depth, st.T, nc)]
            grads, d_pose = render_backward(st, G, Gd)
            gr = {k: v.cpu().numpy().copy() for k, v in grads[0].items()}
            out[cull] = (img, gr)
        for a, b in zip(out["rows"][0], out["box"][0]):
            assert np.array_equal(a, b)
        for k in out["rows"][1]:
            # equal values (the row test may evaluate an extra quadrant that
            # blends nothing: its zero terms leave every sum as it is)
            assert np.array_equal(out["rows"][1][k], out["box"][1][k]), k


def test_split_backward_matches_unsplit(monkeypatch):
    """The backward's split mode (four waves per bin, one per quadrant) against
    the one-wave kernel on a multi-view call: the same gradients up to the
    grouping of the sums (within 1e-5 of the largest entry), and deterministic."""
    sc = synth.cfg3_room_window(n=20_000, n_views=3, W=320, H=180, f=160.0)
    g_rgb, g_d = synth.upstream_grads(sc.cams, 5)
    G = torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_rgb])).cuda()
    Gd = torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_d])).cuda()
    res = {}
    for mode in ("0", "1", "1"):
        monkeypatch.setenv("MGS_BLEND_SPLIT", mode)
        st = run_forward(sc, need_backward=True)
        grads, d_pose = render_backward(st, G, Gd)
        cur = {k: v.cpu().numpy().copy() for k, v in grads[0].items()}
        cur["pose"] = d_pose.cpu().numpy().copy()
        if mode in res:
            for k in cur:
                assert np.array_equal(cur[k], res[mode][k]), k  # deterministic
        res[mode] = cur
    for k in res["0"]:
        a, b = res["0"][k], res["1"][k]
        scale = max(float(np.abs(a).max(initial=0.0)), 1e-30)
        assert np.abs(a - b).max(initial=0.0) <= 1e-5 * scale, (k, np.abs(a - b).max(), scale)


def test_backward_is_deterministic():
    sc = synth.tiny_scene(3000, 160, 120, 34, sh_degree=1, pose=True)
    st = run_forward(sc, need_backward=True)
    g = torch.randn(st.rgb.numel(), device="cuda")
    a, pa = render_backward(st, g)
    b, pb = render_backward(st, g)
    for k in a[0]:
        assert torch.equal(a[0][k], b[0][k]), k
    assert torch.equal(pa, pb)


def test_multiview_one_launch_matches_per_view_oracle():
    sc = synth.cfg3_room_window(n=20_000, n_views=3, W=320, H=180, f=160.0)
    print("case multiview", flush=True)
    st = run_forward(sc, need_backward=True)
    for v, cam in enumerate(sc.cams):
        assert_keys_and_lists(sc, cam, st, v)
        image_parity(sc, cam, st, v)
    g_rgb, g_d = synth.upstream_grads(sc.cams, 3)
    refs = [oracle.forward(sc, c) for c in sc.cams]
    for v in range(3):
        g_rgb[v][:, refs[v]["amb"]] = 0
        g_d[v][refs[v]["amb"]] = 0
    grads, d_pose = render_backward(st, torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_rgb])).cuda(),
                                    torch.from_numpy(np.concatenate([g.reshape(-1) for g in g_d])).cuda())
    tot = None
    for v, cam in enumerate(sc.cams):
        gr = oracle.backward(sc, cam, g_rgb[v], g_d[v])
        grad_parity(d_pose.cpu().numpy()[v], gr["pose"], f"pose view {v}")
        tot = gr if tot is None else {k: tot[k] + gr[k] for k in tot}
    for name in ("means", "scales", "quats", "opac", "sh"):
        grad_parity(grads[0][name].cpu().numpy(), tot[name], name)


def test_mixed_maps_and_resolutions_equal_alone():
    a = synth.tiny_scene(1500, 120, 90, 41, sh_degree=0, pose=True)
    b = synth.tiny_scene(2500, 200, 64, 42, sh_degree=2, pose=True)
    ma, mb = GaussianMap.from_numpy(a), GaussianMap.from_numpy(b)
    va, vb = View.from_camera(a.cams[0], 0), View.from_camera(b.cams[0], 1)
    mixed = render_forward([ma, mb], [vb, va, vb])
    alone_a = render_forward([ma], [View.from_camera(a.cams[0], 0)])
    alone_b = render_forward([mb], [View.from_camera(b.cams[0], 0)])
    torch.cuda.synchronize()
    for v, ref in ((0, alone_b), (1, alone_a), (2, alone_b)):
        for x, y in zip(mixed.view_images(v), ref.view_images(0)):
            assert torch.equal(x, y)


@pytest.mark.parametrize("n_maps,n_views", [(8, 16), (9, 18), (2, 17)])
def test_many_maps_and_views_equal_alone(n_maps, n_views):
    """Calls up to 16 views and 8 maps carry their tables in kernel arguments,
    larger ones copy them: both give every view exactly its one-view image."""
    print(f"case {n_maps} maps, {n_views} views", flush=True)
    scenes = [synth.tiny_scene(400 + 50 * k, 64 + 8 * (k % 3), 48, 300 + k, sh_degree=k % 2, pose=True)
              for k in range(n_maps)]
    maps = [GaussianMap.from_numpy(sc) for sc in scenes]
    views = [View.from_camera(scenes[v % n_maps].cams[0], v % n_maps) for v in range(n_views)]
    mixed = render_forward(maps, views)
    alone = [render_forward([maps[k]], [View.from_camera(scenes[k].cams[0], 0)]) for k in range(n_maps)]
    torch.cuda.synchronize()
    for v in range(n_views):
        for x, y in zip(mixed.view_images(v), alone[v % n_maps].view_images(0)):
            assert torch.equal(x, y), (n_maps, n_views, v)


def test_edge_cases():
    # empty map: background everywhere
    sc = synth.tiny_scene(5, 40, 30, 43)
    empty = sc.subset(np.arange(0))
    st = run_forward(empty, cams=sc.cams, bg=(0.25, 0.5, 0.75, 2.0))
    rgb, depth, T = (x.cpu().numpy() for x in st.view_images(0))
    assert np.all(rgb[0] == 0.25) and np.all(rgb[2] == 0.75) and np.all(depth == 2.0) and np.all(T == 1.0)
    # 1x1 image and a camera facing away (everything culled)
    for W, H, flip in ((1, 1, False), (17, 33, True)):
        sc = synth.tiny_scene(50, W, H, 44, f=30.0)
        if flip:  # rotate the camera by 180 degrees about its x axis: everything is behind it
            sc.cams[0].Tcw = (np.diag([1.0, -1.0, -1.0]) @ sc.cams[0].Tcw).astype(np.float32)
        st = run_forward(sc)
        assert_keys_and_lists(sc, sc.cams[0], st)
        image_parity(sc, sc.cams[0], st, max_amb_frac=1.0)
    # one huge Gaussian covering every tile, with degenerate ones mixed in
    sc = synth.tiny_scene(30, 100, 80, 45)
    sc.scales[0] = [2.0, 2.0, 2.0]
    sc.quats[1] = 0.0
    sc.scales[2, 0] = 0.0
    sc.opac[3] = np.nan
    st = run_forward(sc)
    assert_keys_and_lists(sc, sc.cams[0], st)
    image_parity(sc, sc.cams[0], st)


@pytest.mark.parametrize("bins", ["1x1", "2x1"])
def test_tall_view_ranks_over_several_emission_chunks(bins, monkeypatch):
    """A 96x1400 view (88 tile rows) with a few Gaussians that cover it all:
    their (rank, bin row) items outnumber a wave's 64, so the emission carries
    a rank's written count over several chunks.  Keys, lists and image against
    the oracle."""
    monkeypatch.setenv("MGS_BIN_TILES", bins)
    sc = synth.tiny_scene(400, 96, 1400, 49, sh_degree=0, f=200.0)
    sc.scales[:4] = 2.0
    print(f"case tall view bins={bins}", flush=True)
    st = run_forward(sc)
    assert (int(st.info.bin_tx), int(st.info.bin_ty)) == ((2, 1) if bins == "2x1" else (1, 1))
    assert_keys_and_lists(sc, sc.cams[0], st)
    image_parity(sc, sc.cams[0], st)



@pytest.mark.parametrize("n", [16383, 16400])
def test_depth_sort_long_runs_of_equal_keys(n):
    """Every Gaussian visible, at 50 shared depths: long runs of equal depth
    keys, whose order within a run is the stable pair order, across the
    depth sort's per-wave ranking rounds (the last wave ragged).  Keys, lists
    and image against the oracle."""
    rng = np.random.default_rng(n)
    W, H, f = 160, 120, 150.0
    z = rng.choice(np.linspace(1.0, 6.0, 50), n)
    xr = rng.uniform(-0.8, 0.8, n) * (W / 2) / f
    yr = rng.uniform(-0.8, 0.8, n) * (H / 2) / f
    means = np.stack([xr * z, yr * z, z], axis=1).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(3e-3), np.log(2e-2), size=(n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    opac = rng.uniform(0.2, 0.9, n).astype(np.float32)
    sh = rng.uniform(-1, 1, size=(n, 1, 3)).astype(np.float32)
    Tcw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)
    cam = synth.Camera(W, H, f, f, (W - 1) / 2.0, (H - 1) / 2.0, Tcw)
    sc = synth.Scene(means, scales, q, opac, sh, 0, [cam], f"equal_depths{n}")
    print(f"case equal depth runs n={n}", flush=True)
    st = run_forward(sc)
    assert int(st.info.n_visible) == n
    assert_keys_and_lists(sc, sc.cams[0], st)
    image_parity(sc, sc.cams[0], st)


def test_stage_events_recorded_on_the_stream():
    """Caller events at the stage boundaries: ordered, and the forward's add up
    to its whole call (no waits inside the library)."""
    sc = synth.cfg1_plain_forward()
    m = GaussianMap.from_numpy(sc)
    views = [View.from_camera(c) for c in sc.cams]
    ef = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    eb = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    st = render_forward([m], views, need_backward=True, events=ef)
    npx = sc.cams[0].W * sc.cams[0].H
    render_backward(st, torch.ones(3 * npx, device="cuda"), torch.ones(npx, device="cuda"), events=eb)
    torch.cuda.synchronize()
    f = [ef[i].elapsed_time(ef[i + 1]) for i in range(3)]
    b = [eb[i].elapsed_time(eb[i + 1]) for i in range(2)]
    assert all(x >= 0 for x in f + b) and f[2] > 0 and b[0] > 0
    assert abs(sum(f) - ef[0].elapsed_time(ef[3])) < 1e-2
    assert ef[3].elapsed_time(eb[0]) >= 0


@pytest.mark.parametrize("bins", ["2x1", "2x2"])
def test_larger_list_bins(bins, monkeypatch):
    """Lists per bin of 2x1 or 2x2 tiles: the same keys, ordered subset lists,
    images and gradients as the oracle."""
    monkeypatch.setenv("MGS_BIN_TILES", bins)
    sc = synth.tiny_scene(3000, 200, 150, 47, sh_degree=1, pose=True, log_scale_mu=-2.5)
    cam = sc.cams[0]
    st = run_forward(sc, need_backward=True)
    assert (int(st.info.bin_tx), int(st.info.bin_ty)) == tuple(int(c) for c in bins.split("x"))
    assert_keys_and_lists(sc, cam, st)
    ref, _ = image_parity(sc, cam, st)
    g_rgb, g_d = synth.upstream_grads([cam], 9)
    g_rgb[0][:, ref["amb"]] = 0
    g_d[0][ref["amb"]] = 0
    grads, d_pose = render_backward(st, torch.from_numpy(g_rgb[0].reshape(-1)).cuda(),
                                    torch.from_numpy(g_d[0].reshape(-1)).cuda())
    gref = oracle.backward(sc, cam, g_rgb[0], g_d[0])
    for name in ("means", "scales", "quats", "opac", "sh"):
        grad_parity(grads[0][name].cpu().numpy(), gref[name], name)
    grad_parity(d_pose.cpu().numpy()[0], gref["pose"], "pose")


@pytest.mark.parametrize("bins,size", [("1x1", "small"), ("2x2", "small"), ("1x1", "large")])
def test_wide_and_packed_instances_agree(bins, size, monkeypatch):
    """The packed instance keys (bin, rank and record slot in one word) and the
    wide ones ((bin, rank) keys with the slot as the sort's value) give the
    same lists, images and gradients, bit for bit.  The large case (500k
    Gaussians, 3 views at 1200x680, about 3M instances) runs the tile sort in
    its large-input blocks."""
    monkeypatch.setenv("MGS_BIN_TILES", bins)
    if size == "small":
        sc = synth.cfg3_room_window(n=20_000, n_views=3, W=320, H=180, f=160.0)
    else:
        sc = synth.cfg3_room_window(n=500_000, n_views=3)
    print(f"case wide/packed bins={bins} size={size}", flush=True)
    g = None
    out = {}
    for wide in ("0", "1"):
        monkeypatch.setenv("MGS_WIDE_INSTANCES", wide)
        st = run_forward(sc, need_backward=True)
        kb = int(st.info.inst_bin_bits)
        assert (kb == 0) == (wide == "1"), kb
        if g is None:
            g = torch.randn(st.rgb.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(4))
        grads, d_pose = render_backward(st, g)
        torch.cuda.synchronize()
        out[wide] = (_inst_lists(st), st.rgb.clone(), st.depth.clone(), grads, d_pose)
    if size == "large":
        assert int(st.info.n_instances) >= 1 << 21, int(st.info.n_instances)
    (bp, pp), rgb_p, d_p, gr_p, pose_p = out["0"]
    (bw, pw), rgb_w, d_w, gr_w, pose_w = out["1"]
    assert np.array_equal(bp, bw) and np.array_equal(pp, pw)
    assert torch.equal(rgb_p, rgb_w) and torch.equal(d_p, d_w)
    for k in gr_p[0]:
        assert torch.equal(gr_p[0][k], gr_w[0][k]), k
    assert torch.equal(pose_p, pose_w)
