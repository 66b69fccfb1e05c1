"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and read its forward state; comparison utilities.  Expected values always come
from the oracle."""
import numpy as np
import torch

import oracle
from paper_2509_13536_amd import GaussianMap, View, render_backward, render_forward


def run_forward(scene, cams=None, bg=(0, 0, 0, 0), need_backward=False, maps=None, views=None):
    cams = scene.cams if cams is None else cams
    maps = [GaussianMap.from_numpy(scene)] if maps is None else maps
    views = [View.from_camera(c) for c in cams] if views is None else views
    st = render_forward(maps, views, bg=bg, need_backward=need_backward)
    torch.cuda.synchronize()
    return st


def gpu_keys(st, v=0):
    """Key-path outputs of view v: depth bits, rects, uvr, and the (tile, gid) list."""
    info = st.info
    V = st.views[v]
    P = int(info.n_pairs)
    n_map = st.maps[V.map].n
    base = sum(st.maps[st.views[u].map].n for u in range(v))
    depth = st.ws.view(info.off_pair_depth, P, torch.int32).cpu().numpy().view(np.uint32)[base:base + n_map]
    rect = st.ws.view(info.off_pair_rect, 4 * P, torch.int16).cpu().numpy().view(np.uint16)
    rect = rect.reshape(P, 4)[base:base + n_map].astype(np.int32)
    uvr = st.ws.view(info.off_pair_uvr, 4 * P, torch.float32).cpu().numpy().reshape(P, 4)[base:base + n_map]
    M = int(info.n_instances)
    tiles = st.ws.view(info.off_inst_tile, M, torch.int32).cpu().numpy().view(np.uint32)
    ranks = st.ws.view(info.off_inst_rank, M, torch.int32).cpu().numpy().view(np.uint32)
    rank_pair = st.ws.view(info.off_rank_pair, int(info.n_visible), torch.int32).cpu().numpy().view(np.uint32)
    pairs = rank_pair[ranks].astype(np.int64)
    tile_base = sum(((st.views[u].W + 15) // 16) * ((st.views[u].H + 15) // 16) for u in range(v))
    ntile = ((V.W + 15) // 16) * ((V.H + 15) // 16)
    sel = (tiles >= tile_base) & (tiles < tile_base + ntile)
    return dict(depth=depth, rect=rect, uvr=uvr, tiles=tiles[sel].astype(np.int64) - tile_base,
                gids=pairs[sel] - base)


def oracle_tile_pairs(k):
    """Oracle tile lists flattened to (tile, gid) in tile order."""
    counts = np.diff(k["tile_off"])
    return np.repeat(np.arange(len(counts)), counts), k["tile_gid"].astype(np.int64)


def assert_keys_bit_exact(scene, cam, st, v=0):
    k = oracle.keys(scene, cam)
    g = gpu_keys(st, v)
    exp_depth = np.where(k["valid"], k["depth_bits"], np.uint32(0xFFFFFFFF))
    assert np.array_equal(g["depth"], exp_depth), "depth keys differ"
    assert np.array_equal(g["rect"][k["valid"]], k["rect"][k["valid"]]), "tile rectangles differ"
    assert np.array_equal(g["uvr"][k["valid"], :3].view(np.uint32), k["uvr"][k["valid"]].view(np.uint32)), \
        "image means / radii differ"
    ot, og = oracle_tile_pairs(k)
    assert len(g["tiles"]) == len(ot) == k["M"], (len(g["tiles"]), k["M"])
    assert np.array_equal(g["tiles"], ot), "sorted tile ids differ"
    assert np.array_equal(g["gids"], og), "per-tile depth order differs"
    return k


def gpu_n_contrib(st, v=0):
    V = st.views[v]
    o, n = st.pix_off[v], V.W * V.H
    nc = st.ws.view(st.info.off_n_contrib, int(st.info.n_pixels), torch.int32).cpu().numpy()
    return nc[o:o + n].reshape(V.H, V.W)


def image_parity(scene, cam, st, v=0, bg=(0, 0, 0, 0), atol=1e-4, max_amb_frac=2e-2, amb_atol=0.05):
    """Non-ambiguous pixels: colour and transmittance within atol, depth within
    atol * max depth, and the same last-contributor position.  Ambiguous pixels
    (a decision within the oracle's error-model band): within amb_atol, the size
    of a single skip decision flipping (alpha 1/255 times colour)."""
    ref = oracle.forward(scene, cam, bg=bg)
    rgb, depth, T = (x.cpu().numpy() for x in st.view_images(v))
    ok = ~ref["amb"]
    amb_frac = 1.0 - ok.mean()
    err_rgb = np.abs(rgb - ref["rgb"])[:, ok].max(initial=0.0)
    err_d = np.abs(depth - ref["depth"])[ok].max(initial=0.0)
    err_T = np.abs(T - ref["T"])[ok].max(initial=0.0)
    err_amb = np.abs(rgb - ref["rgb"])[:, ~ok].max(initial=0.0)
    nc_bad = int((gpu_n_contrib(st, v) != ref["n_contrib"])[ok].sum())
    zmax = max(1.0, float(np.abs(ref["depth"]).max(initial=1.0)))
    stats = dict(err_rgb=float(err_rgb), err_depth=float(err_d), err_T=float(err_T), amb=float(amb_frac),
                 err_amb=float(err_amb), nc_mismatch=nc_bad, pixels=int(ok.size))
    print("image parity", stats, flush=True)
    assert amb_frac <= max_amb_frac, f"ambiguous pixel fraction {amb_frac}"
    assert err_rgb <= atol and err_T <= atol, stats
    # depth carries z ~ metres: same absolute bound scaled by the largest depth
    assert err_d <= atol * zmax, stats
    assert nc_bad == 0, stats
    assert err_amb <= amb_atol, stats
    return ref, stats


def grad_parity(got: np.ndarray, ref: np.ndarray, name: str, rel_l2=1e-3, elem=1e-3):
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nref = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / max(nref, 1e-300)
    assert rel <= rel_l2, f"{name}: relative L2 error {rel}"
    bound = elem * np.abs(ref) + elem * np.abs(ref).max(initial=0.0)
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{name}: {bad.sum()} elements outside tolerance, worst {np.abs(got - ref)[bad].max()}"
    return rel
