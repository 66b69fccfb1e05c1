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


def _inst_lists(st):
    """(bin, pair) of every sorted instance, from either instance key format."""
    info = st.info
    M = int(info.n_instances)
    key = st.ws.view(info.off_inst_key, 2 * M, torch.int32).cpu().numpy().view(np.uint64)
    rank_pair = st.ws.view(info.off_rank_pair, int(info.n_visible), torch.int32).cpu().numpy().view(np.uint32)
    tb, rb = int(info.inst_bin_bits), int(info.inst_rank_bits)
    if tb > 0:
        bins = (key & np.uint64((1 << tb) - 1)).astype(np.int64)
        ranks = ((key >> np.uint64(tb)) & np.uint64((1 << rb) - 1)).astype(np.int64)
    else:
        bins = (key >> np.uint64(32)).astype(np.int64)
        ranks = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
    return bins, rank_pair[ranks].astype(np.int64)


def _bins_of(V, info):
    TX, TY = (V.W + 15) // 16, (V.H + 15) // 16
    btx, bty = int(info.bin_tx), int(info.bin_ty)
    BX, BY = (TX + btx - 1) // btx, (TY + bty - 1) // bty
    return btx, bty, BX, BY


def _view_bases(st, v):
    base = sum(st.maps[st.views[u].map].n for u in range(v))
    bin_base = 0
    for u in range(v):
        _, _, BX, BY = _bins_of(st.views[u], st.info)
        bin_base += BX * BY
    return base, bin_base


def gpu_keys(st, v=0):
    """Key-path outputs of view v: depth bits, rects, uvr, and the (bin, gid) lists."""
    info = st.info
    V = st.views[v]
    P = int(info.n_pairs)
    n_map = st.maps[V.map].n
    base, bin_base = _view_bases(st, v)
    depth = st.ws.view(info.off_pair_depth, P, torch.int32).cpu().numpy().view(np.uint32)[base:base + n_map]
    rect = st.ws.view(info.off_pair_rect, 4 * P, torch.int16).cpu().numpy().view(np.uint16)
    rect = rect.reshape(P, 4)[base:base + n_map].astype(np.int32)
    uvr = st.ws.view(info.off_pair_uvr, 4 * P, torch.float32).cpu().numpy().reshape(P, 4)[base:base + n_map]
    bins, pairs = _inst_lists(st)
    _, _, BX, BY = _bins_of(V, info)
    sel = (bins >= bin_base) & (bins < bin_base + BX * BY)
    return dict(depth=depth, rect=rect, uvr=uvr, bins=bins[sel] - bin_base, gids=pairs[sel] - base)


def oracle_tile_pairs(k):
    """Oracle tile lists flattened to (tile, gid) in tile order."""
    counts = np.diff(k["tile_off"])
    return np.repeat(np.arange(len(counts)), counts), k["tile_gid"].astype(np.int64)


def max_alpha_in_tiles(pv, opac, gids, tiles, TX, W, H):
    """fp64 maximum of o exp(power) over the pixel centres of each (Gaussian,
    tile) pair: the concave exponent's maximum over the tile's pixel box (0 when
    the mean lies inside, else on an edge at the clamped stationary point)."""
    u, v = pv[gids, 0], pv[gids, 1]
    A, B, C = pv[gids, 2], pv[gids, 3], pv[gids, 4]
    tx, ty = tiles % TX, tiles // TX
    x0, y0 = 16.0 * tx, 16.0 * ty
    x1, y1 = np.minimum(x0 + 15, W - 1), np.minimum(y0 + 15, H - 1)
    dxl, dxh, dyl, dyh = u - x1, u - x0, v - y1, v - y0

    def pw(dx, dy):
        return -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy

    best = np.full(len(gids), -np.inf)
    for dx in (dxl, dxh):
        best = np.maximum(best, pw(dx, np.clip(-B * dx / C, dyl, dyh)))
    for dy in (dyl, dyh):
        best = np.maximum(best, pw(np.clip(-B * dy / A, dxl, dxh), dy))
    inside = (dxl <= 0) & (dxh >= 0) & (dyl <= 0) & (dyh >= 0)
    best = np.where(inside, 0.0, best)
    return opac[gids].astype(np.float64) * np.exp(best)


def oracle_bin_lists(k, info):
    """The oracle's tile lists gathered into the GPU's list bins: per bin, the
    union of its tiles' Gaussians in the oracle's depth order (depth key, then
    index).  Returns (bin, gid) pairs in bin order and, per oracle tile entry,
    its bin."""
    ot, og = oracle_tile_pairs(k)
    btx, bty = int(info.bin_tx), int(info.bin_ty)
    TX = k["TX"]
    BX = (TX + btx - 1) // btx
    obin = (ot // TX // bty) * BX + (ot % TX) // btx
    depth = k["depth_bits"].astype(np.int64)
    order = np.lexsort((og, depth[og], obin))
    pb, pg = obin[order], og[order]
    keep = np.ones(len(pb), bool)
    keep[1:] = (pb[1:] != pb[:-1]) | (pg[1:] != pg[:-1])
    return pb[keep], pg[keep], ot, og, obin


def assert_keys_and_lists(scene, cam, st, v=0):
    """Depth keys, tile rectangles and image means bit-exact; each GPU list (one
    per bin of bin_tx x bin_ty tiles) is the union of the oracle's tile lists of
    that bin, in the same depth order, less entries whose Gaussian reaches
    alpha < 1/255 at every pixel of every one of its tiles in the bin (checked
    in fp64)."""
    k = oracle.keys(scene, cam)
    g = gpu_keys(st, v)
    exp_depth = np.where(k["valid"], k["depth_bits"], np.uint32(0xFFFFFFFF))
    assert np.array_equal(g["depth"], exp_depth), "depth keys differ"
    assert np.array_equal(g["rect"][k["valid"]], k["rect"][k["valid"]]), "tile rectangles differ"
    assert np.array_equal(g["uvr"][k["valid"], :3].view(np.uint32), k["uvr"][k["valid"]].view(np.uint32)), \
        "image means / radii differ"
    pb, pg, ot, og, obin = oracle_bin_lists(k, st.info)
    n = max(scene.n, 1)
    okey = pb * n + pg
    gkey = g["bins"] * n + g["gids"]
    idx = np.zeros(0, np.int64)
    if len(gkey):
        order = np.argsort(okey)
        pos = np.searchsorted(okey[order], gkey)
        assert len(okey) and np.all(pos < len(okey)), "instance outside the oracle's lists"
        idx = order[pos]
        assert np.array_equal(okey[idx], gkey), "instance outside the oracle's lists"
        assert np.all(np.diff(idx) > 0), "per-bin depth order differs from the oracle's"
    dropped = np.ones(len(okey), bool)
    dropped[idx] = False
    if dropped.any():
        # every oracle tile entry whose (bin, Gaussian) the GPU dropped
        drop_keys = np.sort(okey[dropped])
        te = obin * n + og
        sel = np.isin(te, drop_keys)
        pv = oracle.project_values(scene, cam)
        amax = max_alpha_in_tiles(pv, scene.opac, og[sel], ot[sel], k["TX"], cam.W, cam.H)
        assert np.all(amax < 1.0 / 255.0), f"dropped a reachable tile: max alpha {amax.max()}"
    return k


def last_contributor_gids(st, v, k, ref):
    """Gaussian of the last blended list entry per pixel (-1: none), GPU and oracle."""
    V = st.views[v]
    o, npx = st.pix_off[v], V.W * V.H
    nc = st.ws.view(st.info.off_n_contrib, int(st.info.n_pixels), torch.int32).cpu().numpy()[o:o + npx]
    nc = nc.reshape(V.H, V.W).astype(np.int64)
    base, bin_base = _view_bases(st, v)
    btx, bty, BX, _ = _bins_of(V, st.info)
    yy, xx = np.mgrid[0:V.H, 0:V.W]
    b = (yy // (16 * bty)) * BX + xx // (16 * btx)
    rng = st.ws.view(st.info.off_bin_range, 2 * int(st.info.n_bins), torch.int32).cpu().numpy()
    first = rng.view(np.uint32).reshape(-1, 2)[bin_base + b, 0].astype(np.int64)
    _, pairs = _inst_lists(st)
    gpu = np.where(nc > 0, pairs[np.maximum(first + nc - 1, 0)] - base, -1) if len(pairs) else np.full(nc.shape, -1)
    TX = (V.W + 15) // 16
    tile = (yy // 16) * TX + xx // 16
    onc = ref["n_contrib"].astype(np.int64)
    ofirst = k["tile_off"][tile]
    ogid = k["tile_gid"].astype(np.int64)
    orc = np.where(onc > 0, ogid[np.maximum(ofirst + onc - 1, 0)] if len(ogid) else -1, -1)
    return gpu, orc


def image_parity(scene, cam, st, v=0, bg=(0, 0, 0, 0), atol=1e-4, max_amb_frac=1e-2):
    """Every pixel is checked to atol in colour and transmittance and atol x
    max depth in depth, with the same last blended Gaussian.

    An unflagged pixel is compared with the oracle's render.  A flagged pixel
    (a skip or stop decision inside the oracle's fp32 error band, where a fp32
    renderer may decide either way) must match one of the renders that those
    decisions allow (oracle.forward_alternatives, each decision reversed or
    not), to the same bar.  max_amb_frac only bounds how many pixels take that
    route: the bands flag 0-0.8 % of the pixels of the test scenes."""
    ref = oracle.forward(scene, cam, bg=bg)
    rgb, depth, T = (x.cpu().numpy() for x in st.view_images(v))
    ok = ~ref["amb"]
    amb_frac = 1.0 - ok.mean()
    err_rgb = np.abs(rgb - ref["rgb"])[:, ok].max(initial=0.0)
    err_d = np.abs(depth - ref["depth"])[ok].max(initial=0.0)
    err_T = np.abs(T - ref["T"])[ok].max(initial=0.0)
    g_last, o_last = last_contributor_gids(st, v, oracle.keys(scene, cam), ref)
    nc_bad = int((g_last != o_last)[ok].sum())
    zmax = max(1.0, float(np.abs(ref["depth"]).max(initial=1.0)))
    # flagged pixels: the nearest allowed outcome
    ys, xs = np.nonzero(~ok)
    amb_unmatched, amb_unresolved, n_out = 0, 0, 0
    if len(xs):
        leaves, lgid, nl = oracle.forward_alternatives(scene, cam, xs, ys, bg=bg)
        amb_unresolved = int((nl < 0).sum())
        n_out = int(nl[nl > 0].sum())
        L = leaves.shape[1]
        valid = np.arange(L)[None, :] < nl[:, None]
        d_rgb = np.abs(rgb[:, ys, xs].T[:, None, :] - leaves[:, :, :3]).max(axis=2)
        d_d = np.abs(depth[ys, xs][:, None] - leaves[:, :, 3])
        d_T = np.abs(T[ys, xs][:, None] - leaves[:, :, 4])
        same = lgid == g_last[ys, xs][:, None]
        match = valid & same & (d_rgb <= atol) & (d_T <= atol) & (d_d <= atol * zmax)
        amb_unmatched = int((~match.any(axis=1) & (nl > 0)).sum())
    stats = dict(err_rgb=float(err_rgb), err_depth=float(err_d), err_T=float(err_T), amb=float(amb_frac),
                 amb_pixels=int(len(xs)), amb_outcomes=n_out, amb_unmatched=amb_unmatched,
                 amb_unresolved=amb_unresolved, nc_mismatch=nc_bad, pixels=int(ok.size))
    print("image parity", stats, flush=True)
    assert amb_frac <= max_amb_frac, f"ambiguous pixel fraction {amb_frac}"
    assert err_rgb <= atol and err_T <= atol, stats
    # depth carries z ~ metres: same absolute bound scaled by the largest depth
    assert err_d <= atol * zmax, stats
    assert nc_bad == 0, stats
    assert amb_unresolved == 0 and amb_unmatched == 0, stats
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


def merged_frame_parity(out_q, out_s, o, slots_gpu, slots_oracle, min_margin=1e-3):
    """Rotation and scales of merged Gaussians (Eq. (10)).  Where the oracle's
    frame is decided (canonical_qs_margin of every merge of the chain above
    min_margin: distinct eigenvalues and a clear nearest frame), the GPU must
    carry the same frame, to the precision its own covariance allows.  With
    E = |Sigma(q_gpu, s_gpu) - Sigma_oracle|_2 plus the fp32 rounding of storing
    q and s (4e-7 lam_max), the Davis-Kahan bound puts the GPU's axis c (column
    c of R(q)) within asin(E / gap_c) of the oracle's, gap_c = min_b |lam_c - lam_b|,
    and Weyl's bound puts s_c^2 within E of the oracle's.  Another frame (a
    permutation or sign change of the axes) is 90 or 180 degrees off on some
    axis; q is compared up to its sign through R(q).  Only slots where the bound
    is below 0.1 rad are decisive and counted.  Returns the number checked."""
    from oracle import merge as M
    checked = 0
    worst_ang, worst_s = 0.0, 0.0
    for gs, os_ in zip(slots_gpu, slots_oracle):
        if not (o.frame_margin[os_] > min_margin):
            continue
        qg = np.asarray(out_q[gs], np.float64)
        sg = np.asarray(out_s[gs], np.float64)
        Rg = M.rot(qg)
        Ro = M.rot(o.quats[os_])
        lam = np.asarray(o.scales[os_], np.float64) ** 2
        lmax = lam.max()
        E = np.linalg.norm(M.cov_of(qg, sg) - o.covs[os_], 2) + 4e-7 * lmax
        bounds = [E / min(abs(lam[c] - lam[b]) for b in range(3) if b != c) for c in range(3)]
        if max(bounds) > 0.1:
            continue
        for c in range(3):
            sin_ang = np.linalg.norm(np.cross(Rg[:, c], Ro[:, c]))
            same_dir = Rg[:, c] @ Ro[:, c] > 0
            assert same_dir and sin_ang <= 1.01 * bounds[c] + 1e-12, \
                (gs, os_, c, sin_ang, bounds[c], out_q[gs], o.quats[os_], o.frame_margin[os_])
            worst_ang = max(worst_ang, sin_ang / bounds[c])
            ds = abs(sg[c] ** 2 - lam[c])
            assert ds <= 1.01 * E, (gs, os_, c, ds, E, out_s[gs], o.scales[os_])
            worst_s = max(worst_s, ds / E)
        checked += 1
    print(f"merged frames checked {checked} of {len(slots_gpu)}, worst axis angle / bound {worst_ang:.2f}, "
          f"worst scale^2 error / bound {worst_s:.2f}", flush=True)
    return checked
