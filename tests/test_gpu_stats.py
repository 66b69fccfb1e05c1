"""GPU parity of the Eq. (3) merge-eligibility path (Sec. II-D): the gradient
statistics that mgs_render_backward accumulates and the mask mgs_merge_mask
forms from them, against the oracle.

Bars: view counts bit-exact (they follow the bit-exact key path); summed
gradient norms within the gradient bar (1e-3 relative L2 and element-wise
1e-3 |g*| + 1e-3 max|g*|, upstream gradient zeroed on ambiguous pixels); the
mask bit-exact on the same fp32 statistics (the division and the comparison
are fp32 on both sides); a second call adds exactly the same amounts
(deterministic backward).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import merge as M
from paper_2509_13536_amd import GaussianMap, GradStats, View, merge_mask, render_backward, render_forward, voxel_merge

from gpu_helpers import grad_parity, run_forward

pytestmark = pytest.mark.gpu


def _window(n=20_000, views=3):
    return synth.cfg3_room_window(n=n, n_views=views, W=320, H=180, f=160.0)


def _upstream(sc, seed):
    g_rgb, g_d = synth.upstream_grads(sc.cams, seed)
    for v, cam in enumerate(sc.cams):
        amb = oracle.forward(sc, cam)["amb"]
        g_rgb[v][:, amb] = 0
        g_d[v][amb] = 0
    flat = lambda gs: torch.from_numpy(np.concatenate([g.reshape(-1) for g in gs])).cuda()
    return g_rgb, g_d, flat(g_rgb), flat(g_d)


def test_grad_stats_match_oracle_and_accumulate():
    sc = _window()
    print("case grad stats window 20k x 3", flush=True)
    st = run_forward(sc, need_backward=True)
    g_rgb, g_d, t_rgb, t_d = _upstream(sc, 3)
    stats = GradStats.zeros(sc.n)
    render_backward(st, t_rgb, t_d, stats=[stats])
    torch.cuda.synchronize()
    s1 = stats.grad_norm_sum.cpu().numpy().copy()
    c1 = stats.visible_count.cpu().numpy().copy()
    ref_sum, ref_cnt = oracle.grad_stats(sc, sc.cams, g_rgb, g_d)
    assert np.array_equal(c1, ref_cnt), "view counts differ"
    assert (ref_cnt == 0).any() and (ref_cnt == 3).any() and ((ref_cnt == 1) | (ref_cnt == 2)).any()
    grad_parity(s1, ref_sum, "grad_norm_sum")
    # a second call accumulates the same amounts
    render_backward(st, t_rgb, t_d, stats=[stats], want=())
    torch.cuda.synchronize()
    assert np.array_equal(stats.grad_norm_sum.cpu().numpy(), s1 + s1)
    assert np.array_equal(stats.visible_count.cpu().numpy(), 2 * c1)


def test_grad_stats_per_map_equal_alone():
    a = synth.tiny_scene(1500, 120, 90, 41, sh_degree=0, pose=True)
    b = synth.tiny_scene(2500, 200, 64, 42, sh_degree=2, pose=True)
    ma, mb = GaussianMap.from_numpy(a), GaussianMap.from_numpy(b)
    mixed = render_forward([ma, mb], [View.from_camera(b.cams[0], 1), View.from_camera(a.cams[0], 0)],
                           need_backward=True)
    alone = render_forward([ma], [View.from_camera(a.cams[0], 0)], need_backward=True)
    ga = torch.randn(3 * 120 * 90, device="cuda")
    gb = torch.randn(3 * 200 * 64, device="cuda")
    sm = [GradStats.zeros(a.n), GradStats.zeros(b.n)]
    render_backward(mixed, torch.cat([gb, ga]), stats=sm)
    sa = GradStats.zeros(a.n)
    render_backward(alone, ga, stats=[sa])
    torch.cuda.synchronize()
    assert torch.equal(sm[0].grad_norm_sum, sa.grad_norm_sum)
    assert torch.equal(sm[0].visible_count, sa.visible_count)
    assert int(sm[1].visible_count.sum()) > 0


def test_merge_mask_bit_exact():
    rng = np.random.default_rng(8)
    n = 100_003
    tau = np.float32(1e-3)
    count = rng.integers(0, 6, n).astype(np.int32)
    gsum = (rng.uniform(0, 2.5e-3, n) * np.maximum(count, 1)).astype(np.float32)
    ties = rng.choice(n, 500, replace=False)
    count[ties] = 4
    gsum[ties] = 4 * tau  # average exactly tau: not below it
    kf = rng.integers(0, 12, n).astype(np.int32)
    st = GradStats(torch.from_numpy(gsum).cuda(), torch.from_numpy(count).cuda())
    for kf_arg, lo, hi in ((None, 0, 0), (kf, 3, 8), (kf, 5, 5)):
        got = merge_mask(st, float(tau), None if kf_arg is None else torch.from_numpy(kf_arg).cuda(), lo, hi)
        want = M.merge_mask(gsum, count, tau, kf_index=kf_arg, kf_min=lo, kf_max=hi)
        assert np.array_equal(got.cpu().numpy(), want)
    assert want.any() and not want[ties].any()
    empty = GradStats.zeros(0)
    assert merge_mask(empty).numel() == 0


def test_stats_mask_feed_the_merge():
    sc = _window(n=20_000, views=2)
    print("case stats -> mask -> merge", flush=True)
    st = run_forward(sc, need_backward=True)
    _, _, t_rgb, t_d = _upstream(sc, 4)
    stats = GradStats.zeros(sc.n)
    render_backward(st, t_rgb, t_d, stats=[stats], want=())
    cnt = stats.visible_count.cpu().numpy()
    gsum = stats.grad_norm_sum.cpu().numpy()
    seen = cnt > 0
    tau = float(np.median(gsum[seen] / cnt[seen]))
    mask = merge_mask(stats, tau)
    want = M.merge_mask(gsum, cnt, tau)
    assert np.array_equal(mask.cpu().numpy(), want)
    assert 0 < want.sum() < sc.n
    m = GaussianMap.from_numpy(sc)
    res = voxel_merge(m, mask=mask, voxel_size=0.05)
    o = M.voxel_merge(sc.means, sc.quats, sc.scales, 0.05, eligible=want.astype(bool))
    alive = res.old_to_new.cpu().numpy() >= 0
    cells, ok = M.voxel_cells(sc.means, 0.05, want.astype(bool))
    flagged = np.array([ok[g] and tuple(cells[g]) in o.flagged for g in range(sc.n)])
    assert np.all(alive[want == 0])
    assert (alive != o.alive)[~flagged].sum() == 0
    assert (~o.alive).sum() > 0
