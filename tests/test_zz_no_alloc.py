"""The allocation-free mapping loss (mgs_mapping_loss_noalloc), called through
the C ABI, against mgs_mapping_loss with a workspace on the same inputs: two
calls in a row, the second on a smaller input, each bit-identical to the
workspace entry point (the same kernels, deterministic reductions); and an
input beyond the fixed scratch refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2509_13536_amd import _abi

pytestmark = pytest.mark.gpu


def _inputs(sizes, seed, n_gauss):
    g = torch.Generator().manual_seed(seed)
    npix = sum(w * h for w, h in sizes)
    rgb = torch.rand(3 * npix, generator=g)
    gt = torch.rand(3 * npix, generator=g)
    gt[::7] = rgb[::7]  # equal pixels: the L1 subgradient at 0
    depth = torch.rand(npix, generator=g) * 3 + 0.5
    gtd = torch.rand(npix, generator=g) * 3 + 0.5
    gtd[::5] = 0.0  # missing depth
    scales = torch.exp(torch.randn(n_gauss, 3, generator=g) * 0.5 - 3.5)
    return [t.cuda() for t in (rgb, gt, depth, gtd, scales)]


def _outputs(sizes, n_gauss):
    npix = sum(w * h for w, h in sizes)
    return [torch.full((n,), float("nan"), device="cuda")
            for n in (4 * len(sizes) + 2, 3 * npix, npix, 3 * n_gauss)]


def _p(t):
    return C.c_void_p(t.data_ptr())


def _call_ws(lib, sizes, ins, outs, opts, stream):
    sz = (C.c_int32 * (2 * len(sizes)))(*[x for wh in sizes for x in wh])
    req = C.c_size_t(0)
    st = lib.mgs_mapping_loss(sz, len(sizes), *map(_p, ins[:4]), _p(ins[4]), ins[4].shape[0], C.byref(opts),
                              None, 0, C.byref(req), *map(_p, outs), stream)
    assert st == _abi.MGS_ERR_WORKSPACE
    ws = torch.empty(int(req.value), dtype=torch.uint8, device="cuda")
    st = lib.mgs_mapping_loss(sz, len(sizes), *map(_p, ins[:4]), _p(ins[4]), ins[4].shape[0], C.byref(opts),
                              _p(ws), ws.numel(), C.byref(req), *map(_p, outs), stream)
    assert st == _abi.MGS_OK
    return int(req.value)


def _call_noalloc(lib, sizes, ins, outs, opts, stream):
    sz = (C.c_int32 * (2 * len(sizes)))(*[x for wh in sizes for x in wh])
    req = C.c_size_t(0)
    st = lib.mgs_mapping_loss_noalloc(sz, len(sizes), *map(_p, ins[:4]), _p(ins[4]), ins[4].shape[0],
                                      C.byref(opts), C.byref(req), *map(_p, outs), stream)
    return st, int(req.value)


def test_noalloc_loss_equals_workspace_loss_twice_then_refuses_oversize():
    lib = _abi.load()
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()
    stream = C.c_void_p(s.cuda_stream)
    opts = _abi.LossOpts(0.2, 0.7, 0.3, 0)
    # first call: two views (one 1200x680 keyframe and a ragged one); second: smaller
    for sizes, seed, n_g in (([(1200, 680), (129, 70)], 1, 50_000), ([(97, 33)], 2, 1_000)):
        print(f"noalloc loss: sizes {sizes}, seed {seed}, {n_g} Gaussians", flush=True)
        ins = _inputs(sizes, seed, n_g)
        ref, got = _outputs(sizes, n_g), _outputs(sizes, n_g)
        need = _call_ws(lib, sizes, ins, ref, opts, stream)
        st, req = _call_noalloc(lib, sizes, ins, got, opts, stream)
        assert st == _abi.MGS_OK, lib.mgs_status_string(st)
        assert req == need
        torch.cuda.synchronize()
        for name, a, b in zip(("loss", "d_rgb", "d_depth", "d_scales"), got, ref):
            assert torch.isfinite(b).all(), name
            assert torch.equal(a, b), f"{name}: max diff {(a - b).abs().max().item()}"
    # beyond the scratch: three 1200x680 views need about 88 MB
    sizes = [(1200, 680)] * 3
    ins = _inputs(sizes, 3, 10)
    outs = _outputs(sizes, 10)
    st, req = _call_noalloc(lib, sizes, ins, outs, opts, stream)
    assert st == _abi.MGS_ERR_SCRATCH
    assert req > _abi.MGS_LOSS_SCRATCH_BYTES
    torch.cuda.synchronize()
    assert torch.isnan(outs[0]).all() and torch.isnan(outs[1]).all()  # nothing launched
    assert "scratch" in lib.mgs_status_string(st).decode()
    # more views than the table allows
    sizes = [(8, 8)] * (_abi.MGS_LOSS_NOALLOC_MAX_VIEWS + 1)
    ins = _inputs(sizes, 4, 10)
    outs = _outputs(sizes, 10)
    st, _ = _call_noalloc(lib, sizes, ins, outs, opts, stream)
    assert st == _abi.MGS_ERR_SCRATCH
