"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, its status strings, and the ctypes mirror of every
struct has the header's layout (compiled with gcc from include/memgs.h)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2509_13536_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "memgs.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mgs_[a-z_]+)\s*\(", text)))


def test_header_declares_what_the_binding_uses():
    assert set(_declared_functions()) == set(_abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mgs_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_status_strings_and_version():
    lib = _abi.load()
    assert lib.mgs_status_string(0) == b"ok"
    assert b"workspace" in lib.mgs_status_string(_abi.MGS_ERR_WORKSPACE)
    assert lib.mgs_status_string(12345) == b"unknown status"
    assert lib.mgs_abi_version() >> 16 == 2


STRUCTS = {
    "mgs_gaussians": _abi.Gaussians,
    "mgs_gaussian_grads": _abi.GaussianGrads,
    "mgs_camera": _abi.Camera,
    "mgs_render_opts": _abi.RenderOpts,
    "mgs_forward_info": _abi.ForwardInfo,
    "mgs_gaussians_out": _abi.GaussiansOut,
}


def test_ctypes_layout_matches_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "memgs.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for cname, cls in STRUCTS.items():
        assert int(got[f"{cname} size"]) == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, f"{cname}.{fname}"


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _abi.load()


# ---------------------------------------------------------------- argument checks
# Every check below returns before the library makes any HIP call, so it runs
# here without a GPU; the pointers are placeholders that are never dereferenced.
FAKE = 0x1000


def _maps(n=10, deg=0, quats=FAKE):
    m = (_abi.Gaussians * 1)()
    m[0] = _abi.Gaussians(n, FAKE, FAKE, quats, FAKE, FAKE, deg, 0)
    return m


def _cams(k=1, W=64, H=48, fx=50.0, map_id=0):
    cams = (_abi.Camera * k)()
    for i in range(k):
        T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
        cams[i] = _abi.Camera(W, H, fx, fx, W / 2, H / 2, T, 0.2, map_id)
    return cams


def _fwd(lib, maps, n_maps, cams, n_views, ws_bytes=0, info=None):
    info = info if info is not None else _abi.ForwardInfo()
    st = lib.mgs_render_forward(maps, n_maps, cams, n_views, None, C.c_void_p(FAKE) if ws_bytes else None,
                                ws_bytes, C.byref(info), C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), None)
    return st, info


def test_forward_rejects_bad_arguments():
    lib = _abi.load()
    assert _fwd(lib, _maps(), 1, _cams(), 0)[0] == _abi.MGS_ERR_INVALID_ARG          # no view
    assert _fwd(lib, _maps(), 1, _cams(), 4097)[0] == _abi.MGS_ERR_INVALID_ARG       # too many views
    assert _fwd(lib, _maps(), 0, _cams(), 1)[0] == _abi.MGS_ERR_INVALID_ARG          # no map
    assert _fwd(lib, _maps(deg=4), 1, _cams(), 1)[0] == _abi.MGS_ERR_INVALID_ARG     # SH degree > 3
    assert _fwd(lib, _maps(n=-1), 1, _cams(), 1)[0] == _abi.MGS_ERR_INVALID_ARG      # negative size
    assert _fwd(lib, _maps(quats=FAKE + 4), 1, _cams(), 1)[0] == _abi.MGS_ERR_INVALID_ARG  # quats not 16-byte aligned
    assert _fwd(lib, _maps(), 1, _cams(W=16385), 1)[0] == _abi.MGS_ERR_INVALID_ARG   # image too wide
    assert _fwd(lib, _maps(), 1, _cams(H=0), 1)[0] == _abi.MGS_ERR_INVALID_ARG       # empty image
    assert _fwd(lib, _maps(), 1, _cams(fx=0.0), 1)[0] == _abi.MGS_ERR_INVALID_ARG    # focal length
    assert _fwd(lib, _maps(), 1, _cams(map_id=1), 1)[0] == _abi.MGS_ERR_INVALID_ARG  # map index out of range
    nulls = (_abi.Gaussians * 1)()
    nulls[0] = _abi.Gaussians(10, None, FAKE, FAKE, FAKE, FAKE, 0, 0)
    assert _fwd(lib, nulls, 1, _cams(), 1)[0] == _abi.MGS_ERR_INVALID_ARG            # null attribute


def test_forward_workspace_query():
    """With no workspace the call reports what the projection stage needs and
    fills the sizes it knows, without touching the device."""
    lib = _abi.load()
    st, info = _fwd(lib, _maps(n=1000), 1, _cams(2, W=100, H=40), 2)
    assert st == _abi.MGS_ERR_WORKSPACE
    assert info.ws_required > 0
    assert info.n_pairs == 2000 and info.n_pixels == 2 * 100 * 40 and info.n_views == 2
    assert info.n_bins == 2 * 7 * 3 and (info.bin_tx, info.bin_ty) == (1, 1)


def test_bin_size_follows_the_call(monkeypatch):
    """Calls with 16384 or more 16x16 tiles take bins of 2x1 tiles, smaller
    ones single tiles; MGS_BIN_TILES forces a size."""
    lib = _abi.load()
    monkeypatch.delenv("MGS_BIN_TILES", raising=False)
    # 8 views of 1200x680: 75 x 43 tiles each, 25 800 in all -> 38 x 43 bins per view
    st, info = _fwd(lib, _maps(n=1000), 1, _cams(8, W=1200, H=680), 8)
    assert st == _abi.MGS_ERR_WORKSPACE
    assert (info.bin_tx, info.bin_ty) == (2, 1) and info.n_bins == 8 * 38 * 43
    # 5 of them: 16 125 tiles, below the threshold
    st, info = _fwd(lib, _maps(n=1000), 1, _cams(5, W=1200, H=680), 5)
    assert (info.bin_tx, info.bin_ty) == (1, 1) and info.n_bins == 5 * 75 * 43
    # 64 x 16 tiles of 16 px in each of 16 views: exactly 16384 tiles
    st, info = _fwd(lib, _maps(n=1000), 1, _cams(16, W=1024, H=256), 16)
    assert (info.bin_tx, info.bin_ty) == (2, 1) and info.n_bins == 16 * 32 * 16
    for forced, expect in (("1x1", (1, 1)), ("2x2", (2, 2))):
        monkeypatch.setenv("MGS_BIN_TILES", forced)
        st, info = _fwd(lib, _maps(n=1000), 1, _cams(8, W=1200, H=680), 8)
        assert (info.bin_tx, info.bin_ty) == expect


def test_backward_rejects_inconsistent_state():
    lib = _abi.load()
    _, info = _fwd(lib, _maps(n=1000), 1, _cams(), 1)
    info.need_backward = 1
    grads = _abi.GaussianGrads(FAKE, FAKE, FAKE, FAKE, FAKE)
    P = C.c_void_p(FAKE)

    def bwd(maps, cams, inf):
        return lib.mgs_render_backward(maps, 1, cams, 1, None, C.byref(inf), P, 1 << 30, P, P, None,
                                       C.byref(grads), None, None)
    assert bwd(_maps(n=999), _cams(), info) == _abi.MGS_ERR_INVALID_ARG   # another map size
    assert bwd(_maps(n=1000), _cams(W=65), info) == _abi.MGS_ERR_INVALID_ARG  # another image
    half = _abi.GaussianGrads(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None)
    assert lib.mgs_render_backward(_maps(n=1000), 1, _cams(), 1, None, C.byref(info), P, 1 << 30, P, P, None,
                                   C.byref(half), None, None) == _abi.MGS_ERR_INVALID_ARG  # statistics come in pairs
    info.need_backward = 0
    assert bwd(_maps(n=1000), _cams(), info) == _abi.MGS_ERR_INVALID_ARG  # forward without backward state


def test_merge_mask_rejects_bad_arguments():
    lib = _abi.load()
    P = C.c_void_p(FAKE)

    def mask(n=10, tau=1e-3, gsum=P, cnt=P, out=P):
        return lib.mgs_merge_mask(gsum, cnt, None, n, C.c_float(tau), 0, 5, out, None)
    assert mask(n=-1) == _abi.MGS_ERR_INVALID_ARG
    assert mask(tau=float("nan")) == _abi.MGS_ERR_INVALID_ARG
    assert mask(gsum=None) == _abi.MGS_ERR_INVALID_ARG
    assert mask(cnt=None) == _abi.MGS_ERR_INVALID_ARG
    assert mask(out=None) == _abi.MGS_ERR_INVALID_ARG
    assert mask(n=1 << 31) == _abi.MGS_ERR_TOO_LARGE
    assert mask(n=0, gsum=None, cnt=None, out=None) == _abi.MGS_OK  # nothing to do, nothing launched


def test_merge_rejects_bad_arguments_and_reports_workspace():
    lib = _abi.load()
    g = _abi.Gaussians(1000, FAKE, FAKE, FAKE, FAKE, FAKE, 0, 0)
    out = _abi.GaussiansOut(FAKE, FAKE, FAKE, FAKE, FAKE)
    req, n_out = C.c_size_t(0), C.c_int64(-1)

    def merge(voxel=0.05, chi2=7.815, policy=0, gg=g):
        return lib.mgs_voxel_merge(C.byref(gg), None, C.c_float(voxel), C.c_float(chi2), policy, C.byref(out),
                                   None, None, None, 0, C.byref(req), C.byref(n_out), None)
    assert merge(voxel=0.0) == _abi.MGS_ERR_INVALID_ARG
    assert merge(voxel=float("nan")) == _abi.MGS_ERR_INVALID_ARG
    assert merge(chi2=-1.0) == _abi.MGS_ERR_INVALID_ARG
    assert merge(policy=4) == _abi.MGS_ERR_INVALID_ARG  # flags: BEST_PAIR 1, LBFGS 2
    assert merge(gg=_abi.Gaussians(10, FAKE, FAKE, FAKE, FAKE, FAKE, 5, 0)) == _abi.MGS_ERR_INVALID_ARG
    assert merge() == _abi.MGS_ERR_WORKSPACE and req.value > 1000
    empty = _abi.Gaussians(0, None, None, None, None, None, 0, 0)
    assert merge(gg=empty) == _abi.MGS_OK and n_out.value == 0


def test_mapping_loss_rejects_bad_arguments_and_reports_workspace():
    lib = _abi.load()
    P = C.c_void_p(FAKE)
    req = C.c_size_t(0)

    def call(sizes=(64, 48), n_views=1, depth=None, gtd=None, scales=None, n_g=0, dd=None, ds=None, lam=0.2,
             opts=True):
        sz = (C.c_int32 * len(sizes))(*sizes)
        o = _abi.LossOpts(lam, 1.0, 1.0, 0)
        return lib.mgs_mapping_loss(sz, n_views, P, P, depth, gtd, scales, n_g, C.byref(o) if opts else None,
                                    None, 0, C.byref(req), P, P, dd, ds, None)
    assert call(n_views=0) == _abi.MGS_ERR_INVALID_ARG
    assert call(sizes=(0, 48)) == _abi.MGS_ERR_INVALID_ARG
    assert call(sizes=(64, 16385)) == _abi.MGS_ERR_INVALID_ARG
    assert call(depth=P) == _abi.MGS_ERR_INVALID_ARG                  # depth without its target
    assert call(depth=P, gtd=P) == _abi.MGS_ERR_INVALID_ARG           # depth without its gradient
    assert call(scales=P, n_g=10) == _abi.MGS_ERR_INVALID_ARG         # scales without their gradient
    assert call(n_g=-1) == _abi.MGS_ERR_INVALID_ARG
    assert call(lam=float("nan")) == _abi.MGS_ERR_INVALID_ARG
    assert call(opts=False) == _abi.MGS_ERR_INVALID_ARG
    assert call() == _abi.MGS_ERR_WORKSPACE and req.value >= 36 * 64 * 48


def test_patch_grid_rejects_bad_arguments_and_reports_workspace():
    lib = _abi.load()
    P = C.c_void_p(FAKE)
    req, n_out = C.c_size_t(0), C.c_int64(-1)
    out = _abi.GaussiansOut(FAKE, FAKE, FAKE, FAKE, FAKE)

    def call(cams=None, n_kp=10, kp=P, patch=32, samples=2, min_kp=4, image=P, fx=None):
        cams = cams if cams is not None else _cams(W=100, H=60)
        if fx is not None:
            cams[0].fx = fx
        o = _abi.PgOpts(patch, min_kp, samples, 0.5, 0.5, 0)
        return lib.mgs_patch_grid_sample(cams, kp, kp, n_kp, None, image, C.byref(o), C.byref(out), None, None, 0,
                                         C.byref(req), C.byref(n_out), None)
    assert call(patch=0) == _abi.MGS_ERR_INVALID_ARG
    assert call(samples=0) == _abi.MGS_ERR_INVALID_ARG
    assert call(samples=65) == _abi.MGS_ERR_INVALID_ARG
    assert call(min_kp=-1) == _abi.MGS_ERR_INVALID_ARG
    assert call(n_kp=-1) == _abi.MGS_ERR_INVALID_ARG
    assert call(kp=None) == _abi.MGS_ERR_INVALID_ARG
    assert call(image=None) == _abi.MGS_ERR_INVALID_ARG
    assert call(fx=0.0) == _abi.MGS_ERR_INVALID_ARG
    assert call(cams=_cams(W=0, H=60)) == _abi.MGS_ERR_INVALID_ARG
    assert call() == _abi.MGS_ERR_WORKSPACE and req.value > 0 and n_out.value == 0


def test_adam_rejects_bad_arguments():
    lib = _abi.load()
    out = _abi.GaussiansOut(FAKE, FAKE, FAKE, FAKE, FAKE)
    grads = _abi.GaussianGrads(FAKE, FAKE, FAKE, FAKE, FAKE)

    def call(n=10, deg=0, step=1, b1=0.9, b2=0.999, eps=1e-8, lr0=1e-3, g=grads, o=out):
        opts = _abi.AdamOpts((C.c_float * 5)(lr0, 1e-3, 1e-3, 1e-3, 1e-3), b1, b2, eps, step)
        return lib.mgs_adam_step(C.byref(o), n, deg, C.byref(g), C.byref(o), C.byref(o), C.byref(opts), None)
    assert call(n=-1) == _abi.MGS_ERR_INVALID_ARG
    assert call(deg=4) == _abi.MGS_ERR_INVALID_ARG
    assert call(step=0) == _abi.MGS_ERR_INVALID_ARG
    assert call(b1=1.0) == _abi.MGS_ERR_INVALID_ARG
    assert call(b2=-0.1) == _abi.MGS_ERR_INVALID_ARG
    assert call(eps=-1.0) == _abi.MGS_ERR_INVALID_ARG
    assert call(lr0=float("inf")) == _abi.MGS_ERR_INVALID_ARG
    assert call(o=_abi.GaussiansOut(None, FAKE, FAKE, FAKE, FAKE)) == _abi.MGS_ERR_INVALID_ARG  # means wanted
    none = _abi.GaussianGrads(None, None, None, None, None)
    assert call(g=none) == _abi.MGS_OK  # nothing to update, nothing launched
    assert call(n=0) == _abi.MGS_OK


def test_packed_camera_array_equals_per_view_structs():
    """The binding packs cameras with struct; the bytes must be those of one
    mgs_camera per view filled field by field (ctypes, the header's layout)."""
    import numpy as np
    from paper_2509_13536_amd import api
    rng = np.random.default_rng(4)
    views = []
    for k in range(5):
        T = rng.normal(size=(3, 4)).astype(np.float32)
        views.append(api.View(int(rng.integers(1, 4000)), int(rng.integers(1, 3000)), float(rng.uniform(50, 900)),
                              float(rng.uniform(50, 900)), float(rng.normal()), float(rng.normal()), T,
                              float(rng.uniform(0.01, 1)), k % 3))
    arr = api._views_array(views)
    assert C.sizeof(arr) == len(views) * C.sizeof(_abi.Camera)
    for k, v in enumerate(views):
        assert bytes(arr[k]) == bytes(v.c_struct()), k


def test_backward_refuses_a_workspace_reused_by_a_later_forward():
    """A forward's state lives in its workspace; a later forward on the same
    workspace (or a regrowth) replaces it, and the backward must refuse."""
    import torch

    from paper_2509_13536_amd.api import ForwardState, Workspace
    ws = Workspace("cpu", 1024)
    ws.generation += 1  # what render_forward does after a successful call
    st = ForwardState([], [], (0, 0, 0, 0), None, ws, torch.empty(0), torch.empty(0), torch.empty(0),
                      ws_generation=ws.generation, ws_buf=ws.buf)
    st.check_workspace()
    ws.generation += 1  # a second forward
    with pytest.raises(RuntimeError, match="reused"):
        st.check_workspace()
    ws2 = Workspace("cpu", 256)
    st2 = ForwardState([], [], (0, 0, 0, 0), None, ws2, torch.empty(0), torch.empty(0), torch.empty(0),
                       ws_generation=ws2.generation, ws_buf=ws2.buf)
    ws2.ensure(1 << 20)  # regrown: the old buffer and its state are gone
    with pytest.raises(RuntimeError, match="reused"):
        st2.check_workspace()


def test_roctx_ranges_when_asked(tmp_path):
    """With MGS_ROCTX=1 every entry point opens and closes a roctx range (the
    roctx library looked up at the first call); the calls behave as without."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import tests.test_abi_host as t\n"
        "from paper_2509_13536_amd import _abi\n"
        "lib = _abi.load()\n"
        "for _ in range(3):\n"
        "    assert t._fwd(lib, t._maps(), 1, t._cams(), 0)[0] == _abi.MGS_ERR_INVALID_ARG\n"
        "    assert t._fwd(lib, t._maps(), 1, t._cams(fx=0.0), 1)[0] == _abi.MGS_ERR_INVALID_ARG\n"
        "print('ok')\n" % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    for flag in ("1", "0"):
        env = dict(os.environ, MGS_ROCTX=flag)
        r = subprocess.run(["python3", "-c", code], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
