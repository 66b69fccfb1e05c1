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
    assert lib.mgs_abi_version() >> 16 == 1


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
