"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the C render oracle, every entry point, on a small scene with degenerate
  members (tests/sanitize/oracle_driver.c, gcc);
* the host side of the C ABI: argument validation, workspace sizing and the
  fixed-scratch limits of every entry point, on the paths that end before any
  device work (tests/sanitize/abi_driver.c).  The library is rebuilt with the
  sanitizers on its host code only (hipcc's -Xarch_host); no GPU is touched.

A sanitizer report aborts the driver (-fno-sanitize-recover), so each test
asserts a zero exit status and no report in the output.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
CSRC = os.path.join(ROOT, "paper_2509_13536_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


def _clean(out):
    return "ERROR: AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-o", exe,
                    os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "render_oracle.c"), "-lm"])
    assert rc == 0, out
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and _clean(out), out
    assert "checksum" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_abi_host_code_under_address_and_ub_sanitizers(tmp_path):
    sources = ["render.hip", "merge.hip", "loss.hip", "patch_grid.hip", "adam.hip", "status.hip"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops",
             # the sanitizers instrument the host code only
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", f"-I{INCLUDE}", f"-I{CSRC}"]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        return _run(["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", obj]) + (obj,)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(compile_one, sources))
    for rc, out, _ in results:
        assert rc == 0, out
    lib = str(tmp_path / "libmemgs_san.so")
    rc, out = _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", lib, *[o for _, _, o in results]])
    assert rc == 0, out
    exe = str(tmp_path / "abi_driver")
    rc, out = _run([os.path.join(ROCM, "llvm", "bin", "clang"), "-std=c11", "-O1", "-g",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{INCLUDE}",
                    os.path.join(SAN, "abi_driver.c"), "-o", exe, f"-L{tmp_path}", "-lmemgs_san",
                    f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{ROCM}/lib"])
    assert rc == 0, out
    # the HIP runtime's own allocations outlive main: leak reports off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    rc, out = _run([exe], env=env)
    assert rc == 0 and _clean(out), out
    assert "0 failures" in out
