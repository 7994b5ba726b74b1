"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

- tests/c/host_units.cpp: the overlapping block geometry, the workspace bump
  allocator and the server's first-fit arena allocator (random alloc/release
  sequences against a shadow map), built with g++.
- tests/c/abi_host.c: the C ABI called from C on its host-only paths (status
  strings, block counts, workspace and request sizes, argument errors of every
  entry point, the per-thread error message), linked against a libhdi whose
  host code is built with the sanitizers (the GPU code is built as usual; these
  paths never launch it).

Both programs are built in a temporary directory and must print their "ok"
line and exit 0; any sanitizer report aborts them."""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2401_06747_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-4000:]}\n{p.stderr[-4000:]}"
    return p.stdout


def test_host_units_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_units")
    _run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-o", exe, os.path.join(ROOT, "tests", "c", "host_units.cpp")])
    out = _run([exe], env=ENV)
    assert "host units: ok" in out


def _hip_object(src, out):
    # sanitizers for the host compilation only (-Xarch_host before each)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-c",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", out, src]
    _run(cmd)
    return out


def test_c_abi_host_paths_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _hip_object(s, str(tmp_path / (os.path.basename(s) + ".o"))), srcs))
    lib = str(tmp_path / "libhdi_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-o", lib, *objs])
    exe = str(tmp_path / "abi_host")
    _run([CLANG, "-std=c11", "-O1", "-g", *SAN, "-o", exe, os.path.join(ROOT, "tests", "c", "abi_host.c"),
          "-L", str(tmp_path), "-lhdi_san", "-Wl,-rpath," + str(tmp_path), "-lpthread"])
    out = _run([exe], env=ENV)
    assert "abi host: ok" in out
