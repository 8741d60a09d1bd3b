"""Host AddressSanitizer run of the library's host code (CPU only).

Every HIP source is compiled with the sanitizer on the host pass only
(-Xarch_host; the device code is built but never runs here) into a separate
shared library under
_build/host_asan/; tests/host_asan_driver.cpp then drives the C ABI through
mesh construction and preparation of ragged, hub, multi-class and
disconnected graphs, every validation path, the quadrature schedule and the
network's parameter checks.  Any heap or stack error aborts the driver with
an AddressSanitizer report; leaks are checked at exit as well.
"""

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "host_asan")
LLVM = "/opt/rocm/llvm"


def _tools():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clangxx = os.path.join(LLVM, "bin", "clang++")
    rt = glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    if not (os.path.exists(hipcc) and os.path.exists(clangxx) and rt):
        pytest.skip("hipcc, ROCm clang++ or the clang AddressSanitizer runtime not found")
    return hipcc, clangxx, os.path.dirname(rt[0])


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"


def _build(hipcc, clangxx, rtdir):
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2605_02670_amd", "csrc", "*.hip")))
    # device code is compiled too (the host side registers it) but never runs here
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", f"-I{os.path.join(ROOT, 'include')}"]

    def one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([hipcc, *flags, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(OUT, "libgrf_hostasan.so")
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libsan", "-Xarch_host", "-fsanitize=address",
          *objs,
          f"-Wl,-rpath,{rtdir}", "-o", lib])
    exe = os.path.join(OUT, "host_asan_driver")
    _run([clangxx, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address", "-shared-libsan",
          f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "host_asan_driver.cpp"),
          f"-L{OUT}", "-lgrf_hostasan", f"-Wl,-rpath,{OUT}", f"-Wl,-rpath,{rtdir}", "-o", exe])
    return exe


def test_host_code_under_address_sanitizer():
    exe = _build(*_tools())
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and "PASSED" in r.stdout, out[-4000:]
