"""The library's host code (descriptor checks, tables, factors) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: mr_api.hip is
compiled with both sanitizers on its host side only, linked with the other
objects of the regular build, and tests/host_calls.py runs every host-side
entry point against that library in a child process with the sanitizer
runtime preloaded.  Any report ends the child with a non-zero status."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _asan_runtime():
    if not os.path.exists(CLANG):
        return None
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    objs = sorted(glob.glob(os.path.join(ROOT, "_build", "*.hip.o")))
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None or not objs:
        pytest.skip("needs hipcc, the clang ASan runtime and the regular build's objects (_build)")
    obj = str(tmp_path / "mr_api.o")
    compile_cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Xarch_host", "-fsanitize=address",
                   "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=all",
                   "-Xarch_host", "-fno-omit-frame-pointer",
                   "-I", os.path.join(ROOT, "include"),
                   "-c", os.path.join(ROOT, "paper_1805_03426_amd", "csrc", "mr_api.hip"), "-o", obj]
    r = subprocess.run(compile_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lib = str(tmp_path / "libmrscalar_san.so")
    others = [o for o in objs if not o.endswith("mr_api.hip.o")]
    link_cmd = [CLANG, "-shared", "-shared-libasan", "-fsanitize=address,undefined", "-o", lib, obj] + others + [
        "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link_cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_calls.py"), lib], capture_output=True,
                       text=True, env=env, timeout=600)
    assert r.returncode == 0 and "host calls ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
