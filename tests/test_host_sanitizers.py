"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with the sanitizers on its host side only (hipcc's
-Xarch_host; device code is compiled as usual and never runs here), and the
C driver tests/host_sweep.c sweeps planning, queries, sizing and tuning over
1200 random cells and option sets. Any sanitizer report fails the test. No
GPU is used."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_01083_amd", "csrc")
sys.path.insert(0, os.path.join(ROOT, "paper_2111_01083_amd"))
from build import SOURCES  # noqa: E402  (the library's own source list)


def test_host_entry_points_are_clean_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    clang = "/opt/rocm/llvm/bin/clang" if os.path.exists("/opt/rocm/llvm/bin/clang") else None
    if not hipcc or not clang:
        pytest.skip("hipcc / clang not available")
    lib = str(tmp_path / "libpfmm_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    # one object per source, compiled in parallel; debug info on the host
    # side only (the device code is never run here)
    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([hipcc, "--offload-arch=gfx950", "-c", "-O1", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True, timeout=600)
        return obj
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    # the sanitizer runtimes come with the executable below
    subprocess.run([hipcc, "-shared", "-fPIC", *objs, "-o", lib], check=True, capture_output=True, timeout=120)
    exe = str(tmp_path / "host_sweep")
    subprocess.run([clang, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host_sweep.c"), "-o", exe, lib,
                    "-Wl,-rpath," + str(tmp_path), "-lm"], check=True, capture_output=True, timeout=120)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe, "1200"], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr[-4000:]
    assert "plans made" in res.stdout
