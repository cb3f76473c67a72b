"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with the sanitizers on its host side only (hipcc's
-Xarch_host; device code is compiled as usual and never runs here), and the
C driver tests/host_sweep.c sweeps planning, queries, sizing and tuning over
3000 random cells and option sets. Any sanitizer report fails the test. No
GPU is used."""
import os
import shutil
import subprocess
import sys

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
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    *[os.path.join(CSRC, s) for s in SOURCES], "-o", lib],
                   check=True, capture_output=True, timeout=600)
    exe = str(tmp_path / "host_sweep")
    subprocess.run([clang, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host_sweep.c"), "-o", exe, lib,
                    "-Wl,-rpath," + str(tmp_path), "-lm"], check=True, capture_output=True, timeout=120)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr[-4000:]
    assert "plans made" in res.stdout
