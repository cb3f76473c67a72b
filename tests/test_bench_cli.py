"""bench.py's command-line contract, checked without a GPU: the options the
driver passes exist, and a multi-GPU request ends with a message and a
non-zero status before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_options_exist():
    res = _run("--help")
    assert res.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup"):
        assert opt in res.stdout


def test_more_than_one_gpu_is_refused_with_a_message():
    res = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert res.returncode != 0 and res.stdout == ""
    assert "one GPU" in res.stderr
