"""Host-side argument handling of bench.py (no device is touched: both
checks run before torch is imported)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=60)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_section_is_refused():
    r = _run("--sections", "ttgt,nosuch")
    assert r.returncode == 2
    assert "nosuch" in r.stderr
    assert r.stdout == ""
