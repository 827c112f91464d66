"""The benchmark's command line on the CPU: more than one GPU is refused with a
message and exit status 2 before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_unknown_extra_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--extras", "frame,nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "unknown extras" in r.stderr
