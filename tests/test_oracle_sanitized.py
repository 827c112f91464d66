"""The oracle's pin tests again with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc), in a child process that preloads the ASan
runtime: an out-of-bounds access, a use after free or undefined behaviour in
the oracle's C code ends that run with an error."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["test_oracle_predicate.py", "test_oracle_tree.py", "test_oracle_scan_counts.py", "test_oracle_direct.py",
        "test_oracle_filter.py", "test_oracle_clearance.py", "test_oracle_shard.py", "test_oracle_crop_pad.py",
        "test_oracle_posed.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libcapt_oracle_san.so")
    flags = [f for f in oracle.CFLAGS if f != "-O2"] + ["-O1", "-g", "-fno-omit-frame-pointer",
                                                        "-fsanitize=address,undefined",
                                                        "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, "-o", lib, oracle._SRC, "-lm"])
    env = dict(os.environ, CAPT_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *[os.path.join(ROOT, "tests", f) for f in PINS]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
