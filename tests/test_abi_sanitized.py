"""The host-side ABI checks again against a build of libcapt whose host code
carries AddressSanitizer and UBSan (device code is built as usual and never
launched), in a child process that preloads the ASan runtime: argument
validation, blob parsing and the error paths run under the sanitizers."""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_02807_amd", "csrc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _asan_runtime():
    r = subprocess.run(["hipcc", "-print-resource-dir"], capture_output=True, text=True)
    hits = glob.glob(os.path.join(r.stdout.strip(), "lib", "linux", "libclang_rt.asan-x86_64.so")) if r.returncode == 0 else []
    return hits[0] if hits else None


@pytest.mark.slow
def test_abi_host_checks_under_asan_and_ubsan(tmp_path):
    from paper_2406_02807_amd import build_lib
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    flags = [f for f in build_lib.FLAGS if f != "-O3"] + ["-O1", "-g"] + HOST_SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run(["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", obj], check=True, capture_output=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(build_lib.SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, build_lib.SOURCES))
    lib = str(tmp_path / "libcapt_san.so")
    subprocess.run(["hipcc", f"--offload-arch={build_lib.ARCH}", "-shared", "-fPIC", *HOST_SAN[:4], "-o", lib, *objs],
                   check=True, capture_output=True)
    env = dict(os.environ, CAPT_LIBRARY=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "Sanitizer" not in r.stderr, tail
