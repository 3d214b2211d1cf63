"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libbto is rebuilt with the sanitizers on its host code only (device code is
compiled as usual and never runs here), and the host-side tests of the C
boundary (argument, alias and workspace checks, batch-plan validation,
scratch sizing, tuning tables) run against that build in a child process
with the sanitizer runtime preloaded.  An out-of-bounds access, a use of
freed memory or undefined behaviour fails the child.
"""

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1205_1098_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
# sanitizers on the host side of each translation unit only
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    runtime = _asan_runtime()
    if runtime is None or not os.path.exists(HIPCC):
        pytest.skip("no HIP compiler or no AddressSanitizer runtime")
    base = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(base + ["-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(sources))) as pool:
        objs = list(pool.map(compile_one, sources))
    lib = str(tmp_path / "libbto_san.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN,
                    "-shared-libasan", "-o", lib, *objs], check=True, capture_output=True)

    env = dict(os.environ, LD_PRELOAD=runtime, BTO_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_abi_cpu.py", "test_batch_cpu.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          "-m", "not gpu", *tests], env=env, cwd=ROOT, capture_output=True,
                         text=True, timeout=600)
    report = res.stdout[-3000:] + res.stderr[-3000:]
    assert res.returncode == 0, report
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, report
