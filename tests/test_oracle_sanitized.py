"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with -fsanitize=address,undefined (host code only; the
oracle has no other kind) and every function runs, in a child process with
the ASan runtime preloaded, over empty, ragged and padded shapes with one and
several threads.  Any out-of-bounds access, use of freed memory or undefined
behaviour aborts the child, failing the test.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, sys
import numpy as np
sys.path.insert(0, ROOT)
import oracle
oracle._lib = oracle.bind(ctypes.CDLL(LIB))
rng = np.random.default_rng(3)

def mat(m, n, lda):
    a = np.full((max(m, 1), lda), np.nan)[:m]
    a[:, :n] = rng.uniform(-1, 1, (m, n))
    return a

for threads in (1, 4):
    oracle.set_threads(threads)
    for m, n in [(0, 0), (0, 5), (5, 0), (1, 1), (3, 7), (65, 33), (130, 257), (300, 1)]:
        for pad in (0, 3):
            lda = max(n, 1) + pad
            A = mat(m, n, lda)
            v = lambda k: rng.uniform(-1, 1, k)
            q, s = oracle.bicgk(A, v(n), v(m), lda=lda)
            B, x, w = oracle.gemver(A, v(m), v(n), v(m), v(n), v(m), v(n), 1.5, 0.7, lda=lda)
            y = oracle.atax(A, v(n), lda=lda)
            x2, w2 = oracle.dgemvt(A, v(m), v(n), 1.5, 0.7, lda=lda)
            z = oracle.dgemv(A, v(n), v(m), 1.5, 0.7, lda=lda)
            ldb = max(n, 1) + 2 * pad
            g = oracle.gesummv(A, mat(m, n, ldb), v(n), 1.5, 0.7, m=m, lda=lda, ldb=ldb)
            assert z.shape == g.shape == (m,) and np.all(np.isfinite(z)) and np.all(np.isfinite(g))
            assert q.shape == (m,) and s.shape == (n,) and B.shape[0] == m and y.shape == (n,)
            assert np.all(np.isfinite(q)) and np.all(np.isfinite(s)) and np.all(np.isfinite(w))
    for N in (0, 1, 2, 127, 128, 129, 1000, 4097):
        a, b, c = (rng.uniform(-1, 1, N) for _ in range(3))
        z, r = oracle.axpydot(a, b, c, 1.5)
        w = oracle.waxpby(a, b, 1.5, 0.7)
        x = oracle.vadd(a, b, c)
        assert z.shape == w.shape == x.shape == (N,)
print("sanitized oracle ok")
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "bto_oracle.c")
    import oracle

    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", *flags, "-o", lib, src], check=True)
    script = tmp_path / "child.py"
    script.write_text(f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "sanitized oracle ok" in res.stdout
