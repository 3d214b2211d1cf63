"""CPU oracle for the nine BTO kernels (Table I of the paper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library never does, and this
package never imports the GPU library.

The arithmetic lives in ``bto_oracle.c`` (plain binary64 loops, no fused
multiply-add, sequential matrix reductions, pairwise summation for the long
dot product).  This module only builds that file with gcc and marshals numpy
arrays into it.  Every function takes host float64 arrays in the argument
order of the corresponding C entry point and returns freshly allocated
outputs.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bto_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math"]


def build(verbose: bool = False) -> str:
    """Compile ``bto_oracle.c`` into ``liboracle.so`` (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        _lib = bind(lib)
    return _lib


def bind(lib):
    """Declare the C signatures on a loaded copy of the oracle library."""
    i64, dbl, ptr = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "oracle_bicgk": [i64, i64, ptr, i64, ptr, ptr, ptr, ptr],
        "oracle_gemver": [i64, i64, dbl, dbl, ptr, i64, ptr, ptr, ptr, ptr,
                          ptr, ptr, ptr, i64, ptr, ptr],
        "oracle_atax": [i64, i64, ptr, i64, ptr, ptr],
        "oracle_dgemvt": [i64, i64, dbl, dbl, ptr, i64, ptr, ptr, ptr, ptr],
        "oracle_dgemv": [i64, i64, dbl, dbl, ptr, i64, ptr, ptr, ptr],
        "oracle_gesummv": [i64, i64, dbl, dbl, ptr, i64, ptr, i64, ptr, ptr],
        "oracle_axpydot": [i64, dbl, ptr, ptr, ptr, ptr, ptr],
        "oracle_waxpby": [i64, dbl, ptr, dbl, ptr, ptr],
        "oracle_vadd": [i64, ptr, ptr, ptr, ptr],
        "oracle_set_threads": [ctypes.c_int],
        "oracle_get_threads": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int if name == "oracle_get_threads" else None
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _vec(a, n: int, name: str) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 1 or a.shape[0] != n:
        raise ValueError(f"{name}: expected length {n}, got shape {a.shape}")
    return a


def _mat(A, m: int, n: int, lda: int | None):
    """Accept an (m, lda) array, or an (m, n) array when lda is None."""
    A = np.asarray(A, dtype=np.float64)
    if lda is None:
        A = np.ascontiguousarray(A)
        if A.shape != (m, n):
            raise ValueError(f"A: expected {(m, n)}, got {A.shape}")
        return A, max(n, 1)
    if not A.flags.c_contiguous or A.ndim != 2 or A.shape[0] != m or A.shape[1] != lda:
        raise ValueError("A: expected a contiguous (m, lda) array")
    return A, lda


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def bicgk(A, p, r, lda=None):
    """q = A p ; s = A^T r."""
    m, n = (A.shape[0], p.shape[0])
    A, lda = _mat(A, m, n, lda)
    p, r = _vec(p, n, "p"), _vec(r, m, "r")
    q, s = np.empty(m), np.empty(n)
    _load().oracle_bicgk(m, n, _p(A), lda, _p(p), _p(r), _p(q), _p(s))
    return q, s


def gemver(A, u1, v1, u2, v2, y, z, alpha, beta, lda=None):
    """B = A + u1 v1^T + u2 v2^T ; x = beta B^T y + z ; w = alpha B x."""
    m, n = u1.shape[0], v1.shape[0]
    A, lda = _mat(A, m, n, lda)
    u1, u2, y = _vec(u1, m, "u1"), _vec(u2, m, "u2"), _vec(y, m, "y")
    v1, v2, z = _vec(v1, n, "v1"), _vec(v2, n, "v2"), _vec(z, n, "z")
    ldb = max(n, 1)
    B = np.empty((m, n))
    x, w = np.empty(n), np.empty(m)
    _load().oracle_gemver(m, n, float(alpha), float(beta), _p(A), lda,
                          _p(u1), _p(v1), _p(u2), _p(v2), _p(y), _p(z),
                          _p(B), ldb, _p(x), _p(w))
    return B, x, w


def atax(A, x, lda=None):
    """y = A^T (A x)."""
    m, n = A.shape[0], x.shape[0]
    A, lda = _mat(A, m, n, lda)
    x = _vec(x, n, "x")
    y = np.empty(n)
    _load().oracle_atax(m, n, _p(A), lda, _p(x), _p(y))
    return y


def dgemvt(A, y, z, alpha, beta, lda=None):
    """x = beta A^T y + z ; w = alpha A x."""
    m, n = y.shape[0], z.shape[0]
    A, lda = _mat(A, m, n, lda)
    y, z = _vec(y, m, "y"), _vec(z, n, "z")
    x, w = np.empty(n), np.empty(m)
    _load().oracle_dgemvt(m, n, float(alpha), float(beta), _p(A), lda,
                          _p(y), _p(z), _p(x), _p(w))
    return x, w


def dgemv(A, x, y, alpha, beta, lda=None):
    """z = alpha A x + beta y."""
    m, n = y.shape[0], x.shape[0]
    A, lda = _mat(A, m, n, lda)
    x, y = _vec(x, n, "x"), _vec(y, m, "y")
    z = np.empty(m)
    _load().oracle_dgemv(m, n, float(alpha), float(beta), _p(A), lda, _p(x), _p(y), _p(z))
    return z


def gesummv(A, B, x, alpha, beta, m=None, lda=None, ldb=None):
    """y = alpha A x + beta B x (A and B both m x n)."""
    n = x.shape[0]
    m = np.asarray(A).shape[0] if m is None else m
    A, lda = _mat(A, m, n, lda)
    B, ldb = _mat(B, m, n, ldb)
    x = _vec(x, n, "x")
    y = np.empty(m)
    _load().oracle_gesummv(m, n, float(alpha), float(beta), _p(A), lda, _p(B), ldb, _p(x),
                           _p(y))
    return y


def axpydot(w, v, u, alpha):
    """z = w - alpha v ; r = z^T u (pairwise)."""
    n = w.shape[0]
    w, v, u = _vec(w, n, "w"), _vec(v, n, "v"), _vec(u, n, "u")
    z = np.empty(n)
    r = np.zeros(1)
    _load().oracle_axpydot(n, float(alpha), _p(w), _p(v), _p(u), _p(z), _p(r))
    return z, float(r[0])


def waxpby(x, y, alpha, beta):
    """w = alpha x + beta y."""
    n = x.shape[0]
    x, y = _vec(x, n, "x"), _vec(y, n, "y")
    w = np.empty(n)
    _load().oracle_waxpby(n, float(alpha), _p(x), float(beta), _p(y), _p(w))
    return w


def vadd(w, y, z):
    """x = (w + y) + z."""
    n = w.shape[0]
    w, y, z = _vec(w, n, "w"), _vec(y, n, "y"), _vec(z, n, "z")
    x = np.empty(n)
    _load().oracle_vadd(n, _p(w), _p(y), _p(z), _p(x))
    return x
