"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds none of the kernels' arithmetic: it only turns
(seed, stream, element index) into a double.  It is the one piece of code
that both sides of every parity check consume.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  The k-th output (k = 0, 1, ...) of a
SplitMix64 stream whose state starts at ``s`` is ``mix64(s + (k+1)*G)`` with
``G = 0x9E3779B97F4A7C15``, so the generator is counter based: any element
can be produced without the ones before it.

* A stream is identified by ``(seed, stream)``; its starting state is the
  ``stream``-th output of a SplitMix64 stream started at ``seed``.
* Uniform doubles on [-1, 1): ``d = (x >> 11) * 2**-53`` then ``2*d - 1``;
  both steps are exact in binary64, so every platform gets the same bits.
* Small integers on [lo, hi]: ``lo + ((x >> 11) * (hi-lo+1)) >> 53``, exact
  in 64-bit integer arithmetic.  With entries this small every intermediate
  of the kernels stays an integer below 2**53, so any summation order gives
  the same double.
* A matrix element (i, j) of an m x n matrix is element ``k = i*n + j`` of
  its stream, whatever the leading dimension, so padded layouts hold the
  same values.
"""

from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: default seed of every synthetic workload (the paper's arXiv number)
SEED = 12051098

_CHUNK = 1 << 22


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function, elementwise on uint64 (wrapping)."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_scalar(z: int) -> int:
    """Scalar SplitMix64 output function on a Python int (mod 2**64)."""
    mask = (1 << 64) - 1
    z &= mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    return z ^ (z >> 31)


def stream_state(seed: int, stream: int) -> int:
    """Starting state of stream ``stream`` under ``seed``."""
    return mix64_scalar(seed + (stream + 1) * int(GOLDEN))


def stream_id(config: int, operand: int, instance: int = 0) -> int:
    """Stream number of operand ``operand`` (argument order of the C entry
    point) of instance ``instance`` of workload ``config``."""
    return (instance << 16) | ((config & 0xFF) << 8) | (operand & 0xFF)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _raw_into(state: np.uint64, out: np.ndarray, offset: int) -> None:
    k = np.arange(offset + 1, offset + out.shape[0] + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        out[:] = _mix64(state + k * GOLDEN)


def _convert(x: np.ndarray, kind: str, lo: int, hi: int) -> np.ndarray:
    x = x >> np.uint64(11)
    if kind == "uniform":
        return x.astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0
    if kind == "int":
        span = np.uint64(hi - lo + 1)
        return ((x * span) >> np.uint64(53)).astype(np.int64).astype(np.float64) + lo
    if kind == "unit":
        return x.astype(np.float64) * (2.0 ** -53)
    raise ValueError(f"unknown kind {kind!r}")


def _fill(seed: int, stream: int, out: np.ndarray, offset: int, kind: str,
          lo: int = -2, hi: int = 2) -> None:
    """out[t] = element offset+t of the stream, converted to ``kind``; the
    chunks are independent, so they are filled by a thread pool (numpy
    releases the GIL inside its ufuncs)."""
    state = np.uint64(stream_state(seed, stream))
    count = out.shape[0]

    def one(a: int) -> None:
        b = min(count, a + _CHUNK)
        tmp = np.empty(b - a, dtype=np.uint64)
        _raw_into(state, tmp, offset + a)
        out[a:b] = _convert(tmp, kind, lo, hi)

    starts = range(0, count, _CHUNK)
    if count <= 2 * _CHUNK:
        for a in starts:
            one(a)
    else:
        with cf.ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(one, starts))


def raw(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` raw 64-bit outputs of a stream, starting at element ``offset``."""
    out = np.empty(count, dtype=np.uint64)
    _raw_into(np.uint64(stream_state(seed, stream)), out, offset)
    return out


def uniform(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles uniform on [-1, 1), exact multiples of 2**-52."""
    out = np.empty(count, dtype=np.float64)
    _fill(seed, stream, out, offset, "uniform")
    return out


def small_ints(seed: int, stream: int, count: int, lo: int = -2, hi: int = 2,
               offset: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi], returned as doubles."""
    out = np.empty(count, dtype=np.float64)
    _fill(seed, stream, out, offset, "int", lo, hi)
    return out


def vector(seed: int, stream: int, n: int, kind: str = "uniform") -> np.ndarray:
    """A length-n vector of the given kind ("uniform" or "int")."""
    if kind not in ("uniform", "int"):
        raise ValueError(f"unknown kind {kind!r}")
    out = np.empty(n, dtype=np.float64)
    _fill(seed, stream, out, 0, kind)
    return out


def matrix(seed: int, stream: int, m: int, n: int, lda: int | None = None,
           kind: str = "uniform", pad_value: float = np.nan) -> np.ndarray:
    """An m x n row-major matrix stored in an (m, lda) array.

    Element (i, j) is stream element i*n + j.  Columns n..lda-1 are padding
    filled with ``pad_value`` (NaN by default, so a kernel that reads them
    poisons its result).
    """
    lda = n if lda is None else lda
    if lda < n:
        raise ValueError("lda < n")
    if kind not in ("uniform", "int"):
        raise ValueError(f"unknown kind {kind!r}")
    if lda == n:
        a = np.empty((m, n), dtype=np.float64)
        _fill(seed, stream, a.reshape(-1), 0, kind)
        return a
    a = np.full((m, lda), pad_value, dtype=np.float64)
    dense = np.empty(m * n, dtype=np.float64)
    _fill(seed, stream, dense, 0, kind)
    a[:, :n] = dense.reshape(m, n)
    return a


def log_uniform_int(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integers n = min(hi, floor(lo * (hi/lo)**U)) with U uniform on [0, 1)."""
    u = unit_uniform(seed, stream, count)
    n = np.floor(lo * np.power(hi / lo, u)).astype(np.int64)
    return np.minimum(n, hi)


def unit_uniform(seed: int, stream: int, count: int) -> np.ndarray:
    """Doubles uniform on [0, 1)."""
    out = np.empty(count, dtype=np.float64)
    _fill(seed, stream, out, 0, "unit")
    return out
