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


def raw(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` raw 64-bit outputs of a stream, starting at element ``offset``."""
    state = np.uint64(stream_state(seed, stream))
    out = np.empty(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for lo in range(0, count, _CHUNK):
            hi = min(count, lo + _CHUNK)
            k = np.arange(offset + lo + 1, offset + hi + 1, dtype=np.uint64)
            out[lo:hi] = _mix64(state + k * GOLDEN)
    return out


def uniform(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles uniform on [-1, 1), exact multiples of 2**-52."""
    out = np.empty(count, dtype=np.float64)
    for lo in range(0, count, _CHUNK):
        hi = min(count, lo + _CHUNK)
        x = raw(seed, stream, hi - lo, offset + lo) >> np.uint64(11)
        out[lo:hi] = x.astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0
    return out


def small_ints(seed: int, stream: int, count: int, lo: int = -2, hi: int = 2,
               offset: int = 0) -> np.ndarray:
    """Integers uniform on [lo, hi], returned as doubles."""
    span = np.uint64(hi - lo + 1)
    out = np.empty(count, dtype=np.float64)
    for a in range(0, count, _CHUNK):
        b = min(count, a + _CHUNK)
        x = raw(seed, stream, b - a, offset + a) >> np.uint64(11)
        out[a:b] = ((x * span) >> np.uint64(53)).astype(np.int64) + lo
    return out


def vector(seed: int, stream: int, n: int, kind: str = "uniform") -> np.ndarray:
    """A length-n vector of the given kind ("uniform" or "int")."""
    if kind == "uniform":
        return uniform(seed, stream, n)
    if kind == "int":
        return small_ints(seed, stream, n)
    raise ValueError(f"unknown kind {kind!r}")


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
    a = np.full((m, lda), pad_value, dtype=np.float64)
    rows_per_chunk = max(1, _CHUNK // max(n, 1))
    for i0 in range(0, m, rows_per_chunk):
        i1 = min(m, i0 + rows_per_chunk)
        cnt = (i1 - i0) * n
        if cnt == 0:
            continue
        if kind == "uniform":
            blk = uniform(seed, stream, cnt, offset=i0 * n)
        elif kind == "int":
            blk = small_ints(seed, stream, cnt, offset=i0 * n)
        else:
            raise ValueError(f"unknown kind {kind!r}")
        a[i0:i1, :n] = blk.reshape(i1 - i0, n)
    return a


def log_uniform_int(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integers n = min(hi, floor(lo * (hi/lo)**U)) with U uniform on [0, 1)."""
    u = (raw(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    n = np.floor(lo * np.power(hi / lo, u)).astype(np.int64)
    return np.minimum(n, hi)


def unit_uniform(seed: int, stream: int, count: int) -> np.ndarray:
    """Doubles uniform on [0, 1)."""
    return (raw(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
