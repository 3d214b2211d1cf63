"""Python binding of libbto.so (the C entry points declared in include/bto.h).

Argument marshalling only: every step of every kernel runs in the HIP
library.  Tensors must be float64 on one ROCm device; vectors contiguous,
matrices row-major with unit column stride (any row stride >= n is passed
as the leading dimension).  Outputs and scratch are allocated with torch on
the inputs' device; work is enqueued on the current torch stream of that
device and nothing synchronizes.

Importing this module loads the library and raises ImportError when it has
not been built: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# BTO_LIBRARY points the binding at another build of the same library (the
# tests load a host-sanitized build this way); by default the in-tree one
LIB_PATH = os.environ.get("BTO_LIBRARY") or os.path.join(_HERE, "libbto.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1205_1098_amd.build_lib` "
        "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

FUSED, UNFUSED = 0, 1
FORMS = {"fused": FUSED, "unfused": UNFUSED}
KERNELS = {"bicgk": 0, "gemver": 1, "atax": 2, "dgemvt": 3, "axpydot": 4, "waxpby": 5, "vadd": 6,
           "gemver_contracted": 7, "batax": 8, "dgemv": 9, "gesummv": 10}
STATUS = {0: "success", 1: "invalid argument", 2: "illegal operand overlap",
          3: "workspace too small", 4: "HIP error", 5: "unsupported"}

_i64, _dbl, _ptr, _sz, _int = (ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_int)

class PassDesc(ctypes.Structure):
    """bto_pass_desc: one fused pass over a row-major matrix."""
    _fields_ = [("ops", ctypes.c_int), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("u1", ctypes.c_void_p), ("v1", ctypes.c_void_p),
                ("u2", ctypes.c_void_p), ("v2", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("row_out", ctypes.c_void_p), ("row_scale", ctypes.c_double),
                ("row_add", ctypes.c_void_p), ("row_add_scale", ctypes.c_double),
                ("col_out", ctypes.c_void_p), ("col_scale", ctypes.c_double),
                ("col_add", ctypes.c_void_p), ("col_add_scale", ctypes.c_double)]


PASS_ROWDOT, PASS_COLSUM, PASS_STORE, PASS_CONTRACT, PASS_CHAIN = 1, 2, 4, 8, 16

_SIGS = {
    "bto_version": ([], _int),
    "bto_workspace_bytes": ([_int, _i64, _i64, _int], _sz),
    "bto_status_string": ([_int], ctypes.c_char_p),
    "bto_last_error": ([], ctypes.c_char_p),
    "bto_bicgk": ([_i64, _i64, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_gemver": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _ptr, _ptr,
                    _ptr, _i64, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_gemver_noalloc_max_scratch_bytes": ([], _sz),
    "bto_gemver_noalloc": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _ptr,
                            _ptr, _ptr, _i64, _ptr, _ptr, _int, _ptr], _int),
    "bto_atax": ([_i64, _i64, _ptr, _i64, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_batax": ([_i64, _i64, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_gemver_contracted": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _ptr,
                               _ptr, _ptr, _ptr, _ptr, _sz, _ptr], _int),
    "bto_dgemvt": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _ptr, _sz,
                    _int, _ptr], _int),
    "bto_dgemv": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _ptr, _ptr, _ptr, _sz, _int, _ptr],
                  _int),
    "bto_gesummv": ([_i64, _i64, _dbl, _dbl, _ptr, _i64, _ptr, _i64, _ptr, _ptr, _ptr, _sz, _int,
                     _ptr], _int),
    "bto_lincomb": ([_i64, _int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_dbl), _ptr,
                     _ptr], _int),
    "bto_dot_workspace_bytes": ([_i64], _sz),
    "bto_dot": ([_i64, _ptr, _ptr, _ptr, _ptr, _sz, _ptr], _int),
    "bto_pass_workspace_bytes": ([_int, _i64, _i64], _sz),
    "bto_pass": ([ctypes.POINTER(PassDesc), _ptr, _sz, _ptr], _int),
    "bto_axpydot": ([_i64, _dbl, _ptr, _ptr, _ptr, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_waxpby": ([_i64, _dbl, _ptr, _dbl, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_vadd": ([_i64, _ptr, _ptr, _ptr, _ptr, _ptr, _sz, _int, _ptr], _int),
    "bto_timing_enable": ([_int], _int),
    "bto_timing_collect": ([], _int),
    "bto_timing_only": ([ctypes.c_char_p], _int),
    "bto_timing_count": ([], _int),
    "bto_timing_get": ([_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_i64),
                        ctypes.POINTER(_dbl)], _int),
    "bto_timing_reset": ([], None),
    "bto_probe_copy": ([_ptr, _ptr, _i64, _ptr], _int),
    "bto_probe_read": ([_ptr, _i64, _ptr, _ptr, _sz, _ptr], _int),
    "bto_probe_triad": ([_ptr, _ptr, _ptr, _dbl, _i64, _ptr], _int),
    "bto_probe_read_workspace_bytes": ([_i64], _sz),
    "bto_tune_slot_count": ([], _int),
    "bto_tune_slot_name": ([_int], ctypes.c_char_p),
    "bto_tune_slot_ops": ([_int], _int),
    "bto_tune_get": ([_int, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int)],
                     _int),
    "bto_tune_set": ([_int, _int, _int, _int], _int),
    "bto_tune_get_for": ([_int, _i64, _ptr, _ptr, _ptr], _int),
    "bto_tune_set_for": ([_int, _i64, _int, _int, _int], _int),
    "bto_tune_bucket_count": ([], _int),
    "bto_tune_bucket": ([_i64], _int),
    "bto_tune_shape": ([_int, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                        ctypes.POINTER(_int)], _int),
    "bto_synth_fill": ([_ptr, _i64, _i64, _i64, ctypes.c_uint64, _i64, _int, _int, _int, _ptr],
                       _int),
    "bto_batch_max_n": ([], _i64),
    "bto_batch_plan_create": ([_ptr, _int, _ptr, _ptr], _int),
    "bto_batch_plan_create_empty": ([_int, _i64, _ptr, _ptr], _int),
    "bto_batch_scratch_doubles": ([_ptr, _int, _ptr], _i64),
    "bto_batch_plan_check": ([_ptr, _ptr], _int),
    "bto_batch_plan_error_async": ([_ptr, _ptr, _ptr], _int),
    "bto_batch_plan_reset": ([_ptr, _ptr, _int, _ptr], _int),
    "bto_batch_plan_launch": ([_ptr, _ptr], _int),
    "bto_batch_plan_destroy": ([_ptr], _int),
    "bto_tiled_config_default": ([_ptr], None),
    "bto_tiled_shape_count": ([], _int),
    "bto_tiled_shape": ([_int, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
                         ctypes.POINTER(_int)], _int),
    "bto_tiled_batch_create": ([_ptr, _int, _int, _ptr], _int),
    "bto_tiled_batch_create_config": ([_ptr, _int, _ptr, _ptr], _int),
    "bto_tiled_batch_create_empty": ([_int, _i64, _i64, _ptr, _ptr], _int),
    "bto_tiled_batch_reset": ([_ptr, _ptr, _int, _ptr], _int),
    "bto_tiled_batch_launch": ([_ptr, _ptr], _int),
    "bto_tiled_batch_destroy": ([_ptr], _int),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

#: names of every function the header declares (the library must export all)
EXPORTS = tuple(_SIGS)


class BtoError(RuntimeError):
    """A C entry point returned a status other than BTO_SUCCESS."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _check(status: int) -> None:
    if status != 0:
        raise BtoError(status, _lib.bto_last_error().decode())


class Raw:
    """The entry points on plain integers (device addresses, sizes, a HIP
    stream handle), for callers that keep their own buffers and issue many
    small calls, such as a request server.  The library validates every
    argument as for the tensor wrappers; errors raise BtoError."""

    @staticmethod
    def bicgk(m, n, A, lda, p, r, q, s, ws, ws_bytes, form, stream):
        _check(_lib.bto_bicgk(m, n, A, lda, p, r, q, s, ws, ws_bytes, form, stream))

    @staticmethod
    def gemver(m, n, alpha, beta, A, lda, u1, v1, u2, v2, y, z, B, ldb, x, w, ws, ws_bytes,
               form, stream):
        _check(_lib.bto_gemver(m, n, alpha, beta, A, lda, u1, v1, u2, v2, y, z, B, ldb, x, w,
                               ws, ws_bytes, form, stream))

    @staticmethod
    def atax(m, n, A, lda, x, y, ws, ws_bytes, form, stream):
        _check(_lib.bto_atax(m, n, A, lda, x, y, ws, ws_bytes, form, stream))

    @staticmethod
    def synth_fill(out, rows, cols, ld, state, stream, offset=0, kind=0, lo=-2, hi=2):
        _check(_lib.bto_synth_fill(out, rows, cols, ld, state, offset, kind, lo, hi, stream))


raw = Raw()


def stream_handle(stream) -> int:
    """The HIP stream handle of a torch stream."""
    return int(stream.cuda_stream)


def version() -> int:
    return int(_lib.bto_version())


def _form(form) -> int:
    if isinstance(form, int):
        return form
    try:
        return FORMS[form]
    except KeyError:
        raise ValueError(f"form must be 'fused' or 'unfused', got {form!r}") from None


def workspace_bytes(kernel: str, m: int, n: int, form="fused") -> int:
    return int(_lib.bto_workspace_bytes(KERNELS[kernel], m, n, _form(form)))


def _ptr_of(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check_vec(t: torch.Tensor, name: str, dev, n: int | None = None) -> None:
    """Validate a vector operand; with n, also its length (the C entry points
    take lengths from the matrix extents and cannot check them)."""
    if t.dtype != torch.float64 or t.dim() != 1:
        raise TypeError(f"{name}: expected a 1-D float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: length {t.numel()}, expected {n}")
    if t.device != dev:
        raise ValueError(f"{name}: on {t.device}, expected {dev}")
    if t.numel() > 1 and t.stride(0) != 1:
        raise ValueError(f"{name}: must be contiguous")


def _check_mat(t: torch.Tensor, name: str) -> int:
    """Validate a row-major matrix view and return its leading dimension."""
    if t.dtype != torch.float64 or t.dim() != 2:
        raise TypeError(f"{name}: expected a 2-D float64 tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must live on a ROCm device")
    m, n = t.shape
    if m == 0 or n == 0:
        # no element is read, and torch may give empty tensors any strides
        # (0 among them): every empty matrix gets the smallest even leading
        # dimension, which every entry point and batch accepts and which is
        # the same for an empty output and the empty input it may alias
        k = max(n, 1)
        return k + (k & 1)
    if n > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: needs unit column stride (row-major)")
    if m > 1 and t.stride(0) < max(n, 1):
        raise ValueError(f"{name}: row stride {t.stride(0)} is below the column count {n}")
    # with one row the stride is not used; report it when it is a valid one
    return t.stride(0) if m > 1 or t.stride(0) >= max(n, 1) else max(n, 1)


def _ws(kernel: str, m: int, n: int, form: int, dev, ws):
    need = workspace_bytes(kernel, m, n, form)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev) if need else None
    return ws, need if ws is None else ws.numel()


def _empty(n: int, dev):
    return torch.empty(n, dtype=torch.float64, device=dev)


def bicgk(A, p, r, form="fused", q=None, s=None, ws=None):
    """q = A p ; s = A^T r.  Returns (q, s)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    q = _empty(m, dev) if q is None else q
    s = _empty(n, dev) if s is None else s
    for t, nm, k in ((p, "p", n), (r, "r", m), (q, "q", m), (s, "s", n)):
        _check_vec(t, nm, dev, k)
    f = _form(form)
    ws, wsb = _ws("bicgk", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_bicgk(m, n, _ptr_of(A), lda, _ptr_of(p), _ptr_of(r), _ptr_of(q),
                              _ptr_of(s), _ptr_of(ws), wsb, f, _stream(dev)))
    return q, s


def gemver(A, u1, v1, u2, v2, y, z, alpha, beta, form="fused", B=None, x=None, w=None,
           ws=None):
    """B = A + u1 v1^T + u2 v2^T ; x = beta B^T y + z ; w = alpha B x.

    Pass ``B=A`` for the in-place update.  Returns (B, x, w)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    B = torch.empty((m, n), dtype=torch.float64, device=dev) if B is None else B
    ldb = _check_mat(B, "B")
    if tuple(B.shape) != (m, n) or B.device != dev:
        raise ValueError("B must have A's extents and device")
    x = _empty(n, dev) if x is None else x
    w = _empty(m, dev) if w is None else w
    for t, nm, k in ((u1, "u1", m), (v1, "v1", n), (u2, "u2", m), (v2, "v2", n), (y, "y", m),
                     (z, "z", n), (x, "x", n), (w, "w", m)):
        _check_vec(t, nm, dev, k)
    f = _form(form)
    ws, wsb = _ws("gemver", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_gemver(m, n, float(alpha), float(beta), _ptr_of(A), lda, _ptr_of(u1),
                               _ptr_of(v1), _ptr_of(u2), _ptr_of(v2), _ptr_of(y), _ptr_of(z),
                               _ptr_of(B), ldb, _ptr_of(x), _ptr_of(w), _ptr_of(ws), wsb, f,
                               _stream(dev)))
    return B, x, w


def gemver_noalloc_max_scratch_bytes() -> int:
    return int(_lib.bto_gemver_noalloc_max_scratch_bytes())


def gemver_noalloc(A, u1, v1, u2, v2, y, z, alpha, beta, B, x, w, form="fused"):
    """GEMVER into caller-given outputs B, x, w on the library's own scratch
    (bto_gemver_noalloc): neither this wrapper nor the library allocates.
    Returns (B, x, w)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    ldb = _check_mat(B, "B")
    if tuple(B.shape) != (m, n) or B.device != dev:
        raise ValueError("B must have A's extents and device")
    for t, nm, k in ((u1, "u1", m), (v1, "v1", n), (u2, "u2", m), (v2, "v2", n), (y, "y", m),
                     (z, "z", n), (x, "x", n), (w, "w", m)):
        _check_vec(t, nm, dev, k)
    with torch.cuda.device(dev):
        _check(_lib.bto_gemver_noalloc(m, n, float(alpha), float(beta), _ptr_of(A), lda,
                                       _ptr_of(u1), _ptr_of(v1), _ptr_of(u2), _ptr_of(v2),
                                       _ptr_of(y), _ptr_of(z), _ptr_of(B), ldb, _ptr_of(x),
                                       _ptr_of(w), _form(form), _stream(dev)))
    return B, x, w


def gemver_contracted(A, u1, v1, u2, v2, y, z, alpha, beta, x=None, w=None, ws=None):
    """GEMVER's x and w with B = A + u1 v1^T + u2 v2^T never stored.
    Returns (x, w)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    x = _empty(n, dev) if x is None else x
    w = _empty(m, dev) if w is None else w
    for t, nm, k in ((u1, "u1", m), (v1, "v1", n), (u2, "u2", m), (v2, "v2", n), (y, "y", m),
                     (z, "z", n), (x, "x", n), (w, "w", m)):
        _check_vec(t, nm, dev, k)
    ws, wsb = _ws("gemver_contracted", m, n, 0, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_gemver_contracted(m, n, float(alpha), float(beta), _ptr_of(A), lda,
                                          _ptr_of(u1), _ptr_of(v1), _ptr_of(u2), _ptr_of(v2),
                                          _ptr_of(y), _ptr_of(z), _ptr_of(x), _ptr_of(w),
                                          _ptr_of(ws), wsb, _stream(dev)))
    return x, w


def batax(A, x, beta, form="fused", y=None, ws=None):
    """y = beta A^T (A x)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    y = _empty(n, dev) if y is None else y
    _check_vec(x, "x", dev, n)
    _check_vec(y, "y", dev, n)
    f = _form(form)
    ws, wsb = _ws("batax", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_batax(m, n, float(beta), _ptr_of(A), lda, _ptr_of(x), _ptr_of(y),
                              _ptr_of(ws), wsb, f, _stream(dev)))
    return y


def atax(A, x, form="fused", y=None, ws=None):
    """y = A^T (A x)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    y = _empty(n, dev) if y is None else y
    _check_vec(x, "x", dev, n)
    _check_vec(y, "y", dev, n)
    f = _form(form)
    ws, wsb = _ws("atax", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_atax(m, n, _ptr_of(A), lda, _ptr_of(x), _ptr_of(y), _ptr_of(ws), wsb, f,
                             _stream(dev)))
    return y


def dgemvt(A, y, z, alpha, beta, form="fused", x=None, w=None, ws=None):
    """x = beta A^T y + z ; w = alpha A x.  Returns (x, w)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    x = _empty(n, dev) if x is None else x
    w = _empty(m, dev) if w is None else w
    for t, nm, k in ((y, "y", m), (z, "z", n), (x, "x", n), (w, "w", m)):
        _check_vec(t, nm, dev, k)
    f = _form(form)
    ws, wsb = _ws("dgemvt", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_dgemvt(m, n, float(alpha), float(beta), _ptr_of(A), lda, _ptr_of(y),
                               _ptr_of(z), _ptr_of(x), _ptr_of(w), _ptr_of(ws), wsb, f,
                               _stream(dev)))
    return x, w


def dgemv(A, x, y, alpha, beta, form="fused", z=None, ws=None):
    """z = alpha A x + beta y (z may be y itself)."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    z = _empty(m, dev) if z is None else z
    for t, nm, k in ((x, "x", n), (y, "y", m), (z, "z", m)):
        _check_vec(t, nm, dev, k)
    f = _form(form)
    ws, wsb = _ws("dgemv", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_dgemv(m, n, float(alpha), float(beta), _ptr_of(A), lda, _ptr_of(x),
                              _ptr_of(y), _ptr_of(z), _ptr_of(ws), wsb, f, _stream(dev)))
    return z


def gesummv(A, B, x, alpha, beta, form="fused", y=None, ws=None):
    """y = alpha A x + beta B x (A and B of the same extents; B may be A)."""
    lda = _check_mat(A, "A")
    ldb = _check_mat(B, "B")
    m, n = A.shape
    if tuple(B.shape) != (m, n):
        raise ValueError("A and B must have the same extents")
    dev = A.device
    if B.device != dev:
        raise ValueError("A and B must be on the same device")
    y = _empty(m, dev) if y is None else y
    _check_vec(x, "x", dev, n)
    _check_vec(y, "y", dev, m)
    f = _form(form)
    ws, wsb = _ws("gesummv", m, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_gesummv(m, n, float(alpha), float(beta), _ptr_of(A), lda, _ptr_of(B), ldb,
                                _ptr_of(x), _ptr_of(y), _ptr_of(ws), wsb, f, _stream(dev)))
    return y


def pass_workspace_bytes(ops: int, m: int, n: int) -> int:
    return int(_lib.bto_pass_workspace_bytes(int(ops), m, n))


def fused_pass(ops, A, *, B=None, u1=None, v1=None, u2=None, v2=None, x=None, y=None,
               row_out=None, row_scale=1.0, row_add=None, row_add_scale=1.0,
               col_out=None, col_scale=1.0, col_add=None, col_add_scale=1.0, ws=None):
    """One fused pass over A (bto_pass): the row dots and/or column sums of
    A, or of A + u1 v1^T + u2 v2^T (stored in B with PASS_STORE, never
    formed with PASS_CONTRACT), each reduced with its scale and add.
    Every output must be given; nothing is allocated but the workspace
    when ws is None."""
    lda = _check_mat(A, "A")
    m, n = A.shape
    dev = A.device
    ldb = 0
    if B is not None:
        ldb = _check_mat(B, "B")
        if tuple(B.shape) != (m, n):
            raise ValueError("B must have A's extents")
    for t, nm, k in ((u1, "u1", m), (v1, "v1", n), (u2, "u2", m), (v2, "v2", n), (x, "x", n),
                     (y, "y", m), (row_out, "row_out", m), (row_add, "row_add", m),
                     (col_out, "col_out", n), (col_add, "col_add", n)):
        if t is not None:
            _check_vec(t, nm, dev, k)
    need = pass_workspace_bytes(ops, m, n)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    d = PassDesc(int(ops), m, n, A.data_ptr(), lda, _addr(B), ldb, _addr(u1), _addr(v1),
                 _addr(u2), _addr(v2), _addr(x), _addr(y), _addr(row_out), float(row_scale),
                 _addr(row_add), float(row_add_scale), _addr(col_out), float(col_scale),
                 _addr(col_add), float(col_add_scale))
    with torch.cuda.device(dev):
        _check(_lib.bto_pass(ctypes.byref(d), _ptr_of(ws), ws.numel(), _stream(dev)))


def lincomb(xs, coefs, out=None):
    """out = sum_k coefs[k] * xs[k] (left to right, one pass; up to 8 terms)."""
    if not 1 <= len(xs) <= 8 or len(coefs) != len(xs):
        raise ValueError("1 to 8 vectors, one coefficient each")
    dev = xs[0].device
    n = xs[0].numel()
    out = _empty(n, dev) if out is None else out
    for k, t in enumerate(xs):
        _check_vec(t, f"x{k}", dev, n)
    _check_vec(out, "out", dev, n)
    ptrs = (ctypes.c_void_p * len(xs))(*[t.data_ptr() for t in xs])
    cs = (ctypes.c_double * len(xs))(*[float(c) for c in coefs])
    with torch.cuda.device(dev):
        _check(_lib.bto_lincomb(n, len(xs), ptrs, cs, _ptr_of(out), _stream(dev)))
    return out


def dot(x, y, r=None, ws=None):
    """r = x^T y, into a 1-element tensor on the device."""
    dev = x.device
    n = x.numel()
    r = _empty(1, dev) if r is None else r
    for t, nm, k in ((x, "x", n), (y, "y", n), (r, "r", 1)):
        _check_vec(t, nm, dev, k)
    need = int(_lib.bto_dot_workspace_bytes(n))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        _check(_lib.bto_dot(n, _ptr_of(x), _ptr_of(y), _ptr_of(r), _ptr_of(ws), ws.numel(),
                            _stream(dev)))
    return r


def _addr(t):
    return None if t is None else t.data_ptr()


def axpydot(w, v, u, alpha, form="fused", z=None, r=None, ws=None):
    """z = w - alpha v ; r = z^T u.  Returns (z, r) with r a 1-element tensor."""
    dev = w.device
    n = w.numel()
    z = _empty(n, dev) if z is None else z
    r = _empty(1, dev) if r is None else r
    for t, nm, k in ((w, "w", n), (v, "v", n), (u, "u", n), (z, "z", n), (r, "r", 1)):
        _check_vec(t, nm, dev, k)
    f = _form(form)
    ws, wsb = _ws("axpydot", 0, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_axpydot(n, float(alpha), _ptr_of(w), _ptr_of(v), _ptr_of(u), _ptr_of(z),
                                _ptr_of(r), _ptr_of(ws), wsb, f, _stream(dev)))
    return z, r


def waxpby(x, y, alpha, beta, form="fused", w=None, ws=None):
    """w = alpha x + beta y."""
    dev = x.device
    n = x.numel()
    w = _empty(n, dev) if w is None else w
    for t, nm in ((x, "x"), (y, "y"), (w, "w")):
        _check_vec(t, nm, dev, n)
    f = _form(form)
    ws, wsb = _ws("waxpby", 0, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_waxpby(n, float(alpha), _ptr_of(x), float(beta), _ptr_of(y), _ptr_of(w),
                               _ptr_of(ws), wsb, f, _stream(dev)))
    return w


def vadd(w, y, z, form="fused", x=None, ws=None):
    """x = (w + y) + z."""
    dev = w.device
    n = w.numel()
    x = _empty(n, dev) if x is None else x
    for t, nm in ((w, "w"), (y, "y"), (z, "z"), (x, "x")):
        _check_vec(t, nm, dev, n)
    f = _form(form)
    ws, wsb = _ws("vadd", 0, n, f, dev, ws)
    with torch.cuda.device(dev):
        _check(_lib.bto_vadd(n, _ptr_of(w), _ptr_of(y), _ptr_of(z), _ptr_of(x), _ptr_of(ws),
                             wsb, f, _stream(dev)))
    return x


# ---- measurement support ---------------------------------------------------

def timing_enable(on: bool = True) -> None:
    _check(_lib.bto_timing_enable(1 if on else 0))


def timing_only(name: str | None) -> None:
    """Restrict timing to launches of one kernel name (None: all)."""
    _check(_lib.bto_timing_only(name.encode() if name else None))


def timing_reset() -> None:
    _lib.bto_timing_reset()


def timing_read() -> dict:
    """Wait for recorded events; return {kernel name: (launches, total ms)}."""
    _check(_lib.bto_timing_collect())
    out = {}
    for i in range(_lib.bto_timing_count()):
        name, cnt, ms = ctypes.c_char_p(), _i64(), _dbl()
        _check(_lib.bto_timing_get(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)))
        out[name.value.decode()] = (int(cnt.value), float(ms.value))
    return out


def probe_copy(src, dst) -> None:
    dev = src.device
    with torch.cuda.device(dev):
        _check(_lib.bto_probe_copy(_ptr_of(src), _ptr_of(dst), src.numel(), _stream(dev)))


def probe_triad(a, b, c, s: float) -> None:
    dev = a.device
    with torch.cuda.device(dev):
        _check(_lib.bto_probe_triad(_ptr_of(a), _ptr_of(b), _ptr_of(c), float(s), a.numel(),
                                    _stream(dev)))


def probe_read_workspace_bytes(n: int) -> int:
    return int(_lib.bto_probe_read_workspace_bytes(int(n)))


def probe_read(src, out, ws=None) -> None:
    """out[0] = sum of src (a streaming read in a fixed order)."""
    dev = src.device
    need = probe_read_workspace_bytes(src.numel())
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev) if ws is None else ws
    with torch.cuda.device(dev):
        _check(_lib.bto_probe_read(_ptr_of(src), src.numel(), _ptr_of(out), _ptr_of(ws),
                                   ws.numel(), _stream(dev)))


# ---- tile configuration (the autotuner's knobs) ------------------------------

def tune_slots() -> list:
    """Names of the tunable matrix sweeps, in slot order."""
    return [_lib.bto_tune_slot_name(i).decode() for i in range(_lib.bto_tune_slot_count())]


def tune_slot_ops(slot: int) -> int:
    return int(_lib.bto_tune_slot_ops(slot))


def tune_get(slot: int, size: int = 0) -> tuple:
    """(shape, rb, rev) of a slot for problems with max(m, n) = size (0: the
    16384 bucket)."""
    a, b, c = _int(), _int(), _int()
    _check(_lib.bto_tune_get_for(slot, int(size), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def tune_set(slot: int, shape: int, rb: int, rev: int = 0, size: int = 0) -> None:
    """Set a slot's configuration for the size bucket of `size` (0: all)."""
    _check(_lib.bto_tune_set_for(slot, int(size), shape, rb, rev))


def tune_buckets() -> int:
    return int(_lib.bto_tune_bucket_count())


def tune_bucket(size: int) -> int:
    return int(_lib.bto_tune_bucket(int(size)))


def tune_shape(shape: int) -> dict:
    """kv (16-byte pairs per lane), depth (rows in flight), waves across, waves down."""
    v = [_int() for _ in range(4)]
    _check(_lib.bto_tune_shape(shape, *[ctypes.byref(x) for x in v]))
    return dict(zip(("kv", "depth", "wc", "wr"), (int(x.value) for x in v)))


# ---- synthetic inputs in device memory ---------------------------------------------

def synth_fill(out, state: int, offset: int = 0, kind: str = "uniform", lo: int = -2,
               hi: int = 2) -> None:
    """Fill a 1-D or row-major 2-D float64 tensor in place from a SplitMix64
    stream state (see synth.stream_state); bit-identical to the host side."""
    if out.dim() == 1:
        rows, cols, ld = 1, out.numel(), max(out.numel(), 1)
    else:
        rows, cols = out.shape
        ld = _check_mat(out, "out")
    k = {"uniform": 0, "int": 1}[kind]
    dev = out.device
    with torch.cuda.device(dev):
        _check(_lib.bto_synth_fill(_ptr_of(out), rows, cols, ld, ctypes.c_uint64(state), offset,
                                   k, lo, hi, _stream(dev)))


# ---- batched execution --------------------------------------------------------------

class Desc(ctypes.Structure):
    """bto_batch_desc."""
    _fields_ = [("kind", ctypes.c_int), ("form", ctypes.c_int),
                ("m", _i64), ("n", _i64), ("lda", _i64), ("ldb", _i64),
                ("alpha", _dbl), ("beta", _dbl),
                ("A", _ptr), ("B", _ptr),
                ("inp", _ptr * 6), ("out", _ptr * 2)]


class _Config(ctypes.Structure):
    """bto_batch_config."""
    _fields_ = [("threads", ctypes.c_int), ("wgs_per_cu", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("split_bytes", ctypes.c_int64)]


def batch_max_n() -> int:
    return int(_lib.bto_batch_max_n())


def _batch_descs(instances):
    """Marshal instance dicts into a C array of bto_batch_desc."""
    keep = []
    descs = (Desc * max(len(instances), 1))()
    dev = None
    for i, inst in enumerate(instances):
        d = descs[i]
        A = inst["A"]
        dev = A.device if dev is None else dev
        lda = _check_mat(A, "A")
        d.kind = KERNELS[inst["kind"]]
        d.form = _form(inst.get("form", "fused"))
        d.m, d.n = A.shape
        d.lda = lda
        d.A = A.data_ptr()
        refs = [A]
        if inst["kind"] == "gemver":
            B = inst["B"]
            d.ldb = _check_mat(B, "B")
            d.B = B.data_ptr()
            d.alpha, d.beta = float(inst["alpha"]), float(inst["beta"])
            refs.append(B)
        else:
            d.ldb = lda
        m_, n_ = A.shape
        lens_in, lens_out = {"gemver": ((m_, n_, m_, n_, m_, n_), (n_, m_)),
                             "bicgk": ((n_, m_), (m_, n_)),
                             "atax": ((n_,), (n_,))}.get(inst["kind"], ((), ()))
        if len(inst["in"]) != len(lens_in) or len(inst["out"]) != len(lens_out):
            raise ValueError(f"instance {i}: wrong number of vector operands")
        for k, t in enumerate(inst["in"]):
            _check_vec(t, f"in[{k}]", A.device, lens_in[k])
            d.inp[k] = t.data_ptr()
            refs.append(t)
        for k, t in enumerate(inst["out"]):
            _check_vec(t, f"out[{k}]", A.device, lens_out[k])
            d.out[k] = t.data_ptr()
            refs.append(t)
        keep.append(refs)
    return descs, keep, dev


def batch_scratch_doubles(instances, split_bytes: int = 0) -> int:
    """Scratch a plan needs for these instances (unfused ATAX temporaries and
    the column-sum partials of split instances)."""
    descs = (Desc * max(len(instances), 1))()
    for i, inst in enumerate(instances):
        d = descs[i]
        d.kind = KERNELS[inst["kind"]]
        d.form = _form(inst.get("form", "fused"))
        d.m, d.n = inst["A"].shape if "A" in inst else (inst["m"], inst["n"])
    cfg = _Config(0, 0, 0, int(split_bytes))
    need = _lib.bto_batch_scratch_doubles(ctypes.byref(descs), len(instances), ctypes.byref(cfg))
    if need < 0:
        raise ValueError("bad instance sizes")
    return int(need)


class BatchPlan:
    """Many GEMVER / BiCGK / ATAX instances in one persistent launch.

    `instances` is a list of dicts with keys
        kind ("gemver" | "bicgk" | "atax"), form ("fused" | "unfused"),
        A (2-D tensor), in (list of 1-D tensors), out (list of 1-D tensors),
        and for GEMVER: B (2-D tensor, may be A), alpha, beta
    in the argument order of the single-instance entry points.  The plan keeps
    references to the tensors of its current instances; launch() enqueues the
    batch on the current stream and allocates nothing.  A plan made with
    `BatchPlan.empty` is refilled with `reset` before each launch."""

    def __init__(self, instances, threads: int = 0, wgs_per_cu: int = 0,
                 use_graph: bool = True, split_bytes: int = 0, *, _capacity=None, _scratch=0,
                 _device=None):
        cfg = _Config(threads, wgs_per_cu, 1 if use_graph else 0, int(split_bytes))
        self._plan = ctypes.c_void_p()
        if _capacity is not None:
            self.device = torch.device(_device if _device is not None else "cuda:0")
            self._keep = []
            with torch.cuda.device(self.device):
                _check(_lib.bto_batch_plan_create_empty(int(_capacity), int(_scratch),
                                                        ctypes.byref(cfg), ctypes.byref(self._plan)))
            self.capacity, self.count = int(_capacity), 0
            return
        descs, self._keep, dev = _batch_descs(instances)
        self.device = dev if dev is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            _check(_lib.bto_batch_plan_create(ctypes.byref(descs), len(instances), ctypes.byref(cfg),
                                              ctypes.byref(self._plan)))
        self.capacity = self.count = len(instances)

    @classmethod
    def empty(cls, capacity: int, scratch_doubles: int = 0, threads: int = 0,
              wgs_per_cu: int = 0, use_graph: bool = True, device="cuda:0",
              split_bytes: int = 0) -> "BatchPlan":
        return cls(None, threads, wgs_per_cu, use_graph, split_bytes, _capacity=capacity,
                   _scratch=scratch_doubles, _device=device)

    def check(self) -> None:
        """Wait for the current stream; raise if the last launch's tile waits
        gave up (bto_batch_plan_check)."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        with torch.cuda.device(self.device):
            _check(_lib.bto_batch_plan_check(self._plan, _stream(self.device)))

    def error_async(self, dst: int, stream: int) -> None:
        """Enqueue on the raw `stream` handle a copy of the plan's error word
        into the int at address `dst` (pinned host or device memory)."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        _check(_lib.bto_batch_plan_error_async(self._plan, dst, stream))

    def reset(self, instances) -> None:
        """Replace the instances (copied on the current stream; no allocation)."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        descs, keep, _ = _batch_descs(instances)
        with torch.cuda.device(self.device):
            _check(_lib.bto_batch_plan_reset(self._plan, ctypes.byref(descs), len(instances),
                                             _stream(self.device)))
        self._keep, self.count = keep, len(instances)

    def reset_descs(self, descs, count: int, stream: int, keep=None) -> None:
        """Replace the instances from a filled `Desc` array (device addresses
        as integers) with the copy enqueued on the raw `stream` handle; the
        caller keeps the buffers alive."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        _check(_lib.bto_batch_plan_reset(self._plan, ctypes.byref(descs), count, stream))
        self._keep, self.count = keep or [], count

    def launch_on(self, stream: int) -> None:
        """launch() on a raw HIP stream handle."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        _check(_lib.bto_batch_plan_launch(self._plan, stream))

    def launch(self) -> None:
        if not self._plan:
            raise RuntimeError("plan is closed")
        with torch.cuda.device(self.device):
            _check(_lib.bto_batch_plan_launch(self._plan, _stream(self.device)))

    def close(self) -> None:
        if self._plan:
            _lib.bto_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TiledConfig(ctypes.Structure):
    """bto_tiled_config: the tiled batch's partition parameters."""
    _fields_ = [("store_shape", ctypes.c_int), ("narrow_shape", ctypes.c_int),
                ("wide_shape", ctypes.c_int), ("narrow_n", ctypes.c_int),
                ("store_rb", ctypes.c_int), ("bicgk_rb", ctypes.c_int),
                ("read_rb", ctypes.c_int),
                ("wgs_per_cu", ctypes.c_int), ("use_graph", ctypes.c_int)]

    @classmethod
    def default(cls, **changes) -> "TiledConfig":
        c = cls()
        _lib.bto_tiled_config_default(ctypes.byref(c))
        for k, v in changes.items():
            if k not in {f for f, _ in cls._fields_}:
                raise KeyError(k)
            setattr(c, k, int(v))
        return c

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def tiled_shapes() -> list:
    """The tiled batches' tile shapes: dicts of kv, depth, waves_across,
    waves_down (and the block's column count)."""
    out = []
    for s in range(int(_lib.bto_tiled_shape_count())):
        v = [_int() for _ in range(4)]
        _check(_lib.bto_tiled_shape(s, *[ctypes.byref(x) for x in v]))
        kv, d, wc, wr = (x.value for x in v)
        out.append({"kv": kv, "depth": d, "waves_across": wc, "waves_down": wr,
                    "cols": 128 * kv * wc, "threads": 64 * wc * wr})
    return out


class TiledBatch:
    """Fused GEMVER / BiCGK instances (the dicts BatchPlan takes) run as
    short-lived workgroup tiles, launched per group of tiles (first sweeps,
    their sums, GEMVER's second sweeps, their sums), captured in a HIP graph
    with `use_graph`.  `config` (a TiledConfig) sets the partition; None
    takes the library's defaults (with `use_graph` applied).  launch()
    enqueues the batch on the current stream and allocates nothing.  A plan
    made with `TiledBatch.empty` is refilled with `reset` (or `reset_descs`)
    before each launch."""

    def __init__(self, instances, use_graph: bool = True, config: TiledConfig | None = None, *,
                 _capacity=None, _max_m=0, _max_n=0, _device=None):
        self._plan = ctypes.c_void_p()
        if config is None:
            config = TiledConfig.default(use_graph=1 if use_graph else 0)
        self.config = config
        if _capacity is not None:
            self.device = torch.device(_device if _device is not None else "cuda:0")
            self._keep = []
            with torch.cuda.device(self.device):
                _check(_lib.bto_tiled_batch_create_empty(int(_capacity), int(_max_m), int(_max_n),
                                                         ctypes.byref(config),
                                                         ctypes.byref(self._plan)))
            self.capacity, self.count = int(_capacity), 0
            return
        descs, self._keep, dev = _batch_descs(instances)
        self.device = dev if dev is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            _check(_lib.bto_tiled_batch_create_config(ctypes.byref(descs), len(instances),
                                                      ctypes.byref(config),
                                                      ctypes.byref(self._plan)))
        self.capacity = self.count = len(instances)

    @classmethod
    def empty(cls, capacity: int, max_m: int, max_n: int, config: TiledConfig | None = None,
              device="cuda:0") -> "TiledBatch":
        """A refillable plan for up to `capacity` instances of at most
        max_m x max_n (config.wgs_per_cu must be nonzero)."""
        if config is None:
            config = TiledConfig.default()
            if config.wgs_per_cu == 0:
                config.wgs_per_cu = 2
        return cls(None, config=config, _capacity=capacity, _max_m=max_m, _max_n=max_n,
                   _device=device)

    def reset(self, instances) -> None:
        """Replace the instances (copied on the current stream; no allocation)."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        descs, keep, _ = _batch_descs(instances)
        with torch.cuda.device(self.device):
            _check(_lib.bto_tiled_batch_reset(self._plan, ctypes.byref(descs), len(instances),
                                              _stream(self.device)))
        self._keep, self.count = keep, len(instances)

    def reset_descs(self, descs, count: int, stream: int, keep=None) -> None:
        """Replace the instances from a filled `Desc` array (device addresses
        as integers) with the copy enqueued on the raw `stream` handle; the
        caller keeps the buffers alive."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        _check(_lib.bto_tiled_batch_reset(self._plan, ctypes.byref(descs), count, stream))
        self._keep, self.count = keep or [], count

    def launch_on(self, stream: int) -> None:
        """launch() on a raw HIP stream handle."""
        if not self._plan:
            raise RuntimeError("plan is closed")
        _check(_lib.bto_tiled_batch_launch(self._plan, stream))

    def launch(self) -> None:
        if not self._plan:
            raise RuntimeError("plan is closed")
        with torch.cuda.device(self.device):
            _check(_lib.bto_tiled_batch_launch(self._plan, _stream(self.device)))

    def close(self) -> None:
        if self._plan:
            _lib.bto_tiled_batch_destroy(self._plan)
            self._plan = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
