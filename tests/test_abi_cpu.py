"""Host-side checks of the C boundary that need no GPU: the library loads,
exports every function include/bto.h declares, sizes workspaces, and rejects
bad arguments before it enqueues anything (no kernel is launched here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bto.h")


@pytest.fixture(scope="module")
def bto():
    from paper_1205_1098_amd import bto as b

    return b


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bto_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(bto):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(bto.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), f"libbto.so does not export {name}"
    assert set(names) == set(bto.EXPORTS)


def test_version_and_status_strings(bto):
    assert bto.version() >= 100
    for s in range(6):
        assert bto._lib.bto_status_string(s).decode()


def test_workspace_sizes(bto):
    n = 16384
    for k in ("bicgk", "gemver", "dgemvt"):
        b = bto.workspace_bytes(k, n, n, "fused")
        # partial sums stay a few percent of the 2 GiB matrix
        assert 0 < b < 0.05 * n * n * 8
        assert b % 256 == 0
    assert bto.workspace_bytes("atax", n, n, "fused") < 0.05 * n * n * 8
    assert bto.workspace_bytes("waxpby", 0, 1 << 26, "fused") == 0
    assert bto.workspace_bytes("vadd", 0, 1 << 26, "unfused") == (1 << 26) * 8
    assert bto.workspace_bytes("axpydot", 0, 0, "fused") == 0
    assert bto.workspace_bytes("bicgk", -1, 5, "fused") == 0


FAKE = 1 << 40          # never dereferenced: every case below fails its checks


def _call_bicgk(bto, m, n, A, lda, p, r, q, s, ws, wsb, form=0):
    return bto._lib.bto_bicgk(m, n, A, lda, p, r, q, s, ws, wsb, form, None)


def test_invalid_arguments(bto):
    INV = 1
    v = ctypes.c_void_p
    assert _call_bicgk(bto, -1, 4, v(FAKE), 4, v(FAKE), v(FAKE), v(FAKE), v(FAKE), None, 0) == INV
    assert _call_bicgk(bto, 4, 4, v(FAKE), 3, v(FAKE), v(FAKE), v(FAKE), v(FAKE), None, 0) == INV
    assert _call_bicgk(bto, 4, 4, None, 4, v(FAKE), v(FAKE), v(FAKE), v(FAKE), None, 0) == INV
    assert "NULL" in bto._lib.bto_last_error().decode()
    assert _call_bicgk(bto, 4, 4, v(FAKE), 4, v(FAKE), v(FAKE), v(FAKE), v(FAKE), None, 0,
                       form=7) == INV


def test_alias_detection(bto):
    ALIAS = 2
    v = ctypes.c_void_p
    m = n = 64
    A = FAKE
    p, r = FAKE + (1 << 20), FAKE + (2 << 20)
    q, s = FAKE + (3 << 20), FAKE + (4 << 20)
    ws = FAKE + (8 << 20)
    wsb = bto.workspace_bytes("bicgk", m, n)
    # q overlapping A
    assert _call_bicgk(bto, m, n, v(A), n, v(p), v(r), v(A + 64), v(s), v(ws), wsb) == ALIAS
    # q and s overlapping each other
    assert _call_bicgk(bto, m, n, v(A), n, v(p), v(r), v(q), v(q + 8), v(ws), wsb) == ALIAS
    # workspace overlapping an input
    assert _call_bicgk(bto, m, n, v(A), n, v(p), v(r), v(q), v(s), v(A), wsb) == ALIAS
    # GEMVER: B == A is allowed only with ldb == lda
    lib = bto._lib
    wsg = bto.workspace_bytes("gemver", m, n)
    vec = [v(FAKE + (k << 20)) for k in range(1, 11)]
    st = lib.bto_gemver(m, n, 1.5, 0.7, v(A), n + 2, *vec[:6], v(A), n, vec[6], vec[7],
                        v(ws), wsg, 0, None)
    assert st == ALIAS
    # VADD: partial overlap of x with w is illegal
    st = lib.bto_vadd(100, v(FAKE), v(FAKE + (1 << 20)), v(FAKE + (2 << 20)), v(FAKE + 8),
                      None, 0, 0, None)
    assert st == ALIAS


def test_workspace_too_small(bto):
    WS = 3
    v = ctypes.c_void_p
    m = n = 256
    wsb = bto.workspace_bytes("bicgk", m, n)
    base = FAKE
    st = _call_bicgk(bto, m, n, v(base), n, v(base + (1 << 20)), v(base + (2 << 20)),
                     v(base + (3 << 20)), v(base + (4 << 20)), v(base + (8 << 20)), wsb - 1)
    assert st == WS
    assert "workspace" in bto._lib.bto_last_error().decode()


def test_workspace_checked_before_overlap(bto):
    """A too-small workspace reports WORKSPACE even where the extent it would
    need runs into another operand."""
    v = ctypes.c_void_p
    m = n = 256
    wsb = bto.workspace_bytes("bicgk", m, n)
    base = FAKE
    ws = base + (16 << 20)
    q = ws + 4096            # inside the required extent, past the provided one
    st = _call_bicgk(bto, m, n, v(base), n, v(base + (1 << 20)), v(base + (2 << 20)),
                     v(q), v(base + (4 << 20)), v(ws), 1024)
    assert st == 3


def test_tuning_size_buckets(bto):
    """Tile configurations are kept per size bucket of max(m, n)."""
    nb = bto.tune_buckets()
    assert nb == 8
    assert [bto.tune_bucket(s) for s in (1, 256, 257, 512, 2048, 2049, 16384, 16385, 10**6)] == \
        [0, 0, 1, 1, 3, 4, 6, 7, 7]
    slots = bto.tune_slots()
    p1 = slots.index("gemver_p1")
    saved = {b: bto.tune_get(p1, 256 << b) for b in range(nb)}
    try:
        base = bto.tune_get(p1)                       # the 16384 bucket
        assert base == saved[6]
        other = (10, 64, 0) if base != (10, 64, 0) else (10, 128, 0)
        bto.tune_set(p1, *other, size=3000)           # bucket of 3000: <= 4096
        assert bto.tune_get(p1, 4096) == other and bto.tune_get(p1, 2049) == other
        assert bto.tune_get(p1, 2048) == saved[3] and bto.tune_get(p1) == base
        bto.tune_set(p1, *other)                      # size 0: every bucket
        assert all(bto.tune_get(p1, 256 << b) == other for b in range(nb))
        with pytest.raises(bto.BtoError):
            bto.tune_set(p1, 999, 32, 0, size=1024)   # no such shape
        with pytest.raises(bto.BtoError):
            bto.tune_set(p1, *other, size=-1)
    finally:
        for b, c in saved.items():
            bto.tune_set(p1, *c, size=256 << b)
    assert all(bto.tune_get(p1, 256 << b) == saved[b] for b in range(nb))
    # the row-resident slots take a workgroup size per bucket
    rr = slots.index("bicgk_rowres")
    keep = bto.tune_get(rr, 1024)
    bto.tune_set(rr, 0, 0, 0, size=1024)
    assert bto.tune_get(rr, 1024) == (0, 0, 0) and bto.tune_get(rr, 16384)[0] in (256, 512, 1024)
    bto.tune_set(rr, *keep, size=1024)
    with pytest.raises(bto.BtoError):
        bto.tune_set(slots.index("atax_rowres"), 0, 0, 0, size=1024)   # ATAX has no tile fallback


def test_dgemv_and_gesummv_checks(bto):
    """DGEMV and GESUMMV: workspace sizes and the argument checks, before
    anything is enqueued."""
    v = ctypes.c_void_p
    n = 16384
    wd = bto.workspace_bytes("dgemv", n, n)
    assert 0 < wd < 0.01 * n * n * 8 and wd % 256 == 0
    assert bto.workspace_bytes("dgemv", n, n, "unfused") == wd
    assert bto.workspace_bytes("gesummv", n, n, "fused") == 2 * wd
    assert bto.workspace_bytes("gesummv", n, n, "unfused") == wd + n * 8
    m = k = 256
    base = FAKE
    ptr = lambda i: v(base + (i << 20))
    need = bto.workspace_bytes("dgemv", m, k)

    def dg(A=ptr(0), lda=k, x=ptr(1), y=ptr(2), z=ptr(3), ws=ptr(16), wsb=need, form=0,
           mm=m, nn=k):
        return bto._lib.bto_dgemv(mm, nn, 1.5, 0.7, A, lda, x, y, z, ws, wsb, form, None)

    assert dg(mm=-1) == 1 and dg(nn=-1) == 1
    assert dg(A=None) == 1 and dg(x=None) == 1 and dg(z=None) == 1
    assert dg(lda=k - 1) == 1
    assert dg(form=2) == 1
    assert dg(wsb=need - 1) == 3 and dg(ws=None) == 1
    assert dg(z=ptr(1)) == 2                       # z on top of x
    assert dg(z=v(base + 8)) == 2                  # z inside A
    assert dg(z=v(base + (2 << 20) + 8)) == 2      # z partly over y
    assert dg(z=ptr(16)) == 2                      # z inside the workspace
    assert dg(mm=65535 * 32 + 1, nn=1, lda=1) == 5  # more rows than the grid addresses
    gneed = bto.workspace_bytes("gesummv", m, k, "fused")

    def gs(A=ptr(0), lda=k, B=ptr(4), ldb=k, x=ptr(1), y=ptr(3), ws=ptr(16), wsb=gneed,
           form=0):
        return bto._lib.bto_gesummv(m, k, 1.5, 0.7, A, lda, B, ldb, x, y, ws, wsb, form, None)

    assert gs(B=None) == 1 and gs(ldb=k - 1) == 1 and gs(form=-1) == 1
    assert gs(wsb=gneed - 256) == 3
    assert gs(y=ptr(1)) == 2                       # y on top of x
    assert gs(y=v(base + (4 << 20) + 16)) == 2     # y inside B
    assert gs(y=ptr(0)) == 2                       # y on top of A
    uneed = bto.workspace_bytes("gesummv", m, k, "unfused")
    assert gs(form=1, wsb=uneed - 1) == 3


def test_pass_and_dot_checks(bto):
    """The fused pass and the plain dot: refusals before anything is enqueued."""
    v = ctypes.c_void_p
    m = n = 256
    ptr = lambda i: FAKE + (i << 20)
    R, C, S, K, H = (bto.PASS_ROWDOT, bto.PASS_COLSUM, bto.PASS_STORE, bto.PASS_CONTRACT,
                     bto.PASS_CHAIN)
    assert bto.pass_workspace_bytes(R | C, 16384, 16384) >= bto.workspace_bytes("bicgk", 16384,
                                                                               16384)
    assert bto.pass_workspace_bytes(R | C | H, 300, 40) == bto.workspace_bytes("atax", 300, 40)
    assert bto.pass_workspace_bytes(64, 5, 5) == 0 and bto.pass_workspace_bytes(R, -1, 5) == 0

    def call(ops, wsb=None, **kw):
        d = bto.PassDesc(ops, kw.get("m", m), kw.get("n", n), kw.get("A", ptr(0)),
                         kw.get("lda", n), kw.get("B", ptr(1)), kw.get("ldb", n),
                         kw.get("u1", ptr(2)), kw.get("v1", ptr(3)), kw.get("u2", ptr(4)),
                         kw.get("v2", ptr(5)), kw.get("x", ptr(6)), kw.get("y", ptr(7)),
                         kw.get("row_out", ptr(8)), 1.0, kw.get("row_add"),
                         kw.get("row_add_scale", 1.0), kw.get("col_out", ptr(9)), 1.0,
                         kw.get("col_add"), kw.get("col_add_scale", 1.0))
        need = bto.pass_workspace_bytes(ops, d.m, d.n)
        return bto._lib.bto_pass(ctypes.byref(d), v(ptr(16)), need if wsb is None else wsb,
                                 None)

    assert bto._lib.bto_pass(None, None, 0, None) == 1
    assert call(0) == 1                         # computes nothing
    assert call(64 | R) == 1                    # unknown flag
    assert call(R | S | K) == 1                 # store and contract
    assert call(K) == 1                         # contract without a reduction
    assert call(R | H) == 1                     # chain without column sums
    assert call(R | C | H, y=None, col_add=ptr(10)) == 1     # chain takes no add
    assert call(R | C | K) == 5                 # a contracted pass does one of the two
    assert call(R | K, row_add=ptr(10), row_add_scale=2.0) == 5
    assert call(R, x=None) == 1 and call(C, col_out=None) == 1 and call(S | C, u1=None) == 1
    assert call(R, lda=n - 1) == 1 and call(S, ldb=n - 1) == 1
    assert call(R, wsb=0) == 3
    assert call(R, row_out=ptr(0) + 8) == 2     # row output inside A
    assert call(R | C, col_out=ptr(8)) == 2     # the two outputs meet
    assert call(S | C, B=ptr(0) + 8) == 2       # B overlaps A without being A
    assert call(R, row_add=ptr(8) + 8) == 2     # the add partly over the output
    dn = bto._lib.bto_dot_workspace_bytes(1000)
    assert dn > 0 and bto._lib.bto_dot_workspace_bytes(-1) == 0
    assert bto._lib.bto_dot(-1, v(ptr(0)), v(ptr(1)), v(ptr(2)), v(ptr(16)), dn, None) == 1
    assert bto._lib.bto_dot(1000, None, v(ptr(1)), v(ptr(2)), v(ptr(16)), dn, None) == 1
    assert bto._lib.bto_dot(1000, v(ptr(0)), v(ptr(1)), v(ptr(2)), v(ptr(16)), dn - 1, None) == 3
    assert bto._lib.bto_dot(1000, v(ptr(0)), v(ptr(1)), v(ptr(0) + 8), v(ptr(16)), dn,
                            None) == 2


def test_lincomb_checks(bto):
    """Refusals of the linear combination before anything is enqueued."""
    P = ctypes.c_void_p
    ptrs = lambda *a: (P * len(a))(*[P(x) for x in a])
    cs = lambda k: (ctypes.c_double * k)(*([1.0] * k))
    x = [FAKE + (k << 20) for k in range(9)]
    call = lambda n, k, xs, out: bto._lib.bto_lincomb(n, k, xs, cs(max(k, 1)), P(out), None)
    assert call(10, 0, ptrs(x[0]), x[8]) == 1               # no term
    assert call(10, 9, ptrs(*x), x[8]) == 1                 # more than eight
    assert call(-1, 1, ptrs(x[0]), x[8]) == 1
    assert bto._lib.bto_lincomb(10, 1, None, cs(1), P(x[8]), None) == 1
    assert call(10, 2, ptrs(x[0], 0), x[8]) == 1            # a NULL vector
    assert call(10, 2, ptrs(x[0], x[1]), x[1] + 8) == 2     # out partly over x1
    assert call(10, 2, ptrs(x[0], x[1]), x[0] + 8) == 2     # out partly over x0


def test_contracted_gemver_and_batax_checks(bto):
    """GEMVER without B and BATAX: workspace sizes and the argument checks,
    before anything is enqueued."""
    v = ctypes.c_void_p
    n = 16384
    wc = bto.workspace_bytes("gemver_contracted", n, n)
    assert bto.workspace_bytes("gemver", n, n) < wc < 0.05 * n * n * 8 and wc % 256 == 0
    assert bto.workspace_bytes("batax", n, n, "fused") == bto.workspace_bytes("atax", n, n, "fused")
    assert bto.workspace_bytes("batax", 300, 40, "unfused") == \
        bto.workspace_bytes("atax", 300, 40, "unfused")
    m = k = 256
    base = FAKE
    ptr = lambda i: v(base + (i << 20))
    need = bto.workspace_bytes("gemver_contracted", m, k)

    def gc(A=ptr(0), lda=k, x=ptr(7), w=ptr(8), ws=ptr(16), wsb=need, mm=m, nn=k):
        return bto._lib.bto_gemver_contracted(mm, nn, 1.5, 0.7, A, lda, ptr(1), ptr(2), ptr(3),
                                              ptr(4), ptr(5), ptr(6), x, w, ws, wsb, None)

    assert gc(mm=-1) == 1
    assert gc(A=None) == 1
    assert gc(lda=k - 1) == 1
    assert gc(wsb=need - 1) == 3
    assert gc(x=ptr(5)) == 2                       # x on top of y
    assert gc(w=v(base + 8)) == 2                  # w inside A
    wb = bto.workspace_bytes("batax", m, k, "fused")
    assert bto._lib.bto_batax(m, k, 2.0, ptr(0), k, ptr(1), ptr(1), ptr(16), wb, 0, None) == 2
    assert bto._lib.bto_batax(m, k, 2.0, ptr(0), k, ptr(1), ptr(2), ptr(16), wb - 256, 0,
                              None) == 3
    assert bto._lib.bto_batax(m, k, 2.0, ptr(0), k, ptr(1), ptr(2), ptr(16), wb, 7, None) == 1


def test_noalloc_refuses_beyond_its_scratch(bto):
    """bto_gemver_noalloc checks its scratch need before any HIP call:
    n = m = 16384 fits the 80 MiB exactly, one row more is refused."""
    assert bto.gemver_noalloc_max_scratch_bytes() == 80 << 20
    assert bto.workspace_bytes("gemver", 16384, 16384, "fused") == 80 << 20
    WS = 3
    v = ctypes.c_void_p
    for form in (0, 1):
        st = bto._lib.bto_gemver_noalloc(16385, 16384, 1.5, 0.7, v(FAKE), 16384, v(FAKE),
                                         v(FAKE), v(FAKE), v(FAKE), v(FAKE), v(FAKE), v(FAKE),
                                         16384, v(FAKE), v(FAKE), form, None)
        assert st == WS
        assert "scratch" in bto._lib.bto_last_error().decode()
    assert bto._lib.bto_gemver_noalloc(-1, 4, 1.5, 0.7, v(FAKE), 4, v(FAKE), v(FAKE), v(FAKE),
                                       v(FAKE), v(FAKE), v(FAKE), v(FAKE), 4, v(FAKE), v(FAKE),
                                       0, None) == 1
    assert bto._lib.bto_gemver_noalloc(4, 4, 1.5, 0.7, v(FAKE), 4, v(FAKE), v(FAKE), v(FAKE),
                                       v(FAKE), v(FAKE), v(FAKE), v(FAKE), 4, v(FAKE), v(FAKE),
                                       9, None) == 1
