"""GPU parity: every kernel, both forms, against the CPU oracle.

Tolerance: normwise relative error max|gpu - oracle| / max|oracle| <= 1e-12
per output array (absolute when the oracle output is all zero).  With
integer-valued data every intermediate is an exact integer below 2**53, so
both forms must then equal the oracle bit for bit, whatever the summation
order.
"""

import numpy as np
import pytest

import oracle
from paper_1205_1098_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
SEED = synth.SEED
FORMS = ("fused", "unfused")
ALPHA, BETA = 1.5, 0.7


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto, torch.device("cuda:0")


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    if ref.size == 0:
        return 0.0
    num = float(np.max(np.abs(got - ref)))
    den = float(np.max(np.abs(ref)))
    return num / den if den > 0 else num


def host(t):
    return t.detach().cpu().numpy()


def dmat(torch, dev, A, n):
    """Device copy of an (m, lda) host array, returned as an (m, n) view."""
    full = torch.from_numpy(np.ascontiguousarray(A)).to(dev)
    return full[:, :n]


def dvec(torch, dev, v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(dev)


def inputs(kind, m, n, lda, cfg, kern):
    """Host inputs of one case: A (m, lda) and the vectors in ABI order."""
    sid = lambda op: synth.stream_id(cfg, op, kern)
    A = synth.matrix(SEED, sid(0), m, n, lda=lda, kind=kind)
    vec = lambda op, k: synth.vector(SEED, sid(op), k, kind)
    return A, vec


MSHAPES = [(1, 1), (1, 7), (7, 1), (2, 3), (63, 64), (64, 63), (65, 127), (127, 65),
           (256, 256), (512, 512), (513, 1000), (1000, 513), (300, 4097), (4097, 300),
           (2047, 2049)]
LDA_PAD = [0, 3, 8]


def _lda(n, pad):
    return max(n, 1) + pad


# ---- matrix kernels at small and ragged sizes ------------------------------

@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_bicgk(env, m, n, pad, form):
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 1, 0)
    p, r = vec(1, n), vec(2, m)
    q_ref, s_ref = oracle.bicgk(A, p, r, lda=lda)
    q, s = bto.bicgk(dmat(torch, dev, A, n), dvec(torch, dev, p), dvec(torch, dev, r), form=form)
    assert relerr(host(q), q_ref) <= TOL
    assert relerr(host(s), s_ref) <= TOL


# the fused BiCGK sweeps: the tile kernel (slot value 0) and the row-resident
# kernel at each workgroup size; (140000, 301) gives every workgroup more
# than one 64-row batch of row dots, n = 16385 is too wide to hold a row on
# chip and falls back to the tile kernel
SLOT_BICGK_ROWRES = 9


@pytest.mark.parametrize("threads", [0, 256, 512, 1024])
@pytest.mark.parametrize("m,n,pad,kind", [
    (1, 1, 0, "uniform"), (7, 1, 0, "uniform"), (2, 3, 3, "uniform"), (65, 127, 0, "uniform"),
    (513, 1000, 8, "uniform"), (300, 4097, 3, "uniform"), (1000, 8193, 0, "uniform"),
    (40, 16384, 0, "uniform"), (20, 16385, 0, "uniform"), (140000, 301, 0, "uniform"),
    (999, 2049, 0, "int")])
def test_bicgk_fused_paths(env, threads, m, n, pad, kind):
    torch, bto, dev = env
    assert bto.tune_slots()[SLOT_BICGK_ROWRES] == "bicgk_rowres"
    lda = _lda(n, pad)
    A, vec = inputs(kind, m, n, lda, 1, 7)
    p, r = vec(1, n), vec(2, m)
    q_ref, s_ref = oracle.bicgk(A, p, r, lda=lda)
    saved = {b: bto.tune_get(SLOT_BICGK_ROWRES, 256 << b) for b in range(bto.tune_buckets())}
    bto.tune_set(SLOT_BICGK_ROWRES, threads, 0, 0)
    try:
        q, s = bto.bicgk(dmat(torch, dev, A, n), dvec(torch, dev, p), dvec(torch, dev, r))
        torch.cuda.synchronize()
    finally:
        for b, c in saved.items():
            bto.tune_set(SLOT_BICGK_ROWRES, *c, size=256 << b)
    if kind == "int":
        assert np.array_equal(host(q), q_ref) and np.array_equal(host(s), s_ref)
    else:
        assert relerr(host(q), q_ref) <= TOL
        assert relerr(host(s), s_ref) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_gemver(env, m, n, pad, form):
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 2, 0)
    u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
    B_ref, x_ref, w_ref = oracle.gemver(A, u1, v1, u2, v2, y, z, ALPHA, BETA, lda=lda)
    d = lambda a: dvec(torch, dev, a)
    B, x, w = bto.gemver(dmat(torch, dev, A, n), d(u1), d(v1), d(u2), d(v2), d(y), d(z),
                         ALPHA, BETA, form=form)
    assert relerr(host(B), B_ref) <= TOL
    assert relerr(host(x), x_ref) <= TOL
    assert relerr(host(w), w_ref) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("m,n", [(1, 1), (65, 127), (513, 1000), (2047, 2049)])
def test_gemver_in_place(env, m, n, form):
    """B == A (same array, same leading dimension) gives the out-of-place result,
    and leaves the row padding untouched."""
    torch, bto, dev = env
    lda = n + 5
    A, vec = inputs("uniform", m, n, lda, 2, 1)
    u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
    B_ref, x_ref, w_ref = oracle.gemver(A, u1, v1, u2, v2, y, z, ALPHA, BETA, lda=lda)
    full = torch.from_numpy(A).to(dev)
    Ad = full[:, :n]
    d = lambda a: dvec(torch, dev, a)
    B, x, w = bto.gemver(Ad, d(u1), d(v1), d(u2), d(v2), d(y), d(z), ALPHA, BETA, form=form,
                         B=Ad)
    assert B.data_ptr() == Ad.data_ptr()
    assert relerr(host(Ad), B_ref) <= TOL
    assert relerr(host(x), x_ref) <= TOL and relerr(host(w), w_ref) <= TOL
    assert np.all(np.isnan(host(full)[:, n:]))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES + [(3000, 8192), (700, 8193), (300, 16384)])
def test_atax(env, m, n, pad, form):
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 3, 0)
    x = vec(1, n)
    y_ref = oracle.atax(A, x, lda=lda)
    y = bto.atax(dmat(torch, dev, A, n), dvec(torch, dev, x), form=form)
    assert relerr(host(y), y_ref) <= TOL


@pytest.mark.parametrize("form", FORMS)
def test_atax_wider_than_one_row_on_chip(env, form):
    """n above 16384 backs off to the two-pass form."""
    torch, bto, dev = env
    m, n = 40, 16385
    A, vec = inputs("uniform", m, n, n, 3, 1)
    x = vec(1, n)
    y = bto.atax(dmat(torch, dev, A, n), dvec(torch, dev, x), form=form)
    assert relerr(host(y), oracle.atax(A, x)) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_dgemvt(env, m, n, pad, form):
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 4, 0)
    y, z = vec(1, m), vec(2, n)
    x_ref, w_ref = oracle.dgemvt(A, y, z, ALPHA, BETA, lda=lda)
    x, w = bto.dgemvt(dmat(torch, dev, A, n), dvec(torch, dev, y), dvec(torch, dev, z),
                      ALPHA, BETA, form=form)
    assert relerr(host(x), x_ref) <= TOL
    assert relerr(host(w), w_ref) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("m,n", [(0, 5), (5, 0), (0, 0)])
def test_empty_matrix_extents(env, m, n, form):
    torch, bto, dev = env
    A = torch.zeros((m, n), dtype=torch.float64, device=dev)
    rnd = lambda k, s: dvec(torch, dev, synth.uniform(SEED, s, k))
    q, s = bto.bicgk(A, rnd(n, 1), rnd(m, 2), form=form)
    assert np.all(host(q) == 0) and np.all(host(s) == 0)
    z = rnd(n, 3)
    B, x, w = bto.gemver(A, rnd(m, 4), rnd(n, 5), rnd(m, 6), rnd(n, 7), rnd(m, 8), z,
                         ALPHA, BETA, form=form)
    assert np.array_equal(host(x), host(z)) and np.all(host(w) == 0)
    x2, w2 = bto.dgemvt(A, rnd(m, 9), z, ALPHA, BETA, form=form)
    assert np.array_equal(host(x2), host(z)) and np.all(host(w2) == 0)
    assert np.all(host(bto.atax(A, rnd(n, 10), form=form)) == 0)


# ---- vector kernels ---------------------------------------------------------

VSIZES = [0, 1, 2, 3, 127, 511, 512, 513, 4095, 4096, 4097, 100003, (1 << 20) + 1]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", VSIZES)
def test_vector_kernels(env, n, form):
    torch, bto, dev = env
    v = lambda op: synth.uniform(SEED, synth.stream_id(5, op), n)
    d = lambda a: dvec(torch, dev, a)
    w, vv, u = v(0), v(1), v(2)
    z_ref, r_ref = oracle.axpydot(w, vv, u, ALPHA)
    z, r = bto.axpydot(d(w), d(vv), d(u), ALPHA, form=form)
    assert relerr(host(z), z_ref) <= TOL
    assert relerr(host(r), np.array([r_ref])) <= TOL
    assert relerr(host(bto.waxpby(d(w), d(vv), ALPHA, BETA, form=form)),
                  oracle.waxpby(w, vv, ALPHA, BETA)) <= TOL
    assert relerr(host(bto.vadd(d(w), d(vv), d(u), form=form)), oracle.vadd(w, vv, u)) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n", [1, 2, 4097, 100003])
def test_vector_kernels_misaligned(env, n, form):
    """Views starting one element into an allocation (8-byte, not 16-byte,
    aligned) take the scalar path and give the same results."""
    torch, bto, dev = env
    v = lambda op: synth.uniform(SEED, synth.stream_id(5, op, 1), n + 1)
    w, vv, u = v(0), v(1), v(2)
    d = lambda a: dvec(torch, dev, a)[1:]
    z_ref, r_ref = oracle.axpydot(w[1:], vv[1:], u[1:], ALPHA)
    zbuf = torch.empty(n + 1, dtype=torch.float64, device=dev)
    z, r = bto.axpydot(d(w), d(vv), d(u), ALPHA, form=form, z=zbuf[1:])
    assert relerr(host(z), z_ref) <= TOL and relerr(host(r), np.array([r_ref])) <= TOL
    wbuf = torch.empty(n + 1, dtype=torch.float64, device=dev)
    out = bto.waxpby(d(w), d(vv), ALPHA, BETA, form=form, w=wbuf[1:])
    assert relerr(host(out), oracle.waxpby(w[1:], vv[1:], ALPHA, BETA)) <= TOL
    out = bto.vadd(d(w), d(vv), d(u), form=form, x=wbuf[1:])
    assert relerr(host(out), oracle.vadd(w[1:], vv[1:], u[1:])) <= TOL


@pytest.mark.parametrize("form", FORMS)
def test_vector_exact_aliases(env, form):
    torch, bto, dev = env
    n = 100003
    v = lambda op: synth.uniform(SEED, synth.stream_id(5, op, 2), n)
    w, vv, u = v(0), v(1), v(2)
    d = lambda a: dvec(torch, dev, a)
    wd = d(w)
    z, r = bto.axpydot(wd, d(vv), d(u), ALPHA, form=form, z=wd)          # z == w
    z_ref, r_ref = oracle.axpydot(w, vv, u, ALPHA)
    assert relerr(host(wd), z_ref) <= TOL and relerr(host(r), np.array([r_ref])) <= TOL
    for which in ("x", "y"):
        xd, yd = d(w), d(vv)
        out = xd if which == "x" else yd
        bto.waxpby(xd, yd, ALPHA, BETA, form=form, w=out)
        assert relerr(host(out), oracle.waxpby(w, vv, ALPHA, BETA)) <= TOL
    for which in range(3):
        ins = [d(w), d(vv), d(u)]
        bto.vadd(*ins, form=form, x=ins[which])
        assert relerr(host(ins[which]), oracle.vadd(w, vv, u)) <= TOL


# ---- closed forms, determinism, forms agree ---------------------------------

@pytest.mark.parametrize("form", FORMS)
def test_identity_closed_forms(env, form):
    torch, bto, dev = env
    n = 3001
    I = torch.eye(n, dtype=torch.float64, device=dev)
    x = dvec(torch, dev, synth.uniform(SEED, 77, n))
    assert torch.equal(bto.atax(I, x, form=form), x)
    q, s = bto.bicgk(I, x, x, form=form)
    assert torch.equal(q, x) and torch.equal(s, x)


@pytest.mark.parametrize("form", FORMS)
def test_repeatable_bitwise(env, form):
    torch, bto, dev = env
    m, n = 4097, 3001
    A, vec = inputs("uniform", m, n, n, 6, 0)
    d = lambda a: dvec(torch, dev, a)
    Ad = d(A)
    args = [d(vec(1, m)), d(vec(2, n)), d(vec(3, m)), d(vec(4, n)), d(vec(5, m)), d(vec(6, n))]
    first = [host(t) for t in bto.gemver(Ad, *args, ALPHA, BETA, form=form)]
    again = [host(t) for t in bto.gemver(Ad, *args, ALPHA, BETA, form=form)]
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    q1, s1 = bto.bicgk(Ad, args[1], args[0], form=form)
    q2, s2 = bto.bicgk(Ad, args[1], args[0], form=form)
    assert torch.equal(q1, q2) and torch.equal(s1, s2)
    assert torch.equal(bto.atax(Ad, args[1], form=form), bto.atax(Ad, args[1], form=form))


def test_errors_raise(env):
    torch, bto, dev = env
    A = torch.zeros((64, 64), dtype=torch.float64, device=dev)
    p = torch.zeros(64, dtype=torch.float64, device=dev)
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(bto.BtoError) as e:
        bto.bicgk(A, p, p, ws=small)
    assert e.value.status == 3
    with pytest.raises(bto.BtoError) as e:
        bto.bicgk(A, p, p, q=A[0], s=torch.empty(64, dtype=torch.float64, device=dev))
    assert e.value.status == 2          # q lies inside A
    with pytest.raises(ValueError, match="length"):
        bto.bicgk(A, p, p, s=torch.empty(63, dtype=torch.float64, device=dev))
    with pytest.raises(bto.BtoError) as e:
        buf = torch.zeros(200, dtype=torch.float64, device=dev)
        bto.vadd(buf[:100], buf[100:], buf[100:], x=buf[50:150])
    assert e.value.status == 2


# ---- full-size workloads (the benchmark's launch configuration) -------------

N = 16384
NV = 1 << 26


def _full_matrix_case(env, kind, kern):
    torch, bto, dev = env
    A, vec = inputs(kind, N, N, N, 3, kern)
    return torch, bto, dev, A, vec


@pytest.mark.parametrize("kind", ["uniform", "int"])
def test_full_bicgk_and_atax(env, kind):
    torch, bto, dev, A, vec = _full_matrix_case(env, kind, 10)
    p, r = vec(1, N), vec(2, N)
    Ad, pd, rd = dvec(torch, dev, A), dvec(torch, dev, p), dvec(torch, dev, r)
    q_ref, s_ref = oracle.bicgk(A, p, r)
    y_ref = oracle.atax(A, p)
    outs = {}
    for form in FORMS:
        q, s = bto.bicgk(Ad, pd, rd, form=form)
        y = bto.atax(Ad, pd, form=form)
        outs[form] = (host(q), host(s), host(y))
        for got, ref in zip(outs[form], (q_ref, s_ref, y_ref)):
            if kind == "int":
                assert np.array_equal(got, ref)
            else:
                assert relerr(got, ref) <= TOL
    be = 3.0 if kind == "int" else BETA
    for form in FORMS:
        y = host(bto.batax(Ad, pd, be, form=form))
        if kind == "int":
            assert np.array_equal(y, be * y_ref)
        else:
            assert relerr(y, be * y_ref) <= TOL
    q, s, _ = outs["fused"]
    lhs, rhs = float(r @ q), float(s @ p)
    assert abs(lhs - rhs) <= 1e-12 * float(np.abs(r) @ np.abs(q) + np.abs(s) @ np.abs(p))


@pytest.mark.parametrize("kind", ["uniform", "int"])
def test_full_gemver(env, kind):
    torch, bto, dev, A, vec = _full_matrix_case(env, kind, 11)
    vs = [vec(k, N) for k in range(1, 7)]
    al, be = (2.0, 3.0) if kind == "int" else (ALPHA, BETA)
    B_ref, x_ref, w_ref = oracle.gemver(A, *vs, al, be)
    Ad = dvec(torch, dev, A)
    dv = [dvec(torch, dev, v) for v in vs]
    Bd = torch.empty_like(Ad)
    for form in FORMS:
        B, x, w = bto.gemver(Ad, *dv, al, be, form=form, B=Bd)
        for got, ref in zip((host(B), host(x), host(w)), (B_ref, x_ref, w_ref)):
            if kind == "int":
                assert np.array_equal(got, ref)
            else:
                assert relerr(got, ref) <= TOL
        del B
    x, w = bto.gemver_contracted(Ad, *dv, al, be)
    for got, ref in zip((host(x), host(w)), (x_ref, w_ref)):
        if kind == "int":
            assert np.array_equal(got, ref)
        else:
            assert relerr(got, ref) <= TOL


@pytest.mark.parametrize("kind", ["uniform", "int"])
def test_full_dgemv_gesummv(env, kind):
    torch, bto, dev, A, vec = _full_matrix_case(env, kind, 13)
    B = synth.matrix(SEED, synth.stream_id(3, 9, 13), N, N, kind=kind)
    x, y = vec(1, N), vec(2, N)
    al, be = (2.0, 3.0) if kind == "int" else (ALPHA, BETA)
    z_ref = oracle.dgemv(A, x, y, al, be)
    g_ref = oracle.gesummv(A, B, x, al, be)
    Ad, Bd, xd, yd = (dvec(torch, dev, t) for t in (A, B, x, y))
    for form in FORMS:
        got = (host(bto.dgemv(Ad, xd, yd, al, be, form=form)),
               host(bto.gesummv(Ad, Bd, xd, al, be, form=form)))
        for g, ref in zip(got, (z_ref, g_ref)):
            if kind == "int":
                assert np.array_equal(g, ref)
            else:
                assert relerr(g, ref) <= TOL


@pytest.mark.parametrize("kind", ["uniform", "int"])
def test_full_dgemvt(env, kind):
    torch, bto, dev, A, vec = _full_matrix_case(env, kind, 12)
    y, z = vec(1, N), vec(2, N)
    al, be = (2.0, 3.0) if kind == "int" else (ALPHA, BETA)
    x_ref, w_ref = oracle.dgemvt(A, y, z, al, be)
    Ad, yd, zd = dvec(torch, dev, A), dvec(torch, dev, y), dvec(torch, dev, z)
    for form in FORMS:
        x, w = bto.dgemvt(Ad, yd, zd, al, be, form=form)
        for got, ref in zip((host(x), host(w)), (x_ref, w_ref)):
            if kind == "int":
                assert np.array_equal(got, ref)
            else:
                assert relerr(got, ref) <= TOL


@pytest.mark.parametrize("kind", ["uniform", "int"])
def test_full_vectors(env, kind):
    torch, bto, dev = env
    v = lambda op: synth.vector(SEED, synth.stream_id(3, op, 13), NV, kind)
    w, vv, u = v(0), v(1), v(2)
    al, be = (2.0, 3.0) if kind == "int" else (ALPHA, BETA)
    z_ref, r_ref = oracle.axpydot(w, vv, u, al)
    wx_ref = oracle.waxpby(w, vv, al, be)
    va_ref = oracle.vadd(w, vv, u)
    d = lambda a: dvec(torch, dev, a)
    wd, vd, ud = d(w), d(vv), d(u)
    for form in FORMS:
        z, r = bto.axpydot(wd, vd, ud, al, form=form)
        got = [host(z), host(r), host(bto.waxpby(wd, vd, al, be, form=form)),
               host(bto.vadd(wd, vd, ud, form=form))]
        ref = [z_ref, np.array([r_ref]), wx_ref, va_ref]
        for g, rf in zip(got, ref):
            if kind == "int":
                assert np.array_equal(g, rf)
            else:
                assert relerr(g, rf) <= TOL


# ---- every compiled tile shape in every slot that can run it --------------------
#
# The autotuner may give a slot any shape the library accepts for it; each
# such (slot, shape) runs here once on ragged shapes (odd n takes the
# scalar path, even n with an odd padding the misaligned path) against the
# oracle.  The slot's per-bucket table is restored afterwards.

SLOT_KERNEL = {0: ("bicgk", "fused"), 1: ("bicgk", "unfused"), 2: ("bicgk", "unfused"),
               3: ("gemver", "unfused"), 4: ("gemver", "fused"), 5: ("gemver", "fused"),
               6: ("dgemvt", "fused"), 7: ("dgemvt", "fused")}


def _run_kernel(torch, bto, dev, kernel, form, m, n, pad):
    lda = _lda(n, pad)
    d = lambda a: dvec(torch, dev, a)
    if kernel == "bicgk":
        A, vec = inputs("uniform", m, n, lda, 1, 11)
        p, r = vec(1, n), vec(2, m)
        ref = oracle.bicgk(A, p, r, lda=lda)
        got = bto.bicgk(dmat(torch, dev, A, n), d(p), d(r), form=form)
    elif kernel == "gemver":
        A, vec = inputs("uniform", m, n, lda, 2, 11)
        u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
        ref = oracle.gemver(A, u1, v1, u2, v2, y, z, ALPHA, BETA, lda=lda)
        got = bto.gemver(dmat(torch, dev, A, n), d(u1), d(v1), d(u2), d(v2), d(y), d(z),
                         ALPHA, BETA, form=form)
    elif kernel == "gemver_contracted":
        A, vec = inputs("uniform", m, n, lda, 2, 12)
        u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
        ref = oracle.gemver(A, u1, v1, u2, v2, y, z, ALPHA, BETA, lda=lda)[1:]
        got = bto.gemver_contracted(dmat(torch, dev, A, n), d(u1), d(v1), d(u2), d(v2), d(y),
                                    d(z), ALPHA, BETA)
    elif kernel == "gesummv":     # with DGEMV: both are row-dot sweeps of slot gemv_n
        A, vec = inputs("uniform", m, n, lda, 4, 24)
        B = synth.matrix(SEED, synth.stream_id(4, 9, 24), m, n, lda=lda)
        x, y = vec(1, n), vec(2, m)
        ref = [oracle.dgemv(A, x, y, ALPHA, BETA, lda=lda),
               oracle.gesummv(A, B, x, ALPHA, BETA, m=m, lda=lda, ldb=lda)]
        Ad = dmat(torch, dev, A, n)
        got = [bto.dgemv(Ad, d(x), d(y), ALPHA, BETA, form=form),
               bto.gesummv(Ad, dmat(torch, dev, B, n), d(x), ALPHA, BETA, form=form)]
    else:
        A, vec = inputs("uniform", m, n, lda, 4, 11)
        y, z = vec(1, m), vec(2, n)
        ref = oracle.dgemvt(A, y, z, ALPHA, BETA, lda=lda)
        got = bto.dgemvt(dmat(torch, dev, A, n), d(y), d(z), ALPHA, BETA, form=form)
    torch.cuda.synchronize()
    return [host(g) for g in got], ref


# shapes 0..5 serve the read-only sweeps (shape 1 cannot hold both BiCGK
# vectors), 6..14 the sweeps that store B (slots 3 and 4)
SHAPE_CASES = [(slot, shape) for slot in sorted(SLOT_KERNEL)
               for shape in (range(6, 15) if slot in (3, 4) else range(6))
               if not (slot == 0 and shape == 1)]


@pytest.mark.parametrize("slot,shape", SHAPE_CASES)
def test_every_tile_shape(env, slot, shape):
    torch, bto, dev = env
    kernel, form = SLOT_KERNEL[slot]
    saved = {b: bto.tune_get(slot, 256 << b) for b in range(bto.tune_buckets())}
    saved_rowres = {b: bto.tune_get(SLOT_BICGK_ROWRES, 256 << b)
                    for b in range(bto.tune_buckets())}
    try:
        rb = None
        for cand in (32, 64, 8, 4):
            try:
                bto.tune_set(slot, shape, cand, 1)
                rb = cand
                break
            except bto.BtoError:
                continue
        assert rb is not None, f"slot {slot} refuses shape {shape}"
        if slot == 0:
            bto.tune_set(SLOT_BICGK_ROWRES, 0, 0, 0)     # the tile sweep, not the row-resident one
        for m, n, pad in [(333, 1030, 3), (130, 517, 0), (1, 2, 0)]:
            got, ref = _run_kernel(torch, bto, dev, kernel, form, m, n, pad)
            for g, r in zip(got, ref):
                assert relerr(g, r) <= TOL, (slot, shape, rb, m, n, pad)
            if kernel == "dgemvt":   # the same slots serve GEMVER without B
                got, ref = _run_kernel(torch, bto, dev, "gemver_contracted", form, m, n, pad)
                for g, r in zip(got, ref):
                    assert relerr(g, r) <= TOL, ("contracted", slot, shape, rb, m, n, pad)
            if slot == 1:            # and gemv_n serves DGEMV and GESUMMV
                for f in FORMS:
                    got, ref = _run_kernel(torch, bto, dev, "gesummv", f, m, n, pad)
                    for g, r in zip(got, ref):
                        assert relerr(g, r) <= TOL, ("gesummv", f, shape, rb, m, n, pad)
    finally:
        for b, c in saved.items():
            bto.tune_set(slot, *c, size=256 << b)
        for b, c in saved_rowres.items():
            bto.tune_set(SLOT_BICGK_ROWRES, *c, size=256 << b)


# ---- one fused pass (bto_pass) on every shape of the sweeps that store B ---------
#
# A pass that stores the update and also takes row dots runs the store
# shapes, some of them one 16-byte pair wide per lane: its row-dot partials
# must fit the workspace next to the column-sum partials.

@pytest.mark.parametrize("shape", range(6, 15))
def test_store_pass_every_shape(env, shape):
    torch, bto, dev = env
    slot = 4     # gemver_p1: the configuration a storing pass takes
    saved = {b: bto.tune_get(slot, 256 << b) for b in range(bto.tune_buckets())}
    try:
        for b in range(bto.tune_buckets()):
            bto.tune_set(slot, shape, 32, 1, size=256 << b)
        for m, n, pad in [(513, 1000, 0), (300, 300, 3), (65, 127, 0)]:
            lda = _lda(n, pad)
            A, vec = inputs("uniform", m, n, lda, 2, 25)
            u1, v1, u2, v2, p, r = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, n), vec(6, m)
            B_ref = oracle.gemver(A, u1, v1, u2, v2, r, p, 1.0, 1.0, lda=lda)[0]
            q_ref, s_ref = oracle.bicgk(B_ref, p, r)
            d = lambda a: dvec(torch, dev, a)
            for ops in (bto.PASS_STORE | bto.PASS_ROWDOT,
                        bto.PASS_STORE | bto.PASS_ROWDOT | bto.PASS_COLSUM):
                Bd = torch.empty((m, n), dtype=torch.float64, device=dev)
                q = torch.empty(m, dtype=torch.float64, device=dev)
                s = torch.empty(n, dtype=torch.float64, device=dev)
                kw = dict(B=Bd, u1=d(u1), v1=d(v1), u2=d(u2), v2=d(v2), x=d(p), row_out=q)
                if ops & bto.PASS_COLSUM:
                    kw.update(y=d(r), col_out=s)
                bto.fused_pass(ops, dmat(torch, dev, A, n), **kw)
                assert relerr(host(Bd), B_ref) <= TOL, (shape, m, n, ops)   # FMA may form B
                assert relerr(host(q), q_ref) <= TOL, (shape, m, n, ops)
                if ops & bto.PASS_COLSUM:
                    assert relerr(host(s), s_ref) <= TOL, (shape, m, n, ops)
    finally:
        for b, c in saved.items():
            bto.tune_set(slot, *c, size=256 << b)


# ---- linear combination of up to eight vectors (bto_lincomb) --------------------

@pytest.mark.parametrize("count", range(1, 9))
@pytest.mark.parametrize("n,offset", [(0, 0), (1, 0), (1025, 0), (1 << 20, 1), (4097, 1)])
def test_lincomb(env, count, n, offset):
    """Against sums left to right of the oracle's scaled vectors (WAXPBY with
    a zero second scale is the plain product), and bitwise on integers; the
    output may be one of the inputs."""
    torch, bto, dev = env
    coefs = [1.5 - 0.25 * k for k in range(count)]
    xs = [synth.uniform(SEED, synth.stream_id(5, k, n), n) for k in range(count)]
    ref = oracle.waxpby(xs[0], xs[0], coefs[0], 0.0)
    for k in range(1, count):
        ref = oracle.vadd(ref, oracle.waxpby(xs[k], xs[k], coefs[k], 0.0), np.zeros(n))
    dx = []
    for x in xs:     # offset 1: storage misaligned by one element (scalar path)
        buf = torch.empty(n + offset, dtype=torch.float64, device=dev)
        buf[offset:] = torch.from_numpy(x).to(dev)
        dx.append(buf[offset:])
    out = bto.lincomb(dx, coefs)
    assert relerr(host(out), ref) <= TOL
    ints = [synth.vector(SEED, synth.stream_id(5, 10 + k, n), n, "int") for k in range(count)]
    di = [dvec(torch, dev, v) for v in ints]
    got = bto.lincomb(di, [k - 3.0 for k in range(count)], out=di[-1])   # in place
    want = sum((k - 3) * v.astype(np.int64) for k, v in enumerate(ints))
    assert np.array_equal(host(got), np.asarray(want, dtype=np.float64).reshape(n))


# ---- DGEMV and GESUMMV --------------------------------------------------------

@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_dgemv(env, m, n, pad, form):
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 4, 20)
    x, y = vec(1, n), vec(2, m)
    z_ref = oracle.dgemv(A, x, y, ALPHA, BETA, lda=lda)
    z = bto.dgemv(dmat(torch, dev, A, n), dvec(torch, dev, x), dvec(torch, dev, y), ALPHA, BETA,
                  form=form)
    assert relerr(host(z), z_ref) <= TOL
    # in place: z is y itself, as in the BLAS call
    yd = dvec(torch, dev, y)
    bto.dgemv(dmat(torch, dev, A, n), dvec(torch, dev, x), yd, ALPHA, BETA, form=form, z=yd)
    assert np.array_equal(host(yd), host(z))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_gesummv(env, m, n, pad, form):
    """A and B with different leading dimensions (B's padding is A's + 5)."""
    torch, bto, dev = env
    lda, ldb = _lda(n, pad), _lda(n, pad + 5)
    A, vec = inputs("uniform", m, n, lda, 4, 21)
    B = synth.matrix(SEED, synth.stream_id(4, 9, 21), m, n, lda=ldb)
    x = vec(1, n)
    y_ref = oracle.gesummv(A, B, x, ALPHA, BETA, m=m, lda=lda, ldb=ldb)
    y = bto.gesummv(dmat(torch, dev, A, n), dmat(torch, dev, B, n), dvec(torch, dev, x), ALPHA,
                    BETA, form=form)
    assert relerr(host(y), y_ref) <= TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("m,n", [(1, 1), (65, 127), (513, 1000), (2047, 2049), (3000, 64)])
def test_dgemv_gesummv_integers_exact(env, m, n, form):
    torch, bto, dev = env
    A, vec = inputs("int", m, n, n, 4, 22)
    B = synth.matrix(SEED, synth.stream_id(4, 9, 22), m, n, kind="int")
    x, y = vec(1, n), vec(2, m)
    Ad, Bd, xd = dmat(torch, dev, A, n), dmat(torch, dev, B, n), dvec(torch, dev, x)
    z = bto.dgemv(Ad, xd, dvec(torch, dev, y), 2.0, -3.0, form=form)
    assert np.array_equal(host(z), oracle.dgemv(A, x, y, 2.0, -3.0))
    g = bto.gesummv(Ad, Bd, xd, 2.0, 3.0, form=form)
    assert np.array_equal(host(g), oracle.gesummv(A, B, x, 2.0, 3.0))
    # B may be A itself; with beta = -alpha the two terms cancel exactly
    g = bto.gesummv(Ad, Ad, xd, 2.0, -2.0, form=form)
    assert np.array_equal(host(g), np.zeros(m))


@pytest.mark.parametrize("form", FORMS)
def test_dgemv_gesummv_empty_extents(env, form):
    torch, bto, dev = env
    rnd = lambda k, s: dvec(torch, dev, synth.uniform(SEED, s, k))
    y = rnd(4, 2)
    A = torch.empty((4, 2), dtype=torch.float64, device=dev)[:, :0]
    z = bto.dgemv(A, rnd(0, 1), y, ALPHA, BETA, form=form)
    assert np.array_equal(host(z), BETA * host(y))
    g = bto.gesummv(A, A, rnd(0, 3), ALPHA, BETA, form=form)
    assert np.array_equal(host(g), np.zeros(4))
    E = torch.zeros((0, 5), dtype=torch.float64, device=dev)
    assert bto.dgemv(E, rnd(5, 4), rnd(0, 5), ALPHA, BETA, form=form).numel() == 0
    assert bto.gesummv(E, E, rnd(5, 6), ALPHA, BETA, form=form).numel() == 0


# more row bands than one grid dimension holds with the tuned band height:
# the launch takes taller bands (up to the most rows the entry points take)
@pytest.mark.parametrize("m,n", [(300000, 5), (2097100, 2)])
def test_row_dots_past_the_grid_extent(env, m, n):
    torch, bto, dev = env
    A, vec = inputs("uniform", m, n, n, 4, 23)
    B = synth.matrix(SEED, synth.stream_id(4, 9, 23), m, n)
    x, y, r = vec(1, n), vec(2, m), vec(3, m)
    Ad, Bd, xd = dmat(torch, dev, A, n), dmat(torch, dev, B, n), dvec(torch, dev, x)
    z = bto.dgemv(Ad, xd, dvec(torch, dev, y), ALPHA, BETA)
    assert relerr(host(z), oracle.dgemv(A, x, y, ALPHA, BETA)) <= TOL
    g_ref = oracle.gesummv(A, B, x, ALPHA, BETA)
    for form in FORMS:
        g = bto.gesummv(Ad, Bd, xd, ALPHA, BETA, form=form)
        assert relerr(host(g), g_ref) <= TOL
    q, s = bto.bicgk(Ad, xd, dvec(torch, dev, r), form="unfused")
    q_ref, s_ref = oracle.bicgk(A, x, r)
    assert relerr(host(q), q_ref) <= TOL and relerr(host(s), s_ref) <= TOL


# ---- GEMVER with B contracted away, and BATAX ---------------------------------------

@pytest.mark.parametrize("pad", LDA_PAD)
@pytest.mark.parametrize("m,n", MSHAPES)
def test_gemver_contracted(env, m, n, pad):
    """x and w without B: the oracle's GEMVER (which forms B) gives the
    reference; the two differ only in rounding order."""
    torch, bto, dev = env
    lda = _lda(n, pad)
    A, vec = inputs("uniform", m, n, lda, 2, 5)
    u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
    _, x_ref, w_ref = oracle.gemver(A, u1, v1, u2, v2, y, z, ALPHA, BETA, lda=lda)
    d = lambda a: dvec(torch, dev, a)
    x, w = bto.gemver_contracted(dmat(torch, dev, A, n), d(u1), d(v1), d(u2), d(v2), d(y), d(z),
                                 ALPHA, BETA)
    assert relerr(host(x), x_ref) <= TOL
    assert relerr(host(w), w_ref) <= TOL


@pytest.mark.parametrize("m,n", [(1, 1), (65, 127), (513, 1000), (2047, 2049), (3000, 64)])
def test_gemver_contracted_integers_exact(env, m, n):
    torch, bto, dev = env
    A, vec = inputs("int", m, n, n, 2, 6)
    u1, v1, u2, v2, y, z = vec(1, m), vec(2, n), vec(3, m), vec(4, n), vec(5, m), vec(6, n)
    _, x_ref, w_ref = oracle.gemver(A, u1, v1, u2, v2, y, z, 2.0, 3.0)
    d = lambda a: dvec(torch, dev, a)
    x, w = bto.gemver_contracted(dmat(torch, dev, A, n), d(u1), d(v1), d(u2), d(v2), d(y), d(z),
                                 2.0, 3.0)
    assert np.array_equal(host(x), x_ref) and np.array_equal(host(w), w_ref)


def test_gemver_contracted_empty_extents(env):
    torch, bto, dev = env
    rnd = lambda k, s: dvec(torch, dev, synth.uniform(SEED, s, k))
    z = rnd(5, 3)
    x, w = bto.gemver_contracted(torch.zeros((0, 5), dtype=torch.float64, device=dev), rnd(0, 1),
                                 rnd(5, 2), rnd(0, 4), rnd(5, 5), rnd(0, 6), z, ALPHA, BETA)
    assert np.array_equal(host(x), host(z)) and host(w).size == 0
    A = torch.empty((4, 2), dtype=torch.float64, device=dev)[:, :0]
    x, w = bto.gemver_contracted(A, rnd(4, 1), rnd(0, 2), rnd(4, 4), rnd(0, 5), rnd(4, 6),
                                 rnd(0, 7), ALPHA, BETA)
    assert host(x).size == 0 and np.all(host(w) == 0)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("m,n", [(1, 1), (65, 127), (513, 1000), (4097, 300), (300, 16384)])
def test_batax(env, m, n, form):
    """y = beta A^T A x: the oracle's ATAX, scaled after its reduction."""
    torch, bto, dev = env
    A, vec = inputs("uniform", m, n, n, 3, 7)
    x = vec(1, n)
    y_ref = BETA * oracle.atax(A, x)
    y = bto.batax(dmat(torch, dev, A, n), dvec(torch, dev, x), BETA, form=form)
    assert relerr(host(y), y_ref) <= TOL
    yi = bto.batax(dmat(torch, dev, A, n), dvec(torch, dev, x), 1.0, form=form)
    assert torch.equal(yi, bto.atax(dmat(torch, dev, A, n), dvec(torch, dev, x), form=form))
