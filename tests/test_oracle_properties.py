"""Pins the oracle to closed forms and algebraic invariants, and checks that
its results do not depend on the number of threads."""

import numpy as np
import pytest

from paper_1205_1098_amd import synth

SEED = 3


def U(stream, n):
    return synth.uniform(SEED, stream, n)


def M(stream, m, n):
    return synth.matrix(SEED, stream, m, n)


def INT(stream, n):
    return synth.small_ints(SEED, stream, n)


# ---- closed forms ---------------------------------------------------------

@pytest.mark.parametrize("n", [1, 37, 300])
def test_identity(orc, n):
    I = np.eye(n)
    p, r = U(1, n), U(2, n)
    q, s = orc.bicgk(I, p, r)
    assert np.array_equal(q, p) and np.array_equal(s, r)
    # ATAX with A = I gives y = x
    assert np.array_equal(orc.atax(I, p), p)
    # GEMVER with u = v = 0 and A = I: B = I, x = beta y + z, w = alpha x
    zero = np.zeros(n)
    y, z = U(3, n), U(4, n)
    B, x, w = orc.gemver(I, zero, zero, zero, zero, y, z, 1.5, 0.7)
    assert np.array_equal(B, I)
    assert np.array_equal(x, 0.7 * y + z)
    assert np.array_equal(w, 1.5 * x)
    # DGEMVT with A = I: x = beta y + z, w = alpha x
    x2, w2 = orc.dgemvt(I, y, z, 1.5, 0.7)
    assert np.array_equal(x2, 0.7 * y + z)
    assert np.array_equal(w2, 1.5 * x2)
    # DGEMV with A = I: z = alpha x + beta y
    assert np.array_equal(orc.dgemv(I, y, z, 1.5, 0.7), 1.5 * y + 0.7 * z)
    # GESUMMV with A = I and B the reversal permutation: alpha x + beta (reversed x)
    P = np.ascontiguousarray(I[::-1])
    assert np.array_equal(orc.gesummv(I, P, y, 1.5, 0.7), 1.5 * y + 0.7 * y[::-1])


@pytest.mark.parametrize("n", [2, 64, 257])
def test_permutation_and_diagonal(orc, n):
    perm = np.argsort(U(5, n))
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    x = U(6, n)
    # A^T A = I for a permutation matrix
    assert np.array_equal(orc.atax(P, x), x)
    q, s = orc.bicgk(P, x, x)
    assert np.array_equal(q, x[perm])
    s_expect = np.empty(n)
    s_expect[perm] = x
    assert np.array_equal(s, s_expect)
    d = U(7, n)
    # diag(d): y = d * (d * x), the same two roundings the loops perform
    assert np.array_equal(orc.atax(np.diag(d), x), d * (d * x))


@pytest.mark.parametrize("m,n", [(1, 1), (33, 65), (200, 130)])
def test_rank_one(orc, m, n):
    a, b = INT(8, m), INT(9, n)
    A = np.outer(a, b)
    p, r = INT(10, n), INT(11, m)
    q, s = orc.bicgk(A, p, r)
    assert np.array_equal(q, a * float(b @ p))
    assert np.array_equal(s, b * float(a @ r))
    x = INT(12, n)
    assert np.array_equal(orc.atax(A, x), b * float(a @ a) * float(b @ x))


@pytest.mark.parametrize("m,n", [(7, 5), (128, 96)])
def test_gemver_outer_product_only(orc, m, n):
    u1, v1, y, z = INT(13, m), INT(14, n), INT(15, m), INT(16, n)
    zm, zn = np.zeros(m), np.zeros(n)
    B, x, w = orc.gemver(np.zeros((m, n)), u1, v1, zm, zn, y, z, 2.0, 3.0)
    assert np.array_equal(B, np.outer(u1, v1))
    xe = 3.0 * v1 * float(u1 @ y) + z
    assert np.array_equal(x, xe)
    assert np.array_equal(w, 2.0 * u1 * float(v1 @ xe))


def test_axpydot_zero_v(orc):
    n = 5000
    w, u = INT(17, n), INT(18, n)
    z, r = orc.axpydot(w, np.zeros(n), u, 1.5)
    assert np.array_equal(z, w)
    assert r == float(w @ u)


def test_empty_extents(orc):
    A = np.zeros((0, 4))
    q, s = orc.bicgk(A, U(1, 4), np.zeros(0))
    assert q.shape == (0,) and np.array_equal(s, np.zeros(4))
    A = np.zeros((3, 0))
    q, s = orc.bicgk(A, np.zeros(0), U(2, 3))
    assert np.array_equal(q, np.zeros(3)) and s.shape == (0,)
    z = U(3, 4)
    B, x, w = orc.gemver(np.zeros((0, 4)), *[np.zeros(0), U(4, 4)] * 2,
                         np.zeros(0), z, 1.5, 0.7)
    assert np.array_equal(x, z)
    x, w = orc.dgemvt(np.zeros((3, 0)), U(5, 3), np.zeros(0), 1.5, 0.7)
    assert np.array_equal(w, np.zeros(3))
    assert np.array_equal(orc.atax(np.zeros((0, 4)), U(6, 4)), np.zeros(4))
    z, r = orc.axpydot(np.zeros(0), np.zeros(0), np.zeros(0), 1.5)
    assert r == 0.0
    y = U(7, 3)
    assert np.array_equal(orc.dgemv(np.zeros((3, 0)), np.zeros(0), y, 1.5, 0.7), 0.7 * y)
    assert orc.dgemv(np.zeros((0, 4)), U(8, 4), np.zeros(0), 1.5, 0.7).shape == (0,)
    assert np.array_equal(orc.gesummv(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0), 1.5, 0.7),
                          np.zeros(3))


# ---- invariants -----------------------------------------------------------

@pytest.mark.parametrize("m,n", [(200, 150), (150, 200), (1000, 1000)])
def test_bicgk_invariant(orc, m, n):
    A, p, r = M(20, m, n), U(21, n), U(22, m)
    q, s = orc.bicgk(A, p, r)
    # r^T q = s^T p = r^T A p
    lhs, rhs = float(r @ q), float(s @ p)
    scale = float(np.abs(r) @ np.abs(q) + np.abs(s) @ np.abs(p))
    assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("m,n", [(200, 150), (1000, 1000)])
def test_gemver_invariants(orc, m, n):
    A = M(30, m, n)
    u1, u2, y = U(31, m), U(32, m), U(33, m)
    v1, v2, z = U(34, n), U(35, n), U(36, n)
    al, be = 1.5, 0.7
    B, x, w = orc.gemver(A, u1, v1, u2, v2, y, z, al, be)
    # y^T w = alpha y^T B x = (alpha/beta) (x - z)^T x
    lhs, rhs = float(y @ w), al / be * float((x - z) @ x)
    scale = float(np.abs(y) @ np.abs(w)) + al / be * float(np.abs(x - z) @ np.abs(x))
    assert abs(lhs - rhs) <= 1e-12 * scale
    # B - A has rank at most 2: (B - A) c = u1 (v1.c) + u2 (v2.c)
    c = U(37, n)
    lhs = (B - A) @ c
    rhs = u1 * float(v1 @ c) + u2 * float(v2 @ c)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs)) * n


@pytest.mark.parametrize("m,n", [(300, 200), (1000, 1000)])
def test_dgemvt_atax_invariants(orc, m, n):
    A, y, z = M(40, m, n), U(41, m), U(42, n)
    x, w = orc.dgemvt(A, y, z, 1.5, 0.7)
    lhs, rhs = float(y @ w), 1.5 / 0.7 * float((x - z) @ x)
    scale = float(np.abs(y) @ np.abs(w)) + 1.5 / 0.7 * float(np.abs(x - z) @ np.abs(x))
    assert abs(lhs - rhs) <= 1e-12 * scale
    xv = U(43, n)
    ya = orc.atax(A, xv)
    # x^T A^T A x = |A x|^2 >= 0
    t = A @ xv
    assert float(xv @ ya) > 0
    assert abs(float(xv @ ya) - float(t @ t)) <= 1e-12 * float(t @ t) * 10


def test_axpydot_linearity(orc):
    n = 100000
    w, v, u = U(50, n), U(51, n), U(52, n)
    z, r = orc.axpydot(w, v, u, 1.5)
    rhs = float(w @ u) - 1.5 * float(v @ u)
    assert abs(r - rhs) <= 1e-12 * float(np.abs(z) @ np.abs(u))


# ---- thread-count independence -------------------------------------------

def test_threads_bitwise(orc):
    m, n = 513, 700
    A = M(60, m, n)
    vec = lambda s, k: U(60 + s, k)
    outs = []
    for t in (1, 4):
        orc.set_threads(t)
        outs.append((orc.bicgk(A, vec(1, n), vec(2, m)),
                     orc.gemver(A, vec(3, m), vec(4, n), vec(5, m), vec(6, n),
                                vec(7, m), vec(8, n), 1.5, 0.7),
                     orc.atax(A, vec(9, n)),
                     orc.dgemvt(A, vec(10, m), vec(11, n), 1.5, 0.7)))
    orc.set_threads(1)
    flat = lambda o: np.concatenate([np.ravel(a) for a in
                                     [o[0][0], o[0][1], *o[1], o[2], *o[3]]])
    assert np.array_equal(flat(outs[0]), flat(outs[1]))


@pytest.mark.parametrize("m,n", [(200, 150), (1000, 1000)])
def test_dgemv_gesummv_invariants(orc, m, n):
    A, B = synth.matrix(SEED, 90, m, n), synth.matrix(SEED, 91, m, n)
    x, y, v = U(92, n), U(93, m), U(94, m)
    # the two terms of GESUMMV are symmetric: swapping (A, alpha) and (B, beta)
    # changes nothing, and B = A with beta = -alpha cancels exactly
    assert np.array_equal(orc.gesummv(A, B, x, 1.5, 0.7), orc.gesummv(B, A, x, 0.7, 1.5))
    assert np.array_equal(orc.gesummv(A, A, x, 1.5, -1.5), np.zeros(m))
    # v^T z = alpha (A^T v)^T x + beta v^T y, with A^T v from the column sums
    z = orc.dgemv(A, x, y, 1.5, 0.7)
    _, s = orc.bicgk(A, x, v)
    lhs, rhs = float(v @ z), 1.5 * float(s @ x) + 0.7 * float(v @ y)
    mag = 1.5 * float(np.abs(v) @ (np.abs(A) @ np.abs(x))) + 0.7 * float(np.abs(v) @ np.abs(y))
    assert abs(lhs - rhs) <= 4 * (m + n) * 2.0 ** -53 * mag
    # GESUMMV = alpha A x + beta B x as two DGEMV calls (the BLAS form)
    g = orc.gesummv(A, B, x, 1.5, 0.7)
    two = orc.dgemv(B, x, orc.dgemv(A, x, np.zeros(m), 1.5, 0.0), 0.7, 1.0)
    assert np.max(np.abs(g - two)) <= 4 * 2.0 ** -53 * np.max(
        1.5 * (np.abs(A) @ np.abs(x)) + 0.7 * (np.abs(B) @ np.abs(x)))


# ---- leading dimension ----------------------------------------------------

@pytest.mark.parametrize("m,n,lda", [(5, 3, 4), (64, 65, 80), (130, 257, 300)])
def test_lda_padding_is_ignored(orc, m, n, lda):
    """A padded (m, lda) matrix whose padding is NaN gives bitwise the same
    results as the compact (m, n) matrix with the same elements."""
    Ap = synth.matrix(SEED, 70, m, n, lda=lda)
    Ac = np.ascontiguousarray(Ap[:, :n])
    p, r = U(71, n), U(72, m)
    for a, b in zip(orc.bicgk(Ap, p, r, lda=lda), orc.bicgk(Ac, p, r)):
        assert np.array_equal(a, b)
    assert np.array_equal(orc.atax(Ap, p, lda=lda), orc.atax(Ac, p))
    args = (U(73, m), U(74, n), U(75, m), U(76, n), U(77, m), U(78, n), 1.5, 0.7)
    for a, b in zip(orc.gemver(Ap, *args, lda=lda), orc.gemver(Ac, *args)):
        assert np.array_equal(a, b)
    for a, b in zip(orc.dgemvt(Ap, r, p, 1.5, 0.7, lda=lda), orc.dgemvt(Ac, r, p, 1.5, 0.7)):
        assert np.array_equal(a, b)
    assert np.array_equal(orc.dgemv(Ap, p, r, 1.5, 0.7, lda=lda), orc.dgemv(Ac, p, r, 1.5, 0.7))
    Bp = synth.matrix(SEED, 79, m, n, lda=lda + 5)
    Bc = np.ascontiguousarray(Bp[:, :n])
    assert np.array_equal(orc.gesummv(Ap, Bp, p, 1.5, 0.7, lda=lda, ldb=lda + 5),
                          orc.gesummv(Ac, Bc, p, 1.5, 0.7))
