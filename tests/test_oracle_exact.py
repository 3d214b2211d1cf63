"""Pins the oracle to exact arithmetic: rational brute force on tiny inputs,
hand-worked examples, and exact integer arithmetic at larger sizes.

Each check is independent of the oracle's code: the expected values come
from ``fractions.Fraction`` evaluation of the Table I statements, from the
hand-worked fixtures in ``golden/``, or from numpy's int64 matrix products.
"""

import json
import os

import numpy as np
import pytest

from paper_1205_1098_amd import synth
from tests import exact as ex

SIZES = [1, 2, 3, 5, 8]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _u(stream, n, seed=7):
    return synth.uniform(seed, stream, n)


def _A(stream, m, n, seed=7):
    return synth.matrix(seed, stream, m, n)


@pytest.mark.parametrize("m", SIZES)
@pytest.mark.parametrize("n", SIZES)
def test_bicgk_rational(orc, m, n):
    A, p, r = _A(1, m, n), _u(2, n), _u(3, m)
    q, s = orc.bicgk(A, p, r)
    qe, se = ex.bicgk(A, p, r)
    qa, sa = ex.bicgk_abs(A, p, r)
    for i in range(m):
        assert ex.within(q[i], qe[i], qa[i], n)
    for j in range(n):
        assert ex.within(s[j], se[j], sa[j], m)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (3, 2), (5, 5), (8, 3), (3, 8)])
def test_gemver_rational(orc, m, n):
    A = _A(10, m, n)
    u1, u2, y, = _u(11, m), _u(13, m), _u(15, m)
    v1, v2, z = _u(12, n), _u(14, n), _u(16, n)
    alpha, beta = 1.5, 0.7
    B, x, w = orc.gemver(A, u1, v1, u2, v2, y, z, alpha, beta)
    Be, xe, we = ex.gemver(A, u1, v1, u2, v2, y, z, alpha, beta)
    Ba, xa, wa = ex.gemver(A, u1, v1, u2, v2, y, z, alpha, beta, absolute=True)
    K = 2 * (m + n) + 10
    for i in range(m):
        for j in range(n):
            assert ex.within(B[i, j], Be[i][j], Ba[i][j], 4)
        assert ex.within(w[i], we[i], wa[i], K)
    for j in range(n):
        assert ex.within(x[j], xe[j], xa[j], K)


@pytest.mark.parametrize("m", SIZES)
@pytest.mark.parametrize("n", SIZES)
def test_atax_rational(orc, m, n):
    A, x = _A(20, m, n), _u(21, n)
    y = orc.atax(A, x)
    ye, ya = ex.atax(A, x), ex.atax(A, x, absolute=True)
    for j in range(n):
        assert ex.within(y[j], ye[j], ya[j], m + n + 2)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (3, 2), (5, 5), (8, 3), (3, 8)])
def test_dgemvt_rational(orc, m, n):
    A, y, z = _A(30, m, n), _u(31, m), _u(32, n)
    x, w = orc.dgemvt(A, y, z, 1.5, 0.7)
    xe, we = ex.dgemvt(A, y, z, 1.5, 0.7)
    xa, wa = ex.dgemvt(A, y, z, 1.5, 0.7, absolute=True)
    K = m + n + 6
    for j in range(n):
        assert ex.within(x[j], xe[j], xa[j], K)
    for i in range(m):
        assert ex.within(w[i], we[i], wa[i], K)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (3, 2), (5, 5), (8, 3), (3, 8)])
def test_dgemv_gesummv_rational(orc, m, n):
    A, B, x, y = _A(70, m, n), _A(71, m, n), _u(72, n), _u(73, m)
    z = orc.dgemv(A, x, y, 1.5, -0.7)
    ze, za = ex.dgemv(A, x, y, 1.5, -0.7), ex.dgemv(A, x, y, 1.5, -0.7, absolute=True)
    g = orc.gesummv(A, B, x, 1.5, -0.7)
    ge, ga = ex.gesummv(A, B, x, 1.5, -0.7), ex.gesummv(A, B, x, 1.5, -0.7, absolute=True)
    for i in range(m):
        assert ex.within(z[i], ze[i], za[i], n + 2)
        assert ex.within(g[i], ge[i], ga[i], n + 2)


@pytest.mark.parametrize("n", SIZES + [127, 128, 129, 300])
def test_axpydot_rational(orc, n):
    w, v, u = _u(40, n), _u(41, n), _u(42, n)
    z, r = orc.axpydot(w, v, u, 1.5)
    ze, re_ = ex.axpydot(w, v, u, 1.5)
    za, ra = ex.axpydot(w, v, u, 1.5, absolute=True)
    for k in range(n):
        assert ex.within(z[k], ze[k], za[k], 2)
    assert ex.within(r, re_, ra, n + 3)


@pytest.mark.parametrize("n", SIZES)
def test_waxpby_vadd_rational(orc, n):
    x, y, z = _u(50, n), _u(51, n), _u(52, n)
    w = orc.waxpby(x, y, 1.5, 0.7)
    we, wa = ex.waxpby(x, y, 1.5, 0.7), ex.waxpby(x, y, 1.5, 0.7, absolute=True)
    for k in range(n):
        assert ex.within(w[k], we[k], wa[k], 2)
    s = orc.vadd(x, y, z)
    se, sa = ex.vadd(x, y, z), ex.vadd(x, y, z, absolute=True)
    for k in range(n):
        assert ex.within(s[k], se[k], sa[k], 2)


def test_pairwise_long_dot_error(orc):
    """The long dot product stays within the pairwise-summation bound
    (depth 127 + ceil(log2 N) roundings) of the exactly rounded result."""
    import math
    from fractions import Fraction as F

    n = 1 << 18
    w, v, u = _u(60, n), _u(61, n), _u(62, n)
    z, r = orc.axpydot(w, v, u, 1.5)
    prods = [F(float(a)) * F(float(b)) for a, b in zip(z, u)]
    exact = sum(prods, F(0))
    mag = sum((abs(t) for t in prods), F(0))
    k = 128 + math.ceil(math.log2(n)) + 1
    assert abs(F(r) - exact) <= ex.gamma(k) * mag
    # a sequential sum would be allowed a bound of gamma_n; the pairwise
    # result is typically far below even the tighter bound
    assert abs(F(r) - exact) <= ex.gamma(64) * mag


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_hand_worked(orc):
    g = _golden()
    a = np.array
    c = g["bicgk"]
    q, s = orc.bicgk(a(c["A"], float), a(c["p"], float), a(c["r"], float))
    assert q.tolist() == c["q"] and s.tolist() == c["s"]
    c = g["gemver"]
    B, x, w = orc.gemver(a(c["A"], float), a(c["u1"], float), a(c["v1"], float),
                         a(c["u2"], float), a(c["v2"], float), a(c["y"], float),
                         a(c["z"], float), c["alpha"], c["beta"])
    assert B.tolist() == c["B"] and x.tolist() == c["x"] and w.tolist() == c["w"]
    c = g["atax"]
    assert orc.atax(a(c["A"], float), a(c["x"], float)).tolist() == c["y"]
    c = g["dgemvt"]
    x, w = orc.dgemvt(a(c["A"], float), a(c["y"], float), a(c["z"], float),
                      c["alpha"], c["beta"])
    assert x.tolist() == c["x"] and w.tolist() == c["w"]
    c = g["axpydot"]
    z, r = orc.axpydot(a(c["w"], float), a(c["v"], float), a(c["u"], float), c["alpha"])
    assert z.tolist() == c["z"] and r == c["r"]
    c = g["waxpby"]
    assert orc.waxpby(a(c["x"], float), a(c["y"], float), c["alpha"], c["beta"]).tolist() == c["w"]
    c = g["vadd"]
    assert orc.vadd(a(c["w"], float), a(c["y"], float), a(c["z"], float)).tolist() == c["x"]
    c = g["dgemv"]
    z = orc.dgemv(a(c["A"], float), a(c["x"], float), a(c["y"], float), c["alpha"], c["beta"])
    assert z.tolist() == c["z"]
    c = g["gesummv"]
    y = orc.gesummv(a(c["A"], float), a(c["B"], float), a(c["x"], float), c["alpha"], c["beta"])
    assert y.tolist() == c["y"]


# ---- exact integer arithmetic at sizes that span many blocks -------------

INT_SHAPES = [(300, 257), (257, 300), (1, 513), (513, 1), (1024, 1024)]


def _ints(stream, n, seed=11):
    return synth.small_ints(seed, stream, n)


def _imat(stream, m, n, seed=11):
    return synth.matrix(seed, stream, m, n, kind="int")


@pytest.mark.parametrize("m,n", INT_SHAPES)
def test_integer_exact_matrix_kernels(orc, m, n):
    A = _imat(1, m, n)
    Ai = A.astype(np.int64)
    p, r = _ints(2, n), _ints(3, m)
    q, s = orc.bicgk(A, p, r)
    assert np.array_equal(q, (Ai @ p.astype(np.int64)).astype(float))
    assert np.array_equal(s, (Ai.T @ r.astype(np.int64)).astype(float))

    x = _ints(4, n)
    t = Ai @ x.astype(np.int64)
    assert np.array_equal(orc.atax(A, x), (Ai.T @ t).astype(float))

    u1, u2, y = _ints(5, m), _ints(6, m), _ints(7, m)
    v1, v2, z = _ints(8, n), _ints(9, n), _ints(10, n)
    B, xg, w = orc.gemver(A, u1, v1, u2, v2, y, z, 2.0, 3.0)
    I = lambda a: a.astype(np.int64)
    Bi = Ai + np.outer(I(u1), I(v1)) + np.outer(I(u2), I(v2))
    xi = 3 * (Bi.T @ I(y)) + I(z)
    wi = 2 * (Bi @ xi)
    assert np.abs(wi).max() < 2 ** 53
    assert np.array_equal(B, Bi.astype(float))
    assert np.array_equal(xg, xi.astype(float))
    assert np.array_equal(w, wi.astype(float))

    xd, wd = orc.dgemvt(A, y, z, 2.0, 3.0)
    xi = 3 * (Ai.T @ I(y)) + I(z)
    assert np.array_equal(xd, xi.astype(float))
    assert np.array_equal(wd, (2 * (Ai @ xi)).astype(float))

    Bm = _imat(12, m, n)
    xv, yv = _ints(13, n), _ints(14, m)
    zi = 2 * (Ai @ I(xv)) - 3 * I(yv)
    assert np.array_equal(orc.dgemv(A, xv, yv, 2.0, -3.0), zi.astype(float))
    gi = 2 * (Ai @ I(xv)) + 3 * (I(Bm) @ I(xv))
    assert np.array_equal(orc.gesummv(A, Bm, xv, 2.0, 3.0), gi.astype(float))


@pytest.mark.parametrize("n", [1, 127, 128, 129, 4097, 1 << 20])
def test_integer_exact_vector_kernels(orc, n):
    w, v, u = _ints(20, n), _ints(21, n), _ints(22, n)
    I = lambda a: a.astype(np.int64)
    z, r = orc.axpydot(w, v, u, 2.0)
    zi = I(w) - 2 * I(v)
    assert np.array_equal(z, zi.astype(float))
    assert r == float(int(zi @ I(u)))
    assert np.array_equal(orc.waxpby(w, v, 2.0, 3.0), (2 * I(w) + 3 * I(v)).astype(float))
    assert np.array_equal(orc.vadd(w, v, u), (I(w) + I(v) + I(u)).astype(float))
