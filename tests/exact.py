"""Exact rational evaluation of the Table I kernels (Section V-A).

Used to pin the oracle on tiny inputs: each function evaluates a kernel's
statements in exact arithmetic (``fractions.Fraction``) on the given
doubles, and a second pass with every input replaced by its absolute value
gives the magnitude that bounds the rounding error of any binary64
evaluation order:

    |computed - exact| <= gamma_K * magnitude,   gamma_K = K u / (1 - K u),

where K is the largest number of roundings on any path from an input to the
output and u = 2**-53 (Higham, Accuracy and Stability of Numerical
Algorithms, 2nd ed., section 3.1).
"""

from fractions import Fraction as F

U = F(1, 2 ** 53)


def gamma(k: int) -> F:
    return k * U / (1 - k * U)


def _f(v):
    return [F(float(t)) for t in v]


def _m(A):
    return [[F(float(t)) for t in row] for row in A]


def _abs_v(v):
    return [abs(t) for t in v]


def _abs_m(A):
    return [[abs(t) for t in row] for row in A]


def bicgk(A, p, r):
    A, p, r = _m(A), _f(p), _f(r)
    m, n = len(r), len(p)
    q = [sum((A[i][j] * p[j] for j in range(n)), F(0)) for i in range(m)]
    s = [sum((A[i][j] * r[i] for i in range(m)), F(0)) for j in range(n)]
    return q, s


def gemver(A, u1, v1, u2, v2, y, z, alpha, beta, absolute=False):
    A, u1, v1, u2, v2, y, z = _m(A), _f(u1), _f(v1), _f(u2), _f(v2), _f(y), _f(z)
    alpha, beta = F(float(alpha)), F(float(beta))
    if absolute:
        A, u1, v1, u2, v2, y, z = (_abs_m(A), _abs_v(u1), _abs_v(v1), _abs_v(u2),
                                   _abs_v(v2), _abs_v(y), _abs_v(z))
        alpha, beta = abs(alpha), abs(beta)
    m, n = len(u1), len(v1)
    B = [[A[i][j] + u1[i] * v1[j] + u2[i] * v2[j] for j in range(n)] for i in range(m)]
    x = [beta * sum((B[i][j] * y[i] for i in range(m)), F(0)) + z[j] for j in range(n)]
    w = [alpha * sum((B[i][j] * x[j] for j in range(n)), F(0)) for i in range(m)]
    return B, x, w


def atax(A, x, absolute=False):
    A, x = _m(A), _f(x)
    if absolute:
        A, x = _abs_m(A), _abs_v(x)
    m, n = len(A), len(x)
    t = [sum((A[i][j] * x[j] for j in range(n)), F(0)) for i in range(m)]
    return [sum((A[i][j] * t[i] for i in range(m)), F(0)) for j in range(n)]


def dgemvt(A, y, z, alpha, beta, absolute=False):
    A, y, z = _m(A), _f(y), _f(z)
    alpha, beta = F(float(alpha)), F(float(beta))
    if absolute:
        A, y, z, alpha, beta = _abs_m(A), _abs_v(y), _abs_v(z), abs(alpha), abs(beta)
    m, n = len(y), len(z)
    x = [beta * sum((A[i][j] * y[i] for i in range(m)), F(0)) + z[j] for j in range(n)]
    w = [alpha * sum((A[i][j] * x[j] for j in range(n)), F(0)) for i in range(m)]
    return x, w


def dgemv(A, x, y, alpha, beta, absolute=False):
    A, x, y = _m(A), _f(x), _f(y)
    alpha, beta = F(float(alpha)), F(float(beta))
    if absolute:
        A, x, y, alpha, beta = _abs_m(A), _abs_v(x), _abs_v(y), abs(alpha), abs(beta)
    m, n = len(y), len(x)
    return [alpha * sum((A[i][j] * x[j] for j in range(n)), F(0)) + beta * y[i]
            for i in range(m)]


def gesummv(A, B, x, alpha, beta, absolute=False):
    A, B, x = _m(A), _m(B), _f(x)
    alpha, beta = F(float(alpha)), F(float(beta))
    if absolute:
        A, B, x, alpha, beta = _abs_m(A), _abs_m(B), _abs_v(x), abs(alpha), abs(beta)
    m, n = len(A), len(x)
    return [alpha * sum((A[i][j] * x[j] for j in range(n)), F(0))
            + beta * sum((B[i][j] * x[j] for j in range(n)), F(0)) for i in range(m)]


def axpydot(w, v, u, alpha, absolute=False):
    w, v, u, alpha = _f(w), _f(v), _f(u), F(float(alpha))
    if absolute:
        w, v, u, alpha = _abs_v(w), _abs_v(v), _abs_v(u), abs(alpha)
        z = [w[k] + alpha * v[k] for k in range(len(w))]
    else:
        z = [w[k] - alpha * v[k] for k in range(len(w))]
    return z, sum((z[k] * u[k] for k in range(len(z))), F(0))


def waxpby(x, y, alpha, beta, absolute=False):
    x, y, alpha, beta = _f(x), _f(y), F(float(alpha)), F(float(beta))
    if absolute:
        x, y, alpha, beta = _abs_v(x), _abs_v(y), abs(alpha), abs(beta)
    return [alpha * x[k] + beta * y[k] for k in range(len(x))]


def vadd(w, y, z, absolute=False):
    w, y, z = _f(w), _f(y), _f(z)
    if absolute:
        w, y, z = _abs_v(w), _abs_v(y), _abs_v(z)
    return [w[k] + y[k] + z[k] for k in range(len(w))]


def bicgk_abs(A, p, r):
    q, s = bicgk([[abs(t) for t in row] for row in A], [abs(t) for t in p],
                 [abs(t) for t in r])
    return q, s


def within(computed, exact, magnitude, k: int) -> bool:
    """True when |computed - exact| <= gamma_k * magnitude."""
    return abs(F(float(computed)) - exact) <= gamma(k) * magnitude
