"""The kernels of Table I, BATAX (Fig. 1) and GEMVER with B contracted, in
the input language of Section II, for btoc.compile_spec."""

TABLE_I = {
    "bicgk": """BICGK
in:  A : matrix(row), p : vector(column), r : vector(column)
out: q : vector(column), s : vector(column)
{
  q = A * p
  s = A' * r
}""",
    "gemver": """GEMVER
in:  A : matrix(row), u1 : vector(column), v1 : vector(column), u2 : vector(column),
     v2 : vector(column), y : vector(column), z : vector(column),
     alpha : scalar, beta : scalar
out: B : matrix(row), x : vector(column), w : vector(column)
{
  B = A + u1 * v1' + u2 * v2'
  x = beta * B' * y + z
  w = alpha * B * x
}""",
    "atax": """ATAX
in:  A : matrix(row), x : vector(column)
out: y : vector(column)
{
  y = A' * (A * x)
}""",
    "dgemvt": """DGEMVT
in:  A : matrix(row), y : vector(column), z : vector(column), alpha : scalar, beta : scalar
out: x : vector(column), w : vector(column)
{
  x = beta * A' * y + z
  w = alpha * A * x
}""",
    "dgemv": """DGEMV
in:  A : matrix(row), x : vector(column), y : vector(column), alpha : scalar, beta : scalar
out: z : vector(column)
{
  z = alpha * A * x + beta * y
}""",
    "gesummv": """GESUMMV
in:  A : matrix(row), B : matrix(row), x : vector(column), alpha : scalar, beta : scalar
out: y : vector(column)
{
  y = alpha * A * x + beta * B * x
}""",
    "axpydot": """AXPYDOT
in:  w : vector(column), v : vector(column), u : vector(column), alpha : scalar
out: z : vector(column), r : scalar
{
  z = w - alpha * v
  r = z' * u
}""",
    "waxpby": """WAXPBY
in:  x : vector(column), y : vector(column), alpha : scalar, beta : scalar
out: w : vector(column)
{
  w = alpha * x + beta * y
}""",
    "vadd": """VADD
in:  w : vector(column), y : vector(column), z : vector(column)
out: x : vector(column)
{
  x = w + y + z
}""",
}

# BATAX, the running example of Section II (Fig. 1): y = beta A^T A x
BATAX = """BATAX
in:  A : matrix(row), x : vector(column), beta : scalar
out: y : vector(column)
{
  y = beta * A' * (A * x)
}"""

GEMVER_CONTRACTED = """GEMVERC
in:  A : matrix(row), u1 : vector(column), v1 : vector(column), u2 : vector(column),
     v2 : vector(column), y : vector(column), z : vector(column),
     alpha : scalar, beta : scalar
out: x : vector(column), w : vector(column)
{
  B = A + u1 * v1' + u2 * v2'
  x = beta * B' * y + z
  w = alpha * B * x
}"""

# Programs whose fused passes the library's sweeps cannot run (an update of
# rank three; several row dots and column sums over one matrix): the
# compiler emits their passes as HIP (btoc_gen), built with the package.
GENERATED = {
    "gemver3": """GEMVER3
in:  A : matrix(row), u1 : vector(column), v1 : vector(column), u2 : vector(column),
     v2 : vector(column), u3 : vector(column), v3 : vector(column), y : vector(column),
     z : vector(column), alpha : scalar, beta : scalar
out: B : matrix(row), x : vector(column), w : vector(column)
{
  B = A + u1 * v1' + u2 * v2' + u3 * v3'
  x = beta * B' * y + z
  w = alpha * B * x
}""",
    "gemver3c": """GEMVER3C
in:  A : matrix(row), u1 : vector(column), v1 : vector(column), u2 : vector(column),
     v2 : vector(column), u3 : vector(column), v3 : vector(column), y : vector(column),
     z : vector(column), alpha : scalar, beta : scalar
out: x : vector(column), w : vector(column)
{
  B = A + u1 * v1' + u2 * v2' + u3 * v3'
  x = beta * B' * y + z
  w = alpha * B * x
}""",
    "bicgk2": """BICGK2
in:  A : matrix(row), p1 : vector(column), p2 : vector(column), r1 : vector(column),
     r2 : vector(column)
out: q1 : vector(column), q2 : vector(column), s1 : vector(column), s2 : vector(column)
{
  q1 = A * p1
  q2 = A * p2
  s1 = A' * r1
  s2 = A' * r2
}""",
    "multimv": """MULTIMV
in:  A : matrix(row), x1 : vector(column), x2 : vector(column), x3 : vector(column),
     y : vector(column), alpha : scalar, beta : scalar
out: z1 : vector(column), z2 : vector(column), z3 : vector(column)
{
  z1 = alpha * A * x1 + beta * y
  z2 = A * x2 - y
  z3 = beta * alpha * A * x3
}""",
    "multimv5": """MULTIMV5
in:  A : matrix(row), x1 : vector(column), x2 : vector(column), x3 : vector(column),
     x4 : vector(column), x5 : vector(column), r : vector(column), alpha : scalar
out: z1 : vector(column), z2 : vector(column), z3 : vector(column), z4 : vector(column),
     z5 : vector(column), s : vector(column)
{
  z1 = A * x1
  z2 = alpha * A * x2
  z3 = A * x3
  z4 = A * x4
  z5 = A * x5
  s = A' * r
}""",
    "bicgk2c": """BICGK2C
in:  A : matrix(column), p1 : vector(column), p2 : vector(column), r1 : vector(column),
     r2 : vector(column)
out: q1 : vector(column), q2 : vector(column), s1 : vector(column), s2 : vector(column)
{
  q1 = A * p1
  q2 = A * p2
  s1 = A' * r1
  s2 = A' * r2
}""",
}
