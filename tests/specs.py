"""Kernel specifications for the tests: the library's (Table I, BATAX,
GEMVER with B a temporary) and a few programs of the same language that are
not in the paper's suite."""

from paper_1205_1098_amd.bto_specs import BATAX, GEMVER_CONTRACTED, TABLE_I  # noqa: F401

# programs outside the paper's suite; A is square where both products meet
NOVEL = {
    "both_ways": """BOTHWAYS
in:  A : matrix(row), x : vector(column), w : vector(column)
out: z : vector(column)
{
  z = A * x + A' * w
}""",
    "atax_plus": """ATAXPLUS
in:  A : matrix(row), x : vector(column), z : vector(column)
out: y : vector(column)
{
  y = A' * (A * x) + z
}""",
    "rank1_stored": """RANK1
in:  A : matrix(row), u : vector(column), v : vector(column), p : vector(column),
     r : vector(column)
out: B : matrix(row), q : vector(column), s : vector(column)
{
  B = A + u * v'
  q = B * p
  s = B' * r
}""",
    "rank1_contracted": """RANK1C
in:  A : matrix(row), u : vector(column), v : vector(column), x : vector(column),
     y : vector(column), gamma : scalar
out: w : vector(column)
{
  C = A + u * v'
  w = C * x - gamma * y
}""",
    "two_dots": """TWODOTS
in:  A : matrix(row), x : vector(column)
out: y : vector(column)
{
  t = A * x
  y = 2 * A * t
}""",
    "lin4": """LIN4
in:  w : vector(column), y : vector(column), z : vector(column), v : vector(column),
     a : scalar
out: x : vector(column)
{
  x = a * w + y - 2 * z + v
}""",
    "mixed": """MIXED
in:  A : matrix(row), x : vector(column), y : vector(column), w : vector(column),
     alpha : scalar
out: z : vector(column)
{
  z = -A * x + y - alpha * w
}""",
}
