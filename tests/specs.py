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
    # scaled sums longer than one pass takes (eight terms): the sum so far
    # carries into the next pass
    "lin9": """LIN9
in:  a1 : vector(column), a2 : vector(column), a3 : vector(column), a4 : vector(column),
     a5 : vector(column), a6 : vector(column), a7 : vector(column), a8 : vector(column),
     a9 : vector(column), c : scalar
out: x : vector(column)
{
  x = a1 + 2 * a2 - a3 + c * a4 + a5 - 3 * a6 + a7 + a8 - c * a9
}""",
    "lin16": """LIN16
in:  b1 : vector(column), b2 : vector(column), b3 : vector(column), b4 : vector(column),
     b5 : vector(column), b6 : vector(column), b7 : vector(column), b8 : vector(column),
     b9 : vector(column), b10 : vector(column), b11 : vector(column), b12 : vector(column),
     b13 : vector(column), b14 : vector(column), b15 : vector(column), b16 : vector(column)
out: x : vector(column)
{
  x = b1 + b2 + b3 + b4 + b5 + b6 + b7 + b8 + b9 + b10 + b11 + b12 + b13 + b14 + b15 - b16
}""",
}
