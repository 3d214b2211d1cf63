"""Reference evaluation of a BTO kernel specification on the CPU.

TEST INFRASTRUCTURE ONLY: the tests use it to check what the spec compiler
generates; nothing on the product path imports it, and it imports nothing
from the product.

A specification (the kernel language of Section II, Fig. 1) names its typed
inputs and outputs and a block of assignments.  This module evaluates the
assignments in order, in binary64 with numpy, by their plain meaning:

* a matrix update A + u v' (+ ...) is formed element by element, left to
  right, as Table I's GEMVER defines B;
* a product of a scaled matrix with a vector is reduced first and scaled
  after (every scale applied after its reduction, as in the statements of
  Table I);
* sums of vectors are added left to right;
* a row vector times a column vector is their dot product (a scalar).

Products use numpy's matrix-vector product as a library step.
"""

from __future__ import annotations

import re

import numpy as np

_TOK = re.compile(r"[A-Za-z_][A-Za-z_0-9]*|\d+\.\d*(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?|\S")


def _split(text: str):
    """The header (name, inputs, outputs) and the statement strings."""
    head, _, rest = text.partition("{")
    body, _, _ = rest.rpartition("}")
    words = head.replace(",", " , ").replace(":", " : ").split()
    name = words[0]
    decls = {"in": [], "out": []}
    cur = None
    i = 1
    while i < len(words):
        w = words[i]
        if w in ("in", "out") and i + 1 < len(words) and words[i + 1] == ":":
            cur = w
            i += 2
            continue
        if w == ",":
            i += 1
            continue
        # name : type
        typ = words[i + 2]
        decls[cur].append((w, typ.split("(")[0]))
        i += 3
    stmts = [s.strip() for s in re.split(r"[;\n]", body) if s.strip()]
    return name, decls["in"], decls["out"], stmts


class _Eval:
    def __init__(self, env):
        self.env = env

    def run(self, stmt: str):
        lhs, _, rhs = stmt.partition("=")
        self.toks = _TOK.findall(rhs)
        self.k = 0
        val = self.sum()
        if self.k != len(self.toks):
            raise ValueError(f"cannot read {stmt!r}")
        kind, v = val[0], val[1]
        if kind == "mat":
            if val[2] != 1.0 or val[3]:
                raise ValueError("a matrix assignment must be an update")
            self.env[lhs.strip()] = ("mat", v, 1.0, False)
        elif kind == "vec":
            self.env[lhs.strip()] = ("vec", v)
        elif kind == "scal":
            self.env[lhs.strip()] = ("scal", v)
        else:
            raise ValueError(f"unsupported result in {stmt!r}")

    def peek(self):
        return self.toks[self.k] if self.k < len(self.toks) else None

    def take(self):
        t = self.toks[self.k]
        self.k += 1
        return t

    def sum(self):
        val = self.prod()
        while self.peek() in ("+", "-"):
            op = self.take()
            rhs = self.prod()
            val = self.add(val, rhs, -1.0 if op == "-" else 1.0)
        return val

    def prod(self):
        val = self.unary()
        while self.peek() == "*":
            self.take()
            val = self.mul(val, self.unary())
        return val

    def unary(self):
        if self.peek() == "-":
            self.take()
            return self.mul(("scal", -1.0), self.unary())
        t = self.take()
        if t == "(":
            val = self.sum()
            assert self.take() == ")"
        elif re.match(r"\d", t):
            val = ("scal", float(t))
        else:
            val = self.env[t]
        while self.peek() == "'":
            self.take()
            val = self.transpose(val)
        return val

    @staticmethod
    def transpose(v):
        if v[0] == "mat":
            return ("mat", v[1], v[2], not v[3])
        if v[0] == "vec":
            return ("row", v[1])
        if v[0] == "row":
            return ("vec", v[1])
        return v

    @staticmethod
    def add(a, b, sign):
        if a[0] == "vec" and b[0] == "vec":
            return ("vec", a[1] + sign * b[1] if sign < 0 else a[1] + b[1])
        if a[0] == "mat" and b[0] == "outer":
            if a[2] != 1.0 or a[3] or sign < 0:
                raise ValueError("unsupported update")
            return ("mat", a[1] + b[1], 1.0, False)
        raise ValueError("unsupported sum")

    @staticmethod
    def mul(a, b):
        if a[0] == "scal" and b[0] == "scal":
            return ("scal", a[1] * b[1])
        if a[0] == "scal" or b[0] == "scal":
            s, v = (a, b) if a[0] == "scal" else (b, a)
            if v[0] == "vec":
                return ("vec", s[1] * v[1])
            if v[0] == "mat":
                return ("mat", v[1], v[2] * s[1], v[3])
            raise ValueError("unsupported scaling")
        if a[0] == "vec" and b[0] == "row":
            return ("outer", np.outer(a[1], b[1]))
        if a[0] == "row" and b[0] == "vec":
            return ("scal", float(np.dot(a[1], b[1])))
        if a[0] == "mat" and b[0] == "vec":
            M = a[1].T if a[3] else a[1]
            r = M @ b[1]
            return ("vec", a[2] * r if a[2] != 1.0 else r)
        raise ValueError("unsupported product")


def evaluate(text: str, bound: dict) -> dict:
    """Outputs of the specification for host inputs (numpy float64 arrays
    and floats), by name."""
    _, ins, outs, stmts = _split(text)
    env = {}
    for name, kind in ins:
        v = bound[name]
        if kind == "scalar":
            env[name] = ("scal", float(v))
        elif kind == "matrix":
            env[name] = ("mat", np.asarray(v, dtype=np.float64), 1.0, False)
        else:
            env[name] = ("vec", np.asarray(v, dtype=np.float64))
    ev = _Eval(env)
    for s in stmts:
        ev.run(s)
    return {name: env[name][1] for name, _ in outs}
