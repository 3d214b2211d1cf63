"""A compiler for BTO kernel specifications onto the library's fused passes.

The input is the paper's kernel language (Section II, Fig. 1): a name, the
typed inputs and outputs, and a block of statements over matrices, vectors
and scalars::

    BATAX
    in:  x : vector(column), beta : scalar, A : matrix(row)
    out: y : vector(column)
    { y = beta * A' * (A * x) }

``compile_spec`` parses it, types every expression, builds the dataflow
graph of its operations (matrix-vector products, rank-1 updates, scaled
vector sums) and schedules the products into passes over their matrices by
the legality rules of Section III-D:

* a product needs its vector operand complete before the pass that reads
  the matrix, so a product of a vector that another pass reduces comes
  after that pass (the data and reduction dependences that force GEMVER and
  DGEMVT into two passes);
* the one exception is a row dot feeding the column sums of the same matrix
  row by row (t = A x; y = A' t with t used nowhere else): the row is
  complete when its dot is, so both run in one pass with the row held on
  chip (ATAX and BATAX's one-pass form, Section IV-A);
* products of one matrix at the same point of the schedule share one sweep
  (loop fusion over the operand they share, Section III-E), one row-dot and
  one column-sum vector per sweep;
* a matrix update B = A + u1 v1' + u2 v2' that is an output is formed and
  stored by the first sweep of A; one that is not is contracted (Section
  III-E): products with it read A and add the rank-2 correction.

Scales and vector sums fold into the reduction epilogues of the passes, and
what is left runs as scaled vector sums.  ``form="unfused"`` lowers the same
program the BLAS way: one pass per operation, every temporary stored, each
update applied as its own rank-1 sweep.

Vector statements fuse too: a sum of three vectors is one pass, and a dot
product of a vector just formed as w - alpha v runs in the same pass that
forms it (AXPYDOT).  A matrix stored by columns is planned as the row-major
matrix of its transpose.

The result is a ``Program`` whose ``run`` enqueues the passes on the current
stream through the C entry points (``bto_pass``, ``bto_waxpby``,
``bto_vadd``, ``bto_axpydot``, ``bto_dot``); nothing is computed in Python.
"""

from __future__ import annotations

import re
from dataclasses import dataclass, field

# ---- parsing ----------------------------------------------------------------

_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)|([A-Za-z_]\w*)|(.))")


class SpecError(ValueError):
    """A specification that cannot be compiled."""


def _tokens(text: str):
    out = []
    for line_no, line in enumerate(text.splitlines(), 1):
        line = line.split("%")[0]
        pos = 0
        while pos < len(line):
            m = _TOKEN.match(line, pos)
            if not m or m.end() == pos:
                break
            pos = m.end()
            num, ident, sym = m.groups()
            if num is not None:
                out.append(("num", float(num), line_no))
            elif ident is not None:
                out.append(("id", ident, line_no))
            elif sym is not None and not sym.isspace():
                out.append(("sym", sym, line_no))
        out.append(("nl", None, line_no))
    out.append(("eof", None, -1))
    return out


@dataclass
class Decl:
    name: str
    kind: str          # "matrix", "vector", "scalar"
    orient: str        # "row" or "column" ("" for scalars)


@dataclass
class Spec:
    name: str
    inputs: list
    outputs: list
    statements: list   # (lhs name, expression tree)


class _Parser:
    def __init__(self, text: str):
        self.t = _tokens(text)
        self.i = 0

    def peek(self, skip_nl=True):
        j = self.i
        while skip_nl and self.t[j][0] == "nl":
            j += 1
        return self.t[j]

    def next(self, skip_nl=True):
        while skip_nl and self.t[self.i][0] == "nl":
            self.i += 1
        tok = self.t[self.i]
        self.i += 1
        return tok

    def expect(self, kind, value=None):
        tok = self.next()
        if tok[0] != kind or (value is not None and tok[1] != value):
            raise SpecError(f"line {tok[2]}: expected {value or kind}, got {tok[1]!r}")
        return tok

    def spec(self) -> Spec:
        name = self.expect("id")[1]
        inputs, outputs = [], []
        while True:
            tok = self.peek()
            if tok[0] == "id" and tok[1] in ("in", "out"):
                self.next()
                self.expect("sym", ":")
                (inputs if tok[1] == "in" else outputs).extend(self.decls())
            elif tok == ("sym", "{", tok[2]):
                break
            else:
                raise SpecError(f"line {tok[2]}: expected in:, out: or {{, got {tok[1]!r}")
        self.expect("sym", "{")
        stmts = []
        while True:
            tok = self.peek()
            if tok[0] == "sym" and tok[1] == "}":
                self.next()
                break
            if tok[0] == "sym" and tok[1] == ";":
                self.next()
                continue
            lhs = self.expect("id")[1]
            self.expect("sym", "=")
            stmts.append((lhs, self.expr()))
        if self.peek()[0] != "eof":
            raise SpecError("text after the statement block")
        return Spec(name, inputs, outputs, stmts)

    def decls(self):
        out = []
        while True:
            name = self.expect("id")[1]
            self.expect("sym", ":")
            kind = self.expect("id")[1]
            orient = ""
            if kind in ("vector", "matrix"):
                self.expect("sym", "(")
                orient = self.expect("id")[1]
                self.expect("sym", ")")
                if orient not in ("row", "column"):
                    raise SpecError(f"{name}: orientation {orient!r}")
            elif kind != "scalar":
                raise SpecError(f"{name}: unknown type {kind!r}")
            out.append(Decl(name, kind, orient))
            tok = self.peek(skip_nl=False)
            if tok[0] == "sym" and tok[1] == ",":
                self.next(skip_nl=False)
                continue
            # a declaration list may continue on the next line after a comma only
            return out

    # expr := term (('+'|'-') term)* ; term := unary ('*' unary)* ;
    # unary := '-' unary | postfix ; postfix := atom "'"*
    def expr(self):
        node = self.term()
        while True:
            tok = self.peek(skip_nl=False)
            if tok[0] == "sym" and tok[1] in "+-":
                self.next(skip_nl=False)
                node = (tok[1], node, self.term())
            else:
                return node

    def term(self):
        node = self.unary()
        while True:
            tok = self.peek(skip_nl=False)
            if tok[0] == "sym" and tok[1] == "*":
                self.next(skip_nl=False)
                node = ("*", node, self.unary())
            else:
                return node

    def unary(self):
        tok = self.peek()
        if tok[0] == "sym" and tok[1] == "-":
            self.next()
            return ("neg", self.unary())
        node = self.atom()
        while True:
            tok = self.peek(skip_nl=False)
            if tok[0] == "sym" and tok[1] == "'":
                self.next(skip_nl=False)
                node = ("T", node)
            else:
                return node

    def atom(self):
        tok = self.next()
        if tok[0] == "num":
            return ("num", tok[1])
        if tok[0] == "id":
            return ("sym", tok[1])
        if tok[0] == "sym" and tok[1] == "(":
            node = self.expr()
            self.expect("sym", ")")
            return node
        raise SpecError(f"line {tok[2]}: unexpected {tok[1]!r}")


def parse(text: str) -> Spec:
    return _Parser(text).spec()


# ---- typed values -------------------------------------------------------------
#
# A coefficient is a product of a literal and scalar symbols: (float, tuple).
# A matrix value is a base matrix symbol plus rank-1 terms (u, v), with a
# coefficient and a transpose flag.  A vector value is a linear combination
# of terms: a vector symbol, or a product (matrix value, vector symbol).

ONE = (1.0, ())


def _cmul(a, b):
    return (a[0] * b[0], tuple(sorted(a[1] + b[1])))


@dataclass(frozen=True)
class Mat:
    base: str
    terms: tuple = ()          # ((u, v), ...), u column of length m, v of length n
    coef: tuple = ONE
    trans: bool = False


@dataclass(frozen=True)
class Prod:
    mat: Mat                   # coefficient folded out (ONE)
    vec: str


@dataclass
class Lin:
    terms: list = field(default_factory=list)   # [(coef, Prod | str)]

    def scaled(self, c):
        return Lin([(_cmul(c, k), t) for k, t in self.terms])


@dataclass
class Outer:
    u: str
    v: str


@dataclass
class Dot:
    x: str
    y: str


class _Typer:
    """Turns statement trees into typed values, introducing temporaries for
    products whose vector operand is not a plain symbol."""

    def __init__(self, spec: Spec):
        self.kinds = {}
        self.colmajor = set()        # matrices stored by columns
        declared_col = set()
        for d in spec.inputs + spec.outputs:
            if d.name in self.kinds:
                raise SpecError(f"{d.name} declared twice")
            self.kinds[d.name] = d.kind
            if d.kind == "matrix" and d.orient == "column":
                declared_col.add(d.name)
        self.declared_col = declared_col
        self.colmajor |= {d.name for d in spec.inputs if d.name in declared_col}
        self.inputs = {d.name for d in spec.inputs}
        self.outputs = [d.name for d in spec.outputs]
        self.defs = []               # (name, Lin | Mat) in program order
        self.mats = {}               # matrix symbol -> Mat (inputs map to themselves)
        self.defined = set(self.inputs)
        self.ntemp = 0
        for d in spec.inputs:
            if d.kind == "matrix":
                self.mats[d.name] = Mat(d.name)

    def temp(self):
        self.ntemp += 1
        return f"_t{self.ntemp}"

    def statement(self, lhs, tree):
        if lhs in self.inputs:
            raise SpecError(f"{lhs} is an input and cannot be assigned")
        if lhs in self.defined:
            raise SpecError(f"{lhs} is assigned twice")
        val = self.value(tree)
        if isinstance(val, Mat):
            if val.trans or val.coef != ONE:
                raise SpecError(f"{lhs}: a matrix definition must be A + u v' + ...")
            self.kinds.setdefault(lhs, "matrix")
            if self.kinds[lhs] != "matrix":
                raise SpecError(f"{lhs} is not declared a matrix")
            # an update is stored like the matrix it updates
            if val.base in self.colmajor:
                self.colmajor.add(lhs)
            if lhs in self.outputs and (lhs in self.declared_col) != (val.base in self.colmajor):
                raise SpecError(f"{lhs}: stored by {'columns' if lhs in self.declared_col else 'rows'}"
                                f" but {val.base} is not")
            self.mats[lhs] = val
        elif isinstance(val, Lin):
            self.kinds.setdefault(lhs, "vector")
            if self.kinds[lhs] != "vector":
                raise SpecError(f"{lhs} is not declared a vector")
            self.defs.append((lhs, val))
        elif isinstance(val, Dot):
            if self.kinds.get(lhs) != "scalar" or lhs not in self.outputs:
                raise SpecError(f"{lhs}: a dot product goes to a scalar output")
            self.defs.append((lhs, val))
        else:
            raise SpecError(f"{lhs}: scalar and outer-product results are not supported")
        self.defined.add(lhs)
        if isinstance(val, Mat):
            self.defs.append((lhs, val))

    def value(self, t):
        op = t[0]
        if op == "num":
            return ("scalar", (t[1], ()))
        if op == "sym":
            name = t[1]
            if name not in self.defined:
                raise SpecError(f"{name} is used before it is defined")
            kind = self.kinds[name]
            if kind == "scalar":
                if name not in self.inputs:
                    raise SpecError(f"{name}: a computed scalar cannot scale later statements")
                return ("scalar", (1.0, (name,)))
            if kind == "matrix":
                return self.mats[name]
            return Lin([(ONE, name)])
        if op == "neg":
            return self.scale(self.value(t[1]), (-1.0, ()))
        if op == "T":
            v = self.value(t[1])
            if isinstance(v, Mat):
                return Mat(v.base, v.terms, v.coef, not v.trans)
            if isinstance(v, Lin):
                if len(v.terms) == 1 and isinstance(v.terms[0][1], str) and v.terms[0][0] == ONE:
                    return ("rowvec", v.terms[0][1])
                raise SpecError("only a vector symbol can be transposed")
            if isinstance(v, tuple) and v[0] == "scalar":
                return v
            raise SpecError("transpose of an unsupported value")
        a, b = self.value(t[1]), self.value(t[2])
        if op in "+-":
            if op == "-":
                b = self.scale(b, (-1.0, ()))
            return self.add(a, b)
        return self.mul(a, b)

    def scale(self, v, c):
        if isinstance(v, tuple) and v[0] == "scalar":
            return ("scalar", _cmul(v[1], c))
        if isinstance(v, Lin):
            return v.scaled(c)
        if isinstance(v, Mat):
            return Mat(v.base, v.terms, _cmul(v.coef, c), v.trans)
        raise SpecError("cannot scale this value")

    def add(self, a, b):
        if isinstance(a, Lin) and isinstance(b, Lin):
            return Lin(a.terms + b.terms)
        if isinstance(a, Mat) and isinstance(b, Outer):
            a, b = a, b
        elif isinstance(a, Outer) and isinstance(b, Mat):
            a, b = b, a
        else:
            raise SpecError("only vectors add to vectors, and outer products to a matrix")
        if a.trans or a.coef != ONE:
            raise SpecError("an update applies to an untransposed, unscaled matrix")
        return Mat(a.base, a.terms + ((b.u, b.v),))

    def mul(self, a, b):
        sa = isinstance(a, tuple) and a[0] == "scalar"
        sb = isinstance(b, tuple) and b[0] == "scalar"
        if sa and sb:
            return ("scalar", _cmul(a[1], b[1]))
        if sa:
            return self.scale(b, a[1])
        if sb:
            return self.scale(a, b[1])
        if isinstance(a, Lin) and isinstance(b, tuple) and b[0] == "rowvec":
            if len(a.terms) == 1 and isinstance(a.terms[0][1], str) and a.terms[0][0] == ONE:
                return Outer(a.terms[0][1], b[1])
            raise SpecError("an outer product takes vector symbols")
        if isinstance(a, tuple) and a[0] == "rowvec":
            if (isinstance(b, Lin) and len(b.terms) == 1 and isinstance(b.terms[0][1], str)
                    and b.terms[0][0] == ONE):
                return Dot(a[1], b.terms[0][1])
            raise SpecError("a dot product takes vector symbols; row-vector products are "
                            "not supported")
        if isinstance(a, Mat) and isinstance(b, Lin):
            if len(b.terms) == 1 and isinstance(b.terms[0][1], str) and b.terms[0][0] == ONE:
                vec = b.terms[0][1]
            else:
                vec = self.temp()
                self.kinds[vec] = "vector"
                self.defs.append((vec, b))
                self.defined.add(vec)
            m = Mat(a.base, a.terms, ONE, a.trans)
            return Lin([(a.coef, Prod(m, vec))])
        raise SpecError("unsupported product")


# ---- scheduling -----------------------------------------------------------------

@dataclass
class Pass:
    """One sweep of `base`: a bto_pass call (target "library"), or an
    emitted loop nest (target "generated", whose reductions are the lists
    `rows` and `cols`, any number of each)."""
    level: int
    base: str
    terms: tuple                 # the update, when stored or contracted
    store: str | None = None     # matrix output written by this pass
    contract: bool = False
    chain: bool = False
    row: dict | None = None      # {"x", "out", "scale", "add", "add_scale"}
    col: dict | None = None      # {"y", "out", "scale", "add", "add_scale"}
    rows: list = field(default_factory=list)    # generated: row dots
    cols: list = field(default_factory=list)    # generated: column sums


@dataclass
class VecOp:
    """out = a * x + b * y (bto_waxpby)."""
    level: int
    out: str
    a: tuple
    x: str
    b: tuple
    y: str


@dataclass
class Vadd:
    """out = (a + b) + c in one pass (bto_vadd)."""
    level: int
    out: str
    a: str
    b: str
    c: str


@dataclass
class LinComb:
    """out = sum of c_k t_k, left to right, in one pass (bto_lincomb)."""
    level: int
    out: str
    terms: list


@dataclass
class AxpyDot:
    """z = w - alpha v and r = z . u in one pass (bto_axpydot)."""
    level: int
    z: str
    w: str
    v: str
    alpha: tuple
    u: str
    r: str


@dataclass
class DotOp:
    """r = x . y (bto_dot)."""
    level: int
    r: str
    x: str
    y: str


@dataclass
class Program:
    name: str
    form: str
    inputs: list
    outputs: list
    kinds: dict
    steps: list
    temps: list                   # vector temporaries
    temp_mats: dict               # stored updates that are not outputs: name -> source
    colmajor: set = field(default_factory=set)   # matrices stored by columns
    target: str = "library"       # "library" (bto_pass) or "generated" (emitted passes)

    def describe(self):
        lines = []
        for s in self.steps:
            if isinstance(s, Pass):
                ops = [k for k, on in (("STORE", s.store), ("CONTRACT", s.contract),
                                       ("CHAIN", s.chain), ("ROWDOT", s.row),
                                       ("COLSUM", s.col)) if on]
                if s.rows:
                    ops.append("ROWDOT" + (f"x{len(s.rows)}" if len(s.rows) > 1 else ""))
                if s.cols:
                    ops.append("COLSUM" + (f"x{len(s.cols)}" if len(s.cols) > 1 else ""))
                if s.terms and (s.store or s.contract) and len(s.terms) > 2:
                    ops.append(f"RANK{len(s.terms)}")
                lines.append(f"pass {s.level}: {s.base} {'|'.join(ops)}")
            elif isinstance(s, VecOp):
                lines.append(f"vec {s.level}: {s.out} = a*{s.x} + b*{s.y}")
            elif isinstance(s, Vadd):
                lines.append(f"vadd {s.level}: {s.out} = {s.a} + {s.b} + {s.c}")
            elif isinstance(s, LinComb):
                lines.append(f"lincomb {s.level}: {s.out} = "
                             + " + ".join(f"c*{t}" for _, t in s.terms))
            elif isinstance(s, AxpyDot):
                lines.append(f"axpydot {s.level}: {s.z} = {s.w} - alpha*{s.v}; {s.r} = {s.z}.{s.u}")
            else:
                lines.append(f"dot {s.level}: {s.r} = {s.x}.{s.y}")
        return lines

    def passes(self):
        return [s for s in self.steps if isinstance(s, Pass)]

    def capture(self, ws=None, **bound):
        """The program captured in a HIP graph on these tensors
        (btoc_run.Captured): replay() reruns it with one launch."""
        from . import btoc_run
        return btoc_run.Captured(self, bound, ws)

    def run(self, ws=None, **bound):
        """Enqueue the program on the current stream (see btoc_run.run)."""
        from . import btoc_run
        return btoc_run.run(self, bound, ws)


def search(text: str, bound: dict, **kw):
    """Fastest schedule of `text` on the bound inputs (btoc_run.search)."""
    from . import btoc_run
    return btoc_run.search(text, bound, **kw)


def _uses(defs, name):
    n = 0
    for _, val in defs:
        if isinstance(val, Lin):
            for _, t in val.terms:
                if t == name or (isinstance(t, Prod) and t.vec == name):
                    n += 1
        elif isinstance(val, Mat):
            for u, v in val.terms:
                n += (u == name) + (v == name)
    return n


# The fusion decisions the schedule makes, each of which can be switched off
# (the choices the paper's search explores, Section IV): products of one
# matrix share a sweep; an update that is not an output is contracted; a
# row dot feeding the column sums of its matrix runs row-resident; vector
# statements fuse (three-way sums, AXPYDOT).
DECISIONS = ("share", "contract", "chain", "vector")


#: most rank-1 terms one library pass applies (bto_pass stores or contracts two)
LIBRARY_MAX_TERMS = 2


def compile_spec(text: str, form: str = "fused", off=(), target: str = "library") -> Program:
    """Parse, type and schedule a specification (see the module text).
    `off` names fusion decisions (DECISIONS) not to take in the fused form.
    `target` "library" lowers onto the library's passes (one row dot and one
    column sum per sweep, updates of rank two at most); "generated" plans
    for emitted passes (btoc_gen): products of one matrix at one point of
    the schedule all share a sweep, and an update of any rank is stored or
    formed in registers (contracted) by the sweep that reads it."""
    if form not in ("fused", "unfused"):
        raise SpecError("form must be 'fused' or 'unfused'")
    if target not in ("library", "generated"):
        raise SpecError("target must be 'library' or 'generated'")
    if target == "generated" and form != "fused":
        raise SpecError("generated passes are the fused form")
    if any(d not in DECISIONS for d in off):
        raise SpecError(f"unknown fusion decision in {tuple(off)}")
    spec = parse(text)
    ty = _Typer(spec)
    for lhs, tree in spec.statements:
        ty.statement(lhs, tree)
    for o in ty.outputs:
        if o not in ty.defined:
            raise SpecError(f"output {o} is never assigned")
    fused = form == "fused"
    outputs = set(ty.outputs)
    on = {d: fused and d not in off for d in DECISIONS}
    gen = target == "generated"
    if gen:
        on["chain"] = False        # the row-resident chain is the library's own sweep
    sched = _Scheduler(fused, ty.colmajor, on, generated=gen)
    sched.temps = [n for n, v in ty.defs if isinstance(v, Lin) and n not in outputs]
    for name in ty.inputs:
        sched.avail[name] = 0

    for name, val in ty.defs:
        if name in outputs and isinstance(val, Mat) and not val.terms:
            raise SpecError(f"{name}: a matrix output must update a matrix input")
        if (isinstance(val, Mat) and fused and not gen
                and len(val.terms) > LIBRARY_MAX_TERMS):
            raise SpecError(f"{name}: an update of rank {len(val.terms)} needs generated "
                            f"passes (the library's sweeps apply {LIBRARY_MAX_TERMS} terms)")
    # matrix updates: stored when an output (or always, unfused), else contracted
    for name, val in ty.defs:
        if isinstance(val, Mat) and val.terms and (name in outputs or not on["contract"]):
            sched.store(name, val, name in outputs)

    for name, val in ty.defs:
        if isinstance(val, Lin):
            sched.define(ty, name, val, outputs)
        elif isinstance(val, Dot):
            sched.dot(name, val)

    return Program(spec.name, form, [d.name for d in spec.inputs], ty.outputs, ty.kinds,
                   _ordered(sched.steps), sched.temps, sched.temp_mats, set(ty.colmajor),
                   target)


class _Scheduler:
    """Passes are planned on the matrices as stored: an m x n matrix stored
    by columns is the row-major n x m matrix of its transpose, so its
    products swap row dots and column sums and its updates swap u and v."""

    def __init__(self, fused: bool, colmajor=(), on=None, generated: bool = False):
        self.fused = fused
        self.generated = generated
        self.on = on if on is not None else {d: fused for d in DECISIONS}
        self.colmajor = set(colmajor)
        self.avail = {}          # vector or matrix -> first level that may read it
        self.steps = []
        self.temps = []
        self.temp_mats = {}      # stored updates that are not outputs -> their source
        self.stored = {}         # stored update -> Mat
        self.ntemp = 0

    def temp(self):
        self.ntemp += 1
        name = f"_s{self.ntemp}"
        self.temps.append(name)
        return name

    def phys(self, base, terms):
        """Rank-1 terms of an update as the stored matrix sees them."""
        return tuple((v, u) for u, v in terms) if base in self.colmajor else tuple(terms)

    def store(self, name, val: Mat, is_output: bool):
        lvl = max([self.avail.get(s, 0) for uv in val.terms for s in uv]
                  + [self.avail.get(val.base, 0)])
        self.stored[name] = val
        if not is_output:
            self.temp_mats[name] = val.base
        if self.fused:
            self.steps.append(Pass(lvl, val.base, self.phys(val.base, val.terms), store=name))
            self.avail[name] = lvl    # products over the update may fuse into its pass
        else:
            # the BLAS way: one rank-1 sweep per term, in place after the first
            src = val.base
            for k, uv in enumerate(val.terms):
                self.steps.append(Pass(lvl + k, src, self.phys(val.base, (uv,)), store=name))
                src = name
            self.avail[name] = lvl + len(val.terms)

    def resolve(self, m: Mat):
        """(matrix symbol, contracted terms) that a product of m reads."""
        if not m.terms:
            return m.base, ()
        for name, val in self.stored.items():
            if val.base == m.base and val.terms == m.terms:
                return name, ()
        return m.base, m.terms

    def vec_sum(self, out, terms, lvl):
        """out = sum of c_k t_k: one three-way sum (bto_vadd) when every
        coefficient is 1, one pass per eight terms (bto_lincomb) otherwise,
        or, with vector fusion off, scaled sums of two (bto_waxpby)."""
        if self.on["vector"] and len(terms) == 3 and all(c == ONE for c, _ in terms):
            self.steps.append(Vadd(lvl, out, terms[0][1], terms[1][1], terms[2][1]))
            return
        if self.on["vector"] and len(terms) >= 3:
            # one pass per eight terms: the sum so far is the first of the next
            self.steps.append(LinComb(lvl, out, list(terms[:8])))
            rest = list(terms[8:])
            while rest:
                self.steps.append(LinComb(lvl, out, [(ONE, out)] + rest[:7]))
                rest = rest[7:]
            return
        c0, t0 = terms[0]
        if len(terms) == 1:
            self.steps.append(VecOp(lvl, out, c0, t0, (0.0, ()), t0))
            return
        c1, t1 = terms[1]
        self.steps.append(VecOp(lvl, out, c0, t0, c1, t1))
        for ck, tk in terms[2:]:
            self.steps.append(VecOp(lvl, out, ONE, out, ck, tk))

    def product(self, ty, t: Prod, coef, out, add, add_scale, add_level, outputs):
        """Schedule out = coef * (M v) [+ add_scale * add]; returns the level
        from which out may be read."""
        base, terms = self.resolve(t.mat)
        terms = self.phys(base, terms)
        trans = t.mat.trans != (base in self.colmajor)     # as the stored matrix sees it
        lvl = max(self.avail.get(t.vec, 0), self.avail.get(base, 0), add_level)
        if self.on["chain"] and trans and not t.mat.terms and add is None:
            src = self.chain_source(ty, t, base, outputs)
            if src is not None:
                src.chain = True
                src.row["out"] = None
                src.col = {"y": None, "out": out, "scale": coef, "add": None, "add_scale": ONE}
                if t.vec in self.temps:
                    self.temps.remove(t.vec)
                return src.level + 1
        if terms and add is not None and add_scale != ONE and not self.generated:
            # a contracted sweep adds its vector unscaled: scale it first
            tmp = self.temp()
            self.vec_sum(tmp, [(add_scale, add)], add_level)
            add, add_scale = tmp, ONE
        kind = "col" if trans else "row"
        spec_ = {"x" if kind == "row" else "y": t.vec, "out": out, "scale": coef,
                 "add": add, "add_scale": add_scale}
        p = self.place(lvl, base, terms, kind, spec_)
        return p.level + 1

    def define(self, ty, name, val: Lin, outputs):
        prods = [(c, t) for c, t in val.terms if isinstance(t, Prod)]
        vecs = [(c, t) for c, t in val.terms if isinstance(t, str)]
        vec_level = max([self.avail.get(t, 0) for _, t in vecs] + [0])
        if not prods:
            self.vec_sum(name, vecs, vec_level)
            self.avail[name] = vec_level
            return
        if len(prods) == 1:
            # the vector terms go into the product's epilogue
            c, t = prods[0]
            add, add_scale = None, ONE
            if len(vecs) == 1:
                add_scale, add = vecs[0]
            elif vecs:
                add = self.temp()
                self.vec_sum(add, vecs, vec_level)
            self.avail[name] = self.product(ty, t, c, name, add, add_scale,
                                            vec_level if add else 0, outputs)
            return
        # several products: each into a temporary (free to fuse), then summed
        parts = []
        lvl = vec_level
        for c, t in prods:
            tmp = self.temp()
            lvl = max(lvl, self.product(ty, t, c, tmp, None, ONE, 0, outputs))
            parts.append((ONE, tmp))
        self.vec_sum(name, parts + vecs, lvl)
        self.avail[name] = lvl

    def dot(self, name, d: Dot):
        """r = x . y; fused with the scaled difference that forms one of its
        operands (z = w - alpha v, then z . u: AXPYDOT's one pass)."""
        lvl = max(self.avail.get(d.x, 0), self.avail.get(d.y, 0))
        if self.on["vector"]:
            for z, u in ((d.x, d.y), (d.y, d.x)):
                writers = [i for i, s in enumerate(self.steps) if getattr(s, "out", None) == z]
                if len(writers) != 1:
                    continue
                i = writers[0]
                s = self.steps[i]
                # z = w - alpha v formed in one step, and u ready by then
                if (isinstance(s, VecOp) and s.a == ONE and s.x != s.y and u != z
                        and self.avail.get(u, 0) <= s.level):
                    self.steps[i] = AxpyDot(s.level, z, s.x, s.y, (-s.b[0], s.b[1]), u, name)
                    self.avail[name] = s.level
                    return
        self.steps.append(DotOp(lvl, name, d.x, d.y))
        self.avail[name] = lvl

    def chain_source(self, ty, t: Prod, base, outputs):
        """The pass that forms t.vec as plain row dots of t's matrix, when
        t = A' * (A x) can run as one row-resident pass: t.vec a temporary
        read only here, its pass a plain row dot with nothing fused in."""
        if t.vec in outputs or _uses(ty.defs, t.vec) != 1:
            return None
        for s in self.steps:
            if (isinstance(s, Pass) and s.row and s.row["out"] == t.vec
                    and s.base == base and not s.terms and not s.store
                    and not s.col and not s.chain and s.row["add"] is None
                    and s.row["scale"] == ONE):
                return s
        return None

    def place(self, lvl, base, terms, kind, spec_):
        """Fuse into a pass over the same matrix at the same level that has
        this kind of reduction free (generated passes: any pass over the same
        matrix at that level); otherwise open a pass."""
        if self.generated:
            for s in self.steps:
                if not isinstance(s, Pass) or s.level != lvl:
                    continue
                same = ((s.store is not None and s.store == base and not terms)
                        or (s.store is None and s.base == base and s.terms == terms))
                if same and self.on["share"]:
                    getattr(s, kind + "s").append(spec_)
                    return s
            p = Pass(lvl, base, terms, contract=bool(terms))
            getattr(p, kind + "s").append(spec_)
            self.steps.append(p)
            return p
        if self.on["share"]:
            for s in self.steps:
                if not isinstance(s, Pass) or s.level != lvl or s.chain:
                    continue
                if getattr(s, kind) is not None:
                    continue
                same = ((s.store is not None and s.store == base and not terms)
                        or (s.store is None and s.base == base and s.terms == terms))
                if not same:
                    continue
                other = s.col if kind == "row" else s.row
                if terms and other is not None:
                    continue           # a contracted sweep does one of the two
                setattr(s, kind, spec_)
                return s
        p = Pass(lvl, base, terms, contract=bool(terms))
        setattr(p, kind, spec_)
        self.steps.append(p)
        return p


def _ordered(steps):
    """Program order: by level, passes before the vector sums that read
    their results at the same level (a vector op at level L runs after the
    passes of level L - 1 have finished)."""
    keyed = []
    for i, s in enumerate(steps):
        keyed.append(((s.level, 1 if isinstance(s, Pass) else 0, i), s))
    return [s for _, s in sorted(keyed, key=lambda kv: kv[0])]


def main(argv=None) -> int:
    """python -m paper_1205_1098_amd.btoc SPEC [--unfused] [--off DECISION ...]

    Prints the schedule of a specification file (or of a kernel of the
    library's set: bicgk, gemver, atax, dgemvt, dgemv, gesummv, axpydot,
    waxpby, vadd, batax, gemver_contracted)."""
    import argparse

    from . import bto_specs

    ap = argparse.ArgumentParser(description="schedule of a BTO kernel specification")
    ap.add_argument("spec")
    ap.add_argument("--unfused", action="store_true")
    ap.add_argument("--off", nargs="*", default=[], choices=DECISIONS)
    args = ap.parse_args(argv)
    named = dict(bto_specs.TABLE_I, batax=bto_specs.BATAX,
                 gemver_contracted=bto_specs.GEMVER_CONTRACTED)
    if args.spec in named:
        text = named[args.spec]
    else:
        with open(args.spec) as f:
            text = f.read()
    try:
        prog = compile_spec(text, "unfused" if args.unfused else "fused", tuple(args.off))
    except SpecError as e:
        print(f"error: {e}")
        return 1
    print(f"{prog.name}: {len(prog.passes())} pass(es) over matrices, {len(prog.steps)} step(s)")
    for line in prog.describe():
        print("  " + line)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
