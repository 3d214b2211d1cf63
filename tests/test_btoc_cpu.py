"""The spec compiler on the CPU: parsing, typing, the fusion schedule it
chooses for each program (checked against the pass structure that the
dependences of Section III-D force), its refusals, and the reference
evaluator of specifications that the GPU tests compare with."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import spec_eval
from paper_1205_1098_amd import btoc, synth
from tests import specs

SEED = 7


def _u(stream, n):
    return synth.uniform(SEED, stream, n)


# ---- schedules ----------------------------------------------------------------

SCHEDULES = {
    ("bicgk", "fused"): ["pass 0: A ROWDOT|COLSUM"],
    ("bicgk", "unfused"): ["pass 0: A ROWDOT", "pass 0: A COLSUM"],
    ("gemver", "fused"): ["pass 0: A STORE|COLSUM", "pass 1: B ROWDOT"],
    ("gemver", "unfused"): ["pass 0: A STORE", "pass 1: B STORE", "pass 2: B COLSUM",
                            "pass 3: B ROWDOT"],
    ("atax", "fused"): ["pass 0: A CHAIN|ROWDOT|COLSUM"],
    ("atax", "unfused"): ["pass 0: A ROWDOT", "pass 1: A COLSUM"],
    ("dgemvt", "fused"): ["pass 0: A COLSUM", "pass 1: A ROWDOT"],
    ("dgemv", "fused"): ["pass 0: A ROWDOT"],
    ("gesummv", "fused"): ["pass 0: A ROWDOT", "pass 0: B ROWDOT",
                           "vec 1: y = a*_s1 + b*_s2"],
    ("waxpby", "fused"): ["vec 0: w = a*x + b*y"],
    ("vadd", "fused"): ["vadd 0: x = w + y + z"],
    ("vadd", "unfused"): ["vec 0: x = a*w + b*y", "vec 0: x = a*x + b*z"],
    ("axpydot", "fused"): ["axpydot 0: z = w - alpha*v; r = z.u"],
    ("axpydot", "unfused"): ["vec 0: z = a*w + b*v", "dot 0: r = z.u"],
}


@pytest.mark.parametrize("kernel,form", sorted(SCHEDULES))
def test_table_one_schedules(kernel, form):
    prog = btoc.compile_spec(specs.TABLE_I[kernel], form)
    assert prog.describe() == SCHEDULES[(kernel, form)]


def test_fig1_batax_is_one_row_resident_pass():
    """Fig. 1 as printed: the row dots feed the column sums row by row, so
    the whole kernel is one pass (the max-fuse organism of Section IV-A);
    unfused, the temporary A x is stored and read back."""
    prog = btoc.compile_spec(specs.BATAX)
    assert prog.name == "BATAX" and prog.inputs == ["A", "x", "beta"] and prog.outputs == ["y"]
    assert prog.describe() == ["pass 0: A CHAIN|ROWDOT|COLSUM"]
    assert prog.temps == []
    unf = btoc.compile_spec(specs.BATAX, "unfused")
    assert unf.describe() == ["pass 0: A ROWDOT", "pass 1: A COLSUM"] and len(unf.temps) == 1


def test_contracted_update_reads_A_twice():
    """B not an output: it is never stored, both products read A and add
    the rank-2 correction; x must be complete before w (two passes)."""
    prog = btoc.compile_spec(specs.GEMVER_CONTRACTED)
    assert prog.describe() == ["pass 0: A CONTRACT|COLSUM", "pass 1: A CONTRACT|ROWDOT"]
    unf = btoc.compile_spec(specs.GEMVER_CONTRACTED, "unfused")
    assert unf.temp_mats == {"B": "A"}
    assert unf.describe()[:2] == ["pass 0: A STORE", "pass 1: B STORE"]


NOVEL_SCHEDULES = {
    "both_ways": ["pass 0: A ROWDOT|COLSUM", "vec 1: z = a*_s1 + b*_s2"],
    "atax_plus": ["pass 0: A ROWDOT", "pass 1: A COLSUM"],
    "rank1_stored": ["pass 0: A STORE|ROWDOT|COLSUM"],
    "rank1_contracted": ["vec 0: _s1 = a*y + b*y", "pass 0: A CONTRACT|ROWDOT"],
    "two_dots": ["pass 0: A ROWDOT", "pass 1: A ROWDOT"],
    "mixed": ["vec 0: _s1 = a*y + b*w", "pass 0: A ROWDOT"],
    "lin4": ["lincomb 0: x = c*w + c*y + c*z + c*v"],
    "lin9": ["lincomb 0: x = " + " + ".join(f"c*a{k}" for k in range(1, 9)),
             "lincomb 0: x = c*x + c*a9"],
    "lin16": ["lincomb 0: x = " + " + ".join(f"c*b{k}" for k in range(1, 9)),
              "lincomb 0: x = c*x + " + " + ".join(f"c*b{k}" for k in range(9, 16)),
              "lincomb 0: x = c*x + c*b16"],
}


def test_declarations_over_several_lines():
    """A declaration list may break after a comma and resume on the next
    line; without the comma the next line is not part of the list."""
    prog = btoc.compile_spec("""DOTS
in:
    u : vector(column),
    w : vector(column),
    s : scalar
out:
    r : scalar
{
    r = u' * w
}""")
    assert prog.inputs == ["u", "w", "s"] and prog.outputs == ["r"]
    with pytest.raises(btoc.SpecError):
        btoc.compile_spec("""DOTS
in:
    u : vector(column)
    w : vector(column)
out: r : scalar
{ r = u' * w }""")


@pytest.mark.parametrize("name", sorted(NOVEL_SCHEDULES))
def test_novel_schedules(name):
    prog = btoc.compile_spec(specs.NOVEL[name])
    assert prog.describe() == NOVEL_SCHEDULES[name]


COLUMN_SCHEDULES = {
    "bicgk": ["pass 0: A ROWDOT|COLSUM"],
    "gemver": ["pass 0: A STORE|ROWDOT", "pass 1: B COLSUM"],
    "atax": ["pass 0: A COLSUM", "pass 1: A ROWDOT"],
    "dgemvt": ["pass 0: A ROWDOT", "pass 1: A COLSUM"],
    "dgemv": ["pass 0: A COLSUM"],
}


@pytest.mark.parametrize("kernel", sorted(COLUMN_SCHEDULES))
def test_column_major_schedules(kernel):
    """A matrix stored by columns is swept as its row-major transpose: its
    products swap row dots and column sums.  ATAX then loses its one-pass
    form: A x is a column sum, complete only after the last column, so the
    reduction dependence of Section III-D forces a second pass."""
    text = specs.TABLE_I[kernel].replace("matrix(row)", "matrix(column)")
    prog = btoc.compile_spec(text)
    assert prog.describe() == COLUMN_SCHEDULES[kernel]
    assert "A" in prog.colmajor


def test_column_major_update_swaps_its_terms():
    text = specs.GEMVER_CONTRACTED.replace("matrix(row)", "matrix(column)")
    p = btoc.compile_spec(text).passes()
    assert [(s.contract, s.row is not None, s.col is not None) for s in p] == \
        [(True, True, False), (True, False, True)]
    assert p[0].terms == (("v1", "u1"), ("v2", "u2"))
    bad = specs.TABLE_I["gemver"].replace("A : matrix(row)", "A : matrix(column)")
    with pytest.raises(btoc.SpecError, match="stored by rows"):
        btoc.compile_spec(bad)


VARIANTS = {
    "atax": [((), ["pass 0: A CHAIN|ROWDOT|COLSUM"]),
             (("chain",), ["pass 0: A ROWDOT", "pass 1: A COLSUM"])],
    "bicgk": [(("share",), ["pass 0: A ROWDOT", "pass 0: A COLSUM"])],
    "gemver": [(("share",), ["pass 0: A STORE", "pass 0: B COLSUM", "pass 1: B ROWDOT"])],
    "vadd": [(("vector",), ["vec 0: x = a*w + b*y", "vec 0: x = a*x + b*z"])],
    "axpydot": [(("vector",), ["vec 0: z = a*w + b*v", "dot 0: r = z.u"])],
}


@pytest.mark.parametrize("kernel", sorted(VARIANTS))
def test_fusion_decisions_switch_off(kernel):
    """Each fusion decision the search may switch off gives the schedule
    that decision saves a pass or a step over."""
    for off, sched in VARIANTS[kernel]:
        assert btoc.compile_spec(specs.TABLE_I[kernel], "fused", off).describe() == sched


def test_contraction_switched_off_stores_a_temporary():
    p = btoc.compile_spec(specs.GEMVER_CONTRACTED, "fused", ("contract",))
    assert p.describe() == ["pass 0: A STORE|COLSUM", "pass 1: B ROWDOT"]
    assert p.temp_mats == {"B": "A"}
    with pytest.raises(btoc.SpecError, match="unknown fusion decision"):
        btoc.compile_spec(specs.GEMVER_CONTRACTED, "fused", ("tile",))


def test_unfused_is_one_operation_per_pass():
    for src in list(specs.TABLE_I.values()) + list(specs.NOVEL.values()):
        for s in btoc.compile_spec(src, "unfused").passes():
            assert (s.row is None) + (s.col is None) + (not s.store) >= 2
            assert not s.chain and not s.contract


def test_dot_fuses_only_with_the_difference_that_forms_its_operand():
    """z = w - alpha v then z . u is AXPYDOT's one pass; a dot of an input,
    or of a vector summed in more than one step, is a dot of its own."""
    src = """K
in: w : vector(column), v : vector(column), u : vector(column), x : vector(column)
out: z : vector(column), r : scalar, q : scalar
{
  z = w + v + x
  r = z' * u
  q = u' * w
}"""
    assert btoc.compile_spec(src).describe() == ["vadd 0: z = w + v + x", "dot 0: r = z.u",
                                                 "dot 0: q = u.w"]
    with pytest.raises(btoc.SpecError, match="computed scalar"):
        btoc.compile_spec("""K
in: w : vector(column), u : vector(column)
out: r : scalar, y : vector(column)
{
  r = w' * u
  y = r * w
}""")


@pytest.mark.parametrize("text,message", [
    ("K\nin: x : vector(column)\nout: y : vector(column)\n{ y = A * x }", "before it is defined"),
    ("K\nin: x : vector(column), y : vector(column)\nout: s : vector(column)\n{ s = x' * y }",
     "scalar output"),
    ("K\nin: A : matrix(row), x : vector(column)\nout: y : vector(column)\n{ x = A * x }",
     "input"),
    ("K\nin: A : matrix(row), u : vector(column)\nout: B : matrix(row)\n"
     "{ B = A + u * u' + u * u' + u * u' }", "needs generated"),
    ("K\nin: A : matrix(row), x : vector(column)\nout: y : vector(column), w : vector(column)\n"
     "{ y = A * x }", "never assigned"),
    ("K\nin: A : matrix(row)\nout: B : matrix(row)\n{ B = A }", "must update"),
    ("K\nin: A : matrix(row), u : vector(column)\nout: B : matrix(row)\n{ B = A' + u * u' }",
     "untransposed"),
    ("K\nin: A : matrix(row), x : vector(column)\nout: y : vector(column)\n{ y = A * x x }",
     "expected"),
    ("K\nin: x : tensor(row)\nout: y : vector(column)\n{ y = x }", "unknown type"),
    ("K\nin: A : matrix(row), u : vector(column), x : vector(column)\nout: y : vector(column)\n"
     "{ B = A + u * u'\n B = A\n y = B * x }", "assigned twice"),
    ("K\nin: x : vector(column)\nout: y : vector(column)\n{ y = x\n y = 2 * x }",
     "assigned twice"),
])
def test_refusals(text, message):
    with pytest.raises(btoc.SpecError, match=message):
        btoc.compile_spec(text)


def test_unknown_form():
    with pytest.raises(btoc.SpecError):
        btoc.compile_spec(specs.TABLE_I["dgemv"], "fast")


# ---- the reference evaluator, pinned --------------------------------------------

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _golden_inputs(kernel, case):
    a = lambda v: np.array(v, dtype=float)
    return {k: (a(v) if isinstance(v, list) else float(v)) for k, v in case.items()}


@pytest.mark.parametrize("kernel,outs", [
    ("bicgk", ("q", "s")), ("gemver", ("B", "x", "w")), ("atax", ("y",)),
    ("dgemvt", ("x", "w")), ("dgemv", ("z",)), ("gesummv", ("y",)), ("waxpby", ("w",)),
    ("vadd", ("x",)), ("axpydot", ("z", "r"))])
def test_evaluator_hand_worked(kernel, outs):
    """Table I's specs on the hand-worked fixtures give the hand-worked
    values exactly."""
    case = json.load(open(GOLDEN))[kernel]
    got = spec_eval.evaluate(specs.TABLE_I[kernel], _golden_inputs(kernel, case))
    for o in outs:
        assert np.array_equal(np.atleast_1d(got[o]), np.atleast_1d(np.array(case[o], dtype=float))), \
            (kernel, o)


@pytest.mark.parametrize("m,n", [(1, 1), (7, 5), (64, 130), (300, 257)])
def test_evaluator_agrees_with_the_oracle_kernels(m, n):
    """The spec evaluator and the C oracle are written independently; on
    Table I's kernels they agree to within rounding (normwise 1e-13)."""
    A, B = synth.matrix(SEED, 1, m, n), synth.matrix(SEED, 2, m, n)
    u1, u2, y, r = _u(3, m), _u(4, m), _u(5, m), _u(6, m)
    v1, v2, z, p = _u(7, n), _u(8, n), _u(9, n), _u(10, n)

    def close(a, b):
        a, b = np.asarray(a), np.asarray(b)
        return np.max(np.abs(a - b)) <= 1e-13 * max(np.max(np.abs(b)), 1e-300)

    ev = lambda k, **kw: spec_eval.evaluate(specs.TABLE_I[k], kw)
    q, s = oracle.bicgk(A, p, r)
    g = ev("bicgk", A=A, p=p, r=r)
    assert close(g["q"], q) and close(g["s"], s)
    Bo, xo, wo = oracle.gemver(A, u1, v1, u2, v2, y, z, 1.5, 0.7)
    g = ev("gemver", A=A, u1=u1, v1=v1, u2=u2, v2=v2, y=y, z=z, alpha=1.5, beta=0.7)
    assert np.array_equal(g["B"], Bo) and close(g["x"], xo) and close(g["w"], wo)
    assert close(ev("atax", A=A, x=p)["y"], oracle.atax(A, p))
    xo, wo = oracle.dgemvt(A, y, z, 1.5, 0.7)
    g = ev("dgemvt", A=A, y=y, z=z, alpha=1.5, beta=0.7)
    assert close(g["x"], xo) and close(g["w"], wo)
    assert close(ev("dgemv", A=A, x=p, y=y, alpha=1.5, beta=0.7)["z"],
                 oracle.dgemv(A, p, y, 1.5, 0.7))
    assert close(ev("gesummv", A=A, B=B, x=p, alpha=1.5, beta=0.7)["y"],
                 oracle.gesummv(A, B, p, 1.5, 0.7))
    assert np.array_equal(ev("waxpby", x=p, y=z, alpha=1.5, beta=0.7)["w"],
                          oracle.waxpby(p, z, 1.5, 0.7))
    assert np.array_equal(ev("vadd", w=p, y=z, z=v1)["x"], oracle.vadd(p, z, v1))
    g = ev("axpydot", w=z, v=v1, u=v2, alpha=1.5)
    zo, ro = oracle.axpydot(z, v1, v2, 1.5)
    assert np.array_equal(g["z"], zo) and close([g["r"]], [ro])
    got = spec_eval.evaluate(specs.BATAX, {"A": A, "x": p, "beta": 0.7})["y"]
    assert close(got, 0.7 * oracle.atax(A, p))
    got = spec_eval.evaluate(specs.GEMVER_CONTRACTED, dict(A=A, u1=u1, v1=v1, u2=u2, v2=v2,
                                                             y=y, z=z, alpha=1.5, beta=0.7))
    assert close(got["x"], oracle.gemver(A, u1, v1, u2, v2, y, z, 1.5, 0.7)[1])


def test_evaluator_integers_exact():
    """Small-integer data: every novel program equals its int64 value."""
    m = n = 200
    I = lambda st, k: synth.small_ints(11, st, k)
    A = synth.matrix(11, 1, m, n, kind="int")
    Ai = A.astype(np.int64)
    x, w, z, y, u, v, p, r = (I(k, n) for k in range(2, 10))
    i64 = lambda a: a.astype(np.int64)
    ev = lambda k, **kw: spec_eval.evaluate(specs.NOVEL[k], kw)
    assert np.array_equal(ev("both_ways", A=A, x=x, w=w)["z"], Ai @ i64(x) + Ai.T @ i64(w))
    assert np.array_equal(ev("atax_plus", A=A, x=x, z=z)["y"], Ai.T @ (Ai @ i64(x)) + i64(z))
    Bi = Ai + np.outer(i64(u), i64(v))
    g = ev("rank1_stored", A=A, u=u, v=v, p=p, r=r)
    assert np.array_equal(g["B"], Bi) and np.array_equal(g["q"], Bi @ i64(p))
    assert np.array_equal(g["s"], Bi.T @ i64(r))
    g = ev("rank1_contracted", A=A, u=u, v=v, x=x, y=y, gamma=3.0)
    assert np.array_equal(g["w"], Bi @ i64(x) - 3 * i64(y))
    assert np.array_equal(ev("two_dots", A=A, x=x)["y"], 2 * (Ai @ (Ai @ i64(x))))
    g = ev("mixed", A=A, x=x, y=y, w=w, alpha=2.0)
    assert np.array_equal(g["z"], -(Ai @ i64(x)) + i64(y) - 2 * i64(w))
    g = ev("lin4", w=w, y=y, z=z, v=v, a=3.0)
    assert np.array_equal(g["x"], 3 * i64(w) + i64(y) - 2 * i64(z) + i64(v))


def test_command_line(capsys, tmp_path):
    assert btoc.main(["batax"]) == 0
    assert "pass 0: A CHAIN|ROWDOT|COLSUM" in capsys.readouterr().out
    f = tmp_path / "k.bto"
    f.write_text(specs.NOVEL["two_dots"])
    assert btoc.main([str(f), "--unfused"]) == 0
    assert "pass 1: A ROWDOT" in capsys.readouterr().out
    f.write_text("K\nin: x : vector(column)\nout: y : vector(column)\n{ y = z }")
    assert btoc.main([str(f)]) == 1


def test_bound_output_over_an_input_is_refused():
    """An output bound to memory an input also uses is refused before
    anything runs (it would be written while the input is still read); a
    matrix update bound to exactly the matrix it updates is the in-place
    form and is accepted up to the first library call."""
    torch = pytest.importorskip("torch")
    prog = btoc.compile_spec(specs.NOVEL["lin9"])
    vecs = {f"a{k}": torch.zeros(16, dtype=torch.float64) for k in range(1, 10)}
    with pytest.raises(btoc.SpecError, match="shares memory"):
        prog.run(c=1.5, x=vecs["a9"], **vecs)
    buf = torch.zeros(40, dtype=torch.float64)
    vecs["a3"] = buf[:16]
    with pytest.raises(btoc.SpecError, match="shares memory"):
        prog.run(c=1.5, x=buf[10:26], **vecs)
    g = btoc.compile_spec(specs.TABLE_I["gemver"])
    A = torch.zeros((8, 8), dtype=torch.float64)
    ins = {k: torch.zeros(8, dtype=torch.float64) for k in ("u1", "v1", "u2", "v2", "y", "z")}
    with pytest.raises(btoc.SpecError, match="shares memory"):
        g.run(A=A, B=A[:, :], x=ins["z"], alpha=1.5, beta=0.7, **ins)   # x over input z
    try:
        g.run(A=A, B=A, alpha=1.5, beta=0.7, **ins)                   # in place: not refused
    except btoc.SpecError as e:
        pytest.fail(f"in-place update refused: {e}")
    except Exception:
        pass          # no device here: the first library call fails, as it must
