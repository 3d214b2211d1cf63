"""Compiled specifications on the GPU against the reference evaluation of
the same specification (oracle/spec_eval.py): every Table I kernel, Fig. 1's
BATAX, GEMVER with B contracted, and programs outside the paper's suite,
in both forms, on ragged shapes; integer-valued data must match bitwise."""

import numpy as np
import pytest

from oracle import spec_eval
from paper_1205_1098_amd import synth
from tests import specs

pytestmark = pytest.mark.gpu

TOL = 1e-12
SEED = synth.SEED


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import btoc

    return torch, btoc, torch.device("cuda:0")


# input name -> "A" (an m x n matrix), "m" / "n" (vector lengths) or a scalar value
GEMVER_IN = dict(A="A", u1="m", v1="n", u2="m", v2="n", y="m", z="n", alpha=1.5, beta=0.7)
PROGRAMS = {
    "bicgk": (specs.TABLE_I["bicgk"], dict(A="A", p="n", r="m"), False),
    "gemver": (specs.TABLE_I["gemver"], GEMVER_IN, False),
    "atax": (specs.TABLE_I["atax"], dict(A="A", x="n"), False),
    "dgemvt": (specs.TABLE_I["dgemvt"], dict(A="A", y="m", z="n", alpha=1.5, beta=0.7), False),
    "dgemv": (specs.TABLE_I["dgemv"], dict(A="A", x="n", y="m", alpha=1.5, beta=0.7), False),
    "gesummv": (specs.TABLE_I["gesummv"], dict(A="A", B="A", x="n", alpha=1.5, beta=0.7), False),
    "batax": (specs.BATAX, dict(A="A", x="n", beta=0.7), False),
    "axpydot": (specs.TABLE_I["axpydot"], dict(w="n", v="n", u="n", alpha=1.5), False),
    "waxpby": (specs.TABLE_I["waxpby"], dict(x="n", y="n", alpha=1.5, beta=0.7), False),
    "vadd": (specs.TABLE_I["vadd"], dict(w="n", y="n", z="n"), False),
    "gemver_contracted": (specs.GEMVER_CONTRACTED, GEMVER_IN, False),
    "both_ways": (specs.NOVEL["both_ways"], dict(A="A", x="n", w="m"), True),
    "atax_plus": (specs.NOVEL["atax_plus"], dict(A="A", x="n", z="n"), False),
    "rank1_stored": (specs.NOVEL["rank1_stored"], dict(A="A", u="m", v="n", p="n", r="m"),
                     False),
    "rank1_contracted": (specs.NOVEL["rank1_contracted"],
                         dict(A="A", u="m", v="n", x="n", y="m", gamma=1.25), False),
    "two_dots": (specs.NOVEL["two_dots"], dict(A="A", x="n"), True),
    "mixed": (specs.NOVEL["mixed"], dict(A="A", x="n", y="m", w="m", alpha=0.5), False),
    "lin4": (specs.NOVEL["lin4"], dict(w="n", y="n", z="n", v="n", a=1.5), False),
    "lin9": (specs.NOVEL["lin9"], dict({f"a{k}": "n" for k in range(1, 10)}, c=1.5), False),
    "lin16": (specs.NOVEL["lin16"], {f"b{k}": "n" for k in range(1, 17)}, False),
}
SHAPES = [(1, 1), (65, 127), (513, 1000), (300, 4097), (2047, 2049)]
SQUARE = [(1, 1), (127, 127), (1000, 1000), (2049, 2049)]


def _inputs(kinds, m, n, kind, case):
    host = {}
    for k, (name, what) in enumerate(sorted(kinds.items())):
        stream = synth.stream_id(9, k, case)
        if what == "A":
            # a second matrix operand ("B") gets its own stream
            host[name] = synth.matrix(SEED, stream, m, n, kind=kind)
        elif what in ("m", "n"):
            host[name] = synth.vector(SEED, stream, m if what == "m" else n, kind)
        else:
            host[name] = float(what) if kind == "uniform" else float(round(2 * what) or 2)
    return host


def _relerr(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    if ref.size == 0:
        return 0.0
    den = float(np.max(np.abs(ref)))
    num = float(np.max(np.abs(got - ref)))
    return num / den if den > 0 else num


def _cases():
    out = []
    for name, (_, _, square) in sorted(PROGRAMS.items()):
        for m, n in (SQUARE if square else SHAPES):
            out.append((name, m, n))
    return out


@pytest.mark.parametrize("form", ["fused", "unfused"])
@pytest.mark.parametrize("kind", ["uniform", "int"])
@pytest.mark.parametrize("name,m,n", _cases())
def test_compiled_program(env, name, m, n, kind, form):
    torch, btoc, dev = env
    text, kinds, _ = PROGRAMS[name]
    case = 31 * m + n
    host = _inputs(kinds, m, n, kind, case)
    ref = spec_eval.evaluate(text, host)
    prog = btoc.compile_spec(text, form)
    bound = {k: (torch.from_numpy(np.ascontiguousarray(v)).to(dev) if isinstance(v, np.ndarray)
                 else v) for k, v in host.items()}
    out = prog.run(**bound)
    torch.cuda.synchronize()
    for o, r in ref.items():
        got, r = out[o].cpu().numpy().reshape(np.shape(r)), np.asarray(r)
        if kind == "int":
            assert np.array_equal(got, r), (name, o)
        else:
            assert _relerr(got, r) <= TOL, (name, o, _relerr(got, r))


COLUMN_PROGRAMS = ["bicgk", "gemver", "atax", "dgemvt", "dgemv", "gesummv", "batax",
                   "gemver_contracted", "rank1_stored", "rank1_contracted", "both_ways"]


@pytest.mark.parametrize("form", ["fused", "unfused"])
@pytest.mark.parametrize("kind", ["uniform", "int"])
@pytest.mark.parametrize("m,n", [(65, 127), (513, 1000), (2047, 2049)])
@pytest.mark.parametrize("name", COLUMN_PROGRAMS)
def test_compiled_program_column_major(env, name, m, n, kind, form):
    """The same programs with every matrix stored by columns (tensors with
    unit stride down a column), against the same reference values."""
    torch, btoc, dev = env
    text, kinds, square = PROGRAMS[name]
    if square:
        n = m
    text = text.replace("matrix(row)", "matrix(column)")
    host = _inputs(kinds, m, n, kind, 7 * m + n)
    ref = spec_eval.evaluate(text, host)
    prog = btoc.compile_spec(text, form)
    bound = {}
    for k, v in host.items():
        if isinstance(v, np.ndarray) and v.ndim == 2:
            bound[k] = torch.from_numpy(np.ascontiguousarray(v.T)).to(dev).t()
        elif isinstance(v, np.ndarray):
            bound[k] = torch.from_numpy(v).to(dev)
        else:
            bound[k] = v
    out = prog.run(**bound)
    torch.cuda.synchronize()
    for o, r in ref.items():
        got = out[o].cpu().numpy()
        if kind == "int":
            assert np.array_equal(got, r), (name, o)
        else:
            assert _relerr(got, r) <= TOL, (name, o, _relerr(got, r))


@pytest.mark.parametrize("name", ["gemver_contracted", "atax", "bicgk", "axpydot", "vadd"])
def test_search_times_only_correct_schedules(env, name):
    """Every schedule the search times computes the reference outputs, and
    it returns one of them."""
    torch, btoc, dev = env
    text, kinds, _ = PROGRAMS[name]
    host = _inputs(kinds, 700, 900, "uniform", 3)
    ref = spec_eval.evaluate(text, host)
    bound = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
             for k, v in host.items()}
    best, table = btoc.search(text, bound, reps=2)
    assert len(table) >= 2
    for off, sched, ms in table:
        assert ms > 0
        prog = (btoc.compile_spec(text, "unfused") if off == "unfused"
                else btoc.compile_spec(text, "fused", off))
        assert prog.describe() == sched
        out = prog.run(**bound)
        for o, r in ref.items():
            got = out[o].cpu().numpy().reshape(np.shape(r))
            assert _relerr(got, np.asarray(r)) <= TOL, (name, off, o)
    assert best.describe() in [sched for _, sched, _ in table]


@pytest.mark.parametrize("name", ["gemver", "atax", "axpydot", "gemver_contracted"])
def test_captured_program_replays(env, name):
    """A program captured in a HIP graph: each replay, on inputs rewritten in
    place between replays (with eager work and synchronizations in between),
    gives the bits of the same program run eagerly on the same inputs."""
    torch, btoc, dev = env
    text, kinds, _ = PROGRAMS[name]
    prog = btoc.compile_spec(text)
    d = lambda h: {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
                   for k, v in h.items()}
    bound = d(_inputs(kinds, 300, 200, "uniform", 1))
    cap = prog.capture(**bound)
    for rep in range(3):
        fresh = d(_inputs(kinds, 300, 200, "uniform", 10 + rep))
        for k, t in fresh.items():
            if isinstance(t, torch.Tensor):
                bound[k].copy_(t)
        torch.cuda.synchronize()
        out = cap.replay()
        torch.cuda.synchronize()
        eager = prog.run(**fresh)
        torch.cuda.synchronize()
        for o in eager:
            assert torch.equal(out[o], eager[o]), (name, rep, o)


@pytest.mark.parametrize("name,kind", [("gemver", "int"), ("gemver", "uniform"),
                                       ("gemver_contracted", "uniform"), ("bicgk", "uniform"),
                                       ("atax", "uniform")])
def test_full_size_compiled(env, name, kind):
    """n = 16384, the size the benchmark times the compiled programs at,
    against the C oracle's kernels (integer data bitwise)."""
    import oracle

    torch, btoc, dev = env
    N = 16384
    text, kinds, _ = PROGRAMS[name]
    host = _inputs(kinds, N, N, kind, 99)
    if kind == "int":
        host.update(alpha=2.0, beta=3.0)
    d = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
         for k, v in host.items()}
    out = btoc.compile_spec(text).run(**d)
    h = host
    if name == "gemver":
        B, x, w = oracle.gemver(h["A"], h["u1"], h["v1"], h["u2"], h["v2"], h["y"], h["z"],
                                h["alpha"], h["beta"])
        ref = {"B": B, "x": x, "w": w}
    elif name == "gemver_contracted":
        _, x, w = oracle.gemver(h["A"], h["u1"], h["v1"], h["u2"], h["v2"], h["y"], h["z"],
                                h["alpha"], h["beta"])
        ref = {"x": x, "w": w}
    elif name == "bicgk":
        q, s_ = oracle.bicgk(h["A"], h["p"], h["r"])
        ref = {"q": q, "s": s_}
    else:
        ref = {"y": oracle.atax(h["A"], h["x"])}
    for o, r in ref.items():
        got = out[o].cpu().numpy()
        if kind == "int":
            assert np.array_equal(got, r), (name, o)
        else:
            assert _relerr(got, r) <= TOL, (name, o, _relerr(got, r))


@pytest.mark.parametrize("form", ["fused", "unfused"])
@pytest.mark.parametrize("m,n", [(0, 5), (5, 0), (0, 0)])
@pytest.mark.parametrize("name", ["bicgk", "gemver", "atax", "dgemvt", "dgemv", "gesummv",
                                  "batax", "gemver_contracted", "rank1_stored"])
def test_compiled_program_empty_extents(env, name, m, n, form):
    """m or n = 0: empty sums are 0, and every output is still written."""
    torch, btoc, dev = env
    text, kinds, _ = PROGRAMS[name]
    host = _inputs(kinds, m, n, "uniform", 2)
    ref = spec_eval.evaluate(text, host)
    bound = {}
    for k, v in host.items():
        if isinstance(v, np.ndarray) and v.ndim == 2:
            bound[k] = torch.empty((max(m, 1), max(n, 2)), dtype=torch.float64,
                                   device=dev)[:m, :n]
        elif isinstance(v, np.ndarray):
            bound[k] = torch.from_numpy(v).to(dev)
        else:
            bound[k] = v
    out = btoc.compile_spec(text, form).run(**bound)
    for o, r in ref.items():
        got = out[o].cpu().numpy()
        assert got.shape == np.shape(r), (name, o)
        assert np.array_equal(got, np.asarray(r)), (name, o)


def test_outputs_bound_by_the_caller_receive_the_results(env):
    torch, btoc, dev = env
    text, kinds, _ = PROGRAMS["gemver"]
    host = _inputs(kinds, 300, 200, "uniform", 5)
    d = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
         for k, v in host.items()}
    B = torch.empty((300, 200), dtype=torch.float64, device=dev)
    x = torch.empty(200, dtype=torch.float64, device=dev)
    w = torch.empty(300, dtype=torch.float64, device=dev)
    out = btoc.compile_spec(text).run(**d, B=B, x=x, w=w)
    assert out["B"] is B and out["x"] is x and out["w"] is w
    ref = spec_eval.evaluate(text, host)
    for o, t in (("B", B), ("x", x), ("w", w)):
        assert _relerr(t.cpu().numpy(), ref[o]) <= TOL


def test_wrong_lengths_are_refused_before_launch(env):
    torch, btoc, dev = env
    prog = btoc.compile_spec(specs.TABLE_I["dgemv"])
    A = torch.zeros((40, 30), dtype=torch.float64, device=dev)
    x = torch.zeros(31, dtype=torch.float64, device=dev)
    y = torch.zeros(40, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError, match="length"):
        prog.run(A=A, x=x, y=y, alpha=1.0, beta=1.0)
    with pytest.raises(btoc.SpecError, match="not bound"):
        prog.run(A=A, x=x[:30], alpha=1.0, beta=1.0)
