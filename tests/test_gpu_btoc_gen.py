"""Generated passes on the GPU: every program of bto_specs.GENERATED, run
through its emitted library, against the reference evaluation of the same
specification (oracle/spec_eval.py) on ragged shapes, with integer-valued
data bitwise; every tile shape each pass is compiled for, at its smallest
and a tall band height; the in-place update; and a program compiled for the
library's passes agreeing with its generated form."""

import numpy as np
import pytest

from oracle import spec_eval
from paper_1205_1098_amd import bto_specs, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
SEED = synth.SEED

G3_IN = dict(A="A", u1="m", v1="n", u2="m", v2="n", u3="m", v3="n", y="m", z="n",
             alpha=1.5, beta=0.7)
BICGK2_IN = dict(A="A", p1="n", p2="n", r1="m", r2="m")
PROGRAMS = {
    "gemver3": G3_IN,
    "gemver3c": G3_IN,
    "bicgk2": BICGK2_IN,
    "bicgk2c": BICGK2_IN,
    "multimv": dict(A="A", x1="n", x2="n", x3="n", y="m", alpha=1.5, beta=0.7),
    "multimv5": dict(A="A", x1="n", x2="n", x3="n", x4="n", x5="n", r="m", alpha=1.5),
}
SHAPES = [(1, 1), (2, 3), (65, 127), (300, 517), (513, 1000), (1000, 2049), (2048, 2048)]


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import btoc, btoc_gen

    return torch, btoc, btoc_gen, torch.device("cuda:0")


def _inputs(kinds, m, n, kind, case):
    host = {}
    for k, (name, what) in enumerate(sorted(kinds.items())):
        stream = synth.stream_id(12, k, case)
        if what == "A":
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


def _device(torch, dev, host, colmajor):
    out = {}
    for k, v in host.items():
        if isinstance(v, float):
            out[k] = v
        elif v.ndim == 2 and k in colmajor:
            # stored by columns: an (m, n) view of an (n, m) row-major array
            out[k] = torch.from_numpy(np.ascontiguousarray(v.T)).to(dev).t()
        else:
            out[k] = torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    return out


def _check(torch, prog, got, host, text, exact, what):
    ref = spec_eval.evaluate(text, host)
    for name in prog.outputs:
        g = got[name].cpu().numpy()
        r = np.asarray(ref[name])
        if exact:
            assert np.array_equal(g, r), f"{what}: {name} differs"
        else:
            e = _relerr(g, r)
            assert e <= TOL, f"{what}: {name} relerr {e:.3e}"


@pytest.mark.parametrize("name", sorted(PROGRAMS))
@pytest.mark.parametrize("data", ["uniform", "int"])
def test_generated_matches_spec(env, name, data):
    torch, btoc, gen, dev = env
    text = bto_specs.GENERATED[name]
    prog = btoc.compile_spec(text, target="generated")
    for case, (m, n) in enumerate(SHAPES):
        host = _inputs(PROGRAMS[name], m, n, data, case)
        bound = _device(torch, dev, host, prog.colmajor)
        print(f"{name} {data} {m}x{n}", flush=True)
        got = gen.run(prog, bound)
        torch.cuda.synchronize()
        _check(torch, prog, got, host, text, data == "int", f"{name} {m}x{n}")


@pytest.mark.parametrize("name", sorted(PROGRAMS))
def test_every_shape_and_band(env, name):
    """Each pass under every tile shape it is compiled for, at the smallest
    band height the shape takes and at a tall one (integer data: bitwise)."""
    torch, btoc, gen, dev = env
    text = bto_specs.GENERATED[name]
    prog = btoc.compile_spec(text, target="generated")
    choices = gen.genome_choices(prog)
    m, n = 300, 517
    host = _inputs(PROGRAMS[name], m, n, "int", 99)
    bound = _device(torch, dev, host, prog.colmajor)
    for s in range(len(gen.SHAPES)):
        for pick in (min, max):
            genome = []
            for opts in choices:
                rbs = [rb for sh, rb in opts if sh == s]
                genome.append((s, pick(rbs)))
            got = gen.run(prog, bound, genome=genome)
            torch.cuda.synchronize()
            _check(torch, prog, got, host, text, True, f"{name} genome {genome}")


@pytest.mark.parametrize("name", sorted(PROGRAMS))
def test_empty_extents(env, name):
    """No rows or no columns: no sweep runs, and every output is its
    statement over empty sums (the added vectors, scaled)."""
    torch, btoc, gen, dev = env
    text = bto_specs.GENERATED[name]
    prog = btoc.compile_spec(text, target="generated")
    for case, (m, n) in enumerate(((0, 7), (5, 0), (0, 0))):
        host = _inputs(PROGRAMS[name], m, n, "uniform", 40 + case)
        bound = _device(torch, dev, host, prog.colmajor)
        print(f"{name} empty {m}x{n}", flush=True)
        got = gen.run(prog, bound)
        torch.cuda.synchronize()
        _check(torch, prog, got, host, text, False, f"{name} {m}x{n}")


def test_in_place_update(env):
    """GEMVER3 with B bound to A itself (ldb == lda): the rank-3 update in
    place."""
    torch, btoc, gen, dev = env
    text = bto_specs.GENERATED["gemver3"]
    prog = btoc.compile_spec(text, target="generated")
    m, n = 513, 700
    host = _inputs(G3_IN, m, n, "uniform", 7)
    bound = _device(torch, dev, host, prog.colmajor)
    bound["B"] = bound["A"]
    got = gen.run(prog, bound)
    torch.cuda.synchronize()
    assert got["B"].data_ptr() == bound["A"].data_ptr()
    _check(torch, prog, got, host, text, False, "in place")


def test_generated_agrees_with_library_passes(env):
    """BICGK2 and MULTIMV compiled for the library's passes (two and three
    sweeps) and for generated ones (one sweep): the same results on integer
    data, bitwise."""
    torch, btoc, gen, dev = env
    for name in ("bicgk2", "multimv"):
        text = bto_specs.GENERATED[name]
        lib_prog = btoc.compile_spec(text)
        gen_prog = btoc.compile_spec(text, target="generated")
        assert len(lib_prog.passes()) > len(gen_prog.passes()) == 1
        host = _inputs(PROGRAMS[name], 1000, 1500, "int", 3)
        bound = _device(torch, dev, host, gen_prog.colmajor)
        a = lib_prog.run(**bound)
        b = gen.run(gen_prog, bound)
        torch.cuda.synchronize()
        for o in gen_prog.outputs:
            assert torch.equal(a[o], b[o]), (name, o)


def test_refusals(env):
    """Errors from the generated library's own checks, before any launch."""
    torch, btoc, gen, dev = env
    prog = btoc.compile_spec(bto_specs.GENERATED["bicgk2"], target="generated")
    lib = gen.load(prog)
    assert not lib.config_ok(0, 0, 8)          # 16 waves down need bands of 16 rows or more
    assert not lib.config_ok(0, 4, 65)         # one row group: at most 64 rows per wave
    assert not lib.config_ok(1, 0, 32)         # no such pass
    host = _inputs(BICGK2_IN, 64, 64, "uniform", 1)
    bound = _device(torch, dev, host, prog.colmajor)
    from paper_1205_1098_amd import bto
    with pytest.raises(bto.BtoError):
        gen.run(prog, bound, genome=[(0, 8)])
    with pytest.raises(btoc.SpecError):
        gen.run(prog, bound, genome=[(0, 32), (0, 32)])
