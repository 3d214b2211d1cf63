"""The code generator on the CPU: schedules for generated passes, the
emitted source, and each generated library's C interface (exports, pass
layouts, shapes, workspace sizes, and the argument checks that refuse
before anything is enqueued).  No kernel is launched here."""

import ctypes
import os
import re

import pytest

from paper_1205_1098_amd import bto_specs, btoc, btoc_gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "btog.h")

SCHEDULES = {
    "gemver3": ["pass 0: A STORE|COLSUM|RANK3", "pass 1: B ROWDOT"],
    "gemver3c": ["pass 0: A CONTRACT|COLSUM|RANK3", "pass 1: A CONTRACT|ROWDOT|RANK3"],
    "bicgk2": ["pass 0: A ROWDOTx2|COLSUMx2"],
    "bicgk2c": ["pass 0: A ROWDOTx2|COLSUMx2"],
    "multimv": ["pass 0: A ROWDOTx3"],
    "multimv5": ["pass 0: A ROWDOTx5|COLSUM"],
}
LAYOUTS = {   # per pass: update terms, stored, row dots, column sums
    "gemver3": [(3, 1, 0, 1), (0, 0, 1, 0)],
    "gemver3c": [(3, 0, 0, 1), (3, 0, 1, 0)],
    "bicgk2": [(0, 0, 2, 2)],
    "bicgk2c": [(0, 0, 2, 2)],
    "multimv": [(0, 0, 3, 0)],
    "multimv5": [(0, 0, 5, 1)],
}


def gen(name):
    return btoc.compile_spec(bto_specs.GENERATED[name], target="generated")


@pytest.mark.parametrize("name", sorted(SCHEDULES))
def test_schedules(name):
    prog = gen(name)
    assert prog.describe() == SCHEDULES[name]
    assert [btoc_gen.layout(p) for p in btoc_gen.gen_passes(prog)] == LAYOUTS[name]


def test_library_target_splits_or_refuses():
    """The same programs for the library's passes: one row dot and one
    column sum per sweep (more sweeps), and no update above rank two."""
    assert btoc.compile_spec(bto_specs.GENERATED["bicgk2"]).describe() == [
        "pass 0: A ROWDOT|COLSUM", "pass 0: A ROWDOT|COLSUM"]
    assert len(btoc.compile_spec(bto_specs.GENERATED["multimv"]).passes()) == 3
    with pytest.raises(btoc.SpecError, match="needs generated"):
        btoc.compile_spec(bto_specs.GENERATED["gemver3"])
    with pytest.raises(btoc.SpecError):
        btoc.compile_spec(bto_specs.GENERATED["gemver3"], "unfused", target="generated")
    # the unfused form applies one rank-1 term per sweep, in place after the first
    unf = btoc.compile_spec(bto_specs.GENERATED["gemver3"], "unfused")
    assert [p.store for p in unf.passes()][:3] == ["B", "B", "B"]


def test_emitted_source_writes_out_the_statements():
    src = btoc_gen.emit(gen("gemver3"))
    assert src == btoc_gen.emit(gen("gemver3"))                   # deterministic
    # the rank-3 update, term by term and left to right, stored once
    body = src[src.index("// ---- pass 0"):src.index("// ---- pass 1")]
    assert [int(x) for x in re.findall(r"b\[k\] = b\[k\] \+ su(\d) \* v\1\[k\];", body)] == \
        [0, 1, 2]
    assert body.count("store_pair<VEC, FULL>(brow") == 1
    assert "acc[0][k] += b[k] * sy0;" in body
    # pass 1 reads B and forms no update; x = beta B' y + z: scale beta, add z
    p1 = src[src.index("// ---- pass 1"):]
    assert "su0" not in p1 and "mine[0] = s;" in p1
    assert "1.0 * sc[1]" in body        # beta is the second scalar input
    # every pass is compiled for every tile shape
    for k in range(2):
        for s in range(len(btoc_gen.SHAPES)):
            assert f"case {s}: p{k}_launch<" in src
    # contracted: the update is formed in registers and never stored
    c = btoc_gen.emit(gen("gemver3c"))
    assert "store_pair<VEC, FULL>(brow" not in c
    assert c.count("b[k] = b[k] + su2 * v2[k];") == 2


@pytest.fixture(scope="module")
def libs():
    out = {}
    for name in sorted(SCHEDULES):
        prog = gen(name)
        btoc_gen.build(prog, force=False)
        out[name] = (prog, btoc_gen.load(prog))
    return out


def declared():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(btog_[a-z0-9_]+)\s*\(", text)))


def test_exports_and_tables(libs):
    names = declared()
    assert set(names) == set(btoc_gen.EXPORTS)
    for name, (prog, lib) in libs.items():
        for f in names:
            assert hasattr(lib.lib, f), f"{name}: {f} not exported"
        assert lib.lib.btog_program().decode() == prog.name
        assert lib.lib.btog_pass_count() == len(LAYOUTS[name])
        assert [lib.layout(k) for k in range(len(LAYOUTS[name]))] == LAYOUTS[name]
        assert lib.lib.btog_shape_count() == len(btoc_gen.SHAPES)
        for s, shape in enumerate(btoc_gen.SHAPES):
            v = [ctypes.c_int() for _ in range(4)]
            assert lib.lib.btog_shape(s, *[ctypes.byref(x) for x in v]) == 0
            assert tuple(x.value for x in v) == shape
        assert lib.lib.btog_shape(len(btoc_gen.SHAPES), None, None, None, None) == 1


def test_configs_and_workspace(libs):
    """config_ok agrees with the genomes the search draws from, and the
    workspace is the partial sums: row dots per wave tile and row, column
    sums per band and column, each rounded to 256 bytes."""
    r256 = lambda b: (b + 255) // 256 * 256
    for name, (prog, lib) in libs.items():
        choices = btoc_gen.genome_choices(prog)
        for k, p in enumerate(btoc_gen.gen_passes(prog)):
            allowed = set(choices[k])
            for s in range(len(btoc_gen.SHAPES)):
                for rb in btoc_gen.RB_CHOICES:
                    assert lib.config_ok(k, s, rb) == ((s, rb) in allowed), (name, k, s, rb)
            _, _, P, Q = btoc_gen.layout(p)
            for m, n in ((1, 1), (300, 517), (16384, 16384)):
                for s, rb in choices[k][:: max(1, len(choices[k]) // 7)]:
                    kv, _, wc, wr = btoc_gen.SHAPES[s]
                    ncols = -(-n // (128 * kv))
                    nb = -(-m // rb)
                    want = P * r256(ncols * m * 8) + Q * r256(nb * n * 8)
                    assert lib.workspace_bytes(k, m, n, s, rb) == want
            assert lib.workspace_bytes(k, -1, 5, 0, 32) == 0
            assert lib.workspace_bytes(k, 5, 5, 0, 3) == 0
        assert all(lib.config_ok(k, *g) for k, g in enumerate(btoc_gen.default_genome(prog)))


def test_run_pass_refuses_before_launching(libs):
    prog, lib = libs["multimv"]
    run = lib.lib.btog_run_pass
    a = btoc_gen.PassArgs()
    fake = 1 << 40
    a.m = a.n = a.lda = a.ldb = 64
    a.A = fake
    for q in range(3):
        a.x[q], a.row_out[q] = fake + (q + 1) * (1 << 20), fake + (q + 9) * (1 << 20)
    sc = (ctypes.c_double * 2)(1.5, 0.7)
    a.scalars, a.nscalars = sc, 2
    ws = ctypes.c_void_p(fake + (64 << 20))
    need = lib.workspace_bytes(0, 64, 64, 4, 4)
    assert run(1, ctypes.byref(a), 4, 4, ws, need, None) == 1            # no such pass
    assert run(0, None, 4, 4, ws, need, None) == 1                       # no arguments
    assert run(0, ctypes.byref(a), 4, 65, ws, need, None) == 1           # bad band height
    assert run(0, ctypes.byref(a), 4, 4, ws, need - 1, None) == 3        # workspace too small
    a.nscalars = 1
    assert run(0, ctypes.byref(a), 4, 4, ws, need, None) == 1            # too few scalars
    assert "scalars" in lib.lib.btog_last_error().decode()
    a.nscalars = 2
    a.x[2] = None
    assert run(0, ctypes.byref(a), 4, 4, ws, need, None) == 1            # NULL operand
    a.x[2] = fake
    a.lda = 63
    assert run(0, ctypes.byref(a), 4, 4, ws, need, None) == 1            # lda below n
    a.lda, a.m = 64, (65535 * 4) + 4
    big = lib.workspace_bytes(0, a.m, 64, 4, 4)
    assert run(0, ctypes.byref(a), 4, 4, ws, big, None) == 5             # too many bands
