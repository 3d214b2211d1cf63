"""Batched execution on the GPU: every instance against the oracle, and the
result independent of the schedule (workgroup size, grid, graph replay)."""

import numpy as np
import pytest

import oracle
from paper_1205_1098_amd import batch, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto


def relerr(got, ref):
    ref = np.asarray(ref)
    if ref.size == 0:
        return 0.0
    den = float(np.max(np.abs(ref)))
    num = float(np.max(np.abs(np.asarray(got) - ref)))
    return num / den if den > 0 else num


def reference(spec, alpha, beta):
    A, ins = batch.host_operands(spec)
    if spec.kind == "gemver":
        B, x, w = oracle.gemver(A, *ins, alpha, beta)
        return [x, w], B
    if spec.kind == "bicgk":
        return list(oracle.bicgk(A, *ins)), None
    return [oracle.atax(A, *ins)], None


def check_all(torch, insts, specs, exact):
    for inst, spec in zip(insts, specs):
        outs, B = reference(spec, inst.get("alpha", 0.0), inst.get("beta", 0.0))
        got = [t.cpu().numpy() for t in inst["out"]]
        for g, r in zip(got, outs):
            if exact:
                assert np.array_equal(g, r), (spec.index, spec.kind, spec.n)
            else:
                assert relerr(g, r) <= TOL, (spec.index, spec.kind, spec.n)
        if B is not None:
            gb = inst["B"].cpu().numpy()
            assert np.array_equal(gb, B) if exact else relerr(gb, B) <= TOL


def test_device_fill_matches_host(env):
    torch, bto = env
    st = synth.stream_state(5, 77)
    v = torch.empty(100003, dtype=torch.float64, device="cuda")
    bto.synth_fill(v, st)
    assert np.array_equal(v.cpu().numpy(), synth.uniform(5, 77, 100003))
    full = torch.full((37, 48), float("nan"), dtype=torch.float64, device="cuda")
    bto.synth_fill(full[:, :41], st, kind="int")
    host = full.cpu().numpy()
    assert np.array_equal(host[:, :41], synth.matrix(5, 77, 37, 41, kind="int"))
    assert np.all(np.isnan(host[:, 41:]))
    part = torch.empty(1000, dtype=torch.float64, device="cuda")
    bto.synth_fill(part, st, offset=4096)
    assert np.array_equal(part.cpu().numpy(), synth.uniform(5, 77, 1000, offset=4096))


WEIGHTS = {"gemver": 0.4, "bicgk": 0.4, "atax": 0.2}


@pytest.mark.parametrize("form", ["fused", "unfused"])
@pytest.mark.parametrize("data", ["uniform", "int"])
def test_batch_matches_oracle(env, form, data):
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 120, 64, 2048, WEIGHTS, seed=11, form=form,
                                        data=data)
    plan = bto.BatchPlan(insts)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=(data == "int"))
    plan.close()


def test_batch_edge_sizes(env):
    torch, bto = env
    insts, specs = [], []
    for idx, n in enumerate([1, 2, 3, 63, 64, 65, 127, 129, 1023, 1025, 2047, 2048]):
        for kind in batch.KINDS:
            one, sp = batch.make_instances(torch, bto, 1, n, n, {kind: 1.0}, seed=100 + idx)
            insts += one
            specs += sp
    plan = bto.BatchPlan(insts, use_graph=False)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=False)


# around every change of thread geometry (pairs per thread, threads per row,
# rows spanning several waves), odd and even n, tall and one-row matrices
RECT = [(1, 2048), (3, 2047), (2, 129), (300, 130), (7, 257), (64, 258), (65, 259),
        (9, 513), (33, 515), (5, 1025), (17, 1026), (129, 1027), (5000, 3), (4097, 1),
        (1, 1), (2, 2), (3000, 64), (700, 2000)]


@pytest.mark.parametrize("form", ["fused", "unfused"])
@pytest.mark.parametrize("threads", [256, 512])
def test_batch_rectangular_geometries(env, form, threads):
    torch, bto = env
    insts, specs = [], []
    for k, kind in enumerate(batch.KINDS):
        i, sp = batch.make_instances(torch, bto, len(RECT), 1, 2, {kind: 1.0}, seed=15,
                                     config=20 + k, form=form, shapes=RECT)
        insts += i
        specs += sp
    plan = bto.BatchPlan(insts, threads=threads, use_graph=False)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=False)
    plan.close()


def test_schedule_independence_and_graph_replay(env):
    """For a given workgroup size the results are bit-identical whatever the
    grid, with or without the graph, and on every replay; a different
    workgroup size adds the waves' column sums in another fixed order, so it
    agrees to the tolerance (and both agree with the oracle)."""
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 200, 64, 2048, WEIGHTS, seed=12)
    outs = lambda: [t.clone() for inst in insts for t in inst["out"]]
    by_threads = {}
    for threads, wgs, graph in [(256, 0, True), (256, 1, False), (512, 1, False), (512, 0, True),
                                (256, 3, True)]:
        for inst in insts:
            for t in inst["out"]:
                t.fill_(float("nan"))
        plan = bto.BatchPlan(insts, threads=threads, wgs_per_cu=wgs, use_graph=graph)
        for rep in range(3):
            plan.launch()
            torch.cuda.synchronize()
            cur = outs()
            first = by_threads.setdefault(threads, cur)
            assert all(torch.equal(a, b) for a, b in zip(first, cur)), (threads, wgs, graph, rep)
        plan.close()
        check_all(torch, insts, specs, exact=False)
    for a, b in zip(by_threads[256], by_threads[512]):
        assert relerr(a.cpu().numpy(), b.cpu().numpy()) <= TOL


def test_in_place_gemver_batch(env):
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 40, 64, 1500, {"gemver": 1.0}, seed=13,
                                        in_place=True)
    plan = bto.BatchPlan(insts)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=False)


def test_batch_rejects_overlap(env):
    torch, bto = env
    insts, _ = batch.make_instances(torch, bto, 3, 64, 128, {"bicgk": 1.0}, seed=14)
    # two instances' outputs share an element: views of one buffer, each of
    # its instance's length
    n0, n1 = insts[0]["out"][0].numel(), insts[1]["out"][0].numel()
    buf = torch.empty(n0 + n1 - 1, dtype=torch.float64, device=insts[0]["A"].device)
    insts[0]["out"][0], insts[1]["out"][0] = buf[:n0], buf[n0 - 1:]
    with pytest.raises(bto.BtoError) as e:
        bto.BatchPlan(insts)
    assert e.value.status == 2
    insts[1]["out"][0] = torch.empty(n1 + 1, dtype=torch.float64, device=buf.device)
    with pytest.raises(ValueError, match="length"):
        bto.BatchPlan(insts)


def test_refilled_plan_matches_fresh_plans(env):
    """A plan made empty and refilled before each launch (its graph captured
    once) computes every set of instances exactly as a plan built for that
    set."""
    torch, bto = env
    sets = [batch.make_instances(torch, bto, c, 64, 2048, WEIGHTS, seed=20 + k, config=6 + k)
            for k, c in enumerate([50, 7, 64, 1])]
    sets.insert(2, ([], []))
    outs = lambda insts: [t.clone() for inst in insts for t in inst["out"]]

    def poison(insts):
        for inst in insts:
            for t in inst["out"]:
                t.fill_(float("nan"))

    scratch = max(bto.batch_scratch_doubles(insts) for insts, _ in sets)
    assert scratch > 0     # some instances are split into tiles
    for graph in (True, False):
        plan = bto.BatchPlan.empty(64, scratch, use_graph=graph)
        for insts, specs in sets:
            poison(insts)
            plan.reset(insts)
            plan.launch()
            torch.cuda.synchronize()
            got = outs(insts)
            if insts:
                check_all(torch, insts, specs, exact=False)
                poison(insts)
                fresh = bto.BatchPlan(insts, use_graph=graph)
                fresh.launch()
                torch.cuda.synchronize()
                assert all(torch.equal(a, b) for a, b in zip(got, outs(insts))), graph
                fresh.close()
        many, _ = batch.make_instances(torch, bto, 65, 64, 128, WEIGHTS, seed=30, config=12)
        with pytest.raises(bto.BtoError) as e:
            plan.reset(many)
        assert e.value.status == 1
        plan.close()
    # a plan without scratch refuses instances that need some
    small = bto.BatchPlan.empty(8, 0)
    for form, lo in (("unfused", 64), ("fused", 1500)):
        need, _ = batch.make_instances(torch, bto, 2, lo, lo + 10, {"atax": 1.0}, seed=31,
                                       config=13, form=form)
        assert bto.batch_scratch_doubles(need) > 0
        with pytest.raises(bto.BtoError) as e:
            small.reset(need)
        assert e.value.status == 3
    small.close()


@pytest.mark.parametrize("split", [-1, 0, 64 << 10])
def test_tiled_instances(env, split):
    """Fused instances cut into row tiles (default 2 MiB, or 64 KiB: the most
    tiles) or never cut: every result matches the oracle, is identical on
    replays and other grids, and no tile gave up waiting."""
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 150, 64, 2048, WEIGHTS, seed=16, config=17)
    tall, tspecs = batch.make_instances(torch, bto, 6, 1, 2, {"gemver": 1, "bicgk": 1,
                                                               "atax": 1}, seed=17, config=18,
                                        shapes=[(20000, 33), (9000, 2048), (3001, 1999),
                                                (20000, 1), (17, 2048), (16, 2047)])
    insts += tall
    specs += tspecs
    first = None
    for threads, wgs, graph in [(256, 0, True), (256, 1, False), (512, 0, True)]:
        plan = bto.BatchPlan(insts, threads=threads, wgs_per_cu=wgs, use_graph=graph,
                             split_bytes=split)
        for rep in range(2):
            for inst in insts:
                for t in inst["out"]:
                    t.fill_(float("nan"))
            plan.launch()
            plan.check()
            cur = [t.clone() for inst in insts for t in inst["out"]]
            if threads == 256:
                first = first or cur
                assert all(torch.equal(a, b) for a, b in zip(first, cur)), (threads, wgs, rep)
        check_all(torch, insts, specs, exact=False)
        plan.close()


# ---- tiled batches -----------------------------------------------------------------

TILED_WEIGHTS = {"gemver": 0.5, "bicgk": 0.5}


def _outputs(insts):
    return [t.clone() for inst in insts for t in inst["out"]] + \
        [inst["B"].clone() for inst in insts if "B" in inst]


def _poison(insts):
    for inst in insts:
        for t in inst["out"]:
            t.fill_(float("nan"))
        if "B" in inst and inst["B"].data_ptr() != inst["A"].data_ptr():
            inst["B"].fill_(float("nan"))


@pytest.mark.parametrize("data", ["uniform", "int"])
def test_tiled_batch_matches_oracle(env, data):
    """Random sizes and the shapes around every tile edge (32-row bands,
    128-column blocks, odd n, one row, one column)."""
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 120, 64, 2048, TILED_WEIGHTS, seed=31,
                                        data=data, config=30)
    shapes = [(1, 1), (1, 2048), (2, 2), (31, 127), (32, 128), (33, 129), (64, 255), (65, 257),
              (300, 130), (5000, 3), (4097, 1), (129, 2047), (2048, 2048), (3, 1025)]
    for k, kind in enumerate(TILED_WEIGHTS):
        i, sp = batch.make_instances(torch, bto, len(shapes), 1, 2, {kind: 1.0}, seed=32,
                                     config=31 + k, data=data, shapes=shapes)
        insts += i
        specs += sp
    _poison(insts)
    plan = bto.TiledBatch(insts)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=(data == "int"))
    plan.close()


def test_tiled_batch_in_place_and_empty(env):
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 30, 64, 1500, {"gemver": 1.0}, seed=33,
                                        in_place=True, config=33)
    plan = bto.TiledBatch(insts, use_graph=False)
    plan.launch()
    torch.cuda.synchronize()
    check_all(torch, insts, specs, exact=False)
    plan.close()
    # no rows or no columns: x = z and w = 0 for GEMVER, s = 0 for BiCGK
    dev = "cuda:0"
    z = torch.arange(5, dtype=torch.float64, device=dev) + 1.0
    empty_rows = {"kind": "gemver", "form": "fused", "A": torch.empty((0, 5), dtype=torch.float64,
                                                                        device=dev),
                  "B": torch.empty((0, 5), dtype=torch.float64, device=dev),
                  "in": [torch.empty(0, dtype=torch.float64, device=dev), torch.ones(5, dtype=torch.float64, device=dev),
                         torch.empty(0, dtype=torch.float64, device=dev), torch.ones(5, dtype=torch.float64, device=dev),
                         torch.empty(0, dtype=torch.float64, device=dev), z],
                  "out": [torch.full((5,), float("nan"), dtype=torch.float64, device=dev),
                          torch.empty(0, dtype=torch.float64, device=dev)], "alpha": 2.0, "beta": 3.0}
    no_cols = {"kind": "bicgk", "form": "fused",
               "A": torch.empty((4, 2), dtype=torch.float64, device=dev)[:, :0],
               "in": [torch.empty(0, dtype=torch.float64, device=dev), torch.ones(4, dtype=torch.float64, device=dev)],
               "out": [torch.full((4,), float("nan"), dtype=torch.float64, device=dev),
                       torch.empty(0, dtype=torch.float64, device=dev)]}
    plan = bto.TiledBatch([empty_rows, no_cols])
    plan.launch()
    torch.cuda.synchronize()
    assert torch.equal(empty_rows["out"][0], z)
    assert torch.equal(no_cols["out"][0], torch.zeros(4, dtype=torch.float64, device=dev))
    plan.close()
    for graph in (True, False):          # no instances at all: launches nothing
        plan = bto.TiledBatch([], use_graph=graph)
        plan.launch()
        torch.cuda.synchronize()
        plan.close()


def test_tiled_batch_replays_and_independent_of_the_mix(env):
    """Graph replays and direct launches give the same bits; an instance gives
    the same bits alone as among 200 others."""
    torch, bto = env
    insts, specs = batch.make_instances(torch, bto, 200, 64, 2048, TILED_WEIGHTS, seed=34,
                                        config=34)
    first = None
    for graph in (True, False):
        plan = bto.TiledBatch(insts, use_graph=graph)
        for rep in range(3):
            _poison(insts)
            plan.launch()
            torch.cuda.synchronize()
            cur = _outputs(insts)
            first = first or cur
            assert all(torch.equal(a, b) for a, b in zip(first, cur)), (graph, rep)
        plan.close()
    check_all(torch, insts, specs, exact=False)
    for k in (0, 7, 199):
        alone = [insts[k]]
        _poison(alone)
        plan = bto.TiledBatch(alone)
        plan.launch()
        torch.cuda.synchronize()
        mine = [t for t in insts[k]["out"]]
        lo = sum(len(insts[j]["out"]) for j in range(k))
        assert all(torch.equal(a, b) for a, b in zip(mine, first[lo:lo + len(mine)]))
        plan.close()


def test_tiled_batch_refuses_other_work(env):
    torch, bto = env
    at, _ = batch.make_instances(torch, bto, 2, 64, 128, {"atax": 1.0}, seed=35)
    with pytest.raises(bto.BtoError) as e:
        bto.TiledBatch(at)
    assert e.value.status == 5
    un, _ = batch.make_instances(torch, bto, 2, 64, 128, {"gemver": 1.0}, seed=35,
                                 form="unfused")
    with pytest.raises(bto.BtoError):
        bto.TiledBatch(un)
    ov, _ = batch.make_instances(torch, bto, 3, 64, 128, {"bicgk": 1.0}, seed=36)
    n0, n1 = ov[0]["out"][0].numel(), ov[1]["out"][0].numel()
    buf = torch.empty(n0 + n1 - 1, dtype=torch.float64, device=ov[0]["A"].device)
    ov[0]["out"][0], ov[1]["out"][0] = buf[:n0], buf[n0 - 1:]   # one shared element
    with pytest.raises(bto.BtoError) as e:
        bto.TiledBatch(ov)
    assert e.value.status == 2


# ---- tiled batch configurations and refillable plans ------------------------------

# every tile shape in each role at least once, band heights at the shapes'
# limits, one workgroup per tile and persistent workgroups, graph or not
TILED_CONFIGS = [
    dict(),
    dict(wgs_per_cu=1),
    dict(store_shape=1, narrow_shape=2, wide_shape=8, store_rb=64, bicgk_rb=256, read_rb=64,
         wgs_per_cu=2),
    dict(store_shape=2, narrow_shape=3, wide_shape=9, store_rb=8, bicgk_rb=512, read_rb=64,
         wgs_per_cu=3, use_graph=0),
    dict(store_shape=3, narrow_shape=4, wide_shape=6, store_rb=128, bicgk_rb=4, read_rb=8,
         narrow_n=0, wgs_per_cu=0, use_graph=0),
    dict(store_shape=4, narrow_shape=5, wide_shape=7, store_rb=8, bicgk_rb=100, read_rb=64,
         wgs_per_cu=16),
    dict(store_shape=5, narrow_shape=6, wide_shape=1, store_rb=36, bicgk_rb=64, read_rb=8,
         narrow_n=2048, wgs_per_cu=4),
    dict(store_shape=6, narrow_shape=7, wide_shape=0, store_rb=4, bicgk_rb=1, read_rb=16,
         narrow_n=1000),
    dict(store_shape=7, narrow_shape=8, wide_shape=2, store_rb=32, bicgk_rb=33, read_rb=32,
         wgs_per_cu=1),
    dict(store_shape=8, narrow_shape=9, wide_shape=3, store_rb=12, bicgk_rb=50, read_rb=12,
         wgs_per_cu=2),
    dict(store_shape=9, narrow_shape=1, wide_shape=5, store_rb=1, bicgk_rb=64, read_rb=40,
         wgs_per_cu=8),
    dict(store_shape=10, narrow_shape=10, wide_shape=11, store_rb=64, bicgk_rb=5, read_rb=48,
         wgs_per_cu=2),
    dict(store_shape=11, narrow_shape=11, wide_shape=10, store_rb=7, bicgk_rb=64, read_rb=5),
    dict(store_shape=0, store_rb=16, bicgk_rb=1024, wgs_per_cu=2),
]


def _tiled_set(torch, bto, data, seed, config):
    """Random sizes plus the shapes around every tile edge."""
    insts, specs = batch.make_instances(torch, bto, 40, 64, 2048, TILED_WEIGHTS, seed=seed,
                                        data=data, config=config)
    shapes = [(1, 1), (1, 2048), (2, 2), (31, 127), (33, 129), (65, 257), (300, 130),
              (4097, 1), (129, 2047), (2048, 2048), (3, 1025), (257, 513), (17, 512)]
    for k, kind in enumerate(TILED_WEIGHTS):
        i, sp = batch.make_instances(torch, bto, len(shapes), 1, 2, {kind: 1.0}, seed=seed + 1,
                                     config=config + 1 + k, data=data, shapes=shapes)
        insts += i
        specs += sp
    return insts, specs


@pytest.mark.parametrize("k", range(len(TILED_CONFIGS)))
def test_tiled_configs_match_oracle(env, k):
    """Each configuration against the oracle (1e-12, and bitwise on integer
    data); one workgroup per tile and persistent workgroups give the same
    bits for the same shapes and bands."""
    torch, bto = env
    ch = TILED_CONFIGS[k]
    for data in ("uniform", "int"):
        insts, specs = _tiled_set(torch, bto, data, 40 + k, 40 + 3 * k)
        _poison(insts)
        plan = bto.TiledBatch(insts, config=bto.TiledConfig.default(**ch))
        plan.launch()
        torch.cuda.synchronize()
        check_all(torch, insts, specs, exact=(data == "int"))
        first = _outputs(insts)
        plan.close()
        other = dict(ch, wgs_per_cu=0 if ch.get("wgs_per_cu", 0) else 2)
        _poison(insts)
        plan = bto.TiledBatch(insts, config=bto.TiledConfig.default(**other))
        plan.launch()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(first, _outputs(insts)))
        plan.close()


@pytest.mark.parametrize("graph,wgs", [(1, 2), (0, 2), (0, 0)])
def test_tiled_refills(env, graph, wgs):
    """A refillable plan run on three different sets in a row (the second
    smaller, the third empty, then the first again): every instance against
    the oracle, and bitwise equal to a plan built for that set with the same
    configuration.  In a graph the launches are fixed; without one they are
    sized from each refill (with one workgroup per tile, or persistent)."""
    torch, bto = env
    cfg = bto.TiledConfig.default(wgs_per_cu=wgs, use_graph=graph)
    a, sa = batch.make_instances(torch, bto, 70, 64, 2048, TILED_WEIGHTS, seed=60, config=60)
    b, sb = batch.make_instances(torch, bto, 9, 64, 700, TILED_WEIGHTS, seed=61, config=61)
    plan = bto.TiledBatch.empty(80, 2048, 2048, config=cfg)
    for insts, specs in ((a, sa), (b, sb), ([], []), (a, sa)):
        _poison(insts)
        plan.reset(insts)
        plan.launch()
        torch.cuda.synchronize()
        check_all(torch, insts, specs, exact=False)
        got = _outputs(insts)
        if insts:
            static = bto.TiledBatch(insts, config=cfg)
            _poison(insts)
            static.launch()
            torch.cuda.synchronize()
            assert all(torch.equal(x, y) for x, y in zip(got, _outputs(insts)))
            static.close()
    plan.close()


def test_tiled_refill_limits(env):
    torch, bto = env
    cfg = bto.TiledConfig.default(wgs_per_cu=2)
    insts, _ = batch.make_instances(torch, bto, 5, 64, 300, TILED_WEIGHTS, seed=62, config=62)
    plan = bto.TiledBatch.empty(4, 300, 300, config=cfg)
    with pytest.raises(bto.BtoError) as e:
        plan.reset(insts)                               # five instances, room for four
    assert e.value.status == 1
    # the tables are sized for four instances of 300 x 300 in all: two of
    # 1000 x 1000 need more tiles and scratch than that
    big, _ = batch.make_instances(torch, bto, 2, 1000, 1001, {"gemver": 1.0}, seed=63,
                                  config=63)
    with pytest.raises(bto.BtoError) as e:
        plan.reset(big)
    assert e.value.status == 3
    plan.reset(insts[:4])                               # the plan still works
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    static = bto.TiledBatch(insts[:2])
    with pytest.raises(bto.BtoError) as e:
        static.reset(insts[:1])                         # not refillable
    assert e.value.status == 1
    static.close()
    with pytest.raises(bto.BtoError) as e:
        bto.TiledBatch.empty(4, 300, 300, config=bto.TiledConfig.default(wgs_per_cu=0))
    assert e.value.status == 1
