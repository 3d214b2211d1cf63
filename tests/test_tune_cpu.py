"""The autotuner's search logic on the CPU, driven by a deterministic cost
table in place of device timings: the max-fuse start, the orthogonal search,
the genetic search's reproducibility and legality, the fitness cache and its
resumption, and the final band-height sweep."""

import json
import math

import pytest

from paper_1205_1098_amd import tune

SHAPES = range(11)
RBS = (8, 16, 32, 64, 128, 256)
SLOTS = range(10)


def fake_space():
    sp = tune.Space()
    for slot in SLOTS:
        if slot in (tune.SLOT_ATAX_ROWRES, tune.SLOT_BICGK_ROWRES):
            legal = [(t, 0, 0) for t in ((256, 512, 1024) if slot == tune.SLOT_ATAX_ROWRES
                                         else (0, 256, 512, 1024))]
        else:
            # an uneven legal set, like the library's: some (shape, rb) pairs missing
            legal = [(s, rb, rev) for s in SHAPES for rb in RBS for rev in (0, 1)
                     if not (s % 3 == 1 and rb < 32)]
        sp.legal[slot] = legal
        sp.defaults[slot] = legal[len(legal) // 2]
    return sp


# Each slot has one best configuration; the cost of an organism is the
# form's base cost plus, per slot, its distance from that slot's optimum.
OPT = {slot: (slot % 11, RBS[slot % len(RBS)], slot % 2) for slot in SLOTS}
OPT = {slot: (c[0], 64 if c[0] % 3 == 1 and c[1] < 32 else c[1], c[2]) for slot, c in OPT.items()}
OPT[tune.SLOT_ATAX_ROWRES] = (512, 0, 0)
OPT[tune.SLOT_BICGK_ROWRES] = (256, 0, 0)
BASE = {"fused": 1.0, "unfused": 1.9}


def slot_cost(slot, c):
    o = OPT[slot]
    if slot in (tune.SLOT_ATAX_ROWRES, tune.SLOT_BICGK_ROWRES):
        return 0.0 if c == o else 0.05 + abs(c[0] - o[0]) / 1e4
    return 0.02 * abs(c[0] - o[0]) + 0.01 * abs(math.log2(c[1] / o[1])) + 0.005 * (c[2] != o[2])


class Counter:
    def __init__(self, base=BASE):
        self.calls = 0
        self.base = base

    def __call__(self, kernel, m, n, org):
        self.calls += 1
        return self.base[org.form] + sum(slot_cost(s, c) for s, c in org.slots)


def legal_org(space, kernel, org):
    slots = [s for s, _ in org.slots]
    assert slots == sorted(tune.KERNEL_SLOTS[(kernel, org.form)])
    return all(c in space.legal[s] for s, c in org.slots)


def test_max_fuse_is_fused_with_defaults():
    sp = fake_space()
    t = tune.Tuner(sp, Counter())
    for kernel in ("bicgk", "gemver", "atax", "dgemvt"):
        org = t.max_fuse(kernel)
        assert org.form == "fused"
        assert org.cfg() == {s: sp.defaults[s] for s in tune.KERNEL_SLOTS[(kernel, "fused")]}


@pytest.mark.parametrize("kernel", ["bicgk", "gemver", "atax", "dgemvt"])
def test_orthogonal_finds_separable_optimum(kernel):
    sp = fake_space()
    t = tune.Tuner(sp, Counter())
    best = t.orthogonal(kernel, 1000, 1000)
    assert best.form == "fused"
    assert best.cfg() == {s: OPT[s] for s in tune.KERNEL_SLOTS[(kernel, "fused")]}
    # every legal configuration of every slot was visited once at most
    budget = 2 + sum(len(sp.legal[s]) for s in tune.KERNEL_SLOTS[(kernel, "fused")])
    assert t.evaluations <= budget


def test_orthogonal_both_forms_and_fusion_choice():
    sp = fake_space()
    t = tune.Tuner(sp, Counter({"fused": 2.5, "unfused": 1.0}))   # fusion loses here
    best = t.orthogonal("gemver", 64, 64, forms=["fused", "unfused"])
    assert set(t.form_best) == {"fused", "unfused"}
    assert best.form == "unfused"
    assert t.form_best["fused"].cfg() == {s: OPT[s] for s in
                                          tune.KERNEL_SLOTS[("gemver", "fused")]}
    t2 = tune.Tuner(sp, Counter({"fused": 2.5, "unfused": 1.0}))
    assert t2.orthogonal("gemver", 64, 64).form == "unfused"


def test_mfga_reproducible_and_legal():
    sp = fake_space()
    runs = []
    for _ in range(2):
        ev = Counter()
        t = tune.Tuner(sp, ev, seed=7)
        best = t.mfga("gemver", 512, 512, population=20, generations=6, k=2)
        runs.append((best, ev.calls, dict(t.cache)))
    assert runs[0][0] == runs[1][0] and runs[0][1] == runs[1][1] and runs[0][2] == runs[1][2]
    best = runs[0][0]
    assert legal_org(sp, "gemver", best)
    t = tune.Tuner(sp, Counter(), seed=7)
    mf = t.fitness("gemver", 512, 512, t.max_fuse("gemver"))
    assert t.fitness("gemver", 512, 512, best) <= mf


def test_mutation_and_crossover_stay_legal():
    sp = fake_space()
    t = tune.Tuner(sp, Counter(), seed=3)
    for kernel in ("bicgk", "gemver", "atax", "dgemvt"):
        t._kernel = kernel
        pop = [t.max_fuse(kernel)]
        for i in range(300):
            a, b = t.rng.choice(pop), t.rng.choice(pop)
            child = t.mutate(t.crossover(a, b)) if i % 2 else t.mutate(a)
            assert legal_org(sp, kernel, child), (kernel, child)
            pop.append(child)
        # the four mutation kinds reach both forms and change geometry
        assert {o.form for o in pop} == {"fused", "unfused"}
        assert len({o.slots for o in pop}) > 20


def test_fitness_cache_counts_once_and_resumes(tmp_path):
    sp = fake_space()
    path = str(tmp_path / "cache.json")
    ev = Counter()
    t = tune.Tuner(sp, ev, cache_path=path, seed=1)
    best = t.orthogonal("bicgk", 2048, 2048)
    first = ev.calls
    assert first == t.evaluations == len(t.cache)
    again = t.orthogonal("bicgk", 2048, 2048)        # all cached
    assert again == best and ev.calls == first
    t.save({"note": "x"})
    with open(path) as f:
        data = json.load(f)
    assert data["note"] == "x" and len(data["fitness"]) == first
    ev2 = Counter()
    t2 = tune.Tuner(sp, ev2, cache_path=path, seed=1)  # resume from disk
    assert t2.orthogonal("bicgk", 2048, 2048) == best
    assert ev2.calls == 0
    # another size is another key
    t2.fitness("bicgk", 4096, 4096, best)
    assert ev2.calls == 1


def test_sweep_rb_keeps_shape_and_improves():
    sp = fake_space()
    t = tune.Tuner(sp, Counter())
    slot = tune.SLOT_GEMVER_P1
    o = OPT[slot]
    start = t.organism("gemver", "fused", {slot: (o[0], 8 if (o[0], 8, o[2]) in sp.legal[slot]
                                                  else 32, o[2])})
    best = t.sweep_rb("gemver", 100, 100, start)
    assert best.cfg()[slot][0] == o[0]
    assert best.cfg()[slot][1] == o[1]
    assert t.fitness("gemver", 100, 100, best) <= t.fitness("gemver", 100, 100, start)


def test_apply_sets_every_slot():
    calls = []

    class FakeLib:
        @staticmethod
        def tune_set(slot, shape, rb, rev, size=0):
            calls.append((slot, shape, rb, rev, size))

    sp = fake_space()
    t = tune.Tuner(sp, Counter())
    org = t.orthogonal("gemver", 10, 10)
    tune.apply(FakeLib, org)
    assert calls == [(s, *c, 0) for s, c in org.slots]
    calls.clear()
    tune.apply(FakeLib, org, size=3000)          # only the bucket of 3000
    assert calls == [(s, *c, 3000) for s, c in org.slots]


def test_pruning_by_modeled_partial_bytes():
    """Configurations whose partial sums would outweigh a fraction of the
    matrix pass are not measured (unless nothing else is left)."""
    sp = fake_space()
    sp.ops = {s: 0 for s in SLOTS}
    sp.ops[tune.SLOT_GEMVER_P1] = 4 | 8 | 2        # column sums: partials per row band
    sp.ops[tune.SLOT_GEMVER_P2] = 1                # row dots: partials per wave tile
    sp.kv = {s: 1 + s % 4 for s in SHAPES}
    m = n = 1024
    p1 = sp.pruned(tune.SLOT_GEMVER_P1, m, n, 0.2)
    assert p1 and all(2 * 8 * n * -(-m // c[1]) <= 0.2 * 8 * m * n for c in p1)
    assert len(p1) < len(sp.legal[tune.SLOT_GEMVER_P1])   # rb = 8 (2 MiB of 8) is out
    assert all(c[1] >= 16 for c in p1)
    p2 = sp.pruned(tune.SLOT_GEMVER_P2, 8, 4096, 0.01)
    assert p2 == sp.legal[tune.SLOT_GEMVER_P2] or all(
        sp.partial_bytes(tune.SLOT_GEMVER_P2, c, 8, 4096) <= 0.01 * 8 * 8 * 4096 for c in p2)
    # a search over a pruned space only measures pruned configurations
    seen = []

    def ev(kernel, mm, nn, org):
        seen.append(org.cfg())
        return Counter()(kernel, mm, nn, org)

    t = tune.Tuner(sp, ev, prune=0.2)
    t.orthogonal("gemver", m, n, forms=["fused"])
    assert all(cfg[tune.SLOT_GEMVER_P1] in p1 or cfg[tune.SLOT_GEMVER_P1] ==
               sp.defaults[tune.SLOT_GEMVER_P1] for cfg in seen)


def test_bucket_fitness_sums_the_bucket_sizes():
    calls = []

    def single(kernel, m, n, org):
        calls.append(n)
        return n * 1e-6

    ev = tune.bucket_evaluator(single, {4096: [2400, 3200, 4096]})
    org = tune.Organism("fused", ())
    assert ev("gemver", 4096, 4096, org) == pytest.approx((2400 + 3200 + 4096) * 1e-6)
    assert calls == [2400, 3200, 4096]
    assert ev("gemver", 16384, 16384, org) == pytest.approx(16384e-6)   # ungrouped: itself


def test_batch_knobs_orthogonal_search():
    """The batch plan's knobs are searched one at a time from the library's
    defaults, fusion first; each configuration is measured once."""
    calls = []

    def ev(cfg):
        calls.append(cfg)
        t = 1.0 if cfg["form"] == "fused" else 2.0
        t += {256: 0.0, 512: 0.05}[cfg["threads"]]
        t += {1: 0.2, 2: 0.0, 3: 0.03, 4: 0.1}[cfg["wgs_per_cu"]]
        t += 0.0 if cfg["split_bytes"] == 8 << 20 else 0.02
        return t

    cache = {}
    best, sec, evals = tune.tune_batch(ev, cache=cache)
    defaults = {k: v[0] for k, v in tune.BATCH_SPACE.items()}
    assert best == {**defaults, "form": "fused", "threads": 256, "wgs_per_cu": 2,
                    "split_bytes": 8 << 20}
    assert all(c[k] == defaults[k] for c in calls for k in tune.TILED_KNOBS)
    assert sec == pytest.approx(1.0)
    keys = [json.dumps(c, sort_keys=True) for c in calls]
    assert len(keys) == len(set(keys)) == evals           # no configuration measured twice
    assert evals <= 1 + sum(len(v) - 1 for v in tune.BATCH_SPACE.values())
    again, _, _ = tune.tune_batch(lambda c: pytest.fail("should be cached"), cache=cache)
    assert again == best


def test_space_from_library_keeps_every_bucket():
    """Probing legality sets a slot for all buckets; the per-bucket
    configurations must be as before once the space is built."""

    class FakeBto:
        class BtoError(Exception):
            pass

        NB, NSLOTS, NSHAPES = 8, 10, 15

        def __init__(self):
            self.cfg = {(s, b): (s % 5 + b % 3, 32 << (b % 2), b % 2)
                        for s in range(self.NSLOTS) for b in range(self.NB)}

        def bucket(self, size):
            b = 0
            while b < self.NB - 1 and (256 << b) < size:
                b += 1
            return b

        def tune_shape(self, shape):
            if not 0 <= shape < self.NSHAPES:
                raise self.BtoError("shape out of range")
            return {"kv": 1 + shape % 4, "depth": 2, "wc": 1, "wr": 4}

        def tune_slots(self):
            return [f"slot{s}" for s in range(self.NSLOTS)]

        def tune_buckets(self):
            return self.NB

        def tune_slot_ops(self, slot):
            return slot

        def tune_get(self, slot, size=0):
            return self.cfg[(slot, self.bucket(16384 if size == 0 else size))]

        def tune_set(self, slot, shape, rb, rev=0, size=0):
            if rb not in (0, 32, 64) and slot < 8:
                raise self.BtoError("illegal")
            for b in (range(self.NB) if size == 0 else [self.bucket(size)]):
                self.cfg[(slot, b)] = (shape, rb, rev)

    lib = FakeBto()
    before = dict(lib.cfg)
    sp = tune.Space.from_library(lib)
    assert lib.cfg == before
    assert sorted(sp.kv) == list(range(FakeBto.NSHAPES))
    assert all(sp.legal[s] for s in range(FakeBto.NSLOTS))


def test_batch_knobs_tiled_form_skips_plan_knobs():
    """When the tiled form wins, the persistent plan's knobs (which it does
    not use) are not searched."""
    calls = []

    def ev(cfg):
        calls.append(cfg)
        return {"fused": 1.0, "unfused": 2.0, "tiled": 0.9}[cfg["form"]]

    best, sec, evals = tune.tune_batch(ev)
    assert best["form"] == "tiled" and sec == pytest.approx(0.9)
    assert all(c["threads"] == tune.BATCH_SPACE["threads"][0] and
               c["split_bytes"] == tune.BATCH_SPACE["split_bytes"][0] for c in calls)


def test_batch_knobs_search_the_winning_forms_knobs():
    """With the tiled form best, its partition knobs are searched one after
    another (and the plan's are not); a refused configuration (infinite
    time) is never chosen."""
    seen = []

    def ev(cfg):
        seen.append(cfg)
        if cfg["form"] != "tiled":
            return 2.0
        if cfg["t_store_rb"] == 128:
            return float("inf")            # e.g. refused by the library
        return 1.0 - 0.01 * (cfg["t_store_shape"] == 3) - 0.02 * (cfg["t_read_rb"] == 32)

    best, sec, evals = tune.tune_batch(ev)
    assert best["form"] == "tiled"
    assert best["t_store_shape"] == 3 and best["t_read_rb"] == 32 and best["t_store_rb"] != 128
    assert sec == pytest.approx(0.97)
    assert all(c["threads"] == tune.BATCH_SPACE["threads"][0] for c in seen)
    assert tune.tiled_config_of(best)["store_shape"] == 3
    assert set(tune.tiled_config_of(best)) == {k[2:] for k in tune.TILED_KNOBS}


def test_mfga_genes_finds_the_optimum_and_skips_failures():
    """The genome search over per-pass (shape, band height) genes: from the
    start genome it reaches the optimum of a separable cost, never keeps a
    genome scored infinite (refused or wrong), and measures each genome
    once."""
    choices = [[(s, rb) for s in range(4) for rb in (8, 16, 32, 64)] for _ in range(3)]
    target = ((2, 32), (1, 8), (3, 64))
    seen = []

    def cost(g):
        seen.append(g)
        if g[0] == (0, 64):
            return float("inf")
        return sum(abs(a[0] - b[0]) + abs(a[1] - b[1]) / 8 for a, b in zip(g, target)) + 1.0

    best, fit, evals = tune.mfga_genes(choices, cost, start=((0, 8),) * 3, population=20,
                                       generations=8, seed=5)
    assert best == target and fit == pytest.approx(1.0)
    assert len(seen) == len(set(seen)) == evals
    assert seen[0] == ((0, 8),) * 3
    again, _, _ = tune.mfga_genes(choices, cost, start=((0, 8),) * 3, population=20,
                                  generations=8, seed=5)
    assert again == best                                   # seeded: reproducible


def test_outputs_agree():
    torch = pytest.importorskip("torch")
    ref = [torch.tensor([1.0, -2.0, 4.0], dtype=torch.float64),
           torch.zeros(2, dtype=torch.float64)]
    assert tune.outputs_agree([r.clone() for r in ref], ref)
    near = [ref[0] * (1 + 1e-14), ref[1] + 1e-13]
    assert tune.outputs_agree(near, ref)
    assert not tune.outputs_agree([ref[0] * (1 + 1e-10), ref[1]], ref)
    assert not tune.outputs_agree([torch.tensor([1.0, float("nan"), 4.0], dtype=torch.float64),
                                   ref[1]], ref)


def test_cache_is_keyed_by_environment(tmp_path):
    """A fitness cache written under one device/ROCm/library key is reused
    under the same key and ignored under another."""
    sp = fake_space()
    path = str(tmp_path / "cache.json")
    t = tune.Tuner(sp, Counter(), cache_path=path, env_key="gfx950|rocm 7|abc")
    org = t.max_fuse("bicgk")
    t.fitness("bicgk", 64, 64, org)
    t.save()
    same = tune.Tuner(sp, Counter(), cache_path=path, env_key="gfx950|rocm 7|abc")
    assert same.cache
    other = tune.Tuner(sp, Counter(), cache_path=path, env_key="gfx950|rocm 7|def")
    assert not other.cache
    assert "|" in tune.environment_key(digest="x") and tune.library_digest(None)


def test_tiled_knobs_start_at_the_library_defaults():
    """The first value of each tiled knob is the library's default, so the
    search starts from the configuration the library runs without tuning."""
    from paper_1205_1098_amd import bto

    lib = bto.TiledConfig.default().as_dict()
    assert {k: tune.BATCH_SPACE[k][0] for k in tune.TILED_KNOBS} == \
        {k: lib[k[2:]] for k in tune.TILED_KNOBS}
