"""Autotuner for the fused kernels: the GPU counterpart of the paper's search.

The paper (Section IV) searches loop fusion, the partitioned axis and the
thread count of each loop nest with MFGA: start from the Max-Fuse organism,
build a population by mutation, evolve it by tournament selection (k = 2)
and crossover, cache every fitness, then sweep the global thread count.  It
also shows (Section V-D1) that searching fusion first and the thread count
second, the orthogonal search, finds the same best versions at a fraction of
the cost.

Here an organism is
  form   -- "fused" (the max-fuse point: every statement sharing a matrix pass
            runs in one sweep) or "unfused" (one sweep per BLAS operation);
  slots  -- for each matrix sweep the chosen form launches, its tile
            configuration (shape, rb, rev): the tile shape fixes the lane
            width, rows in flight and the waves across / down a workgroup
            (the partition axis and per-partition parallelism), rb the rows
            per workgroup band (how many partitions: the thread-count knob),
            rev the order the bands are walked.
The four mutation kinds of the paper map to: toggle fusion, change rb
(partition level), change the shape (partition axis), change rev or the
shape's depth (the remaining per-partition parallelism).  Fitness is the
measured time of one call on the device; every result is cached under its
key and the cache persists as JSON, so a later search resumes from it.

The evaluation function is pluggable: on the GPU it sets the configuration
through the library and times the kernel with events; tests drive the same
search with a deterministic cost table on the CPU.
"""

from __future__ import annotations

import json
import os
import random
from dataclasses import dataclass, field

# Slots of the C library (order of bto_tune_slot_name).
SLOT_BICGK_FUSED, SLOT_GEMV_N, SLOT_GEMV_T, SLOT_GER = 0, 1, 2, 3
SLOT_GEMVER_P1, SLOT_GEMVER_P2, SLOT_DGEMVT_P1, SLOT_DGEMVT_P2 = 4, 5, 6, 7
SLOT_ATAX_ROWRES = 8   # its "shape" is the workgroup size of the row-resident sweep
SLOT_BICGK_ROWRES = 9  # likewise for BiCGK; shape 0 selects the tile sweep instead

#: the matrix sweeps each kernel launches in each form
KERNEL_SLOTS = {
    ("bicgk", "fused"): [SLOT_BICGK_ROWRES, SLOT_BICGK_FUSED],
    ("bicgk", "unfused"): [SLOT_GEMV_N, SLOT_GEMV_T],
    ("gemver", "fused"): [SLOT_GEMVER_P1, SLOT_GEMVER_P2],
    ("gemver", "unfused"): [SLOT_GER, SLOT_GEMV_T, SLOT_GEMV_N],
    ("dgemvt", "fused"): [SLOT_DGEMVT_P1, SLOT_DGEMVT_P2],
    ("dgemvt", "unfused"): [SLOT_GEMV_T, SLOT_GEMV_N],
    ("atax", "fused"): [SLOT_ATAX_ROWRES],
    ("atax", "unfused"): [SLOT_GEMV_N, SLOT_GEMV_T],
}

RB_CHOICES = (4, 8, 16, 32, 64, 128, 256, 512)
FORMS = ("fused", "unfused")


@dataclass(frozen=True)
class Organism:
    form: str
    slots: tuple  # ((slot, (shape, rb, rev)), ...) sorted by slot

    def cfg(self) -> dict:
        return dict(self.slots)

    def key(self, kernel: str, m: int, n: int) -> str:
        parts = [f"{kernel}:{m}x{n}:{self.form}"]
        parts += [f"{s}={c[0]}/{c[1]}/{c[2]}" for s, c in self.slots]
        return "|".join(parts)


@dataclass
class Space:
    """The legal tile configurations of every slot (queried from the library,
    which rejects what a slot cannot run), with what the byte model needs."""

    legal: dict = field(default_factory=dict)   # slot -> list[(shape, rb, rev)]
    defaults: dict = field(default_factory=dict)  # slot -> (shape, rb, rev)
    ops: dict = field(default_factory=dict)     # slot -> OP_* bits (0: not a tile sweep)
    kv: dict = field(default_factory=dict)      # shape -> 16-byte pairs per lane

    def partial_bytes(self, slot: int, cfg: tuple, m: int, n: int) -> int:
        """Modeled partial-sum traffic of one sweep (written, then read by the
        finish): row-dot partials per wave tile of 128*kv columns, column-sum
        partials per band of rb rows."""
        ops = self.ops.get(slot, 0)
        shape, rb, _ = cfg
        total = 0
        if ops & 1 and shape in self.kv:
            total += 2 * 8 * m * -(-n // (128 * self.kv[shape]))
        if ops & 2 and rb > 0:
            total += 2 * 8 * n * -(-m // rb)
        return total

    def pruned(self, slot: int, m: int, n: int, ratio: float) -> list:
        """The legal configurations whose partials stay within `ratio` of one
        matrix pass (the coarse analytic pruning the paper applies before
        measuring); all of them if none would."""
        keep = [c for c in self.legal[slot] if self.partial_bytes(slot, c, m, n) <= ratio * 8 * m * n]
        return keep or list(self.legal[slot])

    @classmethod
    def from_library(cls, bto) -> "Space":
        sp = cls()
        nshapes = 0
        while True:                      # the compiled shapes: 0, 1, ... until refused
            try:
                sp.kv[nshapes] = bto.tune_shape(nshapes)["kv"]
            except bto.BtoError:
                break
            nshapes += 1
        nb = bto.tune_buckets()
        for slot in range(len(bto.tune_slots())):
            default = bto.tune_get(slot)
            # legality is probed by setting every bucket; each bucket's own
            # configuration is put back afterwards
            saved = [bto.tune_get(slot, 256 << b) for b in range(nb)]
            sp.defaults[slot] = default
            sp.ops[slot] = bto.tune_slot_ops(slot)
            legal = []
            shapes, rbs = range(nshapes), RB_CHOICES
            if slot == SLOT_ATAX_ROWRES:
                shapes, rbs = (256, 512, 1024), (0,)
            elif slot == SLOT_BICGK_ROWRES:
                shapes, rbs = (0, 256, 512, 1024), (0,)
            for shape in shapes:
                for rb in rbs:
                    for rev in (0, 1):
                        try:
                            bto.tune_set(slot, shape, rb, rev)
                            legal.append((shape, rb, rev))
                        except bto.BtoError:
                            pass
            for b, cfg in enumerate(saved):
                bto.tune_set(slot, *cfg, size=256 << b)
            sp.legal[slot] = legal
        return sp


class Tuner:
    """Search driver.  `evaluate(kernel, m, n, organism) -> seconds` does
    the measurement; results are cached by organism key."""

    def __init__(self, space: Space, evaluate, cache_path: str | None = None, seed: int = 0,
                 prune: float = 0.25, env_key: str = ""):
        self.space = space
        self.prune = prune
        self._kernel, self._m, self._n = None, 1024, 1024   # the GA's current problem
        self.evaluate = evaluate
        self.cache_path = cache_path
        self.cache: dict = {}
        self.rng = random.Random(seed)
        self.evaluations = 0
        # a cache measured on another device, ROCm or build of the library
        # is not reused: its fitness values describe other code
        self.env_key = env_key
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                data = json.load(f)
            if data.get("environment", "") == env_key:
                self.cache = data.get("fitness", {})

    # ---- bookkeeping -------------------------------------------------------
    def fitness(self, kernel: str, m: int, n: int, org: Organism) -> float:
        key = org.key(kernel, m, n)
        if key not in self.cache:
            self.cache[key] = float(self.evaluate(kernel, m, n, org))
            self.evaluations += 1
        return self.cache[key]

    def save(self, extra: dict | None = None) -> None:
        if not self.cache_path:
            return
        data = {"fitness": self.cache, "environment": self.env_key}
        if extra:
            data.update(extra)
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def organism(self, kernel: str, form: str, cfg: dict | None = None) -> Organism:
        slots = KERNEL_SLOTS[(kernel, form)]
        cfg = cfg or {}
        return Organism(form, tuple(sorted((s, tuple(cfg.get(s, self.space.defaults[s])))
                                           for s in slots)))

    # ---- max fuse ----------------------------------------------------------
    def max_fuse(self, kernel: str) -> Organism:
        """Every statement that shares a matrix pass fused, default geometry."""
        return self.organism(kernel, "fused")

    # ---- orthogonal search (fusion first, then geometry) ---------------------
    def orthogonal(self, kernel: str, m: int, n: int, forms=None) -> Organism:
        """Fusion first (the better form at default geometry), then each of
        its slots in turn over every legal configuration.  With `forms`
        given, the geometry of each listed form is searched and the best
        organism over them is returned (per-form bests in self.form_best)."""
        if forms is None:
            forms = [min(FORMS, key=lambda f: self.fitness(kernel, m, n,
                                                           self.organism(kernel, f)))]
        self.form_best = {}
        for form in forms:
            best = self.organism(kernel, form)
            cfg = best.cfg()
            for slot in KERNEL_SLOTS[(kernel, form)]:
                for c in self.space.pruned(slot, m, n, self.prune):
                    trial = self.organism(kernel, form, {**cfg, slot: c})
                    if self.fitness(kernel, m, n, trial) < self.fitness(kernel, m, n, best):
                        best, cfg = trial, trial.cfg()
            self.form_best[form] = best
        return min(self.form_best.values(), key=lambda o: self.fitness(kernel, m, n, o))

    # ---- genetic search -------------------------------------------------------
    def mutate(self, org: Organism) -> Organism:
        kind = self.rng.randrange(4)
        if kind == 0:                                  # add or remove fusion
            form = "unfused" if org.form == "fused" else "fused"
            return self.organism_like(org, form)
        slots = KERNEL_SLOTS[(self._kernel, org.form)]
        if not slots:
            return self.organism_like(org, "unfused" if org.form == "fused" else "fused")
        slot = self.rng.choice(slots)
        shape, rb, rev = org.cfg()[slot]
        legal = self.space.pruned(slot, self._m, self._n, self.prune)
        if kind == 1:                                  # change the partition level (rb)
            pool = [c for c in legal if c[0] == shape and c[2] == rev and c[1] != rb]
        elif kind == 2:                                # change the partition axis (shape)
            pool = [c for c in legal if c[0] != shape and c[1] == rb and c[2] == rev]
        else:                                          # change the walk order
            pool = [c for c in legal if c[0] == shape and c[1] == rb and c[2] != rev]
        if not pool:
            pool = [c for c in legal if c != (shape, rb, rev)] or [(shape, rb, rev)]
        cfg = org.cfg()
        cfg[slot] = self.rng.choice(pool)
        return Organism(org.form, tuple(sorted(cfg.items())))

    def organism_like(self, org: Organism, form: str) -> Organism:
        """An organism of `form` keeping the configurations of slots both share."""
        return self.organism(self._kernel, form, org.cfg())

    def crossover(self, a: Organism, b: Organism) -> Organism:
        """Outermost level first: pick the form from one parent, then each
        slot's configuration from either parent that has that slot."""
        form_parent = a if self.rng.random() < 0.5 else b
        cfg = {}
        for slot in KERNEL_SLOTS[(self._kernel, form_parent.form)]:
            choices = [p.cfg()[slot] for p in (a, b) if slot in p.cfg()]
            cfg[slot] = self.rng.choice(choices)
        return self.organism(self._kernel, form_parent.form, cfg)

    def tournament(self, pop: list, fit, k: int = 2) -> Organism:
        contenders = [self.rng.choice(pop) for _ in range(k)]
        return min(contenders, key=fit)

    def mfga(self, kernel: str, m: int, n: int, population: int = 20, generations: int = 6,
             k: int = 2, mutation_rate: float = 0.3) -> Organism:
        self._kernel, self._m, self._n = kernel, m, n
        fit = lambda o: self.fitness(kernel, m, n, o)
        mf = self.max_fuse(kernel)
        pop = [mf] + [self.mutate(mf) for _ in range(population - 1)]
        best = min(pop, key=fit)
        for _ in range(generations):
            parents = [self.tournament(pop, fit, k) for _ in range(2 * population)]
            children = []
            for i in range(population):
                child = self.crossover(parents[2 * i], parents[2 * i + 1])
                if self.rng.random() < mutation_rate:
                    child = self.mutate(child)
                children.append(child)
            pop = children
            best = min([best] + pop, key=fit)
        return self.sweep_rb(kernel, m, n, best)

    def sweep_rb(self, kernel: str, m: int, n: int, org: Organism) -> Organism:
        """The paper's final global thread-count sweep: for the best organism,
        try every legal band height on every slot with its shape fixed."""
        best = org
        for slot in KERNEL_SLOTS[(kernel, org.form)]:
            shape, _, rev = best.cfg()[slot]
            for c in self.space.pruned(slot, m, n, self.prune):
                if c[0] == shape and c[2] == rev:
                    trial = Organism(best.form, tuple(sorted({**best.cfg(), slot: c}.items())))
                    if self.fitness(kernel, m, n, trial) < self.fitness(kernel, m, n, best):
                        best = trial
        return best


# ---- genomes of generated programs ----------------------------------------------------

def mfga_genes(choices: list, fitness, start=None, population: int = 20, generations: int = 6,
               k: int = 2, mutation_rate: float = 0.3, seed: int = 0) -> tuple:
    """The MFGA of Section IV over a genome of independent genes, gene i
    taking values in choices[i] (for generated programs: one (tile shape,
    band height) per pass).  Starts from `start` (the max-fuse organism's
    default geometry), seeds the population with its mutations, evolves it
    by tournaments of k and per-gene crossover (the best so far kept), then
    refines the winner one gene at a time over all its values.
    `fitness(genome) -> seconds` (infinity for a genome that cannot run or
    gives wrong results); each genome is measured once.  Returns (best
    genome, its fitness, genomes measured)."""
    rng = random.Random(seed)
    cache: dict = {}

    def fit(g):
        g = tuple(g)
        if g not in cache:
            cache[g] = float(fitness(g))
        return cache[g]

    def mutate(g):
        g = list(g)
        i = rng.randrange(len(g))
        shape, rb = g[i]
        kind = rng.randrange(3)
        opts = choices[i]
        if kind == 0:                                   # the partition level (band height)
            pool = [c for c in opts if c[0] == shape and c[1] != rb]
        elif kind == 1:                                 # the partition axis (tile shape)
            same = [c for c in opts if c[0] != shape and c[1] == rb]
            pool = same or [c for c in opts if c[0] != shape]
        else:                                           # anything else
            pool = [c for c in opts if c != (shape, rb)]
        if pool:
            g[i] = rng.choice(pool)
        return tuple(g)

    def crossover(a, b):
        return tuple(rng.choice((x, y)) for x, y in zip(a, b))

    start = tuple(start) if start is not None else tuple(c[0] for c in choices)
    pop = [start] + [mutate(start) for _ in range(population - 1)]
    best = min(pop, key=fit)
    for _ in range(generations):
        parents = [min((rng.choice(pop) for _ in range(k)), key=fit)
                   for _ in range(2 * population)]
        pop = [best]                                    # the best so far survives
        for i in range(population - 1):
            child = crossover(parents[2 * i], parents[2 * i + 1])
            if rng.random() < mutation_rate:
                child = mutate(child)
            pop.append(child)
        best = min(pop, key=fit)
    # refinement: each gene in turn over all its values, the others fixed
    # (the orthogonal search of Section V-D1), until nothing improves; the
    # paper's final sweep of the thread count is the band heights' share
    improved = True
    while improved:
        improved = False
        for i in range(len(best)):
            for c in choices[i]:
                trial = best[:i] + (c,) + best[i + 1:]
                if fit(trial) < fit(best):
                    best, improved = trial, True
    return best, fit(best), len(cache)


def environment_key(bto=None, digest: str = "") -> str:
    """What a measured fitness depends on besides the configuration: the
    device architecture, the ROCm version and a digest of the code timed.
    Caches keyed with it are not reused on another box or build."""
    arch, rocm = "cpu", "none"
    try:
        import torch
        if torch.cuda.is_available():
            arch = torch.cuda.get_device_properties(0).gcnArchName
        rocm = str(getattr(torch.version, "hip", None) or "none")
    except Exception:
        pass
    if not digest and bto is not None:
        digest = library_digest(bto)
    return f"{arch}|rocm {rocm}|{digest}"


def library_digest(bto) -> str:
    """Digest of the library's kernel sources (what a timing depends on)."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def bucket_evaluator(single, groups: dict):
    """Fitness for a size bucket: the summed time over the bucket's sample
    sizes (groups maps the bucket's largest sample to all of them), so a
    configuration is judged over the range it will serve, not at one point."""
    def evaluate(kernel, m, n, org):
        return sum(single(kernel, s, s, org) for s in groups.get(max(m, n), [max(m, n)]))
    return evaluate


# ---- batched execution -------------------------------------------------------------

#: the batch plan's knobs and the values searched (the first is the library default)
BATCH_SPACE = {
    # fuse-or-split of every instance; "tiled": fused, as short-lived tiles
    # (bto_tiled_batch), to which the persistent plan's knobs do not apply
    "form": ["fused", "unfused", "tiled"],
    # the persistent plan (bto_batch_plan)
    "threads": [256, 512],                      # workgroup size
    "wgs_per_cu": [2, 1, 3, 4],                 # persistent workgroups per CU ("threads")
    "split_bytes": [16 << 20, -1, 8 << 20, 32 << 20, 4 << 20],   # row tiles of large instances
    # the tiled form (bto_tiled_config): tile shapes (the partition axis and
    # the per-partition parallelism), band heights (how many partitions) and
    # persistent workgroups (0: one per tile)
    "t_store_shape": [2, 3, 11, 7, 1, 0, 4, 5, 6, 8, 9, 10],
    "t_store_rb": [16, 32, 64, 8, 128, 256, 512],
    "t_bicgk_rb": [64, 32, 128, 256, 512],
    "t_wide_shape": [7, 2, 1, 3, 8, 11, 0],
    "t_narrow_shape": [2, 3, 5, 1, 0],
    "t_read_rb": [64, 32, 128],
    "t_wgs_per_cu": [0, 1, 2, 4],
}
PLAN_KNOBS = ("threads", "wgs_per_cu", "split_bytes")
TILED_KNOBS = ("t_store_shape", "t_store_rb", "t_bicgk_rb", "t_wide_shape", "t_narrow_shape",
               "t_read_rb", "t_wgs_per_cu")


def tiled_config_of(cfg: dict) -> dict:
    """The bto_tiled_config fields of a batch configuration's tiled knobs."""
    return {k[2:]: v for k, v in cfg.items() if k in TILED_KNOBS}


def tune_batch(evaluate, space: dict | None = None, cache: dict | None = None) -> tuple:
    """Orthogonal search over the batch knobs: fusion first, then each knob of
    the winning form in turn over its values, keeping the best so far (the
    paper's orthogonal strategy, Section V-D1).  `evaluate(cfg) -> seconds`
    for a dict cfg (infinity for a configuration that cannot run or gives
    wrong results); results are cached by the configuration.  Returns (best
    cfg, its time, evaluations)."""
    space = BATCH_SPACE if space is None else space
    cache = {} if cache is None else cache

    def fit(cfg):
        key = json.dumps(cfg, sort_keys=True)
        if key not in cache:
            cache[key] = float(evaluate(dict(cfg)))
        return cache[key]

    best = {k: v[0] for k, v in space.items()}
    for knob in space:                        # "form" first: fusion before geometry
        tiled = best.get("form") == "tiled"
        if (tiled and knob in PLAN_KNOBS) or (not tiled and knob in TILED_KNOBS):
            continue                          # knobs of the form not chosen
        for val in space[knob]:
            trial = {**best, knob: val}
            if fit(trial) < fit(best):
                best = trial
    return best, fit(best), len(cache)


# ---- applying results --------------------------------------------------------------

def apply(bto, org: Organism, size: int = 0) -> None:
    """Load an organism's slot configurations into the library, for the size
    bucket of max(m, n) = size (0: every bucket)."""
    for slot, c in org.slots:
        bto.tune_set(slot, *c, size=size)


def outputs_agree(got: list, ref: list, tol: float = 1e-12) -> bool:
    """Every output within `tol` normwise relative error of the reference
    (absolute where the reference is all zero); NaN never agrees."""
    for g, r in zip(got, ref):
        if g.numel() == 0:
            continue
        den = float(r.abs().max())
        num = float((g - r).abs().max())
        err = num / den if den > 0 else num
        if not err <= tol:
            return False
    return True


def gpu_evaluator(bto, torch, make_workload, reps: int = 10, warmup: int = 3, keep: int = 4):
    """An evaluate() that times one call of a kernel on the current device.
    `make_workload(kernel, m, n)` returns an object with run(form) and
    outputs(); the last `keep` workloads stay resident.  Every timed
    variant's outputs are compared with those of the library's default
    configuration (fused form) on the same inputs: a variant that disagrees
    beyond 1e-12, or that the library refuses or that fails, scores
    infinity and is never chosen."""
    cache = {}
    refs = {}

    def evaluate(kernel, m, n, org):
        key = (kernel, m, n)
        if key not in cache:
            if len(cache) >= keep:
                old = next(iter(cache))
                cache.pop(old)
                refs.pop(old, None)
                torch.cuda.empty_cache()
            cache[key] = make_workload(kernel, m, n)
        wl = cache[key]
        if key not in refs:
            wl.run("fused")
            torch.cuda.synchronize()
            refs[key] = [t.clone() for t in wl.outputs()]
        size = max(m, n)
        saved = {s: bto.tune_get(s, size) for s, _ in org.slots}
        try:
            apply(bto, org, size)
            for t in wl.outputs():
                t.fill_(float("nan"))
            for _ in range(warmup):
                wl.run(org.form)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                wl.run(org.form)
            stop.record()
            stop.synchronize()
            if not outputs_agree(wl.outputs(), refs[key]):
                return float("inf")
            return start.elapsed_time(stop) / reps * 1e-3
        except (bto.BtoError, RuntimeError):
            return float("inf")
        finally:
            for s, c in saved.items():
                bto.tune_set(s, *c, size=size)

    return evaluate


# ---- command line: tune on the current device ---------------------------------------

class _MatrixWorkload:
    """Device-resident operands of one matrix kernel (synthetic, seeded)."""

    def __init__(self, bto, torch, synth, kernel, m, n, dev):
        self.bto, self.kernel = bto, kernel
        d = lambda a: torch.from_numpy(a).to(dev)
        sid = lambda op: synth.stream_id(7, op)
        self.A = d(synth.matrix(synth.SEED, sid(0), m, n))
        vm = lambda op: d(synth.uniform(synth.SEED, sid(op), m))
        vn = lambda op: d(synth.uniform(synth.SEED, sid(op), n))
        if kernel == "gemver":
            self.args = [vm(1), vn(2), vm(3), vn(4), vm(5), vn(6)]
            self.B = torch.empty_like(self.A)
            self.x, self.w = vn(7), vm(8)
        elif kernel == "bicgk":
            self.p, self.r, self.q, self.s = vn(1), vm(2), vm(3), vn(4)
        elif kernel == "atax":
            self.xv, self.y = vn(1), vn(2)
        else:
            self.y, self.z, self.x, self.w = vm(1), vn(2), vn(3), vm(4)
        self.ws = {f: torch.empty(max(1, bto.workspace_bytes(kernel, m, n, f)),
                                  dtype=torch.uint8, device=dev) for f in FORMS}

    def outputs(self):
        if self.kernel == "gemver":
            return [self.B, self.x, self.w]
        if self.kernel == "bicgk":
            return [self.q, self.s]
        if self.kernel == "atax":
            return [self.y]
        return [self.x, self.w]

    def run(self, form):
        b, ws = self.bto, self.ws[form]
        if self.kernel == "gemver":
            b.gemver(self.A, *self.args, 1.5, 0.7, form=form, B=self.B, x=self.x, w=self.w, ws=ws)
        elif self.kernel == "bicgk":
            b.bicgk(self.A, self.p, self.r, form=form, q=self.q, s=self.s, ws=ws)
        elif self.kernel == "atax":
            b.atax(self.A, self.xv, form=form, y=self.y, ws=ws)
        else:
            b.dgemvt(self.A, self.y, self.z, 1.5, 0.7, form=form, x=self.x, w=self.w, ws=ws)


HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "bto_tuned.hpp")
TILE_SLOT_NAMES = ["BICGK_FUSED", "GEMV_N", "GEMV_T", "GER", "GEMVER_P1", "GEMVER_P2",
                   "DGEMVT_P1", "DGEMVT_P2"]


def render_defaults(table: dict, nbuckets: int = 8) -> str:
    """The per-bucket default block of bto_tuned.hpp from
    table[slot][bucket] = (shape, rb, rev)."""
    lines = ["// {shape, rb, rev} per slot and size bucket (written by "
             "`python -m paper_1205_1098_amd.tune --write-header`)",
             "#define BTO_TUNED_DEFAULTS                                                "
             "                        \\", "    {                                        "
             "                                                     \\"]
    for slot, name in enumerate(TILE_SLOT_NAMES):
        cfgs = ", ".join("{%d, %d, %d}" % tuple(table[slot][b]) for b in range(nbuckets))
        lines.append(f"        {{{cfgs}}},  /* {name} */ \\")
    lines.append("    }")
    lines.append("")
    lines.append("// workgroup size of the row-resident ATAX and BiCGK sweeps per size bucket")
    lines.append("// (BiCGK: 0 selects the tile sweep of slot bicgk_fused)")
    for slot, macro in ((SLOT_ATAX_ROWRES, "BTO_TUNED_ATAX_ROWRES"),
                        (SLOT_BICGK_ROWRES, "BTO_TUNED_BICGK_ROWRES")):
        vals = ", ".join(str(table[slot][b][0]) for b in range(nbuckets))
        lines.append(f"#define {macro} {{{vals}}}")
    return "\n".join(lines) + "\n"


def write_header(table: dict, path: str = HEADER) -> None:
    """Replace the default block of bto_tuned.hpp (between the size-bucket
    definitions and the end of the namespace)."""
    with open(path) as f:
        text = f.read()
    start = text.index("// {shape, rb, rev} per slot and size bucket")
    end = text.index("}  // namespace bto")
    text = text[:start] + render_defaults(table) + "\n" + text[end:]
    with open(path, "w") as f:
        f.write(text)


def main(argv=None) -> int:
    import argparse
    import time

    import torch

    from paper_1205_1098_amd import bto, synth

    ap = argparse.ArgumentParser(description="tune tile configurations on this device")
    ap.add_argument("--kernels", nargs="+", default=["bicgk", "gemver", "dgemvt", "atax"])
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--sizes", type=int, nargs="*", default=None,
                    help="square sizes to tune, each for its size bucket (instead of --m/--n)")
    ap.add_argument("--strategy", choices=["orth", "mfga"], default="orth")
    ap.add_argument("--cache", default=None, help="fitness cache (JSON) to resume from / write")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--forms", choices=["best", "both", "fused"], default="best",
                    help="search the geometry of the better form only, of both forms, or of "
                         "the fused form")
    ap.add_argument("--prune", type=float, default=0.25,
                    help="skip configurations whose modeled partial-sum traffic exceeds this "
                         "fraction of one matrix pass")
    ap.add_argument("--batch", action="store_true",
                    help="tune the batch plan's knobs on 4096 mixed GEMVER/BiCGK instances "
                         "(n log-uniform on [64, 2048]) instead of the tile slots")
    ap.add_argument("--write-header", action="store_true",
                    help="bake the winners into csrc/bto_tuned.hpp (per size bucket; sizes "
                         "not tuned keep their current configuration)")
    args = ap.parse_args(argv)

    dev = torch.device("cuda:0")
    if args.batch:
        return _tune_batch_main(torch, bto, args)
    space = Space.from_library(bto)
    ev = gpu_evaluator(bto, torch, lambda k, m, n: _MatrixWorkload(bto, torch, synth, k, m, n, dev))
    names = bto.tune_slots()
    nb = bto.tune_buckets()
    table = {s: [bto.tune_get(s, 256 << b) for b in range(nb)] for s in range(len(names))}
    if args.sizes:
        # sizes of one bucket are searched together, judged by their summed time
        groups = {}
        for n in sorted(args.sizes):
            groups.setdefault(bto.tune_bucket(n), []).append(n)
        groups = {max(v): v for v in groups.values()}
        ev = bucket_evaluator(ev, groups)
        shapes = [(n, n) for n in groups]
    else:
        shapes = [(args.m, args.n)]
    tuner = Tuner(space, ev, args.cache, args.seed, args.prune,
                  env_key=environment_key(bto))
    best = {}
    for m, n in shapes:
        for k in args.kernels:
            t0 = time.perf_counter()
            forms = {"both": list(FORMS), "fused": ["fused"], "best": None}[args.forms]
            org = tuner.orthogonal(k, m, n, forms) if args.strategy == "orth" else \
                tuner.mfga(k, m, n)
            apply(bto, org, max(m, n))
            b = bto.tune_bucket(max(m, n))
            for s, c in org.slots:
                table[s][b] = tuple(c)
                if b == nb - 2:        # the largest tuned bucket also serves larger sizes
                    table[s][nb - 1] = tuple(c)
            mf = tuner.fitness(k, m, n, tuner.max_fuse(k))
            got = tuner.fitness(k, m, n, org)
            key = f"{k}:{m}x{n}"
            best[key] = {"form": org.form, "slots": {names[s]: list(c) for s, c in org.slots},
                         "us": round(got * 1e6, 2), "max_fuse_us": round(mf * 1e6, 2),
                         "search_s": round(time.perf_counter() - t0, 2)}
            if args.strategy == "orth" and forms:
                best[key]["per_form"] = {
                    f: {"slots": {names[s]: list(c) for s, c in o.slots},
                        "us": round(tuner.fitness(k, m, n, o) * 1e6, 2)}
                    for f, o in tuner.form_best.items()}
            print(json.dumps({key: best[key]}), flush=True)
            tuner.save({"best": best, "device": torch.cuda.get_device_properties(0).gcnArchName})
    if args.write_header:
        write_header(table)
        print(f"wrote {HEADER}", flush=True)
    return 0


def _tune_batch_main(torch, bto, args) -> int:
    from paper_1205_1098_amd import batch

    sets = {}
    refs = {}

    def outs(insts):
        return [t for inst in insts for t in inst["out"]]

    def evaluate(cfg):
        form = cfg["form"]
        if form not in sets:
            sets.clear()
            torch.cuda.empty_cache()
            sets[form] = batch.make_instances(torch, bto, 4096, 64, 2048,
                                              {"gemver": 0.5, "bicgk": 0.5},
                                              form="fused" if form == "tiled" else form)
            if "ref" not in refs:
                # the reference outputs: the persistent plan's defaults
                # (the instances of every form are generated alike)
                ref_plan = bto.BatchPlan(sets[form][0])
                ref_plan.launch()
                ref_plan.check()
                refs["ref"] = [t.clone() for t in outs(sets[form][0])]
                ref_plan.close()
        insts, _ = sets[form]
        for t in outs(insts):
            t.fill_(float("nan"))
        try:
            if form == "tiled":
                plan = bto.TiledBatch(insts, config=bto.TiledConfig.default(
                    **tiled_config_of(cfg)))
            else:
                plan = bto.BatchPlan(insts, threads=cfg["threads"], wgs_per_cu=cfg["wgs_per_cu"],
                                     split_bytes=cfg["split_bytes"])
        except bto.BtoError as e:          # a configuration the library refuses
            print(json.dumps({"cfg": cfg, "refused": str(e)}), flush=True)
            return float("inf")
        for _ in range(2):
            plan.launch()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            plan.launch()
        b.record()
        b.synchronize()
        ok = outputs_agree(outs(insts), refs["ref"])
        if form != "tiled":
            try:
                plan.check()
            except bto.BtoError:
                ok = False
        plan.close()
        sec = a.elapsed_time(b) / 5 * 1e-3 if ok else float("inf")
        print(json.dumps({"cfg": cfg, "ms": round(sec * 1e3, 3), "checked": ok}), flush=True)
        return sec

    env = environment_key(bto)
    cache = {}
    if args.cache and os.path.exists(args.cache):
        with open(args.cache) as f:
            data = json.load(f)
        if data.get("environment") == env:
            cache = data.get("batch_fitness", {})
    best, sec, evals = tune_batch(evaluate, cache=cache)
    out = {"best": best, "ms": round(sec * 1e3, 3), "evaluations": evals}
    print(json.dumps(out), flush=True)
    if args.cache:
        with open(args.cache, "w") as f:
            json.dump({"batch_fitness": cache, "batch_best": out, "environment": env}, f,
                      indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
