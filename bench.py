"""Benchmark: fused vs unfused FP64 BLAS-1/2 sequences on one MI355X.

One step is one fused GEMVER at n = 16384 (B = A + u1 v1^T + u2 v2^T,
x = beta B^T y + z, w = alpha B x; alpha = 1.5, beta = 0.7) on synthetic
inputs already resident in HBM.  ``value`` is algorithmic HBM bytes per step
(read A, write B, read B, plus every vector once) over the measured time per
step, in GB/s.  Rank 0 prints one JSON line with, besides the headline:

  unfused     the same step in the unfused form (one kernel per BLAS op)
  roofline    the dominant kernel (pass 1 of GEMVER): algorithmic bytes per
              launch over its average duration from HIP events recorded on
              its stream during the timed region, against the 8 TB/s peak;
              traffic = HBM bytes per launch from hardware counters when a
              counter summary for the current kernel source is committed
  suite       every Table I kernel, fused and unfused, at n = 16384 / 2^26
              (DGEMV and GESUMMV included), plus GEMVER with B contracted away
              (against GEMVER's two forms) and BATAX (y = beta A^T A x)
  generated   the same kernels compiled from their specifications (btoc),
              against the hand-written fused entry points
  generated_passes  programs whose fused passes the compiler emits as HIP
              (a rank-3 update, several row dots and column sums per sweep)
              at n = 16384, against their unfused and library lowerings
  stream      measured copy / read / triad ceilings at 2 GiB per array
  batched     4096 GEMVER / BiCGK instances (n log-uniform on [64, 2048]) in
              one persistent graph-captured launch, and the same instances as
              a tiled batch (one graph of launches of short-lived tiles: both
              kinds' first sweeps, their sums, GEMVER's second sweeps, sums)
  serving     Poisson and saturated request streams through the server
              (req/s, p50 / p99 latency): continuous batching with tiled
              batches, with the entry points only, with persistent plans,
              and a one-at-a-time FIFO server
  cpu_baseline  the CPU oracle timed on the host cores on the same workload

Usage: python bench.py [--steps K] [--warmup W] [--workload gemver|bicgk|...]
       [--no-suite] [--no-cpu] [--no-stream] [--no-batch] [--no-serve]
       [--batch-direct] [--no-batch-loop] [--copy-probe] [--row-lengths]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
METRIC = "fused vs unfused HBM GB/s (% peak), GEMVER/BiCGK FP64; batch req/s, p99 latency"
N = 16384
NV = 1 << 26
ALPHA, BETA = 1.5, 0.7
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="gemver",
                    choices=["gemver", "bicgk", "atax", "dgemvt", "axpydot", "waxpby", "vadd"])
    ap.add_argument("--no-suite", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-batch-loop", action="store_true",
                    help="skip the per-instance launch loop the batch is compared with")
    ap.add_argument("--batch-direct", action="store_true",
                    help="launch the batch plan without its HIP graph (hardware counters "
                         "are read per direct dispatch only)")
    ap.add_argument("--no-one-kind", action="store_true",
                    help="skip the batches of one kind at a time (so that a profile of the "
                         "batch sees the mixed batch only)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the 2 GiB copy probe (calibrates hardware byte counters)")
    ap.add_argument("--row-lengths", action="store_true",
                    help="only time the first sweeps per row length: tiled batches of one size "
                         "and one kind, and single tall matrices of the same row length")
    return ap.parse_args()


def copy_probe(torch, bto, reps: int = 3) -> int:
    """Copy 2 GiB `reps` times; prints the bytes each launch moves."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        bto.probe_copy(a, b)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "doubles": n, "read_bytes": n * 8, "write_bytes": n * 8,
                      "launches": reps}), flush=True)
    return 0


def tiled_group_ms(torch, bto, insts, cfg, steps: int = 5) -> dict:
    """Mean time per launch of each group of a tiled batch (first sweeps,
    their sums, second sweeps, their sums), from HIP events around each
    launch on its stream; the plan runs without its graph here so that every
    launch is seen."""
    conf = bto.TiledConfig.default(**{**cfg.as_dict(), "use_graph": 0})
    t = bto.TiledBatch(insts, config=conf)
    t.launch()
    torch.cuda.synchronize()
    bto.timing_reset()
    bto.timing_enable(True)
    for _ in range(steps):
        t.launch()
    torch.cuda.synchronize()
    bto.timing_enable(False)
    times = bto.timing_read()
    bto.timing_reset()
    t.close()
    return {k: round(ms / c, 4) for k, (c, ms) in sorted(times.items())
            if c and k.startswith("bt_")}


ROW_LENGTHS = (256, 512, 1000, 1500, 2000)


def row_length_probe(torch, bto, budget: float = 2.5e9) -> int:
    """The first sweeps at one row length at a time: tiled batches of
    GEMVER-only and of BiCGK-only n x n instances (about `budget` matrix
    bytes each, rows 64-byte aligned as in the mixed batch), next to the
    single-instance sweeps of one tall m x n matrix with the same row length
    and stride.  GB/s count matrix bytes only (GEMVER's first sweep reads A
    and writes B; BiCGK's reads A)."""
    from paper_1205_1098_amd import batch

    dev = torch.device("cuda:0")
    cfg = bto.TiledConfig.default(use_graph=0)
    out = {}
    for n in ROW_LENGTHS:
        ent = {}
        for kind, per in (("gemver", 16 * n * n), ("bicgk", 8 * n * n)):
            count = max(1, int(budget // per))
            insts, _ = batch.make_instances(torch, bto, count, 64, 2048, {kind: 1.0}, config=4,
                                            shapes=[(n, n)] * count)
            ms = tiled_group_ms(torch, bto, insts, cfg)
            ent[f"batch_{kind}"] = {"instances": count, "first_sweep_ms": ms["bt_first"],
                                    "gbs": round(count * per / ms["bt_first"] / 1e6, 1)}
            del insts
            torch.cuda.empty_cache()
        m = int(budget // (16 * n))
        lda = batch._lda(n)
        A = torch.empty((m, lda), dtype=torch.float64, device=dev)[:, :n]
        B = torch.empty((m, lda), dtype=torch.float64, device=dev)[:, :n]
        bto.synth_fill(A, 1)
        vm = [torch.rand(m, dtype=torch.float64, device=dev) for _ in range(3)]
        vn = [torch.rand(n, dtype=torch.float64, device=dev) for _ in range(3)]
        x = torch.empty(n, dtype=torch.float64, device=dev)
        w = torch.empty(m, dtype=torch.float64, device=dev)
        q = torch.empty(m, dtype=torch.float64, device=dev)
        run_g = lambda: bto.gemver(A, vm[0], vn[0], vm[1], vn[1], vm[2], vn[2], 1.5, 0.7, B=B,
                                   x=x, w=w)
        run_b = lambda: bto.bicgk(A, vn[0], vm[0], q=q, s=x)
        for name, fn, per in (("single_gemver_p1", run_g, 16 * m * n),
                              ("single_bicgk", run_b, 8 * m * n)):
            fn()
            torch.cuda.synchronize()
            bto.timing_reset()
            bto.timing_enable(True)
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            bto.timing_enable(False)
            times = bto.timing_read()
            bto.timing_reset()
            key = "gemver_p1" if name == "single_gemver_p1" else max(
                (k for k in times if k.startswith("bicgk")), key=lambda k: times[k][1])
            c, tot = times[key]
            ent[name] = {"rows": m, "kernel": key, "ms": round(tot / c, 4),
                         "gbs": round(per / (tot / c) / 1e6, 1)}
        del A, B, vm, vn, x, w, q
        torch.cuda.empty_cache()
        out[str(n)] = ent
        print(f"row length {n}: {json.dumps(ent)}", file=sys.stderr, flush=True)
    print(json.dumps({"probe": "row_lengths", "budget_bytes": budget, "results": out}),
          flush=True)
    return 0


# ---- algorithmic bytes (each matrix pass the dependencies force, each vector once)

def alg_bytes(kernel: str, form: str, n: int = N, nv: int = NV) -> int:
    M, v, V = n * n * 8, n * 8, nv * 8
    fused = {
        "gemver": 3 * M + 8 * v,     # read A, write B, read B; u1 v1 u2 v2 y z in, x w out
        "bicgk": M + 4 * v,          # read A; p r in, q s out
        "atax": M + 2 * v,           # read A; x in, y out
        "dgemvt": 2 * M + 4 * v,     # two passes over A; y z in, x w out
        "axpydot": 4 * V,            # w v u in, z out
        "waxpby": 3 * V,             # x y in, w out
        "vadd": 4 * V,               # w y z in, x out
        "gemver_contracted": 2 * M + 8 * v,   # two reads of A; B never stored
        "batax": M + 2 * v,          # as ATAX; beta applied after the reduction
        "dgemv": M + 3 * v,          # read A; x y in, z out
        "gesummv": 2 * M + 2 * v,    # read A and B; x in, y out
    }
    unfused = {
        "gemver": 6 * M + 12 * v,    # ger (2M), ger (2M), gemv_t (M), gemv_n (M)
        "bicgk": 2 * M + 4 * v,
        "atax": 2 * M + 4 * v,       # t written and read back
        "dgemvt": 2 * M + 4 * v,
        "axpydot": 5 * V,            # axpy (3V) + dot (2V)
        "waxpby": 5 * V,             # scal (2V) + axpy (3V)
        "vadd": 6 * V,               # add (3V) + add (3V)
        "batax": 2 * M + 4 * v,
        "dgemv": M + 3 * v,          # one BLAS call either way
        "gesummv": 2 * M + 5 * v,    # dgemv (t = alpha A x), dgemv (y = beta B x + t)
    }
    return (fused if form == "fused" else unfused)[kernel]


# dominant kernel of each workload's fused step and its algorithmic bytes per launch
def dominant(kernel: str, n: int = N, nv: int = NV):
    M, v, V = n * n * 8, n * 8, nv * 8
    return {
        "gemver": ("gemver_p1", 2 * M + 5 * v),
        "bicgk": ("bicgk_fused", M + 2 * v),
        "atax": ("atax_rowres", M + v),
        "dgemvt": ("dgemvt_p1", M + v),
        "axpydot": ("axpydot_fused", 4 * V),
        "waxpby": ("ew_waxpby", 3 * V),
        "vadd": ("ew_vadd3", 4 * V),
    }[kernel]


# ---- workloads ------------------------------------------------------------------

# kernels whose suite entry is also timed with inputs that are cold in the
# last-level cache (every matrix kernel)
COLD = ("gemver", "bicgk", "atax", "dgemvt", "gemver_contracted", "batax", "dgemv", "gesummv")

class Workload:
    """Device-resident inputs and outputs of one kernel at bench size."""

    def __init__(self, torch, bto, synth, kernel, dev, shared=None):
        self.kernel, self.bto, self.torch = kernel, bto, torch
        seed = synth.SEED
        sid = lambda op: synth.stream_id(2 if kernel.startswith("gemver") else 3, op)
        d = lambda a: torch.from_numpy(a).to(dev)
        shared = {} if shared is None else shared
        if kernel in ("gemver", "gemver_contracted", "bicgk", "atax", "batax", "dgemvt", "dgemv",
                      "gesummv"):
            if "A" not in shared:
                shared["A"] = d(synth.matrix(seed, sid(0), N, N))
            self.A = shared["A"]
            vec = lambda op: d(synth.uniform(seed, sid(op), N))
            if kernel == "gemver_contracted":
                self.vs = [vec(k) for k in range(1, 7)]
                self.x, self.w = vec(7), vec(8)
            elif kernel == "gemver":
                self.vs = [vec(k) for k in range(1, 7)]
                if "B" not in shared:
                    shared["B"] = torch.empty_like(self.A)
                self.B = shared["B"]
                self.x, self.w = vec(7), vec(8)
            elif kernel == "bicgk":
                self.p, self.r, self.q, self.s = vec(1), vec(2), vec(3), vec(4)
            elif kernel in ("atax", "batax"):
                self.x, self.y = vec(1), vec(2)
            elif kernel == "dgemv":
                self.x, self.y, self.z = vec(1), vec(2), vec(3)
            elif kernel == "gesummv":
                if "B2" not in shared:
                    shared["B2"] = torch.empty_like(self.A)
                    bto.synth_fill(shared["B2"], synth.stream_state(seed, sid(9)))
                self.B2 = shared["B2"]
                self.x, self.y = vec(1), vec(2)
            else:
                self.y, self.z, self.x, self.w = vec(1), vec(2), vec(3), vec(4)
        else:
            vec = lambda op: d(synth.uniform(seed, sid(16 + op), NV))
            self.a, self.b, self.c, self.out = vec(0), vec(1), vec(2), vec(3)
            self.r = torch.zeros(1, dtype=torch.float64, device=dev)
        self.ws = {f: torch.empty(max(1, bto.workspace_bytes(kernel, N, NV if kernel in
                                                                   ("axpydot", "waxpby", "vadd")
                                                                   else N, f)),
                                  dtype=torch.uint8, device=dev) for f in ("fused", "unfused")}

    def run(self, form: str) -> None:
        b, k, ws = self.bto, self.kernel, self.ws[form]
        if k == "gemver":
            b.gemver(self.A, *self.vs, ALPHA, BETA, form=form, B=self.B, x=self.x, w=self.w, ws=ws)
        elif k == "gemver_contracted":
            b.gemver_contracted(self.A, *self.vs, ALPHA, BETA, x=self.x, w=self.w, ws=ws)
        elif k == "batax":
            b.batax(self.A, self.x, BETA, form=form, y=self.y, ws=ws)
        elif k == "dgemv":
            b.dgemv(self.A, self.x, self.y, ALPHA, BETA, form=form, z=self.z, ws=ws)
        elif k == "gesummv":
            b.gesummv(self.A, self.B2, self.x, ALPHA, BETA, form=form, y=self.y, ws=ws)
        elif k == "bicgk":
            b.bicgk(self.A, self.p, self.r, form=form, q=self.q, s=self.s, ws=ws)
        elif k == "atax":
            b.atax(self.A, self.x, form=form, y=self.y, ws=ws)
        elif k == "dgemvt":
            b.dgemvt(self.A, self.y, self.z, ALPHA, BETA, form=form, x=self.x, w=self.w, ws=ws)
        elif k == "axpydot":
            b.axpydot(self.a, self.b, self.c, ALPHA, form=form, z=self.out, r=self.r, ws=ws)
        elif k == "waxpby":
            b.waxpby(self.a, self.b, ALPHA, BETA, form=form, w=self.out, ws=ws)
        else:
            b.vadd(self.a, self.b, self.c, form=form, x=self.out, ws=ws)


def time_stats(torch, fn, steps: int, warmup: int):
    """(median, min) seconds per call of `fn` over `steps` calls after
    `warmup` untimed ones: HIP events recorded on torch's current stream (the
    stream the library launches on) between calls."""
    for _ in range(warmup):
        fn()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for i in range(steps):
        fn()
        evs[i + 1].record()
    torch.cuda.synchronize()
    ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return float(np.median(ms)) * 1e-3, float(min(ms)) * 1e-3


def time_steps(torch, fn, steps: int, warmup: int) -> float:
    """Median seconds per call (see time_stats)."""
    return time_stats(torch, fn, steps, warmup)[0]


# ---- hardware-counter traffic ------------------------------------------------------

def counter_traffic(summary: str):
    """HBM bytes per launch from the committed counter summary `summary`, or
    None when there is none for the current kernel sources."""
    path = os.path.join(PROFILES, summary)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    from paper_1205_1098_amd.profsum import SOURCE_SETS, source_digest

    sources = fields.get("source_set", "")
    if sources not in SOURCE_SETS or fields.get("source_digest") != source_digest(sources):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---- CPU oracle baseline -------------------------------------------------------------

def oracle_bytes(kernel: str, n: int = N) -> int:
    """Bytes the oracle's loops move for one call at size n: the matrix
    passes its unfused statements execute (GEMVER: read A, write B, then
    read B for each product; the others one read of A per product), plus
    each vector once."""
    M, v = n * n * 8, n * 8
    return {"gemver": 4 * M + 10 * v, "bicgk": 2 * M + 4 * v, "atax": 2 * M + 4 * v,
            "dgemvt": 2 * M + 4 * v}[kernel]


def host_cpu() -> dict:
    """The host CPU's model name and logical CPU count (from /proc/cpuinfo)."""
    model, count = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    count += 1
                    model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"model": model, "logical_cpus": count or (os.cpu_count() or 0)}


def cpu_baseline(kernel: str, target_s: float):
    """The oracle on the host cores, on the same workload (one full call at
    n = 16384 on host data): with every thread the process may use, and with
    one thread; the median of 3 calls or more (repeated up to about
    `target_s` seconds with all threads), in GB/s of the bytes its loops move."""
    import oracle
    from paper_1205_1098_amd import synth

    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    seed = synth.SEED
    sid = lambda op: synth.stream_id(2, op)
    A = synth.matrix(seed, sid(0), N, N)
    vs = [synth.uniform(seed, sid(k), N) for k in range(1, 7)]

    def call():
        if kernel == "gemver":
            oracle.gemver(A, *vs, ALPHA, BETA)
        elif kernel == "bicgk":
            oracle.bicgk(A, vs[0], vs[1])
        elif kernel == "atax":
            oracle.atax(A, vs[0])
        else:
            oracle.dgemvt(A, vs[0], vs[1], ALPHA, BETA)

    def leg(t: int, budget: float, cap: int):
        oracle.set_threads(t)
        used = int(oracle.get_threads())
        times = []
        while len(times) < 3 or (sum(times) < budget and len(times) < cap):
            t0 = time.perf_counter()
            call()
            times.append(time.perf_counter() - t0)
        med = float(np.median(times))
        return {"threads": used, "calls": len(times), "median_ms": round(med * 1e3, 2),
                "min_ms": round(min(times) * 1e3, 2),
                "gbs": round(oracle_bytes(kernel) / med / 1e9, 3)}

    full = leg(threads, target_s, 200)
    one = leg(1, 0.0, 3)
    del A
    # a vector kernel at N = 2^26 beside it: AXPYDOT, whose unfused loops
    # move 5 vectors (axpy: w, v in, z out; dot: z, u in); the oracle's
    # vector loops run on one thread (its pairwise dot is one recursion)
    oracle.set_threads(1)
    xs = [synth.uniform(seed, sid(10 + k), NV) for k in range(3)]
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.axpydot(*xs, ALPHA)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    vector = {"kernel": f"axpydot N={NV}", "threads": 1, "calls": 3,
              "median_ms": round(med * 1e3, 2), "gbs": round(5 * NV * 8 / med / 1e9, 3)}
    del xs
    cpu = host_cpu()
    return {
        "value": full["gbs"],
        "unit": "GB/s",
        "cores": full["threads"],
        "kind": "oracle",
        "sample": f"{full['calls']} full {kernel} n={N} calls on host data with {full['threads']} "
                  f"threads (median {full['median_ms']} ms) and 3 with 1 thread (median "
                  f"{one['median_ms']} ms); GB/s of the {oracle_bytes(kernel)} bytes its "
                  "unfused loops move per call",
        "cpu_model": cpu["model"],
        "logical_cpus": cpu["logical_cpus"],
        "all_threads": full,
        "one_thread": one,
        "bytes_per_call": oracle_bytes(kernel),
        "vector": vector,
    }


# the compiled specifications timed against the hand-written fused entry
# points (same algorithmic bytes); input name -> "A", "B" (matrices), "m" /
# "n" (vectors) or a scalar value
GENERATED = {
    "gemver": dict(A="A", u1="m", v1="n", u2="m", v2="n", y="m", z="n", alpha=ALPHA, beta=BETA),
    "gemver_contracted": dict(A="A", u1="m", v1="n", u2="m", v2="n", y="m", z="n",
                              alpha=ALPHA, beta=BETA),
    "bicgk": dict(A="A", p="n", r="m"),
    "atax": dict(A="A", x="n"),
    "batax": dict(A="A", x="n", beta=BETA),
    "dgemvt": dict(A="A", y="m", z="n", alpha=ALPHA, beta=BETA),
    "dgemv": dict(A="A", x="n", y="m", alpha=ALPHA, beta=BETA),
    "gesummv": dict(A="A", B="B", x="n", alpha=ALPHA, beta=BETA),
    "axpydot": dict(w="V", v="V", u="V", alpha=ALPHA),
    "waxpby": dict(x="V", y="V", alpha=ALPHA, beta=BETA),
    "vadd": dict(w="V", y="V", z="V"),
}


def bench_generated(torch, bto, synth, shared, suite) -> dict:
    """Each kernel compiled from its specification (btoc) and run through
    the fused-pass entry point, against the suite's hand-written fused time."""
    from paper_1205_1098_amd import bto_specs, btoc

    dev = shared["A"].device
    out = {}
    texts, bounds = {}, {}
    for k, kinds in GENERATED.items():
        text = {"batax": bto_specs.BATAX, "gemver_contracted": bto_specs.GEMVER_CONTRACTED}.get(
            k, bto_specs.TABLE_I.get(k))
        prog = btoc.compile_spec(text, "fused")
        length = NV if "V" in kinds.values() else N
        bound = {}
        for j, (name, what) in enumerate(sorted(kinds.items())):
            if what == "A":
                bound[name] = shared["A"]
            elif what == "B":
                bound[name] = shared["B2"]
            elif what in ("m", "n", "V"):
                bound[name] = torch.from_numpy(synth.uniform(synth.SEED, 900 + j, length)).to(dev)
            else:
                bound[name] = what
        for o in prog.outputs:   # outputs preallocated: the loop allocates nothing
            if prog.kinds[o] == "matrix":
                bound[o] = shared["B"]
            else:
                bound[o] = torch.empty(1 if prog.kinds[o] == "scalar" else length,
                                       dtype=torch.float64, device=dev)
        ws = torch.empty(max(bto.pass_workspace_bytes(o, N, N) for o in range(1, 32)),
                         dtype=torch.uint8, device=dev)
        sec = time_steps(torch, lambda: prog.run(ws=ws, **bound), 20, 3)
        hand = suite.get(k, {}).get("fused_ms")
        ent = {"passes": len(prog.passes()), "ms": round(sec * 1e3, 4),
               "gbs": round(alg_bytes(k, "fused") / sec / 1e9, 1),
               "vs_hand_fused": round(hand / (sec * 1e3), 3) if hand else None}
        if k in ("gemver", "bicgk", "atax", "dgemv"):
            # the same program with its matrices stored by columns (transposed
            # views of the same storage): the schedule follows the layout
            cprog = btoc.compile_spec(text.replace("matrix(row)", "matrix(column)"), "fused")
            cb = {name: (t.t() if isinstance(t, torch.Tensor) and t.dim() == 2 else t)
                  for name, t in bound.items()}
            csec = time_steps(torch, lambda: cprog.run(ws=ws, **cb), 20, 3)
            ent["column_major"] = {"passes": len(cprog.passes()), "ms": round(csec * 1e3, 4),
                                   "vs_row_major": round(sec / csec, 3)}
        out[k] = ent
        texts[k], bounds[k] = text, bound
    # the empirical search over fusion decisions, on the same inputs
    search = {}
    for k in ("gemver_contracted", "atax", "bicgk", "axpydot"):
        best, table = btoc.search(texts[k], bounds[k], reps=5, ws=ws)
        search[k] = {"best": best.describe(),
                     "variants": [{"off": off if isinstance(off, str) else list(off),
                                   "steps": len(sched), "ms": round(ms, 4)}
                                  for off, sched, ms in table]}
    out["search"] = search
    # at small sizes a program costs its launches: eager calls against one
    # captured HIP graph replay per call
    small = {}
    for k in ("gemver", "bicgk", "atax"):
        ns = 512
        prog = btoc.compile_spec(texts[k], "fused")
        sb = {}
        for j, (name, what) in enumerate(sorted(GENERATED[k].items())):
            if what == "A":
                sb[name] = torch.from_numpy(synth.matrix(synth.SEED, 950 + j, ns, ns)).to(dev)
            elif what in ("m", "n"):
                sb[name] = torch.from_numpy(synth.uniform(synth.SEED, 950 + j, ns)).to(dev)
            else:
                sb[name] = what
        for o in prog.outputs:
            sb[o] = (torch.empty((ns, ns), dtype=torch.float64, device=dev)
                     if prog.kinds[o] == "matrix" else torch.empty(ns, dtype=torch.float64,
                                                                   device=dev))
        eager = time_steps(torch, lambda: prog.run(ws=ws, **sb), 200, 20)
        cap = prog.capture(**sb)
        graph = time_steps(torch, cap.replay, 200, 20)
        small[k] = {"n": ns, "eager_us": round(eager * 1e6, 2), "graph_us": round(graph * 1e6, 2),
                    "speedup": round(eager / graph, 2)}
        del cap
    out["graph_small"] = small
    return out


def bench_generated_passes(torch, bto, n: int = N) -> dict:
    """The programs whose fused passes the compiler generates as HIP
    (bto_specs.GENERATED) at n x n: the generated library under its searched
    genome (and under the structural one), against the same program lowered
    unfused onto the library's passes and, where the library can run it
    fused, against that lowering (more sweeps)."""
    from paper_1205_1098_amd import bto_specs, btoc, btoc_gen

    dev = torch.device("cuda:0")
    out = {}
    for name, text in bto_specs.GENERATED.items():
        prog = btoc.compile_spec(text, target="generated")
        bound = btoc_gen.synthetic_bound(prog, n, dev)
        first = btoc_gen.run(prog, bound)
        bound.update(first)                  # outputs preallocated for the timed loops
        genome = btoc_gen.default_genome(prog)
        heur = btoc_gen.heuristic_genome(prog)
        sec = time_steps(torch, lambda: btoc_gen.run(prog, bound, genome), 20, 3)
        sec_h = sec if heur == genome else time_steps(
            torch, lambda: btoc_gen.run(prog, bound, heur), 20, 3)
        nbytes = btoc_gen.alg_bytes(prog, n, n)
        ent = {"passes": len(prog.passes()), "schedule": prog.describe(),
               "genome": [list(g) for g in genome],
               "tuned": btoc_gen.tuned_genome(prog) is not None,
               "alg_gb": round(nbytes / 1e9, 3), "ms": round(sec * 1e3, 4),
               "gbs": round(nbytes / sec / 1e9, 1),
               "pct_peak": round(100 * nbytes / sec / 1e9 / PEAK_GBS, 1),
               "structural_genome_ms": round(sec_h * 1e3, 4)}
        unf = btoc.compile_spec(text, "unfused")
        sec_u = time_steps(torch, lambda: unf.run(**bound), 10, 2)
        ent["unfused"] = {"passes": len(unf.passes()), "ms": round(sec_u * 1e3, 4),
                          "speedup": round(sec_u / sec, 3)}
        try:
            lib_prog = btoc.compile_spec(text)
        except btoc.SpecError as e:
            ent["library_fused"] = {"refused": str(e)}
        else:
            sec_l = time_steps(torch, lambda: lib_prog.run(**bound), 10, 2)
            ent["library_fused"] = {"passes": len(lib_prog.passes()),
                                    "ms": round(sec_l * 1e3, 4),
                                    "speedup": round(sec_l / sec, 3)}
        out[name] = ent
        print(f"generated {name}: {ent['ms']} ms, {ent['gbs']} GB/s", file=sys.stderr,
              flush=True)
        del bound, first
        torch.cuda.empty_cache()
    return out


def stream_probes(torch, bto, dev) -> dict:
    """The copy, read and triad probes over 2 GiB arrays (GB/s of the bytes
    each moves): the read probe's figure is its read kernel alone, timed with
    HIP events, without the one-workgroup finish that adds its partials."""
    n = 1 << 28   # 2 GiB per array
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.ones(n, dtype=torch.float64, device=dev)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    st = {}
    s = time_steps(torch, lambda: bto.probe_copy(b, a), 10, 2)
    st["copy_gbs"] = round(2 * n * 8 / s / 1e9, 1)
    rws = torch.empty(bto.probe_read_workspace_bytes(n), dtype=torch.uint8, device=dev)
    s = time_steps(torch, lambda: bto.probe_read(b, out, rws), 10, 2)
    st["read_call_gbs"] = round(n * 8 / s / 1e9, 1)
    bto.timing_reset()
    bto.timing_only("probe_read")
    bto.timing_enable(True)
    for _ in range(10):
        bto.probe_read(b, out, rws)
    torch.cuda.synchronize()
    bto.timing_enable(False)
    cnt, tot = bto.timing_read().get("probe_read", (0, 0.0))
    bto.timing_reset()
    bto.timing_only(None)
    st["read_gbs"] = round(n * 8 / (tot / cnt * 1e-3) / 1e9, 1) if cnt else st["read_call_gbs"]
    s = time_steps(torch, lambda: bto.probe_triad(a, b, c, 0.5), 10, 2)
    st["triad_gbs"] = round(3 * n * 8 / s / 1e9, 1)
    del a, b, c, rws
    torch.cuda.empty_cache()
    return st


def bench_batched(torch, bto, count: int, with_loop: bool = True, graph: bool = True,
                  with_one_kind: bool = True) -> dict:
    """4096 GEMVER / BiCGK instances (n log-uniform on [64, 2048], kinds by a
    fair seeded coin) in one graph-captured persistent launch, then as tiled
    batches; then 4096 instances of one kind at a time (all GEMVER, all
    BiCGK) in both forms."""
    from paper_1205_1098_amd import batch

    insts, specs = batch.make_instances(torch, bto, count, 64, 2048,
                                        {"gemver": 0.5, "bicgk": 0.5}, config=4)
    total = sum(batch.alg_bytes(s.kind, s.m, s.n) for s in specs)
    out_list = [t for inst in insts for t in inst["out"]]
    # every output array flattened into one buffer, and each element's array
    # index: the comparison below is a handful of launches, not one per array
    outs = lambda: torch.cat([t.reshape(-1) for t in out_list])
    seg = torch.repeat_interleave(
        torch.arange(len(out_list), device=out_list[0].device),
        torch.tensor([t.numel() for t in out_list], device=out_list[0].device))
    print(f"batched: {count} instances built", file=sys.stderr, flush=True)
    plan = bto.BatchPlan(insts, use_graph=graph)
    sec, sec_min = time_stats(torch, plan.launch, 10, 2)
    # the last timed launch completed every bounded wait (raises otherwise),
    # so its outputs are those of the batch
    try:
        plan.check()
        checked = True
    except bto.BtoError as e:
        print(f"batched: {e}", file=sys.stderr, flush=True)
        checked = False
    persistent = outs()
    plan.close()
    print("batched: persistent plan timed", file=sys.stderr, flush=True)
    # the same instances as short-lived workgroup tiles (GEMVER's first
    # sweeps and BiCGK's in one launch, then the finishes and GEMVER's second
    # sweeps), under the tuned configuration; outputs start as NaN
    torch._foreach_zero_(out_list)
    torch._foreach_add_(out_list, float("nan"))
    tiled_cfg = bto.TiledConfig.default(use_graph=1 if graph else 0)
    tiled = bto.TiledBatch(insts, config=tiled_cfg)
    sec_tiled, sec_tiled_min = time_stats(torch, tiled.launch, 10, 2)
    torch.cuda.synchronize()
    tiled_outs = outs()
    tiled.close()
    group_ms = tiled_group_ms(torch, bto, insts, tiled_cfg)
    print("batched: tiled batch timed", file=sys.stderr, flush=True)
    # the two forms add in different orders: they agree to the parity
    # tolerance (each is checked against the oracle by the GPU tests);
    # per array, max |difference| over max |persistent|
    k = len(out_list)
    amax = lambda v: torch.zeros(k, dtype=v.dtype, device=v.device).scatter_reduce(
        0, seg, v, "amax", include_self=True)
    den = amax(persistent.abs())
    num = amax((persistent - tiled_outs).abs())
    rel = torch.where(den > 0, num / torch.where(den > 0, den, 1.0), num)
    nan = bool(torch.isnan(tiled_outs).any() or torch.isnan(persistent).any())
    worst = float("inf") if nan else float(rel.max())
    del persistent, tiled_outs, seg
    # the same instances launched one entry-point call at a time
    def loop():
        for inst in insts:
            if inst["kind"] == "gemver":
                bto.gemver(inst["A"], *inst["in"], inst["alpha"], inst["beta"], B=inst["B"],
                           x=inst["out"][0], w=inst["out"][1])
            else:
                bto.bicgk(inst["A"], *inst["in"], q=inst["out"][0], s=inst["out"][1])
    sec_loop = time_steps(torch, loop, 2, 1) if with_loop else None
    del insts, out_list, outs
    torch.cuda.empty_cache()
    # the same sizes with every instance of one kind
    one_kind = {}
    for kind in ("gemver", "bicgk") if with_one_kind else ():
        ki, ks = batch.make_instances(torch, bto, count, 64, 2048, {kind: 1.0}, config=4)
        kb = sum(batch.alg_bytes(s.kind, s.m, s.n) for s in ks)
        kp = bto.BatchPlan(ki, use_graph=graph)
        ksec, _ = time_stats(torch, kp.launch, 5, 2)
        kp.check()
        kp.close()
        kt = bto.TiledBatch(ki, config=bto.TiledConfig.default(use_graph=1 if graph else 0))
        ktsec, _ = time_stats(torch, kt.launch, 5, 2)
        kt.close()
        one_kind[kind] = {
            "alg_gb": round(kb / 1e9, 3),
            "persistent": {"ms_per_batch": round(ksec * 1e3, 3),
                           "inst_per_s": round(count / ksec, 1),
                           "gbs": round(kb / ksec / 1e9, 1)},
            "tiled": {"ms_per_batch": round(ktsec * 1e3, 3),
                      "inst_per_s": round(count / ktsec, 1),
                      "gbs": round(kb / ktsec / 1e9, 1)},
        }
        print(f"batched: {count} {kind} instances timed", file=sys.stderr, flush=True)
        del ki, kp, kt
        torch.cuda.empty_cache()
    return {
        "instances": count,
        "gemver": sum(1 for s in specs if s.kind == "gemver"),
        "n_range": [64, 2048],
        "alg_gb": round(total / 1e9, 3),
        "ms_per_batch": round(sec * 1e3, 3),
        "min_ms": round(sec_min * 1e3, 3),
        "checked": checked and worst <= 2e-12,
        "check": "bto_batch_plan_check after the timed launches: every bounded wait of the last "
                 "launch completed; tiled outputs against persistent ones (normwise, per array)",
        "tiled_vs_persistent_max_relerr": worst,
        "inst_per_s": round(count / sec, 1),
        "gbs": round(total / sec / 1e9, 1),
        "pct_peak": round(100 * total / sec / 1e9 / PEAK_GBS, 1),
        "traffic": counter_traffic("batch_mixed4096_counters.txt") if count == 4096 else None,
        "tiled": {
            "ms_per_batch": round(sec_tiled * 1e3, 3),
            "min_ms": round(sec_tiled_min * 1e3, 3),
            "inst_per_s": round(count / sec_tiled, 1),
            "gbs": round(total / sec_tiled / 1e9, 1),
            "pct_peak": round(100 * total / sec_tiled / 1e9 / PEAK_GBS, 1),
            "speedup_vs_persistent": round(sec / sec_tiled, 3),
            "config": tiled_cfg.as_dict(),
            "launch_ms": group_ms,
            "launch_ms_how": "mean per launch of each group, HIP events around each launch, "
                             "plan run without its graph in a separate loop",
            "traffic": counter_traffic("tiled_batch_mixed4096_counters.txt")
            if count == 4096 else None,
        },
        "per_instance_loop_ms": round(sec_loop * 1e3, 2) if sec_loop else None,
        "speedup_vs_loop": round(sec_loop / sec, 2) if sec_loop else None,
        "best": {"form": "tiled" if sec_tiled < sec else "persistent",
                 "ms_per_batch": round(min(sec, sec_tiled) * 1e3, 3),
                 "inst_per_s": round(count / min(sec, sec_tiled), 1),
                 "gbs": round(total / min(sec, sec_tiled) / 1e9, 1),
                 "pct_peak": round(100 * total / min(sec, sec_tiled) / 1e9 / PEAK_GBS, 1)},
        "one_kind": one_kind,
    }


def bench_serving(torch, bto, count: int, warmup: int) -> dict:
    """Requests for BiCGK / GEMVER / ATAX (weights .4/.4/.2) over a pool of 64
    device-resident matrices with n log-uniform on [256, 16384]: all at once
    (saturated throughput), then Poisson arrivals at 0.7 of what the entry
    points alone sustain, served with continuous batching by three routes
    (tiled batches for small GEMVER/BiCGK, the default; entry points only;
    persistent batch plans) and by a one-at-a-time FIFO server.  The default
    and entry-point routes serve the same arrivals three times each,
    alternating, and report medians (run-to-run spread of p50 is ~25%)."""
    from paper_1205_1098_amd import serve

    GiB = 1 << 30
    sizes = serve.pool_sizes(64, 256, 16384)
    pool = serve.MatrixPool(torch, bto, sizes)
    total = warmup + count

    def once(executor, reqs, slots, lanes):
        executor.start()
        srv = serve.Server(executor, budget_bytes=32 * GiB, slots=slots, lanes=lanes)
        t0 = time.perf_counter()
        srv.run(reqs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = serve.summarize(reqs, warmup)
        out["wall_s"] = round(wall, 3)
        out["steps"] = srv.steps
        out["mean_step_size"] = round(float(np.mean(srv.step_sizes)), 2) if srv.step_sizes else 0
        out["peak_gib"] = round(srv.peak_bytes / GiB, 2)
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}

    # continuous batching over the single-instance entry points on two lanes
    ex = serve.GpuExecutor(torch, bto, pool, batch_n=0)
    print("serving: saturated run, entry points only", file=sys.stderr, flush=True)
    once(ex, serve.make_requests(min(total, 2000), sizes, rate=None, first_rid=900000), 64, 2)
    direct_sat = once(ex, serve.make_requests(total, sizes, rate=None), 64, 2)
    # one offered load for every route: 0.7 of what the entry points alone sustain
    lam = 0.7 * direct_sat["req_per_s"]
    print(f"serving: Poisson runs at {lam:.0f} req/s", file=sys.stderr, flush=True)
    # the default: GEMVER and BiCGK requests of n <= 2048 in refillable tiled
    # batches (one graph launch per step), the rest through the entry points
    tiled_ex = serve.GpuExecutor(torch, bto, pool)
    print("serving: runs with tiled batches", file=sys.stderr, flush=True)
    once(tiled_ex, serve.make_requests(min(total, 2000), sizes, rate=None, first_rid=800000),
         64, 2)
    sat = once(tiled_ex, serve.make_requests(total, sizes, rate=None), 64, 2)
    # the same arrivals through both routes, alternating, three times each:
    # each route reports the run of median p50 and the medians of p50 and p99
    runs = {"direct": [], "tiled": []}
    for _ in range(3):
        for name, e in (("direct", ex), ("tiled", tiled_ex)):
            runs[name].append(once(e, serve.make_requests(total, sizes, rate=lam,
                                                          first_rid=total), 64, 2))

    def median_run(rs):
        pick = sorted(rs, key=lambda r: r["p50_ms"])[len(rs) // 2]
        return dict(pick, p50_ms_median=float(np.median([r["p50_ms"] for r in rs])),
                    p99_ms_median=float(np.median([r["p99_ms"] for r in rs])),
                    p50_ms_runs=[r["p50_ms"] for r in rs], p99_ms_runs=[r["p99_ms"] for r in rs])

    direct_poisson, poisson = median_run(runs["direct"]), median_run(runs["tiled"])
    ex.close()
    lam_own = 0.7 * sat["req_per_s"]
    poisson_own = once(tiled_ex, serve.make_requests(total, sizes, rate=lam_own,
                                                     first_rid=2 * total), 64, 2)
    tiled_ex.close()
    # requests of n <= 2048 through refillable persistent plans instead
    plan_ex = serve.GpuExecutor(torch, bto, pool, batch_form="persistent")
    print("serving: runs with persistent batch plans", file=sys.stderr, flush=True)
    plan_sat = once(plan_ex, serve.make_requests(total, sizes, rate=None), 64, 2)
    plan_poisson = once(plan_ex, serve.make_requests(total, sizes, rate=lam, first_rid=total),
                        64, 2)
    plan_ex.close()
    # the same arrivals served one at a time, first come first served
    fifo_ex = serve.GpuExecutor(torch, bto, pool, lanes=1, batch_n=0)
    print("serving: one-at-a-time FIFO run", file=sys.stderr, flush=True)
    fifo = once(fifo_ex, serve.make_requests(total, sizes, rate=lam, first_rid=total), 1, 1)
    fifo_ex.close()
    res = {
        "pool": len(sizes), "pool_gb": round(pool.bytes / 1e9, 2), "n_range": [256, 16384],
        "weights": serve.WEIGHTS, "budget_gib": 32, "slots": 64, "lanes": 2,
        "requests": count, "warmup": warmup, "seed": serve.synth.SEED,
        "route": f"GEMVER/BiCGK with n <= {int(bto.batch_max_n())} in refillable tiled "
                 "batches, the rest through the fused entry points",
        "saturated": sat, "poisson_rate": round(lam, 1), "poisson": poisson,
        "poisson_own_rate": {"rate": round(lam_own, 1), "result": poisson_own},
        "entry_points_only": {"saturated": direct_sat, "poisson": direct_poisson},
        "persistent_plans": {"batch_n": int(bto.batch_max_n()), "saturated": plan_sat,
                             "poisson": plan_poisson},
        "fifo": fifo,
    }
    del pool
    return res


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of these kernels is a design note, not a measured path.", file=sys.stderr)
        return 2

    import torch

    from paper_1205_1098_amd import bto, synth

    if args.copy_probe:
        return copy_probe(torch, bto)
    if args.row_lengths:
        return row_length_probe(torch, bto)
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    shared = {}
    main_wl = Workload(torch, bto, synth, args.workload, dev, shared)

    # timed region: K fused steps and nothing else.  One HIP event is recorded
    # on torch's current stream (the stream the library launches on) between
    # steps, so step i's time is the time between events i and i + 1; the
    # headline is the median of those K times.
    for _ in range(args.warmup):
        main_wl.run("fused")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        main_wl.run("fused")
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    sec = float(np.median(step_ms)) * 1e-3

    # the dominant kernel's launch time, from a separate loop of K steps with
    # HIP events around that kernel alone (on the stream it is launched on)
    dom_name, dom_bytes = dominant(args.workload)
    if dom_name == "bicgk_fused" and bto.tune_get(bto.tune_slots().index("bicgk_rowres"), N)[0]:
        dom_name = "bicgk_rowres"   # the row-resident sweep serves fused BiCGK at this size
    bto.timing_reset()
    bto.timing_only(dom_name)
    bto.timing_enable(True)
    for _ in range(args.steps):
        main_wl.run("fused")
    torch.cuda.synchronize()
    bto.timing_enable(False)
    times = bto.timing_read()
    bto.timing_reset()
    bto.timing_only(None)

    fused_bytes = alg_bytes(args.workload, "fused")
    value = fused_bytes / sec / 1e9
    launches, total_ms = times.get(dom_name, (0, 0.0))
    dom_ms = total_ms / launches if launches else float("nan")
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = counter_traffic(f"{dom_name}_n16384_counters.txt")

    sec_unf = time_steps(torch, lambda: main_wl.run("unfused"), max(3, args.steps // 2), 2)
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "timing": {"method": "median of K per-step HIP-event intervals on the launching "
                             "stream; no other events in the timed loop",
                   "min_ms": round(min(step_ms), 4), "max_ms": round(max(step_ms), 4),
                   "wall_mean_ms": round(wall * 1e3, 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (SplitMix64 uniform[-1,1), seed 12051098), resident in HBM",
        "config": {"workload": f"{args.workload} fused FP64 n={N}" if args.workload in
                   ("gemver", "bicgk", "atax", "dgemvt") else f"{args.workload} fused FP64 N=2^26",
                   "alpha": ALPHA, "beta": BETA, "form": "fused",
                   "alg_bytes_per_step": fused_bytes},
        "pct_peak": round(100 * value / PEAK_GBS, 2),
        "unfused": {
            "ms_per_step": round(sec_unf * 1e3, 4),
            "gbs_same_bytes": round(fused_bytes / sec_unf / 1e9, 2),
            "gbs_own_bytes": round(alg_bytes(args.workload, "unfused") / sec_unf / 1e9, 2),
            "fused_speedup": round(sec_unf / sec, 3),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": round(achieved, 2),
            "peak": PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": dom_bytes,
            "avg_launch_ms": round(dom_ms, 5),
            "launches_timed": launches,
            "how": "mean of HIP-event pairs around the kernel on its stream, in a separate "
                   "loop of K steps after the headline loop",
        },
        "kernel_ms": {k: round(ms / c, 5) for k, (c, ms) in times.items() if c},
        "device": {"name": props.name, "cus": props.multi_processor_count,
                   "hbm_gib": round(props.total_memory / 2 ** 30, 1)},
    }

    if not args.no_suite:
        suite = {}
        # a second set of matrices (other streams, filled in place): the cold
        # timings alternate between the two sets, so each step reads 2 GiB
        # matrices that the 256 MB last-level cache cannot hold from the step
        # before; the warm timings re-run one set as a plain loop would
        alt = {"A": torch.empty_like(shared["A"])}
        bto.synth_fill(alt["A"], synth.stream_state(synth.SEED, synth.stream_id(3, 40)))
        for k in ("gemver", "bicgk", "atax", "dgemvt", "axpydot", "waxpby", "vadd",
                  "gemver_contracted", "batax", "dgemv", "gesummv"):
            wl = main_wl if k == args.workload else Workload(torch, bto, synth, k, dev, shared)
            wl2 = Workload(torch, bto, synth, k, dev, alt) if k in COLD else None
            ent = {}
            for form in ("fused",) if k == "gemver_contracted" else ("fused", "unfused"):
                s, smin = time_stats(torch, lambda: wl.run(form), 20, 3)
                ent[form + "_ms"] = round(s * 1e3, 4)
                ent[form + "_min_ms"] = round(smin * 1e3, 4)
                ent[form + "_gbs"] = round(alg_bytes(k, form) / s / 1e9, 1)
                if wl2 is not None:
                    flip = [0]

                    def alternate():
                        (wl if flip[0] == 0 else wl2).run(form)
                        flip[0] ^= 1
                    sc = time_steps(torch, alternate, 20, 4)
                    ent[form + "_cold_ms"] = round(sc * 1e3, 4)
                    ent[form + "_cold_gbs"] = round(alg_bytes(k, form) / sc / 1e9, 1)
            ent["fused_pct_peak"] = round(100 * ent["fused_gbs"] / PEAK_GBS, 1)
            if wl2 is not None:
                ent["fused_cold_pct_peak"] = round(100 * ent["fused_cold_gbs"] / PEAK_GBS, 1)
                if "unfused_cold_ms" in ent:
                    ent["speedup_cold"] = round(ent["unfused_cold_ms"] / ent["fused_cold_ms"], 3)
            del wl2
            if k == "gemver_contracted":
                # same x and w as GEMVER, without storing B
                g = suite["gemver"]
                ent["vs_gemver_fused"] = round(g["fused_ms"] / ent["fused_ms"], 3)
                ent["vs_gemver_unfused"] = round(g["unfused_ms"] / ent["fused_ms"], 3)
            else:
                ent["speedup"] = round(ent["unfused_ms"] / ent["fused_ms"], 3)
            suite[k] = ent
            if wl is not main_wl and k in ("axpydot", "waxpby", "vadd"):
                del wl
        alt.clear()
        result["suite"] = suite
        # BiCGK at 512 x 512 (2 MiB: resident in the caches, so not an HBM
        # figure): the entry point's fused and unfused forms, which cost
        # their launches
        ns = 512
        A5 = torch.from_numpy(synth.matrix(synth.SEED, synth.stream_id(1, 0), ns, ns)).to(dev)
        p5 = torch.from_numpy(synth.uniform(synth.SEED, synth.stream_id(1, 1), ns)).to(dev)
        r5 = torch.from_numpy(synth.uniform(synth.SEED, synth.stream_id(1, 2), ns)).to(dev)
        q5, s5 = torch.empty_like(r5), torch.empty_like(p5)
        ws5 = torch.empty(max(bto.workspace_bytes("bicgk", ns, ns, "fused"),
                              bto.workspace_bytes("bicgk", ns, ns, "unfused")),
                          dtype=torch.uint8, device=dev)
        small = {"workload": "bicgk 512x512 (cache-resident)"}
        for form in ("fused", "unfused"):
            sec5 = time_steps(torch, lambda: bto.bicgk(A5, p5, r5, form=form, q=q5, s=s5,
                                                       ws=ws5), 200, 20)
            small[form + "_us"] = round(sec5 * 1e6, 2)
            small[form + "_gbs"] = round(alg_bytes("bicgk", form, ns) / sec5 / 1e9, 1)
        small["speedup"] = round(small["unfused_us"] / small["fused_us"], 3)
        result["small_bicgk"] = small
        del A5, p5, r5, q5, s5, ws5
        result["generated"] = bench_generated(torch, bto, synth, shared, suite)

    # the STREAM probes, after the suite: the ceilings each kernel is set
    # against (kernels measured first in a run read a few per cent faster, so
    # the suite keeps that place)
    st = None
    if not args.no_stream:
        st = stream_probes(torch, bto, dev)
        result["stream"] = st
        result["pct_of_copy_probe"] = round(100 * result["value"] / st["copy_gbs"], 1)
    if st is not None:
        # each kernel against the probe of its own traffic: read-only sweeps
        # against the read probe, sweeps that also write against the copy
        # probe, three-input vector kernels against the triad
        def ceiling(k):
            if k in ("gemver",):
                return "copy"
            if k in ("axpydot", "vadd", "waxpby"):
                return "triad"
            return "read"
        for k, ent in result.get("suite", {}).items():
            probe = ceiling(k)
            ent["ceiling"] = {"probe": probe,
                              "pct": round(100 * ent["fused_gbs"] / st[probe + "_gbs"], 1)}

    shared.clear()
    del main_wl
    torch.cuda.empty_cache()
    if not args.no_suite:
        result["generated_passes"] = bench_generated_passes(torch, bto)
        torch.cuda.empty_cache()
    if not args.no_batch:
        result["batched"] = bench_batched(torch, bto, args.batch_count, not args.no_batch_loop,
                                          not args.batch_direct, not args.no_one_kind)
        torch.cuda.empty_cache()
    if not args.no_serve:
        result["serving"] = bench_serving(torch, bto, args.serve_requests, args.serve_warmup)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args.workload if args.workload in
                                              ("gemver", "bicgk", "atax", "dgemvt") else "gemver",
                                              args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
