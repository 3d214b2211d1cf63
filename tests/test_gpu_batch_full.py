"""The batched workload at the size the benchmark times: 4096 fused GEMVER /
BiCGK instances (kinds by a fair seeded coin, n log-uniform on [64, 2048],
seed 12051098), in one persistent graph-captured launch with the default
configuration and as a tiled batch (four graph-captured launches).

Every instance that the persistent plan cuts into row tiles (matrix above
16 MiB) and a seeded sample of 64 others are compared with the oracle:
within 1e-12 (normwise per output) for uniform data, bitwise for integer
data.  The outputs are copied to the host after the same launches the
benchmark times (a graph replay after warm-up launches), and the plan's
bounded waits are checked."""

import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from paper_1205_1098_amd import batch, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
COUNT = 4096
WEIGHTS = {"gemver": 0.5, "bicgk": 0.5}
SPLIT_BYTES = 16 << 20      # the persistent plan's default row-tile threshold
SAMPLE = 64


def relerr(got, ref):
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    return num / den if den > 0 else num


def checked_indices(specs):
    split = [s.index for s in specs if s.m * s.n * 8 > SPLIT_BYTES]
    rest = np.array([s.index for s in specs if s.m * s.n * 8 <= SPLIT_BYTES])
    pick = synth.unit_uniform(synth.SEED, synth.stream_id(4, 252), SAMPLE)
    sample = sorted({int(rest[int(u * len(rest))]) for u in pick})
    return split, sample


def reference(spec, alpha, beta):
    A, ins = batch.host_operands(spec)
    if spec.kind == "gemver":
        B, x, w = oracle.gemver(A, *ins, alpha, beta)
        return [x, w], B
    return list(oracle.bicgk(A, *ins)), None


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto


def run_both(torch, bto, data):
    """Build the workload, run both forms as the benchmark does, and return
    (specs, checked indices, {form: {index: host outputs}}, alpha, beta)."""
    insts, specs = batch.make_instances(torch, bto, COUNT, 64, 2048, WEIGHTS, config=4,
                                        data=data)
    assert [s.n for s in specs] == batch.sizes_and_kinds(COUNT, 64, 2048, WEIGHTS, synth.SEED,
                                                         4)[0]
    split, sample = checked_indices(specs)
    assert len(split) > 300 and len(sample) >= SAMPLE - 4
    want = split + sample
    got = {}

    def grab():
        out = {}
        for k in want:
            inst = insts[k]
            vecs = [t.cpu().numpy() for t in inst["out"]]
            B = inst["B"].cpu().numpy() if inst["kind"] == "gemver" else None
            out[k] = (vecs, B)
        return out

    def poison():
        for inst in insts:
            for t in inst["out"]:
                t.fill_(float("nan"))
            if inst["kind"] == "gemver":
                inst["B"].fill_(float("nan"))

    poison()
    plan = bto.BatchPlan(insts)            # the benchmark's configuration
    for _ in range(3):
        plan.launch()
    plan.check()
    got["persistent"] = grab()
    plan.close()
    poison()
    tiled = bto.TiledBatch(insts)
    for _ in range(3):
        tiled.launch()
    torch.cuda.synchronize()
    got["tiled"] = grab()
    tiled.close()
    alpha, beta = (2.0, 3.0) if data == "int" else (batch.ALPHA, batch.BETA)
    del insts
    torch.cuda.empty_cache()
    return specs, want, got, alpha, beta


@pytest.mark.parametrize("data", ["uniform", "int"])
def test_bench_batch_against_oracle(env, data):
    torch, bto = env
    specs, want, got, alpha, beta = run_both(torch, bto, data)
    print(f"config 4 ({data}): checking {len(want)} of {COUNT} instances", flush=True)

    def check(k):
        spec = specs[k]
        outs, B = reference(spec, alpha, beta)
        bad = []
        for form, res in got.items():
            vecs, gB = res[k]
            for j, (g, r) in enumerate(zip(vecs, outs)):
                ok = np.array_equal(g, r) if data == "int" else relerr(g, r) <= TOL
                if not ok:
                    bad.append((form, k, spec.kind, spec.n, f"out{j}", relerr(g, r)))
            if B is not None:
                ok = np.array_equal(gB, B) if data == "int" else relerr(gB, B) <= TOL
                if not ok:
                    bad.append((form, k, spec.kind, spec.n, "B", relerr(gB, B)))
        return bad

    with cf.ThreadPoolExecutor(16) as ex:
        bad = [b for res in ex.map(check, want) for b in res]
    assert not bad, bad[:10]
