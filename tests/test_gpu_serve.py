"""Serving on the GPU: every request's result matches the oracle, and a
request computes the same bits alone as in a mix of other requests."""

import numpy as np
import pytest

import oracle
from paper_1205_1098_amd import serve
from paper_1205_1098_amd.batch import ALPHA, BETA

pytestmark = pytest.mark.gpu

TOL = 1e-12
GiB = 1 << 30
# both sides of the batched / single-instance boundary (n <= 2048 batched)
SIZES = [256, 301, 777, 2048, 2049, 3001, 5000, 9000]


@pytest.fixture(scope="module")
def pool():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto, serve.MatrixPool(torch, bto, SIZES)


@pytest.fixture(scope="module", params=["direct", "tiled", "persistent"])
def env(pool, request):
    """Small requests through the single-instance entry points, or through
    refillable batches (n <= 2048): tiled (GEMVER and BiCGK; ATAX takes its
    entry point) or persistent plans (every kind)."""
    torch, bto, mats = pool
    route = request.param
    ex = serve.GpuExecutor(torch, bto, mats, keep_outputs=True,
                           batch_n=0 if route == "direct" else None,
                           batch_form="persistent" if route == "persistent" else "tiled")
    yield torch, bto, mats, ex
    ex.close()


def batched(ex, r):
    return r.n <= ex.batch_max and (ex.batch_form == "persistent" or r.kind != "atax")


def relerr(got, ref):
    den = float(np.max(np.abs(ref)))
    num = float(np.max(np.abs(got - ref)))
    return num / den if den > 0 else num


_host = {}


def reference(req):
    if req.pool not in _host:
        _host[req.pool] = serve.host_matrix(req.pool, req.n)
    A = _host[req.pool]
    ins = serve.host_inputs(req)
    if req.kind == "bicgk":
        return oracle.bicgk(A, *ins)
    if req.kind == "gemver":
        return oracle.gemver(A, *ins, ALPHA, BETA)
    return (oracle.atax(A, *ins),)


def serve_all(torch, ex, reqs, **kw):
    ex.start()
    srv = serve.Server(ex, budget_bytes=kw.pop("budget", 32 * GiB), **kw)
    srv.run(reqs)
    torch.cuda.synchronize()
    return srv


@pytest.mark.parametrize("rate", [None, 20000.0], ids=["burst", "poisson"])
def test_mix_matches_oracle_and_alone(env, rate):
    torch, bto, pool, ex = env
    reqs = serve.make_requests(48, SIZES, rate=rate, first_rid=1000 if rate else 0)
    print(f"serving {len(reqs)} requests, rate {rate}", flush=True)
    srv = serve_all(torch, ex, reqs, slots=32)
    assert all(r.state == "done" for r in reqs), [(r.rid, r.kind, r.n, r.state, r.error)
                                                  for r in reqs if r.state != "done"]
    # the mix really mixed: some step launched several requests together
    steps = {}
    for r in reqs:
        steps.setdefault((r.step, r.batched), []).append(r)
    assert any(len(g) > 1 for g in steps.values())
    assert all(r.batched == batched(ex, r) for r in reqs)
    if ex.batch_max:
        assert any(len(g) > 1 for (_, b), g in steps.items() if b)
    assert all(r.latency > 0 for r in reqs)
    for r in reqs:
        ref = reference(r)
        for got, want in zip(r.outputs, ref):
            assert relerr(got.cpu().numpy(), np.asarray(want)) <= TOL, (r.rid, r.kind, r.n)
    # each request alone, through a fresh server on the same executor
    for r in reqs:
        alone = serve.Request(r.rid, r.kind, r.pool, r.n, 0.0)
        serve_all(torch, ex, [alone], slots=32)
        assert alone.state == "done"
        for a, b in zip(alone.outputs, r.outputs):
            assert torch.equal(a, b), (r.rid, r.kind, r.n)


def test_budget_limits_inflight(env):
    torch, bto, pool, ex = env
    reqs = serve.make_requests(40, SIZES, rate=None, first_rid=5000)
    budget = 3 * serve.footprint("gemver", max(SIZES))
    srv = serve_all(torch, ex, reqs, slots=4, budget=budget)
    assert all(r.state == "done" for r in reqs)
    assert srv.peak_bytes <= budget and srv.peak_slots <= 4
    assert srv.used_bytes == 0 and srv.used_slots == 0
    # completion times never precede arrival or launch order within a lane
    assert all(r.done >= r.launched - 1e-3 for r in reqs)


def test_persistent_error_words_read_per_launch(pool):
    """The persistent route checks each batched launch's error word without
    synchronizing: a good launch leaves 0 in its slot, and its requests
    finish as done; every slot is returned."""
    torch, bto, mats = pool
    ex = serve.GpuExecutor(torch, bto, mats, batch_form="persistent")
    try:
        free = len(ex.free_errs)
        ex.errs.fill_(7)
        reqs = serve.make_requests(24, SIZES, rate=None, first_rid=7000)
        serve_all(torch, ex, reqs, slots=16)
        assert all(r.state == "done" for r in reqs)
        assert any(r.batched for r in reqs)
        assert len(ex.free_errs) == free
        used = [k for k in range(len(ex.errs_np)) if ex.errs_np[k] != 7]
        assert used and all(ex.errs_np[k] == 0 for k in used)
    finally:
        ex.close()
