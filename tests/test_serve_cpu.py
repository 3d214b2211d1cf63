"""The serving scheduler on a virtual clock (no GPU): admission by memory
budget and slots, arrival-order fairness, continuous batching, cancellation,
injected launch failures, queue time-outs, and the workload generator."""

import math

import numpy as np
import pytest

from paper_1205_1098_amd import serve, synth
from tests.serve_fake import FakeExecutor

GiB = 1 << 30


def run(reqs, ex=None, **kw):
    ex = ex or FakeExecutor()
    srv = serve.Server(ex, **kw)
    srv.run(reqs)
    return srv, ex


def test_footprint():
    # vectors rounded to 8 doubles per row; GEMVER adds its n x ld matrix
    assert serve.footprint("atax", 256) == 2 * 256 * 8
    assert serve.footprint("bicgk", 100) == serve._round512(4 * 104 * 8)
    assert serve.footprint("gemver", 16384) == 8 * 16384 * 8 + 16384 * 16384 * 8


def test_pool_sizes_log_uniform():
    sizes = np.array(serve.pool_sizes(4000, 256, 16384))
    assert sizes.min() >= 256 and sizes.max() <= 16384
    # log-uniform on [256, 16384]: median near sqrt(256 * 16384) = 2048,
    # and a quarter of the mass per factor 2.83
    assert 1800 < np.median(sizes) < 2300
    frac = np.mean(sizes <= 2048)
    assert abs(frac - 0.5) < 0.03
    assert serve.pool_sizes(64, 256, 16384) == serve.pool_sizes(64, 256, 16384)


def test_requests_mix_and_arrivals():
    sizes = serve.pool_sizes(64, 256, 16384)
    reqs = serve.make_requests(20000, sizes, rate=5000.0)
    kinds = [r.kind for r in reqs]
    for k, w in serve.WEIGHTS.items():
        assert abs(kinds.count(k) / len(kinds) - w) < 0.015
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() * 5000.0 - 1.0) < 0.03        # Poisson: mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05     # exponential: cv = 1
    assert all(r.n == sizes[r.pool] for r in reqs)
    assert [r.rid for r in reqs] == list(range(20000))
    again = serve.make_requests(20000, sizes, rate=5000.0)
    assert [(r.kind, r.pool, r.arrival) for r in again] == [(r.kind, r.pool, r.arrival)
                                                            for r in reqs]
    assert all(r.arrival == 0.0 for r in serve.make_requests(10, sizes, rate=None))


def test_host_inputs_are_consecutive_stream_slices():
    r = serve.Request(7, "gemver", 0, 33, 0.0)
    ins = serve.host_inputs(r)
    assert len(ins) == 6
    whole = synth.uniform(synth.SEED, synth.stream_id(serve.CONFIG, serve.OP_REQ, 7), 6 * 33)
    assert np.array_equal(np.concatenate(ins), whole)


def test_budget_and_slots_never_exceeded():
    sizes = serve.pool_sizes(64, 256, 16384)
    reqs = serve.make_requests(600, sizes, rate=2e5)
    budget = 5 * GiB
    srv, ex = run(reqs, budget_bytes=budget, slots=8)
    assert all(r.state == "done" for r in reqs)
    assert srv.peak_bytes <= budget and ex.max_live <= budget
    assert srv.peak_slots <= 8
    assert srv.used_bytes == 0 and srv.used_slots == 0 and ex.live_bytes == 0
    # the budget binds: without it more would have been in flight
    srv2, ex2 = run(serve.make_requests(600, sizes, rate=2e5), budget_bytes=64 * GiB, slots=8)
    assert ex2.max_live > budget


def test_admission_in_arrival_order_and_no_starvation():
    # a 2 GiB GEMVER at the head of the queue blocks the small requests
    # behind it until it fits; nothing overtakes it
    big = serve.Request(0, "gemver", 0, 16384, 0.0)
    small = [serve.Request(i, "atax", 1, 300, 1e-6 * i) for i in range(1, 40)]
    first = [serve.Request(100 + i, "gemver", 2, 12000, 0.0) for i in range(1)]
    first[0].arrival = -1e-6
    reqs = first + [big] + small
    srv, ex = run(reqs, budget_bytes=int(2.3 * GiB), slots=64)
    assert all(r.state == "done" for r in reqs)
    order = sorted(reqs, key=lambda r: r.arrival)
    assert srv.admit_order == [r.rid for r in order]
    # the big one could only start after the first GEMVER finished
    assert big.admitted >= first[0].done
    assert all(s.admitted >= big.admitted for s in small)


def test_continuous_batching_groups_pending_work():
    # requests that arrive while the host is launching a step go out
    # together in the next one
    sizes = [256, 512, 1024, 2048, 4096, 16384]
    reqs = serve.make_requests(400, sizes, rate=1e6)
    srv, ex = run(reqs, ex=FakeExecutor(launch_cost=30e-6), budget_bytes=32 * GiB, slots=64)
    assert all(r.state == "done" for r in reqs)
    assert max(srv.step_sizes) > 1
    small_groups = [g for _, g in ex.launched if len(g) > 1]
    assert small_groups, "no step batched several small requests"
    by_rid = {r.rid: r for r in reqs}
    for g in small_groups:
        assert all(by_rid[i].n <= 2048 for i in g)
    # lanes alternate by step
    lanes = {by_rid[g[0]].step % 2 == lane for lane, g in ex.launched}
    assert lanes == {True}
    # only requests larger than the batch limit go alone
    assert all(r.batched == (r.n <= 2048) for r in reqs)


def test_over_budget_request_rejected():
    reqs = [serve.Request(0, "bicgk", 0, 256, 0.0),
            serve.Request(1, "gemver", 1, 16384, 0.0),
            serve.Request(2, "atax", 0, 256, 0.0)]
    srv, ex = run(reqs, budget_bytes=1 * GiB, slots=4)
    assert [r.state for r in reqs] == ["done", "failed", "done"]
    assert "budget" in reqs[1].error
    assert 1 not in srv.admit_order


def test_injected_launch_failure_releases_resources():
    sizes = [256, 1024, 4096]
    reqs = serve.make_requests(200, sizes, rate=1e5)
    fail = {5, 17, 18, 120}
    ex = FakeExecutor(fail_rids=fail)
    srv, _ = run(reqs, ex=ex, budget_bytes=1 * GiB, slots=6)
    for r in reqs:
        if r.rid in fail:
            assert r.state == "failed" and "injected" in r.error
        else:
            assert r.state == "done"
    assert srv.used_bytes == 0 and srv.used_slots == 0
    assert ex.live_bytes == 0 and not ex.live


def test_cancellation():
    sizes = [4096]
    reqs = serve.make_requests(30, sizes, rate=None, weights={"bicgk": 1.0})
    ex = FakeExecutor()
    srv = serve.Server(ex, budget_bytes=1 * GiB, slots=2, lanes=1)
    for r in reqs:
        srv.submit(r)
    srv.pump()                      # admits and launches the first two
    assert [r.state for r in reqs[:3]] == ["launched", "launched", "pending"]
    srv.cancel(reqs[0])             # running: cancelled on completion
    srv.cancel(reqs[2])             # waiting: cancelled at once
    assert reqs[2].state == "cancelled" and reqs[2].step == -1
    while srv.busy():
        if not srv.pump():
            ex.idle(math.inf)
    assert reqs[0].state == "cancelled" and not math.isnan(reqs[0].done)
    assert all(r.state == "done" for r in reqs[1:2] + reqs[3:])
    assert srv.used_bytes == 0 and ex.live_bytes == 0


def test_queue_timeout():
    # slow device, one slot: the queue backs up and late requests time out
    sizes = [8192]
    reqs = serve.make_requests(50, sizes, rate=1e5, weights={"atax": 1.0})
    ex = FakeExecutor(bandwidth=1e11)
    per = reqs[0].bytes / 1e11
    srv, _ = run(reqs, ex=ex, budget_bytes=1 * GiB, slots=1, lanes=1, timeout=5 * per)
    states = [r.state for r in reqs]
    assert "failed" in states and "done" in states
    for r in reqs:
        if r.state == "failed":
            assert "timed out" in r.error and r.step == -1
            assert r.done - r.arrival > 5 * per
        else:
            assert r.admitted - r.arrival <= 5 * per + 1e-12
    assert srv.used_slots == 0


def test_results_follow_their_own_inputs():
    # every request's outputs are the oracle's on its own regenerated inputs
    sizes = [8, 33, 64, 130]
    reqs = serve.make_requests(40, sizes, rate=1e6)
    import oracle
    srv, _ = run(reqs, ex=FakeExecutor(compute=True, batch_max=64), budget_bytes=GiB, slots=16)
    for r in reqs:
        A = serve.host_matrix(r.pool, r.n)
        ins = serve.host_inputs(r)
        if r.kind == "atax":
            ref = (oracle.atax(A, *ins),)
        elif r.kind == "bicgk":
            ref = oracle.bicgk(A, *ins)
        else:
            ref = oracle.gemver(A, *ins, 1.5, 0.7)
        assert all(np.array_equal(a, b) for a, b in zip(r.outputs, ref))


def test_summary_statistics():
    reqs = []
    for i in range(100):
        r = serve.Request(i, "atax", 0, 256, arrival=0.001 * i)
        r.state, r.done = "done", 0.001 * i + 0.0005 + 1e-5 * i
        reqs.append(r)
    s = serve.summarize(reqs, warmup=10)
    lat = np.array([0.0005 + 1e-5 * i for i in range(10, 100)]) * 1e3
    assert s["measured"] == 90
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    ends = sorted(r.done for r in reqs)
    assert s["req_per_s"] == pytest.approx(90 / (ends[-1] - ends[9]))


def test_device_error_fails_its_launch_group():
    """A launch that completes with an error (a batched launch whose bounded
    wait gave up) fails every request of that launch, never marks them done,
    and releases their memory and slots; other launches are unaffected."""
    sizes = [300, 500, 9000]
    reqs = serve.make_requests(60, sizes, rate=None)
    bad = {r.rid for r in reqs if r.n <= 2048}
    victim = min(bad)
    ex = FakeExecutor(device_fail_rids={victim})
    srv, ex = run(reqs, ex, budget_bytes=64 * GiB, slots=8)
    failed = [r for r in reqs if r.state == "failed"]
    assert failed and all("gave up" in r.error for r in failed)
    assert any(r.rid == victim for r in failed)
    # exactly the requests launched together with the victim failed
    group = next(g for _, g in ex.launched if victim in g)
    assert {r.rid for r in failed} == set(group)
    assert all(r.state == "done" for r in reqs if r.rid not in group)
    assert srv.used_bytes == 0 and srv.used_slots == 0 and ex.live_bytes == 0
