"""A fake serving executor for the scheduler's CPU tests.

It runs on a virtual clock: a launch group occupies the (single, modelled)
device for its algorithmic bytes at a fixed bandwidth plus a fixed
overhead, groups execute in launch order, and the clock only moves when the
scheduler idles.  With `compute=True` it evaluates every request with the
oracle on the request's regenerated inputs.  It also keeps its own account
of the device memory it holds, so the tests can check the budget from the
executor's side, not only from the scheduler's bookkeeping.
"""

import math

import oracle
from paper_1205_1098_amd import serve
from paper_1205_1098_amd.batch import ALPHA, BETA


class Token:
    __slots__ = ("done", "reqs")

    def __init__(self, done, reqs):
        self.done, self.reqs = done, reqs


class FakeExecutor:
    def __init__(self, bandwidth=6.4e12, overhead=10e-6, batch_max=2048, fail_rids=(),
                 compute=False, launch_cost=0.0, device_fail_rids=()):
        self.t = 0.0
        self.device_free = 0.0
        self.bw = bandwidth
        self.overhead = overhead
        self.batch_max = batch_max
        self.fail = set(fail_rids)
        # requests whose launch completes with an error (a batched launch
        # whose error word is set): every request of that launch fails
        self.device_fail = set(device_fail_rids)
        self.compute = compute
        self.launch_cost = launch_cost
        self.open = set()
        self.live = {}            # rid -> bytes held
        self.live_bytes = 0
        self.max_live = 0
        self.launched = []        # (lane, [rids]) per launch group

    def now(self):
        return self.t

    def footprint(self, req):
        return serve.footprint(req.kind, req.n)

    def _run(self, reqs):
        start = max(self.t, self.device_free)
        cost = sum(r.bytes for r in reqs) / self.bw + self.overhead
        self.device_free = start + cost
        tok = Token(self.device_free, list(reqs))
        self.open.add(tok)
        if self.compute:
            for r in reqs:
                A = serve.host_matrix(r.pool, r.n)
                ins = serve.host_inputs(r)
                if r.kind == "bicgk":
                    r.outputs = oracle.bicgk(A, *ins)
                elif r.kind == "gemver":
                    r.outputs = oracle.gemver(A, *ins, ALPHA, BETA)
                else:
                    r.outputs = (oracle.atax(A, *ins),)
        return tok

    def launch(self, reqs, lane):
        self.t += self.launch_cost
        tokens, failed, small, large = [], [], [], []
        for r in reqs:
            assert r.rid not in self.live, "launched twice"
            self.live[r.rid] = r.footprint
            self.live_bytes += r.footprint
            self.max_live = max(self.max_live, self.live_bytes)
            if r.rid in self.fail:
                failed.append((r, "injected launch failure"))
                continue
            (small if r.n <= self.batch_max else large).append(r)
        if small:
            for r in small:
                r.batched = True
            tok = self._run(small)
            tokens.append((tok, small, ("batch", lane)))
            self.launched.append((lane, [r.rid for r in small]))
        for r in large:
            tok = self._run([r])
            tokens.append((tok, [r], ("direct", lane)))
            self.launched.append((lane, [r.rid]))
        return tokens, failed

    def poll(self, tok):
        if self.t >= tok.done:
            self.open.discard(tok)
            if any(r.rid in self.device_fail for r in tok.reqs):
                return tok.done, "a tile of the batched launch gave up waiting"
            return tok.done
        return None

    def release(self, req):
        b = self.live.pop(req.rid, None)
        if b is not None:
            self.live_bytes -= b

    def idle(self, until):
        nxt = min((t.done for t in self.open), default=math.inf)
        target = min(until, nxt)
        if target == math.inf:
            raise RuntimeError("scheduler idles with nothing in flight and nothing to come")
        self.t = max(self.t, target)
