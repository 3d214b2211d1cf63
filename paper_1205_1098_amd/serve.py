"""Serving BiCGK / GEMVER / ATAX requests with continuous batching.

Each request names a kernel and a matrix from a device-resident pool (the
use case of an iterative solver: the same A, fresh vectors each time) and
brings fresh input vectors.  The scheduler:

* admits requests in arrival order while the device memory they own
  (vectors, and GEMVER's updated matrix B) fits a byte budget and a slot is
  free.  The head of the queue is never overtaken, so no request starves; a
  request larger than the whole budget is rejected at once, and one that has
  waited longer than the time-out is failed without running;
* at every step launches all admitted requests that have not been launched
  yet: those with at most `batch_max_n` columns together, as one batch (by
  default a tiled batch: every instance cut into workgroup tiles that spread
  over the whole GPU, in one graph launch; or a persistent batched launch
  with one workgroup per instance), the others each through its
  single-instance entry point.  Steps alternate between streams (lanes), so
  a step's work overlaps the previous step's;
* takes a request's completion from an event recorded after its launch
  group: the request's latency is that event's time minus its arrival, and
  its memory and slot are released.

The batched and single-instance paths are deterministic, so a request's
result does not depend on the other requests served with it: a request
computes the same bits alone as in any mix.

The executor (device work, clock, completion) is a separate object, so the
scheduling policy is testable on the CPU with a virtual clock;
`GpuExecutor` is the one that runs the HIP library.
"""

from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import synth
from .batch import ALPHA, BETA, IN_LENGTHS, OUT_LENGTHS, alg_bytes

KINDS = ("bicgk", "gemver", "atax")
WEIGHTS = {"bicgk": 0.4, "gemver": 0.4, "atax": 0.2}
CONFIG = 5                 # stream-id namespace of the serving workload
OP_POOL, OP_REQ = 0, 1     # operand ids: pool matrices, request vectors


def _ld(n: int) -> int:
    return max(8, (n + 7) // 8 * 8)   # rows and vectors start on 64-byte boundaries


def _round512(b: int) -> int:
    return (b + 511) // 512 * 512


# ---- requests and workloads ---------------------------------------------------------

@dataclass(eq=False)
class Request:
    rid: int
    kind: str
    pool: int                  # index of the matrix in the pool
    n: int                     # the matrix is n x n
    arrival: float             # seconds on the server clock
    state: str = "new"         # pending, admitted, launched, done, failed, cancelled
    error: str | None = None
    admitted: float = math.nan
    launched: float = math.nan
    done: float = math.nan
    step: int = -1
    batched: bool = False
    footprint: int = 0
    cancel_requested: bool = False
    outputs: tuple = ()
    bufs: object = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def bytes(self) -> int:
        return alg_bytes(self.kind, self.n, self.n, "fused")


def pool_sizes(count: int, lo: int, hi: int, seed: int = synth.SEED) -> list:
    """Sizes of the matrix pool: n log-uniform on [lo, hi]."""
    return [int(v) for v in synth.log_uniform_int(seed, synth.stream_id(CONFIG, 240), count,
                                                  lo, hi)]


def make_requests(count: int, sizes: list, rate: float | None, seed: int = synth.SEED,
                  weights: dict | None = None, first_rid: int = 0) -> list:
    """`count` requests over a pool with the given sizes.  Kinds are drawn
    with `weights`, pool indices uniformly, and arrivals form a Poisson
    process of `rate` per second (all at time 0 when `rate` is None)."""
    weights = WEIGHTS if weights is None else weights
    names = list(weights)
    cum = np.cumsum([weights[k] for k in names])
    cum = cum / cum[-1]
    u_kind = synth.unit_uniform(seed, synth.stream_id(CONFIG, 241, first_rid), count)
    u_pool = synth.unit_uniform(seed, synth.stream_id(CONFIG, 242, first_rid), count)
    if rate is None:
        arrivals = np.zeros(count)
    else:
        u_gap = synth.unit_uniform(seed, synth.stream_id(CONFIG, 243, first_rid), count)
        arrivals = np.cumsum(-np.log1p(-u_gap) / rate)
    reqs = []
    for i in range(count):
        kind = names[int(np.searchsorted(cum, u_kind[i], side="right"))]
        p = min(int(u_pool[i] * len(sizes)), len(sizes) - 1)
        reqs.append(Request(first_rid + i, kind, p, sizes[p], float(arrivals[i])))
    return reqs


def footprint(kind: str, n: int) -> int:
    """Device bytes a request owns while admitted: its vectors and, for
    GEMVER, the updated matrix B."""
    ldv = _ld(n)
    vec = (len(IN_LENGTHS[kind]) + len(OUT_LENGTHS[kind])) * ldv * 8
    mat = n * _ld(n) * 8 if kind == "gemver" else 0
    return _round512(vec) + (_round512(mat) if mat else 0)


# ---- host-side regeneration (for checking results) ----------------------------------

def host_matrix(pool_index: int, n: int, seed: int = synth.SEED) -> np.ndarray:
    return synth.matrix(seed, synth.stream_id(CONFIG, OP_POOL, pool_index), n, n)


def host_inputs(req: Request, seed: int = synth.SEED) -> list:
    """The request's input vectors, in the entry point's argument order:
    input j is elements [j*n, (j+1)*n) of the request's stream."""
    sid = synth.stream_id(CONFIG, OP_REQ, req.rid)
    return [synth.uniform(seed, sid, req.n, offset=j * req.n)
            for j in range(len(IN_LENGTHS[req.kind]))]


# ---- the scheduler ------------------------------------------------------------------

class LaunchError(RuntimeError):
    pass


class Server:
    """Admission, continuous batching and completion over an executor.

    The executor provides
        now() -> float                        server clock, seconds
        launch(reqs, lane) -> (tokens, failed)
            start the requests' device work on `lane`; `tokens` are
            (token, [requests], queue) triples, `failed` (request, message)
            pairs.  Tokens of one queue complete in launch order (a queue is
            a device stream), so only the oldest of each queue is polled
        poll(token) -> float | (float, str | None) | None
                                              completion time (and an error
                                              that fails the token's requests),
                                              None if running
        release(req)                          free the request's device memory
        idle(until)                           wait (or advance a virtual clock)
                                              until `until`, a completion, or a
                                              short while, whichever is first
    """

    def __init__(self, executor, budget_bytes: int, slots: int = 64, lanes: int = 2,
                 timeout: float | None = None, max_batch: int | None = None):
        if slots < 1 or lanes < 1 or budget_bytes <= 0:
            raise ValueError("slots, lanes and budget must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.lanes = int(lanes)
        self.timeout = timeout
        self.max_batch = max_batch if max_batch is not None else self.slots
        self.pending: deque = deque()
        self.ready: list = []           # admitted, not launched
        self.inflight: dict = {}        # queue -> deque of (token, [requests])
        self.ninflight = 0
        self.used_bytes = 0
        self.used_slots = 0
        self.peak_bytes = 0
        self.peak_slots = 0
        self.steps = 0
        self.step_sizes: list = []
        self.admit_order: list = []
        self.finished: list = []

    # -- bookkeeping --
    def _finish(self, req: Request, state: str, when: float, error: str | None = None):
        req.state = state
        req.error = error
        req.done = when
        self.finished.append(req)

    def _release(self, req: Request):
        # after _finish, so the executor sees the final state
        self.ex.release(req)
        self.used_bytes -= req.footprint
        self.used_slots -= 1

    def submit(self, req: Request) -> None:
        req.footprint = self.ex.footprint(req)
        if req.footprint > self.budget:
            self._finish(req, "failed", self.ex.now(), "larger than the memory budget")
            return
        req.state = "pending"
        self.pending.append(req)

    def cancel(self, req: Request) -> None:
        """Cancel a request: at once while it waits, else when its launch
        group completes (device work cannot be recalled)."""
        if req.state == "pending":
            self.pending.remove(req)
            self._finish(req, "cancelled", self.ex.now())
        elif req.state == "admitted":
            self.ready.remove(req)
            self._finish(req, "cancelled", self.ex.now())
            self._release(req)
        elif req.state == "launched":
            req.cancel_requested = True

    # -- one scheduling pass --
    def pump(self) -> bool:
        """Complete, expire, admit and launch; True if anything changed."""
        changed = False
        now = self.ex.now()
        # completions, oldest first on each queue
        if self.ninflight:
            for dq in self.inflight.values():
                while dq:
                    token, reqs = dq[0]
                    res = self.ex.poll(token)
                    if res is None:
                        break
                    t, err = res if isinstance(res, tuple) else (res, None)
                    dq.popleft()
                    self.ninflight -= 1
                    changed = True
                    for r in reqs:
                        if err is not None:
                            self._finish(r, "failed", t, err)
                        else:
                            self._finish(r, "cancelled" if r.cancel_requested else "done", t)
                        self._release(r)
        # queue time-outs, oldest first (requests are submitted in arrival
        # order); only requests that have not started can time out
        if self.timeout is not None:
            while self.pending and now - self.pending[0].arrival > self.timeout:
                self._finish(self.pending.popleft(), "failed", now, "timed out in the queue")
                changed = True
        # admission, strictly in arrival order
        while self.pending:
            head = self.pending[0]
            if self.used_slots >= self.slots or self.used_bytes + head.footprint > self.budget:
                break
            self.pending.popleft()
            self.used_bytes += head.footprint
            self.used_slots += 1
            self.peak_bytes = max(self.peak_bytes, self.used_bytes)
            self.peak_slots = max(self.peak_slots, self.used_slots)
            head.state = "admitted"
            head.admitted = now
            self.admit_order.append(head.rid)
            self.ready.append(head)
            changed = True
        # launch everything admitted as one step
        while self.ready:
            group, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
            lane = self.steps % self.lanes
            for r in group:
                r.state, r.launched, r.step = "launched", now, self.steps
            try:
                tokens, failed = self.ex.launch(group, lane)
            except LaunchError as e:
                tokens, failed = [], [(r, str(e)) for r in group]
            for r, msg in failed:
                self._finish(r, "failed", self.ex.now(), msg)
                self._release(r)
            for token, treqs, queue in tokens:
                dq = self.inflight.get(queue)
                if dq is None:
                    dq = self.inflight[queue] = deque()
                dq.append((token, treqs))
                self.ninflight += 1
            self.step_sizes.append(len(group))
            self.steps += 1
            changed = True
        return changed

    def busy(self) -> bool:
        return bool(self.pending or self.ready or self.ninflight)

    def run(self, requests: list) -> list:
        """Serve `requests` (sorted by arrival) open-loop: each is submitted
        once the clock passes its arrival time.  Returns them, finished."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        i = 0
        total = len(reqs)
        while i < total or self.busy():
            now = self.ex.now()
            while i < total and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            if not self.pump():
                self.ex.idle(reqs[i].arrival if i < total else math.inf)
        return reqs


# ---- reports ------------------------------------------------------------------------

def summarize(reqs: list, warmup: int = 0) -> dict:
    """Latency percentiles and throughput over the requests after the first
    `warmup` (by arrival); throughput counts completions between the
    warmup-th completion and the last one."""
    done = [r for r in reqs if r.state == "done"]
    order = sorted(reqs, key=lambda r: r.arrival)
    measured = [r for r in order[warmup:] if r.state == "done"]
    out = {"requests": len(reqs), "completed": len(done),
           "failed": sum(r.state == "failed" for r in reqs),
           "cancelled": sum(r.state == "cancelled" for r in reqs)}
    if not measured:
        return out
    lat = np.array([r.latency for r in measured]) * 1e3
    ends = np.sort([r.done for r in done])
    k = min(max(warmup, 1), len(ends)) - 1
    window = ends[-1] - ends[k]
    count = len(ends) - 1 - k
    if window <= 0 or count <= 0:
        window, count = ends[-1] - min(r.arrival for r in done), len(ends)
    nbytes = sum(r.bytes for r in measured)
    span = max(r.done for r in measured) - min(r.arrival for r in measured)
    out.update({
        "measured": len(measured),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "max_ms": float(lat.max()),
        "req_per_s": count / window if window > 0 else math.nan,
        "gb_per_s": nbytes / span / 1e9 if span > 0 else math.nan,
        "batched_fraction": sum(r.batched for r in measured) / len(measured),
    })
    return out


# ---- the GPU executor ---------------------------------------------------------------

class MatrixPool:
    """Device-resident n x n matrices (row stride rounded up to 8 doubles),
    filled by the library's generator from their own streams."""

    def __init__(self, torch, bto, sizes: list, seed: int = synth.SEED, device="cuda:0"):
        self.sizes = list(sizes)
        self.mats, self.ptrs, self.lds = [], [], []
        dev = torch.device(device)
        for i, n in enumerate(self.sizes):
            full = torch.empty((n, _ld(n)), dtype=torch.float64, device=dev)
            A = full[:, :n]
            bto.synth_fill(A, synth.stream_state(seed, synth.stream_id(CONFIG, OP_POOL, i)))
            self.mats.append(A)
            self.ptrs.append(A.data_ptr())
            self.lds.append(_ld(n))
        self.bytes = sum(n * _ld(n) * 8 for n in self.sizes)


_NIN = {k: len(v) for k, v in IN_LENGTHS.items()}
_NOUT = {k: len(v) for k, v in OUT_LENGTHS.items()}


class _Bufs:
    """A request's device memory: one block of vectors (inputs, then
    outputs, each row `ldv` doubles) and GEMVER's B; addresses as ints."""
    __slots__ = ("block", "B", "ldv", "ins", "outs", "Bp")


class GpuExecutor:
    """Runs requests with libbto on the current device.

    Per request: one allocation for its vectors (plus B for GEMVER) and one
    generator launch for its inputs; then the requests of a step with at
    most `batch_max_n` columns go into a refillable batch plan (a ring of
    them per lane, so refilling one never waits for the step just launched)
    on the lane's batch stream, and the others through the fused entry
    points on the lane's direct stream, so a long batch never holds up a
    large request or the reverse.  Tiled batches (the default) take GEMVER
    and BiCGK; ATAX requests then take their entry point.  A persistent
    plan's launch is followed by an asynchronous copy of its error word, so
    a request whose batched launch gave up a bounded wait fails instead of
    returning invalid results.  Calls take device addresses directly (no
    tensor views per call).  Completion comes from pooled timing events: a
    request's finish time is the device's, not the moment the host noticed.
    """

    def __init__(self, torch, bto, pool: MatrixPool, lanes: int = 2, capacity: int = 64,
                 plans_per_lane: int = 4, batch_n: int | None = None, threads: int = 0,
                 wgs_per_cu: int = 0, seed: int = synth.SEED, keep_outputs: bool = False,
                 device="cuda:0", batch_form: str = "tiled", tiled_config=None):
        """`batch_n`: requests with at most this many columns go through the
        batch plans (None: the library's limit; 0: none).  `batch_form`:
        "tiled" (refillable tiled batches, for GEMVER and BiCGK; ATAX
        requests take their entry point) or "persistent" (refillable
        persistent plans, every kind; `threads` and `wgs_per_cu` are their
        knobs).  `tiled_config`: a TiledConfig for the tiled batches (None:
        the library's defaults, launched without a graph)."""
        self.torch, self.bto, self.pool = torch, bto, pool
        self.dev = torch.device(device)
        if self.dev.index not in (None, torch.cuda.current_device()):
            raise ValueError("the executor runs on the current device")
        if batch_form not in ("tiled", "persistent"):
            raise ValueError("batch_form must be 'tiled' or 'persistent'")
        self.seed = seed
        self.keep = keep_outputs
        self.capacity = capacity
        self.batch_form = batch_form
        limit = int(bto.batch_max_n())
        self.batch_max = limit if batch_n is None else int(batch_n)
        if not 0 <= self.batch_max <= limit:
            raise ValueError(f"batch_n must be in [0, {limit}]")
        batch = self.batch_max > 0
        self.direct = [torch.cuda.Stream(self.dev) for _ in range(lanes)]
        self.hdirect = [bto.stream_handle(st) for st in self.direct]
        self.errs = None
        if batch:
            self.bstreams = [torch.cuda.Stream(self.dev) for _ in range(lanes)]
            self.hbatch = [bto.stream_handle(st) for st in self.bstreams]
            if batch_form == "tiled":
                # launched without a graph, each refill sizes its launches and
                # skips empty groups: a step with one small request costs the
                # launches its entry point would
                cfg = tiled_config if tiled_config is not None else \
                    bto.TiledConfig.default(use_graph=0)
                self.plans = [[bto.TiledBatch.empty(capacity, self.batch_max, self.batch_max,
                                                    config=cfg, device=self.dev)
                               for _ in range(plans_per_lane)] for _ in range(lanes)]
            else:
                # scratch for the tile partials of a full plan of the largest
                # batched requests
                small = [n for n in set(pool.sizes) if n <= self.batch_max]
                per = max((bto.batch_scratch_doubles([{"kind": k, "m": n, "n": n}])
                           for k in KINDS for n in small), default=0)
                self.plans = [[bto.BatchPlan.empty(capacity, capacity * per, threads, wgs_per_cu,
                                                   True, self.dev)
                               for _ in range(plans_per_lane)] for _ in range(lanes)]
                # each launch's error word lands in its own slot of pinned
                # memory, read when the launch's event has completed
                nslots = 4096
                self.errs = torch.zeros(nslots, dtype=torch.int32, pin_memory=True)
                self.errs_np = self.errs.numpy()
                self.free_errs = list(range(nslots))
            self.descs = [[(bto.Desc * capacity)() for _ in range(plans_per_lane)]
                          for _ in range(lanes)]
        self.ring = [0] * lanes
        # the workspace a size needs is not monotone in n (it follows the
        # launch shape chosen for it): take the largest over the pool
        self.wsb = max((bto.workspace_bytes(k, n, n, "fused") for k in KINDS
                        for n in set(pool.sizes)), default=0)
        self.ws = [torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=self.dev)
                   for _ in range(lanes)]
        self.wsp = [w.data_ptr() for w in self.ws]
        self.events: list = []
        self.graveyard: list = []      # (event, bufs) of failed requests
        self.ref = torch.cuda.Event(enable_timing=True)
        self.t0 = time.perf_counter()
        self.start()

    def start(self) -> None:
        """Re-zero the clock (waits for the device to be idle)."""
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self.ref.record(self.direct[0])
        torch.cuda.synchronize(self.dev)
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def footprint(self, req: Request) -> int:
        return footprint(req.kind, req.n)

    def _event(self, stream):
        ev = self.events.pop() if self.events else self.torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        return ev

    def _alloc(self, req: Request, hstream: int) -> _Bufs:
        torch, n, kind = self.torch, req.n, req.kind
        ldv = _ld(n)
        nin, nout = _NIN[kind], _NOUT[kind]
        b = _Bufs()
        b.ldv = ldv
        b.block = torch.empty((nin + nout) * ldv, dtype=torch.float64, device=self.dev)
        base = b.block.data_ptr()
        step = 8 * ldv
        b.ins = [base + step * j for j in range(nin)]
        b.outs = [base + step * (nin + j) for j in range(nout)]
        if kind == "gemver":
            b.B = torch.empty(n * ldv, dtype=torch.float64, device=self.dev)
            b.Bp = b.B.data_ptr()
        else:
            b.B, b.Bp = None, 0
        state = synth.stream_state(self.seed, synth.stream_id(CONFIG, OP_REQ, req.rid))
        self.bto.raw.synth_fill(base, nin, n, ldv, state, hstream)
        return b

    def _desc(self, d, req: Request) -> None:
        b, n = req.bufs, req.n
        d.kind = self.bto.KERNELS[req.kind]
        d.form = 0
        d.m = d.n = n
        d.lda = self.pool.lds[req.pool]
        d.A = self.pool.ptrs[req.pool]
        if req.kind == "gemver":
            d.ldb, d.B, d.alpha, d.beta = b.ldv, b.Bp, ALPHA, BETA
        else:
            d.ldb, d.B = d.lda, None
        for j, p in enumerate(b.ins):
            d.inp[j] = p
        for j, p in enumerate(b.outs):
            d.out[j] = p

    def _direct(self, req: Request, lane: int) -> None:
        raw, b, n = self.bto.raw, req.bufs, req.n
        A, lda = self.pool.ptrs[req.pool], self.pool.lds[req.pool]
        ws, wsb, h = self.wsp[lane], self.wsb, self.hdirect[lane]
        if req.kind == "bicgk":
            raw.bicgk(n, n, A, lda, b.ins[0], b.ins[1], b.outs[0], b.outs[1], ws, wsb, 0, h)
        elif req.kind == "gemver":
            raw.gemver(n, n, ALPHA, BETA, A, lda, *b.ins, b.Bp, b.ldv, b.outs[0], b.outs[1],
                       ws, wsb, 0, h)
        else:
            raw.atax(n, n, A, lda, b.ins[0], b.outs[0], ws, wsb, 0, h)

    def _reap(self) -> None:
        self.graveyard = [(ev, b) for ev, b in self.graveyard if not ev.query()]

    def _bury(self, req: Request, stream) -> None:
        # device work may still use a failed request's buffers (its input
        # fill): free them only once the stream has passed this point
        if req.bufs is not None:
            self.graveyard.append((self._event(stream), req.bufs))
            req.bufs = None

    def launch(self, reqs: list, lane: int):
        if self.graveyard:
            self._reap()
        tokens, failed, small = [], [], []
        bst = self.bstreams[lane] if self.batch_max else None
        for r in reqs:
            is_small = r.n <= self.batch_max and (self.batch_form == "persistent" or
                                                  r.kind != "atax")
            stream = bst if is_small else self.direct[lane]
            try:
                r.bufs = self._alloc(r, self.hbatch[lane] if is_small else self.hdirect[lane])
            except Exception as e:   # allocation or generator failure
                failed.append((r, f"{type(e).__name__}: {e}"))
                self._bury(r, stream)
                continue
            if is_small:
                small.append(r)
                continue
            try:
                self._direct(r, lane)
            except Exception as e:
                failed.append((r, f"{type(e).__name__}: {e}"))
                self._bury(r, stream)
                continue
            tokens.append((self._event(stream), [r], ("direct", lane)))
        if small:
            k = self.ring[lane]
            self.ring[lane] = (k + 1) % len(self.plans[lane])
            plan, descs = self.plans[lane][k], self.descs[lane][k]
            slot = None
            try:
                for i, r in enumerate(small):
                    self._desc(descs[i], r)
                plan.reset_descs(descs, len(small), self.hbatch[lane])
                plan.launch_on(self.hbatch[lane])
                if self.errs is not None:
                    # a persistent plan's bounded waits: its error word
                    # after this launch, checked when the launch completes
                    slot = self.free_errs.pop()
                    plan.error_async(self.errs.data_ptr() + 4 * slot, self.hbatch[lane])
            except Exception as e:
                if slot is not None:
                    self.free_errs.append(slot)
                for r in small:
                    failed.append((r, f"{type(e).__name__}: {e}"))
                    self._bury(r, bst)
            else:
                for r in small:
                    r.batched = True
                ev = self._event(bst)
                tokens.append((ev if slot is None else (ev, slot), small, ("batch", lane)))
        return tokens, failed

    def poll(self, token):
        ev, slot = token if isinstance(token, tuple) else (token, None)
        if not ev.query():
            return None
        t = self.ref.elapsed_time(ev) * 1e-3
        self.events.append(ev)
        if slot is None:
            return t
        bad = int(self.errs_np[slot]) != 0
        self.free_errs.append(slot)
        if bad:
            return t, "a tile of the batched launch gave up waiting; its results are not valid"
        return t, None

    def release(self, req: Request) -> None:
        b = req.bufs
        if b is None:
            return
        if self.keep and req.state == "done":
            n, ldv = req.n, b.ldv
            nin, nout = _NIN[req.kind], _NOUT[req.kind]
            rows = b.block.view(nin + nout, ldv)
            outs = tuple(rows[nin + j, :n] for j in range(nout))
            req.outputs = ((b.B.view(n, ldv)[:, :n],) if b.B is not None else ()) + outs
        req.bufs = None

    def idle(self, until: float) -> None:
        # spin briefly: completions are polled on the next pass
        end = min(until, self.now() + 20e-6)
        while self.now() < end:
            pass

    def close(self) -> None:
        self.torch.cuda.synchronize(self.dev)
        self.graveyard = []
        if self.batch_max:
            for ring in self.plans:
                for p in ring:
                    p.close()
