"""Batched workloads: many GEMVER / BiCGK / ATAX instances of uneven size.

`make_instances` builds a seeded set of instances directly in device memory
(each operand filled from its own SplitMix64 stream by the library's fill
kernel, bit-identical to `synth` on the host), so that any single instance
can be regenerated on the host for checking.  Sizes are square with n drawn
log-uniformly from [lo, hi]; kinds are drawn with the given weights.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import synth

KINDS = ("gemver", "bicgk", "atax")
ALPHA, BETA = 1.5, 0.7

# operand lengths in the entry points' argument order: "m" rows, "n" columns
IN_LENGTHS = {"gemver": ("m", "n", "m", "n", "m", "n"), "bicgk": ("n", "m"), "atax": ("n",)}
OUT_LENGTHS = {"gemver": ("n", "m"), "bicgk": ("m", "n"), "atax": ("n",)}


@dataclass
class Spec:
    """What is needed to regenerate one instance on the host."""
    index: int
    kind: str
    m: int
    n: int
    config: int
    seed: int
    data: str


def sizes_and_kinds(count: int, lo: int, hi: int, weights: dict, seed: int, config: int):
    n = synth.log_uniform_int(seed, synth.stream_id(config, 250), count, lo, hi)
    u = synth.unit_uniform(seed, synth.stream_id(config, 251), count)
    names = list(weights)
    cum = np.cumsum([weights[k] for k in names])
    cum = cum / cum[-1]
    kinds = [names[int(np.searchsorted(cum, x, side="right"))] for x in u]
    return [int(v) for v in n], kinds


def alg_bytes(kind: str, m: int, n: int, form: str = "fused") -> int:
    """Algorithmic HBM bytes of one instance (each forced matrix pass once,
    each vector once)."""
    M = m * n * 8
    if kind == "gemver":
        passes = 3 if form == "fused" else 6
        return passes * M + 8 * (3 * m + 3 * n) + 8 * (m + n)
    if kind == "bicgk":
        return (1 if form == "fused" else 2) * M + 8 * 2 * (m + n)
    return (1 if form == "fused" else 2) * M + 8 * 2 * n


def _lda(n: int) -> int:
    return max(8, (n + 7) // 8 * 8)   # rows start on 64-byte boundaries


def make_instances(torch, bto, count: int, lo: int, hi: int, weights: dict,
                   seed: int = synth.SEED, config: int = 4, form: str = "fused",
                   data: str = "uniform", device="cuda:0", in_place: bool = False,
                   shapes: list | None = None):
    """Build `count` instances on `device`; returns (instances, specs).
    With `shapes` given, instance i is shapes[i] = (m, n) instead of square
    with a drawn n (the kinds are still drawn)."""
    dev = torch.device(device)
    sizes, kinds = sizes_and_kinds(count, lo, hi, weights, seed, config)
    dims = shapes if shapes is not None else [(n, n) for n in sizes]
    instances, specs = [], []
    for idx, ((m, n), kind) in enumerate(zip(dims, kinds)):
        state = lambda op: synth.stream_state(seed, synth.stream_id(config, op, idx))
        lda = _lda(n)
        full = torch.empty((max(m, 1), lda), dtype=torch.float64, device=dev)[:m]
        A = full[:, :n]
        bto.synth_fill(A, state(0), kind=data)
        inst = {"kind": kind, "form": form, "A": A, "in": [], "out": []}
        length = {"m": m, "n": n}
        for op, ln in enumerate(IN_LENGTHS[kind], start=1):
            v = torch.empty(length[ln], dtype=torch.float64, device=dev)
            bto.synth_fill(v, state(op), kind=data)
            inst["in"].append(v)
        for ln in OUT_LENGTHS[kind]:
            inst["out"].append(torch.empty(length[ln], dtype=torch.float64, device=dev))
        if kind == "gemver":
            if in_place:
                inst["B"] = A
            else:
                inst["B"] = torch.empty((m, lda), dtype=torch.float64, device=dev)[:, :n]
            inst["alpha"], inst["beta"] = (2.0, 3.0) if data == "int" else (ALPHA, BETA)
        instances.append(inst)
        specs.append(Spec(idx, kind, m, n, config, seed, data))
    return instances, specs


def host_operands(spec: Spec):
    """Regenerate an instance's inputs on the host: (A, [inputs])."""
    sid = lambda op: synth.stream_id(spec.config, op, spec.index)
    A = synth.matrix(spec.seed, sid(0), spec.m, spec.n, kind=spec.data)
    length = {"m": spec.m, "n": spec.n}
    ins = [synth.vector(spec.seed, sid(op), length[ln], spec.data)
           for op, ln in enumerate(IN_LENGTHS[spec.kind], start=1)]
    return A, ins
