"""Runs a compiled specification (btoc.Program) on a ROCm device.

Every step is one call of the C library on the current torch stream: a
fused pass (``bto_pass``) or a scaled vector sum (``bto_waxpby``).  This
module only binds names to tensors, allocates what the program writes and
is not given, and evaluates the scalar coefficients (products of input
scalars and literals) on the host.
"""

from __future__ import annotations

import ctypes

import torch

from . import bto
from .btoc import AxpyDot, DotOp, LinComb, Pass, SpecError, Vadd, VecOp


def _coef(c, scalars):
    v = c[0]
    for s in c[1]:
        v *= scalars[s]
    return v


def run(prog, bound: dict, ws=None, gen=None) -> dict:
    """Enqueue the program.  `bound` maps every input to a tensor (matrices
    (m, n) float64, row-major, or column-major where the specification says
    matrix(column), i.e. unit stride down a column; vectors 1-D float64) or
    a float (scalars); an output may be bound too, to a tensor of the right
    shape and layout that receives it.  Returns the outputs by name; a
    column-major matrix is returned as an (m, n) view of its storage.

    Passes run on matrices as stored: a column-major matrix is handed to the
    library as the row-major matrix of its transpose.  `gen` = (generated
    library, its passes, genome) runs the matrix passes in a library emitted
    by btoc_gen instead of bto_pass.

    A bound output may not share memory with any bound input (an output is
    written while inputs are still read)."""
    env, scalars = {}, {}
    dev = None
    for name in prog.inputs:
        if name not in bound:
            raise SpecError(f"input {name} is not bound")
        if prog.kinds[name] == "scalar":
            scalars[name] = float(bound[name])
        else:
            t = bound[name]
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
                raise SpecError(f"{name}: expected a float64 tensor")
            want = 2 if prog.kinds[name] == "matrix" else 1
            if t.dim() != want:
                raise SpecError(f"{name}: expected a {want}-D tensor")
            dev = t.device if dev is None else dev
            env[name] = _stored(name, t, prog)
    if dev is None:
        raise SpecError("the program has no tensor input")
    given = {o: bound[o] for o in prog.outputs if o in bound}
    _check_overlaps(prog, bound, given)
    zeros = {}

    def zero(k):
        if k not in zeros:
            zeros[k] = torch.zeros(k, dtype=torch.float64, device=dev)
        return zeros[k]

    def vec_out(name, k):
        if name in env:
            t = env[name]
        elif name in given:
            t = given[name]
        else:
            t = torch.empty(k, dtype=torch.float64, device=dev)
        if t.dim() != 1 or t.numel() != k:
            raise SpecError(f"{name}: expected a vector of length {k}")
        env[name] = t
        return t

    def mat_out(name, m, n):
        t = env.get(name)
        if t is None and name in given:
            t = _stored(name, given[name], prog)
        if t is None:
            t = torch.empty((m, n), dtype=torch.float64, device=dev)
        if tuple(t.shape) != (m, n):
            raise SpecError(f"{name}: expected an ({m}, {n}) matrix")
        env[name] = t
        return t

    def get(name):
        if name not in env:
            raise SpecError(f"{name} is read before it is written")
        return env[name]

    if gen is not None:
        lib, gpasses, genome = gen
        gindex = {id(p): k for k, p in enumerate(gpasses)}
        scal = [scalars[n] for n in prog.inputs if prog.kinds[n] == "scalar"]
        scal_c = (ctypes.c_double * max(len(scal), 1))(*scal)

        def gen_ws(s, m, n):
            k = gindex[id(s)]
            return lib.workspace_bytes(k, m, n, *genome[k])

        need = max([gen_ws(s, *_shape(s, env)) for s in prog.steps
                    if isinstance(s, Pass) and s.base in env] + [1])
    else:
        need = max([bto.pass_workspace_bytes(_ops(s), *_shape(s, env)) for s in prog.steps
                    if isinstance(s, Pass) and s.base in env] + [1])
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)

    for s in prog.steps:
        if isinstance(s, VecOp):
            x, y = get(s.x), get(s.y)
            out = vec_out(s.out, x.numel())
            bto.waxpby(x, y, _coef(s.a, scalars), _coef(s.b, scalars), w=out)
            continue
        if isinstance(s, Vadd):
            a = get(s.a)
            bto.vadd(a, get(s.b), get(s.c), x=vec_out(s.out, a.numel()))
            continue
        if isinstance(s, LinComb):
            xs = [get(t) for _, t in s.terms]
            bto.lincomb(xs, [_coef(c, scalars) for c, _ in s.terms],
                        out=vec_out(s.out, xs[0].numel()))
            continue
        if isinstance(s, AxpyDot):
            w = get(s.w)
            bto.axpydot(w, get(s.v), get(s.u), _coef(s.alpha, scalars),
                        z=vec_out(s.z, w.numel()), r=vec_out(s.r, 1))
            continue
        if isinstance(s, DotOp):
            bto.dot(get(s.x), get(s.y), r=vec_out(s.r, 1))
            continue
        A = get(s.base)
        m, n = A.shape
        if gen is not None:
            k = gindex[id(s)]
            shape, rb = genome[k]
            need = gen_ws(s, m, n)
            if ws.numel() < need:
                ws = torch.empty(need, dtype=torch.uint8, device=dev)
            _gen_pass(lib, k, s, A, m, n, shape, rb, get, vec_out, mat_out, scal_c, len(scal),
                      ws, dev)
            continue
        kw = {}
        if s.store or s.contract:
            us = [get(u) for u, _ in s.terms] + [zero(m)] * (2 - len(s.terms))
            vs = [get(v) for _, v in s.terms] + [zero(n)] * (2 - len(s.terms))
            kw.update(u1=us[0], v1=vs[0], u2=us[1], v2=vs[1])
        if s.store:
            kw["B"] = mat_out(s.store, m, n)
        if s.row is not None:
            r = s.row
            kw["x"] = get(r["x"])
            if r["out"] is not None:
                kw["row_out"] = vec_out(r["out"], m)
                kw["row_scale"] = _coef(r["scale"], scalars)
                if r["add"] is not None:
                    kw["row_add"] = get(r["add"])
                    kw["row_add_scale"] = _coef(r["add_scale"], scalars)
        if s.col is not None:
            c = s.col
            if c["y"] is not None:
                kw["y"] = get(c["y"])
            kw["col_out"] = vec_out(c["out"], n)
            kw["col_scale"] = _coef(c["scale"], scalars)
            if c["add"] is not None:
                kw["col_add"] = get(c["add"])
                kw["col_add_scale"] = _coef(c["add_scale"], scalars)
        # the workspace need depends on the pass's extents, known only now
        k = bto.pass_workspace_bytes(_ops(s), m, n)
        if ws.numel() < k:
            ws = torch.empty(k, dtype=torch.uint8, device=dev)
        bto.fused_pass(_ops(s), A, ws=ws, **kw)
    return {o: (env[o].t() if o in prog.colmajor else env[o]) for o in prog.outputs}


def _gen_pass(lib, k, s, A, m, n, shape, rb, get, vec_out, mat_out, scal_c, nscal, ws, dev):
    """One pass in a generated library (btog_run_pass), operands bound by
    the pass's structure: update terms, row dots, column sums."""
    from .btoc_gen import PassArgs

    a = PassArgs()
    a.m, a.n = m, n
    a.lda = bto._check_mat(A, "A")
    a.A = A.data_ptr()
    keep = [A]
    if s.store or s.contract:
        for r, (u, v) in enumerate(s.terms):
            tu, tv = get(u), get(v)
            bto._check_vec(tu, u, dev, m)
            bto._check_vec(tv, v, dev, n)
            a.u[r], a.v[r] = tu.data_ptr(), tv.data_ptr()
            keep += [tu, tv]
    if s.store:
        B = mat_out(s.store, m, n)
        a.ldb = bto._check_mat(B, "B")
        a.B = B.data_ptr()
        keep.append(B)
    else:
        a.ldb = a.lda
    for q, r in enumerate(s.rows):
        x = get(r["x"])
        bto._check_vec(x, r["x"], dev, n)
        out = vec_out(r["out"], m)
        a.x[q], a.row_out[q] = x.data_ptr(), out.data_ptr()
        if r["add"] is not None:
            add = get(r["add"])
            bto._check_vec(add, r["add"], dev, m)
            a.row_add[q] = add.data_ptr()
    for q, c in enumerate(s.cols):
        y = get(c["y"])
        bto._check_vec(y, c["y"], dev, m)
        out = vec_out(c["out"], n)
        a.y[q], a.col_out[q] = y.data_ptr(), out.data_ptr()
        if c["add"] is not None:
            add = get(c["add"])
            bto._check_vec(add, c["add"], dev, n)
            a.col_add[q] = add.data_ptr()
    a.scalars = scal_c
    a.nscalars = nscal
    with torch.cuda.device(dev):
        st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        lib._check(lib.lib.btog_run_pass(k, ctypes.byref(a), shape, rb,
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), st))


def _span(t):
    """[lo, hi) bytes of a tensor's storage that it can touch."""
    if t.numel() == 0:
        return None
    lo = t.data_ptr()
    hi = lo + 8 * (1 + sum((d - 1) * st for d, st in zip(t.shape, t.stride())))
    return lo, hi


def _check_overlaps(prog, bound, given):
    """Refuse an output bound to memory that a bound input also uses, except
    a matrix update bound to exactly the matrix it updates (in place, as
    the library's GEMVER allows B == A)."""
    in_place = {(s.store, s.base) for s in prog.steps if isinstance(s, Pass) and s.store}
    ins = [(n, _span(bound[n])) for n in prog.inputs
           if prog.kinds[n] != "scalar" and isinstance(bound.get(n), torch.Tensor)]
    for o, t in given.items():
        if not isinstance(t, torch.Tensor):
            continue
        so = _span(t)
        if so is None:
            continue
        for n, si in ins:
            if si is None or not (si[0] < so[1] and so[0] < si[1]):
                continue
            u = bound[n]
            exact = (t.data_ptr() == u.data_ptr() and t.shape == u.shape
                     and t.stride() == u.stride())
            if (o, n) in in_place and exact:
                continue
            raise SpecError(f"output {o} shares memory with input {n}")


def _stored(name, t, prog):
    """The row-major matrix the library sweeps for matrix `name`: the tensor
    itself, or for a column-major one the transpose view of its storage."""
    if t.dim() != 2 or name not in prog.colmajor:
        return t
    m, n = t.shape
    if t.numel() > 0 and m > 1 and t.stride(0) != 1:
        raise SpecError(f"{name}: declared matrix(column) but not stored by columns")
    return t.t()


def _shape(s, env):
    return tuple(env[s.base].shape)


def _ops(s: Pass) -> int:
    ops = 0
    if s.row is not None:
        ops |= bto.PASS_ROWDOT
    if s.col is not None:
        ops |= bto.PASS_COLSUM
    if s.store:
        ops |= bto.PASS_STORE
    if s.contract:
        ops |= bto.PASS_CONTRACT
    if s.chain:
        ops |= bto.PASS_CHAIN
    return ops


def search(text: str, bound: dict, reps: int = 5, warmup: int = 1, ws=None):
    """Empirical search over the fusion decisions (the paper's search,
    Section IV, over this compiler's choices): compile every distinct
    schedule that switching decisions off gives, plus the unfused form,
    time each on the bound inputs (HIP events on the current stream, `reps`
    runs after `warmup`), and return (fastest program, [(decisions off,
    schedule, ms per run)]).  Every variant computes the same outputs."""
    import itertools

    from .btoc import DECISIONS, compile_spec

    variants, seen = [], set()
    for k in range(len(DECISIONS) + 1):
        for off in itertools.combinations(DECISIONS, k):
            prog = compile_spec(text, "fused", off)
            key = tuple(prog.describe())
            if key not in seen:
                seen.add(key)
                variants.append((off, prog))
    unf = compile_spec(text, "unfused")
    if tuple(unf.describe()) not in seen:
        variants.append(("unfused", unf))
    table = []
    for off, prog in variants:
        for _ in range(warmup):
            prog.run(ws=ws, **bound)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            prog.run(ws=ws, **bound)
        e1.record()
        e1.synchronize()
        table.append((off, prog.describe(), e0.elapsed_time(e1) / reps, prog))
    best = min(table, key=lambda t: t[2])
    return best[3], [(off, d, ms) for off, d, ms, _ in table]


class Captured:
    """A compiled program captured once in a HIP graph on fixed tensors.

    `replay()` enqueues every pass of the program as one graph launch on the
    current stream.  The tensors bound at capture are the program's inputs
    and outputs from then on: to run on new data, copy it into them first.
    Scalars are taken at capture.  Temporaries and the workspace belong to
    the capture and stay allocated with it."""

    def __init__(self, prog, bound: dict, ws=None):
        first = run(prog, bound, ws)                    # outputs allocated eagerly
        self.bound = dict(bound)
        self.bound.update(first)
        self.outputs = first
        dev = next(t.device for t in first.values())
        if ws is None:
            need = max([bto.pass_workspace_bytes(_ops(s), *_shape(s, _env_of(prog, self.bound)))
                        for s in prog.steps if isinstance(s, Pass)] + [1])
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.ws = ws
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            run(prog, self.bound, self.ws)              # warm-up off the capture
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            run(prog, self.bound, self.ws)

    def replay(self) -> dict:
        self.graph.replay()
        return self.outputs


def _env_of(prog, bound):
    """Stored views of the bound matrices (for workspace sizing)."""
    return {k: _stored(k, v, prog) for k, v in bound.items() if isinstance(v, torch.Tensor)}
