"""bto_gemver_noalloc: GEMVER on the library's own device scratch.

Called through the C-ABI (the ctypes binding), its outputs are compared
with bto_gemver's on the same inputs (the same kernels and tile
configurations, so bitwise equal) and with the oracle (normwise relative
error <= 1e-12 per output array), on two calls in a row with the second
smaller, in both forms.  The largest size that fits its scratch runs once;
one row more is refused before anything is enqueued.
"""

import numpy as np
import pytest

import oracle
from paper_1205_1098_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
ALPHA, BETA = 1.5, 0.7
CFG = 61     # the synthetic streams of this file


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto, torch.device("cuda:0")


def relerr(got, ref):
    if ref.size == 0:
        return 0.0
    num = float(np.max(np.abs(got - ref)))
    den = float(np.max(np.abs(ref)))
    return num / den if den > 0 else num


def host_case(m, n, lda, case):
    sid = lambda op: synth.stream_id(CFG, op, case)
    A = synth.matrix(synth.SEED, sid(0), m, n, lda=lda)
    vecs = [synth.uniform(synth.SEED, sid(1 + k), m if k in (0, 2, 4) else n)
            for k in range(6)]          # u1, v1, u2, v2, y, z
    return A, vecs


def device_case(torch, dev, A, vecs, n):
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(dev)[:, :n]
    return Ad, [torch.from_numpy(v).to(dev) for v in vecs]


def nan_outputs(torch, dev, m, n, ldb):
    B = torch.full((m, ldb), float("nan"), dtype=torch.float64, device=dev)[:, :n]
    x = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    w = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
    return B, x, w


def test_scratch_limit_reported(env):
    _, bto, _ = env
    assert bto.gemver_noalloc_max_scratch_bytes() == 80 << 20
    assert bto.workspace_bytes("gemver", 16384, 16384) <= 80 << 20
    assert bto.workspace_bytes("gemver", 16385, 16384) > 80 << 20


@pytest.mark.parametrize("form", ["fused", "unfused"])
def test_two_calls_second_smaller(env, form):
    """Two calls in a row, the second on a smaller problem (so the scratch
    still holds partials of the first), each bitwise equal to bto_gemver on
    the same inputs and within 1e-12 of the oracle."""
    torch, bto, dev = env
    cases = []
    for case, (m, n, pad) in enumerate([(3001, 2500, 5), (700, 1103, 0)]):
        A, vecs = host_case(m, n, n + pad, case)
        Ad, vd = device_case(torch, dev, A, vecs, n)
        ref = bto.gemver(Ad, *vd, ALPHA, BETA, form=form)
        cases.append((m, n, A, vecs, Ad, vd, ref, nan_outputs(torch, dev, m, n, n + 2)))
    torch.cuda.synchronize()
    for m, n, A, vecs, Ad, vd, ref, got in cases:       # back to back
        bto.gemver_noalloc(Ad, *vd, ALPHA, BETA, *got, form=form)
    torch.cuda.synchronize()
    for m, n, A, vecs, Ad, vd, ref, got in cases:
        Bo, xo, wo = oracle.gemver(A, *vecs, ALPHA, BETA, lda=A.shape[1])
        for name, g, r, o in zip(("B", "x", "w"), got, ref, (Bo, xo, wo)):
            gh, rh = g.cpu().numpy(), r.cpu().numpy()
            assert np.array_equal(gh, rh), f"{form} {m}x{n} {name}: differs from bto_gemver"
            e = relerr(gh, o)
            assert e <= TOL, f"{form} {m}x{n} {name}: relerr {e:.3e} against the oracle"


def test_in_place_and_empty(env):
    """B == A (in place), then the empty extents: m = 0 gives x = z, n = 0
    gives w = 0."""
    torch, bto, dev = env
    m, n = 513, 1000
    A, vecs = host_case(m, n, n, 7)
    Bo, xo, wo = oracle.gemver(A, *vecs, ALPHA, BETA)
    Ad, vd = device_case(torch, dev, A, vecs, n)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    w = torch.empty(m, dtype=torch.float64, device=dev)
    bto.gemver_noalloc(Ad, *vd, ALPHA, BETA, Ad, x, w)
    torch.cuda.synchronize()
    for g, o in ((Ad, Bo), (x, xo), (w, wo)):
        assert relerr(g.cpu().numpy(), o) <= TOL
    z = vd[5]
    e = torch.empty((0, n), dtype=torch.float64, device=dev)
    x0 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    none = torch.empty(0, dtype=torch.float64, device=dev)
    bto.gemver_noalloc(e, none, vd[1], none, vd[3], none, z, ALPHA, BETA,
                       torch.empty((0, n), dtype=torch.float64, device=dev), x0, none)
    w0 = torch.full((m,), float("nan"), dtype=torch.float64, device=dev)
    e2 = torch.empty((m, 0), dtype=torch.float64, device=dev)
    bto.gemver_noalloc(e2, vd[0], none, vd[2], none, vd[4], none, ALPHA, BETA,
                       torch.empty((m, 0), dtype=torch.float64, device=dev), none, w0)
    torch.cuda.synchronize()
    assert torch.equal(x0, z)
    assert torch.equal(w0, torch.zeros_like(w0))


def test_largest_fitting_size(env):
    """n = m = 16384 needs exactly the scratch the library holds: bitwise
    equal to bto_gemver, integer data, so also equal to the oracle on a
    sample of rows and columns computed one by one."""
    torch, bto, dev = env
    m = n = 16384
    g = torch.Generator(device="cpu").manual_seed(5)
    Ad = torch.randint(-2, 3, (m, n), generator=g, dtype=torch.int8).to(dev).double()
    vd = [torch.randint(-2, 3, (k,), generator=g, dtype=torch.int8).to(dev).double()
          for k in (m, n, m, n, m, n)]
    ref = bto.gemver(Ad, *vd, 2.0, 3.0)
    got = nan_outputs(torch, dev, m, n, n)
    bto.gemver_noalloc(Ad, *vd, 2.0, 3.0, *got)
    torch.cuda.synchronize()
    for g_, r_ in zip(got, ref):
        assert torch.equal(g_, r_)
    del ref
    # exact sample: x_j = 3 * sum_i B_ij y_i + z_j and w_i = 2 * sum_j B_ij x_j
    B, x, w = (t.cpu().numpy() for t in got)
    u1, v1, u2, v2, y, z = (t.cpu().numpy() for t in vd)
    A = Ad.cpu().numpy()
    rows = [0, 1, 8191, 16383]
    for i in rows:
        assert np.array_equal(B[i], (A[i] + u1[i] * v1) + u2[i] * v2)
        assert w[i] == 2.0 * float(np.dot(B[i], x))
    for j in [0, 5, 12345, 16383]:
        assert x[j] == 3.0 * float(np.dot(B[:, j], y)) + z[j]


def test_too_large_refused(env):
    """One row more than fits is refused before anything is enqueued (the
    pointers are never touched)."""
    _, bto, _ = env
    fake = 1 << 40
    st = bto._lib.bto_gemver_noalloc(16385, 16384, ALPHA, BETA, fake, 16384, fake, fake, fake,
                                     fake, fake, fake, fake, 16384, fake, fake, 0, None)
    assert st == 3
    assert "scratch" in bto._lib.bto_last_error().decode()
