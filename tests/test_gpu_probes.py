"""The bandwidth probes (copy, read, triad): exact results on seeded data."""

import math

import numpy as np
import pytest

from paper_1205_1098_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1205_1098_amd import bto

    return torch, bto


# whole 256 KiB chunks, a ragged tail, shorter than one chunk, and empty
@pytest.mark.parametrize("n", [0, 1, 7, 32767, 32768, 32769, 3 * 32768 + 5, 1 << 20])
def test_read_probe_sum(env, n):
    """The read probe's sum of small integers is exact in any order; of
    uniform doubles it is within n ulp-sized steps of the exact sum."""
    torch, bto = env
    ints = synth.small_ints(synth.SEED, 700, n, -100, 100)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    bto.probe_read(torch.from_numpy(ints).cuda(), out)
    assert out.item() == float(ints.sum())
    uni = synth.uniform(synth.SEED, 701, n)
    bto.probe_read(torch.from_numpy(uni).cuda(), out)
    exact = math.fsum(uni)
    bound = 2.0 ** -53 * max(n, 1) * float(np.abs(uni).sum())
    assert abs(out.item() - exact) <= bound


def test_read_probe_misaligned(env):
    """A source that starts 8 bytes past a 16-byte boundary takes the
    element path."""
    torch, bto = env
    ints = synth.small_ints(synth.SEED, 702, 70001, -3, 3)
    buf = torch.from_numpy(np.concatenate([[0.0], ints])).cuda()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    bto.probe_read(buf[1:], out)
    assert out.item() == float(ints.sum())


def test_copy_and_triad(env):
    torch, bto = env
    n = 100003
    b = torch.from_numpy(synth.uniform(synth.SEED, 703, n)).cuda()
    c = torch.from_numpy(synth.uniform(synth.SEED, 704, n)).cuda()
    a = torch.full_like(b, float("nan"))
    bto.probe_copy(b, a)
    assert torch.equal(a, b)
    bto.probe_triad(a, b, c, 0.5)
    assert torch.equal(a, b + 0.5 * c)
