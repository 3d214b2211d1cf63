"""The seeded generator: published SplitMix64 values, ranges, and
independence of how the work is split into chunks and threads."""

import numpy as np

from paper_1205_1098_amd import synth


def test_splitmix64_reference_values():
    # SplitMix64 started at state 0: its first outputs, as published with the
    # reference implementation (Vigna, xoshiro/splitmix64.c)
    first = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    mixed = [synth.mix64_scalar((k + 1) * int(synth.GOLDEN)) for k in range(3)]
    assert mixed == first
    vec = synth._mix64(np.arange(1, 4, dtype=np.uint64) * synth.GOLDEN)
    assert [int(v) for v in vec] == first


def test_ranges_and_exactness():
    u = synth.uniform(1, 2, 100000)
    assert u.min() >= -1.0 and u.max() < 1.0
    # every value is an exact multiple of 2**-52
    assert np.all(np.floor(u * 2.0 ** 52) == u * 2.0 ** 52)
    assert abs(u.mean()) < 0.01
    k = synth.small_ints(1, 3, 100000)
    assert set(np.unique(k).tolist()) == {-2.0, -1.0, 0.0, 1.0, 2.0}


def test_offsets_threads_and_layouts_agree():
    n = (1 << 23) + 12345            # several chunks: the threaded path
    full = synth.uniform(9, 4, n)
    part = synth.uniform(9, 4, 1000, offset=(1 << 22) - 500)
    assert np.array_equal(full[(1 << 22) - 500:(1 << 22) + 500], part)
    A = synth.matrix(9, 4, 7, 11)
    assert np.array_equal(A.ravel(), full[:77])
    Ap = synth.matrix(9, 4, 7, 11, lda=16)
    assert np.array_equal(Ap[:, :11], A) and np.all(np.isnan(Ap[:, 11:]))


def test_streams_differ_and_sizes_log_uniform():
    a, b = synth.uniform(1, 0, 64), synth.uniform(1, 1, 64)
    assert not np.array_equal(a, b)
    n = synth.log_uniform_int(5, 6, 20000, 64, 2048)
    assert n.min() >= 64 and n.max() <= 2048
    # log-uniform: about half of the mass below the geometric mean
    assert 0.45 < np.mean(n < np.sqrt(64 * 2048)) < 0.55
