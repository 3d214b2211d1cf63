"""Batch plan validation on the host: bad instances are rejected before any
device work (fake pointers, never dereferenced)."""

import ctypes

import pytest

FAKE = 1 << 40
MB = 1 << 20


@pytest.fixture(scope="module")
def bto():
    from paper_1205_1098_amd import bto as b

    return b


def desc(bto, kind, m, n, lda, base):
    d = bto.Desc()
    d.kind = bto.KERNELS[kind]
    d.form = 0
    d.m, d.n, d.lda, d.ldb = m, n, lda, lda
    d.alpha, d.beta = 1.5, 0.7
    d.A = base
    d.B = base + 64 * MB
    for k in range(6):
        d.inp[k] = base + (128 + k) * MB
    for k in range(2):
        d.out[k] = base + (160 + k) * MB
    return d


def create(bto, descs):
    arr = (bto.Desc * len(descs))(*descs)
    plan = ctypes.c_void_p()
    cfg = bto._Config(256, 2, 0, 0)
    return bto._lib.bto_batch_plan_create(ctypes.byref(arr), len(descs), ctypes.byref(cfg),
                                          ctypes.byref(plan))


def test_max_n(bto):
    assert bto.batch_max_n() == 2048


def test_rejects_wide_instances(bto):
    assert create(bto, [desc(bto, "gemver", 10, 2049, 2050, FAKE)]) == 5


def test_rejects_odd_or_short_lda(bto):
    assert create(bto, [desc(bto, "bicgk", 10, 100, 101, FAKE)]) == 1
    assert create(bto, [desc(bto, "bicgk", 10, 100, 98, FAKE)]) == 1


def test_rejects_unsupported_kind(bto):
    d = desc(bto, "bicgk", 10, 100, 100, FAKE)
    d.kind = bto.KERNELS["vadd"]
    assert create(bto, [d]) == 5


def test_rejects_misaligned_matrix(bto):
    assert create(bto, [desc(bto, "atax", 10, 100, 100, FAKE + 8)]) == 1


def test_rejects_cross_instance_output_overlap(bto):
    a = desc(bto, "bicgk", 10, 100, 100, FAKE)
    b = desc(bto, "bicgk", 10, 100, 100, FAKE + 1024 * MB)
    b.out[0] = a.out[0] + 16          # instance 1 writes into instance 0's q
    assert create(bto, [a, b]) == 2
    c = desc(bto, "bicgk", 10, 100, 100, FAKE + 2048 * MB)
    c.out[1] = a.A                    # instance 2 writes over instance 0's matrix
    assert create(bto, [a, c]) == 2


def test_rejects_bad_config(bto):
    arr = (bto.Desc * 1)(desc(bto, "bicgk", 10, 100, 100, FAKE))
    plan = ctypes.c_void_p()
    cfg = bto._Config(384, 2, 0, 0)
    assert bto._lib.bto_batch_plan_create(ctypes.byref(arr), 1, ctypes.byref(cfg),
                                          ctypes.byref(plan)) == 1


def scratch(bto, descs, split=0):
    arr = (bto.Desc * max(len(descs), 1))(*descs)
    cfg = bto._Config(0, 0, 0, split)
    return bto._lib.bto_batch_scratch_doubles(ctypes.byref(arr), len(descs), ctypes.byref(cfg))


def test_scratch_sizes(bto):
    small = desc(bto, "gemver", 100, 100, 104, FAKE)
    assert scratch(bto, [small]) == 0                    # fits one workgroup: no tiles
    unf = desc(bto, "atax", 100, 70, 70, FAKE)
    unf.form = 1
    assert scratch(bto, [unf]) == 128                    # m rounded up to 32
    big = desc(bto, "bicgk", 20000, 2000, 2000, FAKE)    # 320 MB > 16 MiB: tiled
    rows = -(-(16 << 20) // (8 * 2000))                  # rows per 16 MiB tile
    rows = max(rows, -(-20000 // 64))
    rows = -(-rows // 8) * 8
    tiles = -(-20000 // rows)
    assert scratch(bto, [big]) == tiles * 2016           # one partial (n rounded to 32) per tile
    assert scratch(bto, [big], split=-1) == 0            # never split
    # at most 64 tiles: 20000 / 64 -> 313 rows, rounded up to 320 -> 63 tiles
    assert scratch(bto, [big], split=1 << 20) == 63 * 2016
    assert scratch(bto, [big, unf, small]) == tiles * 2016 + 128
    neg = desc(bto, "bicgk", -1, 10, 10, FAKE)
    assert scratch(bto, [neg]) == -1
    assert bto._lib.bto_batch_scratch_doubles(None, -1, None) == -1


def test_rejects_misaligned_vectors(bto):
    d = desc(bto, "gemver", 10, 100, 100, FAKE)
    d.inp[2] = d.inp[2] + 8
    assert create(bto, [d]) == 1
    d = desc(bto, "bicgk", 10, 100, 100, FAKE)
    d.out[1] = d.out[1] + 8
    assert create(bto, [d]) == 1


def test_empty_plan_argument_checks(bto):
    plan = ctypes.c_void_p()
    cfg = bto._Config(0, 0, 0, 0)
    lib = bto._lib
    assert lib.bto_batch_plan_create_empty(1 << 30, 0, ctypes.byref(cfg), ctypes.byref(plan)) == 1
    assert lib.bto_batch_plan_create_empty(-1, 0, ctypes.byref(cfg), ctypes.byref(plan)) == 1
    assert lib.bto_batch_plan_create_empty(4, -5, ctypes.byref(cfg), ctypes.byref(plan)) == 1
    assert lib.bto_batch_plan_create_empty(4, 0, ctypes.byref(cfg), None) == 1
    arr = (bto.Desc * 1)(desc(bto, "bicgk", 10, 100, 100, FAKE))
    assert lib.bto_batch_plan_reset(None, ctypes.byref(arr), 1, None) == 1
    assert lib.bto_batch_plan_launch(None, None) == 1
    assert lib.bto_batch_plan_check(None, None) == 1
    bad = bto._Config(0, 9, 0, 0)                     # more than 8 workgroups per CU
    assert lib.bto_batch_plan_create_empty(4, 0, ctypes.byref(bad), ctypes.byref(plan)) == 1


def create_tiled(bto, descs):
    arr = (bto.Desc * max(len(descs), 1))(*descs)
    plan = ctypes.c_void_p()
    return bto._lib.bto_tiled_batch_create(ctypes.byref(arr), len(descs), 0, ctypes.byref(plan))


def test_tiled_batch_validation(bto):
    """The tiled form takes fused GEMVER and BiCGK only, and checks instances
    as the persistent plan does, before any device work."""
    assert bto._lib.bto_tiled_batch_create(None, 0, 0, None) == 1          # plan is NULL
    assert create_tiled(bto, [desc(bto, "atax", 10, 100, 100, FAKE)]) == 5
    un = desc(bto, "gemver", 10, 100, 100, FAKE)
    un.form = 1
    assert create_tiled(bto, [un]) == 5
    assert create_tiled(bto, [desc(bto, "gemver", 10, 2049, 2050, FAKE)]) == 5
    assert create_tiled(bto, [desc(bto, "bicgk", 10, 100, 101, FAKE)]) == 1
    a = desc(bto, "bicgk", 10, 100, 100, FAKE)
    b = desc(bto, "bicgk", 10, 100, 100, FAKE + 1024 * MB)
    b.out[0] = a.out[0]
    assert create_tiled(bto, [a, b]) == 2
    plan = ctypes.c_void_p()
    assert bto._lib.bto_tiled_batch_create(None, -1, 0, ctypes.byref(plan)) == 1
    assert bto._lib.bto_tiled_batch_launch(None, None) == 1
    assert bto._lib.bto_tiled_batch_destroy(None) == 0


def test_tiled_batch_refuses_more_tiles_than_a_launch_indexes(bto):
    """An instance whose tiles would not fit an int launch index is refused
    before any list is built (fake, non-overlapping addresses)."""
    m, n = 1 << 40, 2048
    d = bto.Desc()
    d.kind = bto.KERNELS["gemver"]
    d.form = 0
    d.m, d.n, d.lda, d.ldb = m, n, n, n
    d.alpha, d.beta = 1.5, 0.7
    d.A = 1 << 40
    d.B = 1 << 56
    for k in range(6):
        d.inp[k] = (1 << 57) + k * (1 << 45)
    for k in range(2):
        d.out[k] = (1 << 58) + k * (1 << 45)
    assert create_tiled(bto, [d]) == 5
    assert "tiles" in bto._lib.bto_last_error().decode()


def test_tiled_config_validation(bto):
    """Configurations are checked before any device work: shapes, band
    heights (GEMVER's first sweeps, BiCGK's, the second sweeps) against the
    shapes' row groups (and at most 64 rows per wave where rows are dotted),
    workgroups per compute unit, the graph flag."""
    shapes = bto.tiled_shapes()
    assert len(shapes) == bto._lib.bto_tiled_shape_count() >= 4
    d = bto.TiledConfig.default()
    assert 0 <= d.store_shape < len(shapes) and d.use_graph == 1
    arr = (bto.Desc * 1)()
    plan = ctypes.c_void_p()
    bad = [dict(store_shape=len(shapes)), dict(wide_shape=-1), dict(narrow_shape=99),
           dict(store_rb=0), dict(bicgk_rb=0), dict(read_rb=-4), dict(narrow_n=-1),
           dict(wgs_per_cu=17),
           dict(wgs_per_cu=-1), dict(use_graph=2)]
    for s, sh in enumerate(shapes):
        wr = sh["waves_down"]
        if wr > 1:
            bad.append(dict(store_shape=s, store_rb=wr + 1))
            bad.append(dict(store_shape=s, store_rb=wr, bicgk_rb=wr + 1))
        bad.append(dict(wide_shape=s, read_rb=65 * wr))       # 65 rows per wave
        bad.append(dict(store_shape=s, store_rb=wr, bicgk_rb=65 * wr))
    for ch in bad:
        c = bto.TiledConfig.default(**ch)
        assert bto._lib.bto_tiled_batch_create_config(ctypes.byref(arr), 0, ctypes.byref(c),
                                                      ctypes.byref(plan)) == 1, ch
        assert bto._lib.bto_tiled_batch_create_empty(4, 64, 64, ctypes.byref(c),
                                                     ctypes.byref(plan)) == 1, ch
    c = bto.TiledConfig.default(wgs_per_cu=0)
    assert bto._lib.bto_tiled_batch_create_empty(4, 64, 64, ctypes.byref(c),
                                                 ctypes.byref(plan)) == 1
    assert "persistent" in bto._lib.bto_last_error().decode()
    c = bto.TiledConfig.default(wgs_per_cu=0, use_graph=0)     # sized per refill: accepted
    assert bto._lib.bto_tiled_batch_create_empty(4, 64, 64, ctypes.byref(c),
                                                 ctypes.byref(plan)) == 4   # no device here
    c = bto.TiledConfig.default(wgs_per_cu=2)
    assert bto._lib.bto_tiled_batch_create_empty(-1, 64, 64, ctypes.byref(c),
                                                 ctypes.byref(plan)) == 1
    assert bto._lib.bto_tiled_batch_create_empty(4, 64, 2049, ctypes.byref(c),
                                                 ctypes.byref(plan)) == 5
    assert bto._lib.bto_tiled_batch_reset(None, None, 0, None) == 1
    assert bto._lib.bto_tiled_shape(len(shapes), None, None, None, None) == 1
