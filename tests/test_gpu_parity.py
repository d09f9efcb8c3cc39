"""Device hierarchy vs the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import compare_hierarchy
from tests.helpers import (Q, clustered, from_positions, morton_py, particles, small_mixed_scaled,
                           uniform)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0904_3662_amd import ahf
    c = ahf.Context(0)
    yield c
    c.close()


def run_case(ctx, p, connectivity=26, labels=True):
    from paper_0904_3662_amd import ahf
    print(f"case {p.name} n={p.n} g={p.g} Lmax={p.max_levels} conn={connectivity}", flush=True)
    levels, order = oracle.build(p, connectivity=connectivity, labels=labels)
    h, dev = ahf.build_snapshot(ctx, p, labels=labels, connectivity=connectivity)
    m_max = 1.0 if p.mass is None else float(np.max(p.mass))
    compare_hierarchy(h, p.n, levels, order, m_max=m_max, labels=labels)
    h.free()
    return levels


def test_small_mixed_32k_full_parity(ctx):
    # 32^3 particles, 70% uniform + 8 NFW halos, 32^3 domain grid, 4 levels
    levels = run_case(ctx, synth.small_mixed(0))
    assert len(levels) >= 3


@pytest.mark.parametrize("conn", [26, 18, 6])
def test_clustered_connectivities(ctx, conn):
    run_case(ctx, clustered(3, 20000, n_clumps=6, spread=0.01, g=4, thr=5, max_levels=5), conn)


@pytest.mark.parametrize("seed,g,Lmax", [(1, 1, 4), (2, 2, 4), (3, 3, 3), (4, 6, 2)])
def test_uniform_various_grids(ctx, seed, g, Lmax):
    run_case(ctx, uniform(seed, 5000, g=g, thr=5, max_levels=Lmax))


def test_heavy_cells_multichunk(ctx):
    # 40000 particles in one domain cell (40 chunks of 1024) plus background
    rng = np.random.Generator(np.random.PCG64(5))
    core = np.array([0.53, 0.41, 0.77]) + rng.normal(0, 0.004, (40000, 3))
    bg = rng.random((3000, 3))
    p = from_positions(np.concatenate([core, bg]), g=3, thr=5, max_levels=6)
    p.name = "heavy"
    run_case(ctx, p)


def test_full_refinement_and_no_refinement(ctx):
    run_case(ctx, uniform(7, 3000, g=2, thr=-1.0, max_levels=3))
    run_case(ctx, uniform(8, 3000, g=4, thr=1e9, max_levels=3))


def test_per_particle_mass(ctx):
    p = clustered(9, 8000, g=3, thr=4, max_levels=4)
    p.mass = (np.random.Generator(np.random.PCG64(10)).random(p.n) + 0.5).astype(np.float32)
    run_case(ctx, p)


def test_ragged_and_tiny_inputs(ctx):
    for n in (1, 2, 63, 64, 65, 4095, 4097):
        run_case(ctx, clustered(100 + n, n, g=2, thr=2, max_levels=3))


def test_empty_input(ctx):
    run_case(ctx, particles([], [], [], g=3, thr=5, max_levels=3))


def test_coincident_chain_to_cap(ctx):
    K = 100
    x = 123457
    f = np.float32(0.375)
    p = particles([x] * K, [x + 999] * K, [x + 77777] * K, [f] * K, [f] * K, [f] * K, g=2,
                  thr=5, max_levels=19)
    run_case(ctx, p)


def sort_layout(n, key_bits):
    """(index width, number of (key, index) passes) of the device radix sort."""
    ib = 1
    while ib < 32 and (1 << ib) < n:
        ib += 1
    q = 0
    while key_bits - 8 * q > 64 - ib:
        q += 1
    return ib, q


# every pass layout of the sort: packed words from the start (q = 0), and
# one, two or three (key, index) passes before packing
@pytest.mark.parametrize("n,g,Lmax,q", [(5000, 3, 6, 0), (70000, 7, 10, 1),
                                        (100000, 7, 14, 2), (300000, 7, 14, 3)])
def test_particle_order_every_sort_layout(ctx, n, g, Lmax, q):
    from paper_0904_3662_amd import ahf
    B = g + Lmax
    assert sort_layout(n, 3 * B)[1] == q
    print(f"sort layout case n={n} B={B} q={q}", flush=True)
    rng = np.random.Generator(np.random.PCG64(n))
    X = rng.integers(0, Q, n, dtype=np.uint32)
    Y = rng.integers(0, Q, n, dtype=np.uint32)
    Z = rng.integers(0, Q, n, dtype=np.uint32)
    # a fifth of the particles repeat earlier positions: equal keys keep index order
    dup = rng.random(n) < 0.2
    src = rng.integers(0, n, n)
    for a in (X, Y, Z):
        a[dup] = a[src[dup]]
    p = particles(X, Y, Z, g=g, thr=1e30, max_levels=Lmax)
    h, _ = ahf.build_snapshot(ctx, p, labels=False)
    order = h.order_numpy(n)
    s = 21 - B
    keys = morton_py(X >> s, Y >> s, Z >> s, B)
    want = np.lexsort((np.arange(n), keys)).astype(np.uint32)
    assert np.array_equal(order, want)
    assert int(h.level_numpy(0)["cell_count"].sum()) == n
    h.free()


def test_bit_identical_reruns(ctx):
    from paper_0904_3662_amd import ahf
    p = small_mixed_scaled(4, 30000, g=4, max_levels=5)
    h1, dev = ahf.build_snapshot(ctx, p)
    h2, _ = ahf.build_snapshot(ctx, p, dev=dev)
    assert h1.num_levels() == h2.num_levels()
    for L in range(h1.num_levels()):
        a, b = h1.level_numpy(L), h2.level_numpy(L)
        for k, v in a.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, b[k]), (L, k)
            else:
                assert v == b[k], (L, k)
    h1.free()
    h2.free()


def test_invalid_coordinate_is_reported(ctx):
    from paper_0904_3662_amd import ahf
    p = uniform(11, 100, g=3, thr=5, max_levels=2)
    p.X[5] = Q  # one past the 21-bit range
    with pytest.raises(ahf.AhfError) as e:
        ahf.build_snapshot(ctx, p)
    assert e.value.code == ahf.AHF_EINVAL


def test_bad_parameters_rejected_before_launch(ctx):
    from paper_0904_3662_amd import ahf
    p = uniform(12, 100, g=3, thr=5, max_levels=2)
    dev = ahf.snapshot_to_device(p)
    for kw in (dict(g=0), dict(g=11, max_levels=0), dict(g=10, max_levels=12),
               dict(connectivity=7), dict(dom_ref=float("nan"))):
        args = dict(g=3, dom_ref=5.0, ref_ref=5.0, max_levels=2, connectivity=26)
        args.update(kw)
        with pytest.raises(ahf.AhfError) as e:
            ahf.build_hierarchy(ctx, *dev[:6], dev[6], **args)
        assert e.value.code == ahf.AHF_EINVAL


@pytest.mark.parametrize("conn", [26, 18, 6])
def test_labels_match_oracle_on_repeated_builds(ctx, conn):
    # the union-find runs concurrently; every build must give the oracle's labels
    from paper_0904_3662_amd import ahf
    p = clustered(13, 30000, n_clumps=10, spread=0.015, g=4, thr=4, max_levels=5)
    levels, order = oracle.build(p, connectivity=conn)
    dev = ahf.snapshot_to_device(p)
    for _ in range(5):
        h, _ = ahf.build_snapshot(ctx, p, connectivity=conn, dev=dev)
        compare_hierarchy(h, p.n, levels, order)
        h.free()


# every tuning gives the oracle's hierarchy (integers exactly, the field within
# tolerance): light/heavy thresholds down to a few particles per cell, and both
# level-1 batch sizes
TUNINGS = [dict(heavy_level0=4, heavy_level1=2, heavy_deeper=3, batch_level1=4,
                sort_skip_digits=1),
           dict(heavy_level0=16, heavy_level1=8, heavy_deeper=16, batch_level1=2,
                sort_skip_digits=0),
           dict(heavy_level0=64, heavy_level1=64, heavy_deeper=64, batch_level1=4,
                sort_skip_digits=-1)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=["t4-2-3-b4", "t16-8-16-b2", "t64-b4"])
def test_tunings_match_oracle(tuning):
    from paper_0904_3662_amd import ahf
    with ahf.Context(0) as c:
        c.set_tuning([(0, tuning)])
        assert c.tuning(12345) == tuning
        run_case(c, synth.small_mixed(0))
        rng = np.random.Generator(np.random.PCG64(15))
        core = np.array([0.31, 0.62, 0.18]) + rng.normal(0, 0.01, (20000, 3))
        p = from_positions(np.concatenate([core, rng.random((20000, 3))]), g=5, thr=5,
                           max_levels=6)
        p.name = "clump-on-uniform"
        run_case(c, p)
        c.set_tuning([])
        assert c.tuning(12345)["heavy_level1"] == 64


# The sort may leave the lowest key digits out and then sort every run of
# particles that only those digits order: with one and two digits left out,
# on a deep clustered input (short runs), one with 300 coincident particles
# and a tight clump (long runs, ties) and a shallow one, the oracle's
# hierarchy and particle order, ties included, synced and sized ahead.
SKIP_CASES = [
    ("clumps-8lev", lambda: clustered(51, 60000, n_clumps=6, spread=0.006, frac=0.8, g=4, thr=4,
                                      max_levels=8)),
    ("chain-ties", lambda: coincident_chain(52)),
    ("shallow", lambda: uniform(53, 20000, g=4, thr=5, max_levels=8)),
]


def coincident_chain(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = np.concatenate([np.repeat([[0.2, 0.7, 0.4]], 300, axis=0),
                          np.array([0.6, 0.3, 0.9]) + rng.normal(0, 0.002, (5000, 3)),
                          rng.random((8000, 3))]) % 1.0
    return from_positions(pts, g=3, thr=3, max_levels=9)


@pytest.mark.parametrize("skip", [1, 2])
@pytest.mark.parametrize("name,make", SKIP_CASES, ids=[c[0] for c in SKIP_CASES])
def test_sort_with_skipped_digits_matches_oracle(name, make, skip):
    from paper_0904_3662_amd import ahf
    p = make()
    levels, order = oracle.build(p)
    dev = ahf.snapshot_to_device(p)
    t = dict(heavy_level0=64, heavy_level1=64, heavy_deeper=64, batch_level1=2,
             sort_skip_digits=skip)
    with ahf.Context(0) as c:
        c.set_tuning([(0, t)])
        c.set_planning(True)
        for rep in range(2):  # synced, then sized ahead
            h, _ = ahf.build_snapshot(c, p, dev=dev)
            compare_hierarchy(h, p.n, levels, order)
            info = h.build_info()
            bits = 3 * min(p.g + p.max_levels, 21) - 8 * skip
            assert info["sort_key_bits"] == bits and info["sort_passes"] == (bits + 7) // 8
            h.free()


# Builds sized ahead (planning switched on): the second build of a snapshot
# class is enqueued with no host wait per level and gives the oracle's
# hierarchy; a plan too small for the next snapshot is detected on the device
# and that build is redone.
def test_planned_build_matches_oracle_without_host_waits():
    from paper_0904_3662_amd import ahf
    cases = [synth.small_mixed(0),
             clustered(21, 40000, n_clumps=8, spread=0.01, g=4, thr=5, max_levels=6)]
    with ahf.Context(0) as c:
        c.set_planning(True)
        for p in cases:
            levels, order = oracle.build(p)
            dev = ahf.snapshot_to_device(p)
            h1, _ = ahf.build_snapshot(c, p, dev=dev)
            i1 = h1.build_info()
            assert i1["planned"] == 0 and i1["host_waits"] >= 1
            compare_hierarchy(h1, p.n, levels, order)
            h1.free()
            for rep in range(2):
                h2, _ = ahf.build_snapshot(c, p, dev=dev)
                i2 = h2.build_info()
                assert i2["planned"] == 1 and i2["host_waits"] == 0 and i2["replanned"] == 0, i2
                compare_hierarchy(h2, p.n, levels, order)
                h2.free()


def test_plan_too_small_is_redone():
    from paper_0904_3662_amd import ahf
    # same size class and parameters, but the second snapshot refines far more
    sparse = uniform(31, 30000, g=4, thr=5, max_levels=5)
    dense = clustered(32, 30000, n_clumps=4, spread=0.004, frac=0.9, g=4, thr=5, max_levels=5)
    levels, order = oracle.build(dense)
    with ahf.Context(0) as c:
        c.set_planning(True)
        ahf.build_snapshot(c, sparse)[0].free()
        h, _ = ahf.build_snapshot(c, dense)
        info = h.build_info()
        assert info["replanned"] == 1 and info["planned"] == 0, info
        compare_hierarchy(h, dense.n, levels, order)
        h.free()
        # the plan has learned: the next build of the dense snapshot is planned
        h, _ = ahf.build_snapshot(c, dense)
        assert h.build_info()["planned"] == 1
        compare_hierarchy(h, dense.n, levels, order)
        h.free()
        # a plan deeper than the snapshot: the extra levels stay empty
        h, _ = ahf.build_snapshot(c, sparse)
        info = h.build_info()
        assert info["planned"] == 1, info
        sl, so = oracle.build(sparse)
        compare_hierarchy(h, sparse.n, sl, so)
        h.free()


def test_planned_build_with_masses_and_substructure():
    from paper_0904_3662_amd import ahf
    p = clustered(33, 20000, n_clumps=6, spread=0.01, g=4, thr=4, max_levels=5)
    p.mass = (np.random.Generator(np.random.PCG64(34)).random(p.n) + 0.5).astype(np.float32)
    levels, order = oracle.build(p)
    with ahf.Context(0) as c:
        c.set_planning(True)
        dev = ahf.snapshot_to_device(p)
        for rep in range(3):
            h, _ = ahf.build_snapshot(c, p, dev=dev, substructure=True)
            assert h.build_info()["planned"] == (1 if rep else 0)
            compare_hierarchy(h, p.n, levels, order, m_max=float(np.max(p.mass)))
            h.free()
