"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's formulas: they use closed forms (cell-centre
TSC weights, partition of unity, first moment), exact special cases (uniform
lattice, coincident particles, thresholds that refine nothing or everything),
invariants (mass conservation per level, count nesting, translation by a
whole domain cell, input permutation) and an independent dense brute force on
tiny inputs.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from tests.helpers import (Q, clustered, demorton_py, from_positions, morton_py,
                           particles, small_mixed_scaled, uniform)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def field_dict(lev):
    return {int(k): float(m) for k, m in zip(lev.field_key, lev.field_mass)}


def coords(key, bits):
    x, y, z = demorton_py(np.array([key], np.uint64), bits)
    return int(x[0]), int(y[0]), int(z[0])


def load_centre_fixture():
    rows = []
    with open(os.path.join(GOLD, "tsc_cell_centre.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            dx, dy, dz, num, den = (int(v) for v in line.split())
            rows.append(((dx, dy, dz), Fraction(num, den)))
    return rows


# ---------------------------------------------------------------- TSC weights

def test_cell_centre_weights_match_fixture():
    g = 3
    cx, cy, cz = 3, 5, 2
    half = 1 << (21 - g - 1)
    p = particles([cx * (Q >> g) + half], [cy * (Q >> g) + half], [cz * (Q >> g) + half],
                  g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    f = field_dict(levels[0])
    n = 1 << g
    fixture = load_centre_fixture()
    assert sum(v for _, v in fixture) == 1
    for (dx, dy, dz), v in fixture:
        k = int(morton_py([(cx + dx) % n], [(cy + dy) % n], [(cz + dz) % n], g)[0])
        assert f[k] == float(v), ((dx, dy, dz), f[k], v)
    assert sum(1 for v in f.values() if v != 0.0) == 27


def test_cell_corner_weights_half_half_zero():
    # u = 0 on every axis: cells i-1 and i get 1/2 per axis, cell i+1 gets 0
    g = 3
    c = 4
    p = particles([c * (Q >> g)], [c * (Q >> g)], [c * (Q >> g)], g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    f = field_dict(levels[0])
    nz = {k: v for k, v in f.items() if v != 0.0}
    assert len(nz) == 8
    for k, v in nz.items():
        x, y, z = coords(k, g)
        assert {x, y, z} <= {c - 1, c}
        assert v == 0.125


@pytest.mark.parametrize("seed", range(5))
def test_partition_of_unity_and_first_moment(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = 4
    pos = rng.random((1, 3))
    p = from_positions(pos, g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    lev = levels[0]
    n = 1 << g
    assert abs(lev.field_mass.sum() - 1.0) < 1e-15
    # first moment about the particle: sum_c M(c) (centre_c - x) = 0 per axis
    X = np.array([int(p.X[0]), int(p.Y[0]), int(p.Z[0])])
    f = np.array([float(p.fx[0]), float(p.fy[0]), float(p.fz[0])])
    xpos = (X + f) / float(Q >> g)  # in cell units
    home = X >> (21 - g)
    mom = np.zeros(3)
    for k, m in zip(lev.field_key, lev.field_mass):
        if m == 0.0:
            continue
        c = np.array(coords(int(k), g))
        d = (c - home + n // 2) % n - n // 2  # unwrapped offset of the cell from home
        mom += m * (home + d + 0.5 - xpos)
    assert np.all(np.abs(mom) < 1e-14), mom
    # second moment: TSC variance is 1/4 cell^2 plus the offsets' own spread
    # (sum_a w_a (a + 1/2 - u)^2 = 1/4 for every u)
    var = np.zeros(3)
    for k, m in zip(lev.field_key, lev.field_mass):
        if m == 0.0:
            continue
        c = np.array(coords(int(k), g))
        d = (c - home + n // 2) % n - n // 2
        var += m * (home + d + 0.5 - xpos) ** 2
    assert np.all(np.abs(var - 0.25) < 1e-14), var


def test_periodic_wrap_low_corner():
    # a particle in cell 0 with u < 1/2 gives weight (1-u)^2/2 per axis to cell 2^b - 1
    g = 3
    u = 0.25
    lo = int(u * (Q >> g))
    p = particles([lo], [lo], [lo], g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    f = field_dict(levels[0])
    top = (1 << g) - 1
    k = int(morton_py([top], [top], [top], g)[0])
    assert f[k] == (0.5 * (1 - u) ** 2) ** 3


def test_uniform_lattice_gives_uniform_field_exactly():
    # one particle per cell, same in-cell offset (exact binary fractions):
    # every cell receives exactly one particle mass
    g = 4
    n = 1 << g
    off = np.array([0.25, 0.625, 0.5]) * (Q >> g)
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = (ix.ravel() * (Q >> g) + off[0]).astype(np.uint32)
    Y = (iy.ravel() * (Q >> g) + off[1]).astype(np.uint32)
    Z = (iz.ravel() * (Q >> g) + off[2]).astype(np.uint32)
    p = particles(X, Y, Z, g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    assert np.all(levels[0].field_mass == 1.0)
    assert np.all(levels[0].cell_count == 1)


def test_uniform_lattice_random_offset_close():
    g = 3
    n = 1 << g
    rng = np.random.Generator(np.random.PCG64(3))
    fr = rng.random(3)
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pos = np.stack([(ix.ravel() + fr[0]) / n, (iy.ravel() + fr[1]) / n,
                    (iz.ravel() + fr[2]) / n], axis=1)
    p = from_positions(pos, g=g, thr=1e9, max_levels=0)
    levels, _ = oracle.build(p)
    assert np.max(np.abs(levels[0].field_mass - 1.0)) < 1e-14


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("maker", ["uniform", "clustered", "mixed"])
def test_mass_conservation_and_count_nesting(maker):
    if maker == "uniform":
        p = uniform(11, 3000, g=3, thr=5, max_levels=4)
    elif maker == "clustered":
        p = clustered(12, 3000, g=3, thr=5, max_levels=4)
    else:
        p = small_mixed_scaled(0, 4096, g=4, max_levels=3)
    levels, order = oracle.build(p)
    assert levels[0].cell_count.sum() == p.n
    assert levels[0].n_particles == p.n
    for lv in levels:
        tot = lv.field_mass.sum()
        assert abs(tot - lv.n_particles) <= 1e-12 * max(1, lv.n_particles)
        assert abs(lv.total_cell_mass - lv.total_particle_mass) <= 1e-12 * max(1, lv.n_particles)
        assert lv.cell_count.sum() == lv.n_particles
        # the field lives on S plus its ghost ring; every S cell is in it
        assert set(lv.cell_key.tolist()) <= set(lv.field_key.tolist())
        ghosts = set(lv.field_key[lv.field_ghost == 1].tolist())
        assert ghosts.isdisjoint(set(lv.cell_key.tolist()))
    for a, b in zip(levels[:-1], levels[1:]):
        parents = a.cell_key[a.cell_flag == 1]
        assert np.array_equal(b.cell_key.reshape(-1, 8)[:, 0] >> np.uint64(3), parents)
        assert np.array_equal(b.cell_count.reshape(-1, 8).sum(axis=1),
                              a.cell_count[a.cell_flag == 1])
        assert b.n_particles == a.cell_count[a.cell_flag == 1].sum()


def test_threshold_extremes():
    p = uniform(5, 500, g=2, thr=1e9, max_levels=3)
    levels, _ = oracle.build(p)
    assert len(levels) == 1 and levels[0].cell_flag.sum() == 0
    p = uniform(5, 500, g=2, thr=-1.0, max_levels=3)
    levels, _ = oracle.build(p)
    assert len(levels) == 4
    for L, lv in enumerate(levels):
        assert len(lv.cell_key) == 8 ** L * 2 ** (3 * 2)
        assert lv.n_particles == 500
        # the whole box is refined, so no ghost cells
        assert lv.field_ghost.sum() == 0


def test_start_is_count_of_smaller_keys_and_order_is_stable_sort():
    p = clustered(21, 2000, g=3, thr=5, max_levels=3)
    levels, order = oracle.build(p)
    B = p.g + p.max_levels
    keys = morton_py(p.X >> (21 - B), p.Y >> (21 - B), p.Z >> (21 - B), B)
    ref = np.lexsort((np.arange(p.n), keys))
    assert np.array_equal(order, ref.astype(np.uint32))
    for lv in levels:
        b = lv.bits
        ck = keys >> np.uint64(3 * (B - b))
        exp = np.searchsorted(np.sort(ck), lv.cell_key, side="left")
        assert np.array_equal(lv.cell_start, exp.astype(np.uint32))


def _level_maps(levels):
    out = []
    for lv in levels:
        x, y, z = demorton_py(lv.cell_key, lv.bits)
        cells = {(int(a), int(b), int(c)): (int(n), int(fl))
                 for a, b, c, n, fl in zip(x, y, z, lv.cell_count, lv.cell_flag)}
        fx, fy, fz = demorton_py(lv.field_key, lv.bits)
        field = {(int(a), int(b), int(c)): float(m) for a, b, c, m in
                 zip(fx, fy, fz, lv.field_mass)}
        out.append((cells, field))
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_translation_by_one_domain_cell(axis):
    # the exact form of the paper's shifted-distribution check (Sect. 3.2): a
    # whole-domain-cell shift leaves every in-cell offset unchanged, so the
    # hierarchy is the same, displaced by one cell at level 0 and 2^L at level L
    p = small_mixed_scaled(3, 3000, g=3, max_levels=3)
    levels, _ = oracle.build(p)
    q = particles(p.X.copy(), p.Y.copy(), p.Z.copy(), p.fx, p.fy, p.fz, g=p.g, thr=p.dom_ref,
                  max_levels=p.max_levels)
    arr = [q.X, q.Y, q.Z][axis]
    arr[:] = (arr.astype(np.int64) + (Q >> p.g)) % Q
    levels2, _ = oracle.build(q)
    assert len(levels) == len(levels2)
    for L, ((c1, f1), (c2, f2)) in enumerate(zip(_level_maps(levels), _level_maps(levels2))):
        n = 1 << (p.g + L)
        s = 1 << L

        def sh(t):
            t = list(t)
            t[axis] = (t[axis] + s) % n
            return tuple(t)
        assert {sh(k): v for k, v in c1.items()} == c2
        assert {sh(k): v for k, v in f1.items()} == f2
    # labels: the same partition, possibly renumbered
    for L in range(1, len(levels)):
        a, b = levels[L], levels2[L]
        xa = demorton_py(a.cell_key, a.bits)
        pa = {}
        for i in range(len(a.cell_key)):
            t = [int(xa[0][i]), int(xa[1][i]), int(xa[2][i])]
            t[axis] = (t[axis] + (1 << L)) % (1 << a.bits)
            pa[tuple(t)] = int(a.cell_patch[i])
        xb = demorton_py(b.cell_key, b.bits)
        pairs = set()
        for i in range(len(b.cell_key)):
            pairs.add((pa[(int(xb[0][i]), int(xb[1][i]), int(xb[2][i]))], int(b.cell_patch[i])))
        assert len(pairs) == a.n_patches == b.n_patches


def test_input_permutation_invariance():
    p = clustered(31, 2500, g=3, thr=5, max_levels=3)
    levels, order = oracle.build(p)
    perm = np.random.Generator(np.random.PCG64(4)).permutation(p.n)
    q = p.subset(perm)
    levels2, order2 = oracle.build(q)
    assert len(levels) == len(levels2)
    for a, b in zip(levels, levels2):
        assert np.array_equal(a.cell_key, b.cell_key)
        assert np.array_equal(a.cell_count, b.cell_count)
        assert np.array_equal(a.cell_flag, b.cell_flag)
        assert np.array_equal(a.cell_patch, b.cell_patch)
        assert np.array_equal(a.field_key, b.field_key)
        np.testing.assert_allclose(a.field_mass, b.field_mass, rtol=1e-13, atol=1e-300)
    # the permutation maps the same particles to the same runs of equal keys:
    # within a run, the stable sort of q orders them by their index in q, that
    # of p by their index in p, so the runs hold the same particles and p's
    # run is ascending
    B = p.g + p.max_levels
    k1 = morton_py(p.X >> (21 - B), p.Y >> (21 - B), p.Z >> (21 - B), B)[order]
    k2 = morton_py(q.X >> (21 - B), q.Y >> (21 - B), q.Z >> (21 - B), B)[order2]
    assert np.array_equal(k1, k2)
    assert np.any(k1[1:] == k1[:-1]), "the case should have ties"
    mapped = perm[order2].astype(np.int64)
    runs_sorted = mapped[np.lexsort((mapped, k1))]
    assert np.array_equal(runs_sorted, order.astype(np.int64))


# ---------------------------------------------------------------- special cases

def test_coincident_particles_refine_to_the_cap_as_one_chain():
    K = 20
    g, Lmax = 2, 5
    x = 123457
    f = np.float32(0.375)
    p = particles([x] * K, [x + 999] * K, [x + 77777] * K, [f] * K, [f] * K, [f] * K,
                  g=g, thr=5, max_levels=Lmax)
    levels, _ = oracle.build(p)
    assert len(levels) == Lmax + 1
    for L, lv in enumerate(levels):
        assert lv.n_particles == K
        if L < Lmax:
            assert lv.cell_flag.sum() == 1
        if L >= 1:
            assert len(lv.cell_key) == 8
            assert lv.n_patches == 1
            assert lv.patch_parent[0] == (-1 if L == 1 else 0)
            assert lv.patch_nparticles[0] == K
        # field = K times the single-particle TSC weights: 27 non-zero values
        nz = lv.field_mass[lv.field_mass != 0]
        assert len(nz) == 27
        assert abs(nz.sum() - K) < 1e-12


def test_two_far_clumps_make_two_roots():
    rng = np.random.Generator(np.random.PCG64(8))
    a = np.array([0.2, 0.2, 0.2]) + rng.normal(0, 0.003, (200, 3))
    b = np.array([0.7, 0.7, 0.7]) + rng.normal(0, 0.003, (200, 3))
    p = from_positions(np.concatenate([a, b]), g=3, thr=5, max_levels=4)
    levels, _ = oracle.build(p)
    assert levels[1].n_patches == 2
    assert list(levels[1].patch_parent) == [-1, -1]
    for lv in levels[2:]:
        assert np.all(lv.patch_parent >= 0)


def test_empty_input():
    p = particles([], [], [], g=3, thr=5, max_levels=3)
    levels, order = oracle.build(p)
    assert len(levels) == 1 and len(order) == 0
    assert levels[0].field_mass.sum() == 0.0


def test_bad_parameters_rejected():
    p = uniform(1, 10, g=3, thr=5, max_levels=3)
    with pytest.raises(ValueError):
        oracle.build(p, g=10, max_levels=12)
    with pytest.raises(ValueError):
        oracle.build(p, connectivity=7)
    with pytest.raises(ValueError):
        oracle.build(p, dom_ref=float("nan"))


# ---------------------------------------------------------------- brute force

CASES = [
    ("uniform-g1", lambda: uniform(1, 60, g=1, thr=5, max_levels=3)),
    ("uniform-g2", lambda: uniform(2, 400, g=2, thr=5, max_levels=3)),
    ("clustered-g2", lambda: clustered(3, 500, g=2, thr=5, max_levels=3, spread=0.02)),
    ("clustered-g3", lambda: clustered(4, 600, g=3, thr=3, max_levels=2, spread=0.03)),
    ("mixed-g3", lambda: small_mixed_scaled(5, 800, g=3, max_levels=3)),
    ("one-cell", lambda: from_positions(np.full((30, 3), 0.51) +
                                        np.random.Generator(np.random.PCG64(6)).normal(0, 1e-4, (30, 3)),
                                        g=2, thr=5, max_levels=3)),
    ("wrap-corner", lambda: from_positions((np.random.Generator(np.random.PCG64(7)).normal(0, 0.01, (300, 3))) % 1.0,
                                           g=2, thr=4, max_levels=3)),
    ("massive", lambda: particles(*[np.random.Generator(np.random.PCG64(9)).integers(0, Q, 300)
                                    for _ in range(3)],
                                  mass=np.random.Generator(np.random.PCG64(10)).random(300) + 0.5,
                                  g=2, thr=4, max_levels=2)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("conn", [26, 18, 6])
def test_oracle_matches_dense_brute_force(name, make, conn):
    p = make()
    levels, _ = oracle.build(p, connectivity=conn)
    bf = brute.brute(p, p.g, p.dom_ref, p.ref_ref, p.max_levels, conn=conn)
    assert len(levels) == len(bf)
    for lv, d in zip(levels, bf):
        b = lv.bits
        assert b == d["bits"]
        x, y, z = demorton_py(lv.cell_key, b)
        mask = np.zeros_like(d["inS"])
        mask[x.astype(int), y.astype(int), z.astype(int)] = True
        assert np.array_equal(mask, d["inS"])
        assert np.array_equal(lv.cell_count, d["count"][x.astype(int), y.astype(int), z.astype(int)])
        assert np.array_equal(lv.cell_flag.astype(bool), d["flag"][x.astype(int), y.astype(int), z.astype(int)])
        ex, ey, ez = (v.astype(int) for v in demorton_py(lv.field_key, b))
        emask = np.zeros_like(d["inE"])
        emask[ex, ey, ez] = True
        assert np.array_equal(emask, d["inE"])
        ref = d["mass"][ex, ey, ez]
        assert np.all(np.abs(lv.field_mass - ref) <= 1e-12 * np.maximum(ref, 1e-300) + 1e-300)
        outside = d["mass"].copy()
        outside[ex, ey, ez] = 0.0
        assert np.all(outside == 0.0)
        assert lv.n_particles == d["n_particles"]
        if lv.level >= 1:
            assert np.array_equal(lv.cell_patch, d["patch"][x.astype(int), y.astype(int), z.astype(int)])
            assert lv.n_patches == len(d["patch_minkey"])
            assert list(lv.patch_parent) == d["patch_parent"]
            for pid, mk in enumerate(d["patch_minkey"]):
                assert int(lv.cell_key[lv.cell_patch == pid].min()) == mk
            # per-patch statistics, summed cell by cell on the dense grid
            assert list(lv.patch_ncells.astype(int)) == d["patch_ncells"]
            assert list(lv.patch_nparticles.astype(int)) == d["patch_nparticles"]
            np.testing.assert_allclose(lv.patch_mass, d["patch_mass"], rtol=1e-12, atol=0)
            assert sum(d["patch_ncells"]) == len(lv.cell_key)
            assert sum(d["patch_nparticles"]) == lv.n_particles


# ---------------------------------------------------------------- probe

def test_probe_agrees_with_build_on_every_cell():
    p = small_mixed_scaled(2, 3000, g=3, max_levels=3)
    levels, _ = oracle.build(p)
    pr = oracle.Probe(p)
    for lv in levels:
        fd = field_dict(lv)
        S = set(lv.cell_key.tolist())
        for i, k in enumerate(lv.cell_key):
            r = pr.cell(lv.level, int(k))
            assert r["in_S"] and r["in_E"]
            assert r["count"] == lv.cell_count[i]
            assert r["start"] == lv.cell_start[i]
            assert r["flag"] == bool(lv.cell_flag[i])
            assert abs(r["mass"] - fd[int(k)]) <= 1e-12 * max(1.0, fd[int(k)])
        for k, m in list(fd.items())[:500]:
            r = pr.cell(lv.level, k)
            assert r["in_E"]
            assert r["in_S"] == (k in S)
            assert abs(r["mass"] - m) <= 1e-12 * max(1.0, m)
    pr.close()
