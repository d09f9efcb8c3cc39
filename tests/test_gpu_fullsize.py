"""Full-size device builds (the 16.8M and 134M workloads, in the launch
configuration bench.py times) checked against the oracle one cell at a time
and against invariants that hold at any size."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import ABS_FLOOR, REL_TOL, brick_cells
from tests.helpers import demorton_py, morton_py

pytestmark = pytest.mark.gpu

N_SAMPLE = int(os.environ.get("AHF_FULLSIZE_SAMPLES", "250"))


@pytest.fixture(scope="module")
def ctx():
    from paper_0904_3662_amd import ahf
    c = ahf.Context(0)
    yield c
    c.close()


def neighbour_keys(keys, bits, dx, dy, dz):
    x, y, z = demorton_py(keys, bits)
    m = np.uint64((1 << bits) - 1)
    def sh(a, d):
        return ((a.astype(np.int64) + d) & int(m)).astype(np.uint64)
    return morton_py(sh(x, dx), sh(y, dy), sh(z, dz), bits)


def adjacency_components(keys, bits, conn=26):
    """Connected components of the cells `keys` (sorted) with scipy: returns
    the component of every cell, numbered by smallest key."""
    n = len(keys)
    rows, cols = [], []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                s = abs(dx) + abs(dy) + abs(dz)
                if s == 0 or (conn == 6 and s > 1) or (conn == 18 and s > 2):
                    continue
                if (dx, dy, dz) < (0, 0, 0):
                    continue
                nk = neighbour_keys(keys, bits, dx, dy, dz)
                pos = np.searchsorted(keys, nk)
                pos = np.minimum(pos, n - 1)
                hit = keys[pos] == nk
                rows.append(np.nonzero(hit)[0])
                cols.append(pos[hit])
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    g = sp.coo_matrix((np.ones(len(r), np.int8), (r, c)), shape=(n, n)).tocsr()
    ncomp, lab = connected_components(g, directed=False)
    # renumber by smallest member (cells are in key order)
    first = np.full(ncomp, n, np.int64)
    np.minimum.at(first, lab, np.arange(n))
    order = np.argsort(first)
    rank = np.empty(ncomp, np.int64)
    rank[order] = np.arange(ncomp)
    return rank[lab], ncomp


def check_fullsize(ctx, snap, seed):
    from paper_0904_3662_amd import ahf
    print(f"full-size case {snap.name}: n={snap.n}", flush=True)
    h, dev = ahf.build_snapshot(ctx, snap)
    nlev = h.num_levels()
    levels = [h.level_numpy(L) for L in range(nlev)]
    order = h.order_numpy(snap.n)
    print(f"built {nlev} levels", flush=True)
    rng = np.random.Generator(np.random.PCG64(seed))

    # particle order: a permutation, keys non-decreasing, ties by input index
    B = snap.g + snap.max_levels
    assert np.array_equal(np.sort(order), np.arange(snap.n, dtype=np.uint32))
    keys = morton_py(snap.X[order] >> (21 - B), snap.Y[order] >> (21 - B),
                     snap.Z[order] >> (21 - B), B)
    dk = np.diff(keys.astype(np.uint64))
    assert np.all(keys[1:] >= keys[:-1])
    tie = keys[1:] == keys[:-1]
    assert np.all(order[1:][tie] > order[:-1][tie])
    del dk

    # invariants on every level
    assert levels[0]["n_particles"] == snap.n
    for L, d in enumerate(levels):
        assert int(d["cell_count"].sum()) == d["n_particles"]
        assert abs(d["total_cell_mass"] - d["total_particle_mass"]) <= 1e-6 * max(1.0, d["total_particle_mass"])
        assert d["total_particle_mass"] == float(d["n_particles"])
        if L + 1 < nlev:
            e = levels[L + 1]
            ref = d["cell_key"][d["cell_refined"] == 1]
            assert np.array_equal(e["cell_key"].reshape(-1, 8)[:, 0] >> np.uint64(3), ref)
            assert np.array_equal(e["cell_count"].reshape(-1, 8).sum(axis=1).astype(np.int64),
                                  d["cell_count"][d["cell_refined"] == 1].astype(np.int64))
        else:
            assert d["n_refined"] == 0
    print("invariants ok", flush=True)

    # sampled cells against the oracle, one by one
    probe = oracle.Probe(snap)
    for L, d in enumerate(levels):
        nS = len(d["cell_key"])
        bkeys, bvals = brick_cells(d)
        for i in rng.choice(nS, size=min(N_SAMPLE, nS), replace=False):
            k = int(d["cell_key"][i])
            r = probe.cell(L, k)
            assert r["in_S"], (L, k)
            assert r["count"] == int(d["cell_count"][i]), (L, k)
            assert r["start"] == int(d["cell_start"][i]), (L, k)
            assert r["flag"] == bool(d["cell_refined"][i]), (L, k)
        for j in rng.choice(len(bkeys), size=min(N_SAMPLE, len(bkeys)), replace=False):
            k = int(bkeys[j])
            r = probe.cell(L, k)
            got = float(bvals[j])
            if not r["in_E"]:
                assert got == 0.0, (L, k, got)
            else:
                assert abs(got - r["mass"]) <= REL_TOL * r["mass"] + ABS_FLOOR, (L, k, got, r["mass"])
        print(f"level {L}: sampled cells match the oracle", flush=True)
    probe.close()

    # labels: the exact partition into connected components
    for L in range(1, nlev):
        d = levels[L]
        keys_L = d["cell_key"]
        if len(keys_L) <= 2_000_000:
            comp, ncomp = adjacency_components(keys_L, d["bits"])
            assert ncomp == d["n_patches"], (L, ncomp, d["n_patches"])
            assert np.array_equal(comp, d["cell_patch"].astype(np.int64)), L
        else:
            # a level this large is checked on its refined parents, whose
            # components lifted to their children are those of S_L
            pv = levels[L - 1]
            pk = pv["cell_key"][pv["cell_refined"] == 1]
            comp, ncomp = adjacency_components(pk, pv["bits"])
            assert ncomp == d["n_patches"], (L, ncomp, d["n_patches"])
            assert np.array_equal(np.repeat(comp, 8), d["cell_patch"].astype(np.int64)), L
        cells = np.bincount(d["cell_patch"], minlength=d["n_patches"])
        assert np.array_equal(cells, d["patch_ncells"].astype(np.int64))
        parts = np.bincount(d["cell_patch"], weights=d["cell_count"].astype(np.float64),
                            minlength=d["n_patches"])
        assert np.array_equal(parts.astype(np.uint64), d["patch_nparticles"])
        if L == 1:
            assert np.all(d["patch_parent"] == -1)
        else:
            pv = levels[L - 1]
            first = np.full(d["n_patches"], len(keys_L), np.int64)
            np.minimum.at(first, d["cell_patch"], np.arange(len(keys_L)))
            parent_keys = keys_L[first] >> np.uint64(3)
            pos = np.searchsorted(pv["cell_key"], parent_keys)
            assert np.array_equal(pv["cell_patch"][pos], d["patch_parent"])
        print(f"level {L}: {d['n_patches']} patches match the exact components", flush=True)
    h.free()
    return levels


@pytest.mark.timeout(900)
def test_fullsize_16m(ctx):
    # 256^3 particles, 128^3 domain grid, threshold 5, up to 10 levels
    check_fullsize(ctx, synth.snapshot_16m(1), seed=21)


@pytest.mark.timeout(900)
def test_largest_tiled_grid_g8(ctx):
    # 3M uniform particles on a 256^3 domain grid refined wherever a cell holds
    # a particle: about 2.7M refined level-0 cells, more than 1/8 of the grid,
    # so levels 0 and 1 both take the dense tile deposit at its largest grid
    # (level-1 tiles of 8^3 cells over the whole 512^3 grid)
    rng = np.random.Generator(np.random.PCG64(808))
    X, fx = synth.quantize(rng.random(3_000_000))
    Y, fy = synth.quantize(rng.random(3_000_000))
    Z, fz = synth.quantize(rng.random(3_000_000))
    snap = synth.Snapshot(X, Y, Z, fx, fy, fz, None, 8, 0.0, 0.0, 2, "uniform-3M-g8")
    levels = check_fullsize(ctx, snap, seed=23)
    assert 8 * levels[0]["n_refined"] >= 1 << 24


@pytest.fixture(scope="module")
def snap134():
    # 512^3 particles: 70% lattice, 30% in 20000 NFW hosts with 5 Plummer
    # subhalos each; generated once for the tests below (about a minute)
    print("generating the 134M snapshot", flush=True)
    return synth.snapshot_134m(2)


@pytest.mark.timeout(1500)
def test_fullsize_134m_subsample_parity(ctx, snap134):
    # the 134M workload's seeded 64^3 subsample, full oracle parity
    from tests.gpu_compare import compare_hierarchy
    from paper_0904_3662_amd import ahf
    s = snap134
    idx = np.sort(np.random.Generator(np.random.PCG64(64)).choice(s.n, 64 ** 3, replace=False))
    sub = s.subset(idx, "134M-subsample-64^3")
    print(f"case {sub.name}: n={sub.n}", flush=True)
    levels, order = oracle.build(sub)
    h, _ = ahf.build_snapshot(ctx, sub)
    compare_hierarchy(h, sub.n, levels, order)
    h.free()


@pytest.mark.timeout(1500)
def test_fullsize_134m(ctx, snap134):
    # 512^3 particles, 256^3 domain grid, threshold 5, up to 12 levels
    check_fullsize(ctx, snap134, seed=22)
