"""Pins of the oracle's density refinement criterion (Sect. 2.1 read
literally: a cell is refined where its TSC particle density, in particles per
cell, exceeds the threshold): closed forms, independence of particle masses,
and equality with the dense brute force."""
import numpy as np
import pytest

import oracle
from oracle import brute
from tests.helpers import Q, clustered, demorton_py, from_positions, particles, uniform

MARGIN = 1e-9  # a case must keep every cell's density this far from its threshold


def lattice(nside, offset, g):
    # one particle per cell of a nside^3 grid at a common offset (in cells)
    i = np.arange(nside)
    x, y, z = np.meshgrid(i, i, i, indexing="ij")
    pos = (np.stack([x.ravel(), y.ravel(), z.ravel()], 1) + offset) / nside
    return pos


def test_lattice_density_is_one_per_cell():
    pos = lattice(8, 0.3, 3)
    p = from_positions(pos, g=3, thr=0.5, max_levels=1)
    levels, _ = oracle.build(p, density=True)
    assert np.all(levels[0].cell_flag == 1)          # density 1 > 0.5 everywhere
    levels, _ = oracle.build(p, density=True, dom_ref=1.5)
    assert len(levels) == 1 and np.all(levels[0].cell_flag == 0)


def test_coincident_particles_at_a_cell_centre():
    # K particles at the centre of one level-0 cell: that cell holds K * 27/64
    K = 10
    c = (5 + 0.5) / 8
    p = from_positions(np.full((K, 3), c), g=3, thr=0.0, max_levels=1)
    exact = K * 27.0 / 64.0
    lv, _ = oracle.build(p, density=True, dom_ref=exact - 1e-6)
    assert int(lv[0].cell_flag.sum()) == 1
    lv, _ = oracle.build(p, density=True, dom_ref=exact + 1e-6)
    assert int(lv[0].cell_flag.sum()) == 0
    # the count criterion would refine it at any threshold below K
    lv, _ = oracle.build(p, dom_ref=exact + 1e-6)
    assert int(lv[0].cell_flag.sum()) == 1


def test_criterion_counts_particles_not_mass():
    p = clustered(81, 3000, g=3, thr=2.5, max_levels=3)
    a, _ = oracle.build(p, density=True)
    p.mass = (np.random.Generator(np.random.PCG64(82)).random(p.n) * 10 + 0.1).astype(np.float32)
    b, _ = oracle.build(p, density=True)
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert np.array_equal(x.cell_key, y.cell_key)
        assert np.array_equal(x.cell_flag, y.cell_flag)


def margin_ok(bf, p):
    for d in bf:
        thr = p.dom_ref if d["level"] == 0 else p.ref_ref
        v = d["number"][d["inS"]]
        if len(v) and np.min(np.abs(v - thr)) <= MARGIN * max(1.0, abs(thr)):
            return False
    return True


CASES = [
    ("uniform-g2", lambda: uniform(83, 400, g=2, thr=4.3, max_levels=3)),
    ("clustered-g2", lambda: clustered(84, 500, g=2, thr=3.7, max_levels=3, spread=0.02)),
    ("clustered-g3", lambda: clustered(85, 700, g=3, thr=2.2, max_levels=2, spread=0.03)),
    ("wrap-corner", lambda: from_positions(
        (np.random.Generator(np.random.PCG64(86)).normal(0, 0.01, (300, 3))) % 1.0,
        g=2, thr=3.1, max_levels=3)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_density_criterion_matches_dense_brute_force(name, make):
    p = make()
    bf = brute.brute(p, p.g, p.dom_ref, p.ref_ref, p.max_levels, density=True)
    assert margin_ok(bf, p)
    levels, _ = oracle.build(p, density=True)
    assert len(levels) == len(bf)
    assert len(levels) >= 2
    for lv, d in zip(levels, bf):
        b = lv.bits
        x, y, z = (v.astype(int) for v in demorton_py(lv.cell_key, b))
        mask = np.zeros_like(d["inS"])
        mask[x, y, z] = True
        assert np.array_equal(mask, d["inS"])
        assert np.array_equal(lv.cell_flag.astype(bool), d["flag"][x, y, z])
        ex, ey, ez = (v.astype(int) for v in demorton_py(lv.field_key, b))
        ref = d["mass"][ex, ey, ez]
        assert np.all(np.abs(lv.field_mass - ref) <= 1e-12 * np.maximum(ref, 1e-300) + 1e-300)
        if lv.level >= 1:
            assert np.array_equal(lv.cell_patch, d["patch"][x, y, z])
