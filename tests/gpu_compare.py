"""Comparison of a device hierarchy with the oracle (shared by the GPU tests
and the smoke check).  Integer outputs must match bit for bit; the FP32 field
within 1e-5 relative of the FP64 oracle plus an absolute floor of 1e-30 times
the largest particle mass (FP32 underflow of triple-tail products)."""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-5
ABS_FLOOR = 1e-30


def brick_cells(d):
    """(keys, values) of every cell stored in the device bricks of a level."""
    bk = d["brick_key"].astype(np.uint64)
    keys = (bk[:, None] << np.uint64(3)) | np.arange(8, dtype=np.uint64)[None, :]
    return keys.reshape(-1), d["brick_mass"].astype(np.float64)


def compare_level(d, lv, m_max=1.0, labels=True):
    """Raise AssertionError on the first difference between device level `d`
    (dict from Hierarchy.level_numpy) and oracle level `lv`."""
    L = lv.level
    assert d["bits"] == lv.bits, (L, d["bits"], lv.bits)
    assert np.array_equal(d["cell_key"], lv.cell_key), f"level {L}: cell keys differ"
    assert np.array_equal(d["cell_count"], lv.cell_count), f"level {L}: counts differ"
    assert np.array_equal(d["cell_start"], lv.cell_start), f"level {L}: starts differ"
    assert np.array_equal(d["cell_refined"], lv.cell_flag), f"level {L}: refinement flags differ"
    assert d["n_particles"] == lv.n_particles, (L, d["n_particles"], lv.n_particles)
    # field: every oracle cell of E_L is stored, within tolerance; every other
    # stored cell is exactly zero
    keys, vals = brick_cells(d)
    order = np.argsort(keys, kind="stable")
    ks, vs = keys[order], vals[order]
    assert np.all(ks[1:] > ks[:-1]), f"level {L}: duplicated brick cells"
    pos = np.searchsorted(ks, lv.field_key)
    assert np.all(pos < len(ks)) and np.array_equal(ks[np.minimum(pos, len(ks) - 1)], lv.field_key), \
        f"level {L}: a cell of E_L is missing from the bricks"
    got = vs[pos]
    ref = lv.field_mass
    err = np.abs(got - ref)
    bound = REL_TOL * np.abs(ref) + ABS_FLOOR * m_max
    bad = np.nonzero(err > bound)[0]
    assert len(bad) == 0, (f"level {L}: {len(bad)} field cells out of tolerance; worst rel "
                           f"{np.max(err / np.maximum(ref, 1e-300)):.3e} at key {lv.field_key[bad[0]]}")
    rest = np.ones(len(ks), bool)
    rest[pos] = False
    assert np.all(vs[rest] == 0.0), f"level {L}: non-zero mass outside E_L"
    # brick -> S map: a brick belongs to S_L exactly when its parent is refined
    bc = d["brick_cell"].astype(np.int64)
    inS = bc >= 0
    if inS.any():
        assert np.array_equal(d["cell_key"][bc[inS]], d["brick_key"][inS] << np.uint64(3))
    assert int(inS.sum()) * 8 == len(d["cell_key"])
    # totals
    assert abs(d["total_cell_mass"] - lv.total_cell_mass) <= 1e-6 * max(lv.total_cell_mass, 1e-300)
    assert abs(d["total_particle_mass"] - lv.total_particle_mass) <= 1e-12 * max(lv.total_particle_mass, 1e-300)
    if labels and L >= 1:
        assert d["n_patches"] == lv.n_patches, (L, d["n_patches"], lv.n_patches)
        assert np.array_equal(d["cell_patch"], lv.cell_patch), f"level {L}: patch ids differ"
        assert np.array_equal(d["patch_parent"], lv.patch_parent), f"level {L}: patch parents differ"
        assert np.array_equal(d["patch_ncells"].astype(np.uint64), lv.patch_ncells)
        assert np.array_equal(d["patch_nparticles"], lv.patch_nparticles)
        np.testing.assert_allclose(d["patch_mass"], lv.patch_mass, rtol=1e-9, atol=0)


def compare_hierarchy(h, n, levels, order, m_max=1.0, labels=True):
    assert h.num_levels() == len(levels), (h.num_levels(), len(levels))
    assert np.array_equal(h.order_numpy(n), order), "particle order differs"
    for lv in levels:
        compare_level(h.level_numpy(lv.level), lv, m_max=m_max, labels=labels)
