"""Device builds with the paper-literal density criterion (refine where a
cell's TSC particle number exceeds the threshold) against the oracle.  The
flags then rest on floating point: each case keeps every cell of S_L at least
EPS (relative) away from its level's threshold in the FP64 oracle, nudging
the thresholds until it does, so the FP32 device field must decide every flag
the same way; then everything (cells, flags, field, labels) must match."""
import numpy as np
import pytest

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import compare_hierarchy
from tests.helpers import clustered, small_mixed_scaled, uniform

pytestmark = pytest.mark.gpu

EPS = 2e-5  # twice the field tolerance


@pytest.fixture(scope="module")
def ctx():
    from paper_0904_3662_amd import ahf
    c = ahf.Context(0)
    yield c
    c.close()


def clear_of_threshold(levels, dom, ref, max_levels):
    for lv in levels:
        if lv.level >= max_levels:
            continue  # the level cap refines nothing, whatever the density
        thr = dom if lv.level == 0 else ref
        fk = lv.field_key
        pos = np.searchsorted(fk, lv.cell_key)
        num = lv.field_mass[pos]                 # unit masses: mass = particle number
        if len(num) and np.min(np.abs(num - thr)) <= EPS * max(1.0, abs(thr)):
            return False
    return True


def oracle_with_margin(p):
    for _ in range(8):
        levels, order = oracle.build(p, density=True)
        if clear_of_threshold(levels, p.dom_ref, p.ref_ref, p.max_levels):
            return levels, order
        p.dom_ref *= 1.000371
        p.ref_ref *= 1.000529
    raise AssertionError("no threshold with a margin found")


CASES = [
    ("clustered-g4", lambda: clustered(91, 30000, n_clumps=9, spread=0.02, g=4, thr=3.3,
                                       max_levels=6)),
    ("clustered-g3-deep", lambda: clustered(92, 15000, n_clumps=5, spread=0.004, g=3, thr=2.6,
                                            max_levels=8)),
    ("mixed-32k", lambda: small_mixed_scaled(4, 32768, g=5, max_levels=4)),
    ("uniform-g3", lambda: uniform(93, 6000, g=3, thr=9.4, max_levels=4)),
    ("uniform-g4", lambda: uniform(94, 40000, g=4, thr=11.3, max_levels=3)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_density_criterion_matches_oracle(ctx, name, make):
    from paper_0904_3662_amd import ahf
    p = make()
    if name == "mixed-32k":
        p.dom_ref, p.ref_ref = 3.7, 2.9
    levels, order = oracle_with_margin(p)
    print(f"density case {name}: n={p.n} thresholds {p.dom_ref:.6f} {p.ref_ref:.6f}, "
          f"{len(levels)} levels", flush=True)
    assert len(levels) >= 2
    h, _ = ahf.build_snapshot(ctx, p, density_criterion=True)
    compare_hierarchy(h, p.n, levels, order)
    h.free()


def test_density_criterion_needs_equal_masses(ctx):
    from paper_0904_3662_amd import ahf
    p = uniform(95, 3000, g=3, thr=2.0, max_levels=3)
    p.mass = np.ones(p.n, np.float32)
    with pytest.raises(ahf.AhfError) as e:
        ahf.build_snapshot(ctx, p, density_criterion=True)
    assert e.value.code == ahf.AHF_EINVAL


@pytest.mark.timeout(900)
def test_fullsize_16m_density_criterion(ctx):
    # full size: every flag equals the rule applied to the device's own field
    # (in double precision), levels nest, masses are conserved
    from paper_0904_3662_amd import ahf
    s = synth.snapshot_16m(1)
    h, _ = ahf.build_snapshot(ctx, s, density_criterion=True)
    nlev = h.num_levels()
    assert nlev >= 4
    for L in range(nlev):
        d = h.level_numpy(L)
        thr = s.dom_ref if L == 0 else s.ref_ref
        bk = d["brick_key"].astype(np.uint64)
        keys = ((bk[:, None] << np.uint64(3)) | np.arange(8, dtype=np.uint64)[None, :]).reshape(-1)
        order = np.argsort(keys)
        pos = order[np.searchsorted(keys[order], d["cell_key"])]
        num = d["brick_mass"].astype(np.float64)[pos]
        can_refine = L < s.max_levels and s.g + L < 21
        want = ((num > thr) & can_refine).astype(np.uint8)
        assert np.array_equal(d["cell_refined"], want), L
        assert abs(d["total_cell_mass"] - d["total_particle_mass"]) <= 1e-6 * d["total_particle_mass"]
        if L + 1 < nlev:
            e = h.level_numpy(L + 1)
            ref = d["cell_key"][d["cell_refined"] == 1]
            assert np.array_equal(e["cell_key"].reshape(-1, 8)[:, 0] >> np.uint64(3), ref)
    h.free()
