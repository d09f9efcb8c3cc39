"""Device classification of the grid tree into host structures and
substructures against the oracle (exact integers)."""
import numpy as np
import pytest

import oracle
from oracle.substructure import classify, classify_levels
from paper_0904_3662_amd import synth
from tests.helpers import clustered, small_mixed_scaled, uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0904_3662_amd import ahf
    c = ahf.Context(0)
    yield c
    c.close()


def device_tree(h):
    nlev = h.num_levels()
    lv = [h.level_numpy(L) for L in range(nlev)]
    parents = [np.zeros(0, np.int32)] + [lv[L]["patch_parent"] for L in range(1, nlev)]
    counts = [np.zeros(0, np.uint64)] + [lv[L]["patch_nparticles"] for L in range(1, nlev)]
    return lv, parents, counts


def check_against(h, ps, st):
    s = h.structures()
    assert s["n_structures"] == len(st["host"])
    for k in ("host", "level", "patch", "depth"):
        assert np.array_equal(s[k], st[k]), k
    for L in range(1, h.num_levels()):
        got = h.level_numpy(L)["patch_struct"]
        assert np.array_equal(got, ps[L]), L


CASES = [
    ("clustered-g4", lambda: clustered(61, 30000, n_clumps=9, spread=0.02, g=4, thr=4, max_levels=6)),
    ("clustered-g3-deep", lambda: clustered(62, 15000, n_clumps=5, spread=0.005, g=3, thr=2,
                                            max_levels=9)),
    ("mixed-32k", lambda: small_mixed_scaled(3, 32768, g=5, max_levels=4)),
    ("uniform-dense", lambda: uniform(63, 6000, g=3, thr=2, max_levels=4)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_classification_matches_oracle(ctx, name, make):
    from paper_0904_3662_amd import ahf
    p = make()
    print(f"substructure case {name}: n={p.n}", flush=True)
    levels, _ = oracle.build(p)
    ps, st = classify_levels(levels)
    h, dev = ahf.build_snapshot(ctx, p, substructure=True)
    check_against(h, ps, st)
    # the same through the explicit call on a labelled hierarchy
    h2, _ = ahf.build_snapshot(ctx, p, dev=dev)
    assert h2.level_numpy(1)["patch_struct"] is None
    h2.classify(ctx)
    check_against(h2, ps, st)
    h.free()
    h2.free()


def test_substructure_needs_labels(ctx):
    from paper_0904_3662_amd import ahf
    p = uniform(64, 2000, g=3, thr=3, max_levels=3)
    with pytest.raises(ahf.AhfError) as e:
        ahf.build_snapshot(ctx, p, labels=False, substructure=True)
    assert e.value.code == ahf.AHF_EINVAL
    h, _ = ahf.build_snapshot(ctx, p, labels=False)
    with pytest.raises(ahf.AhfError) as e:
        h.classify(ctx)
    assert e.value.code == ahf.AHF_EINVAL
    h.free()


@pytest.mark.timeout(900)
def test_fullsize_16m_classification(ctx):
    # the device tree itself is checked against exact components elsewhere;
    # here its classification must equal the oracle rule applied to it
    from paper_0904_3662_amd import ahf
    s = synth.snapshot_16m(1)
    h, _ = ahf.build_snapshot(ctx, s, substructure=True)
    lv, parents, counts = device_tree(h)
    ps, st = classify(parents, counts)
    check_against(h, ps, st)
    print(f"16.8M: {len(st['host'])} structures, max depth {int(st['depth'].max())}", flush=True)
    h.free()


def test_served_classification(ctx):
    from paper_0904_3662_amd import ahf
    s = synth.subvolume(71, 200000)
    with ahf.Server(ctx, n_streams=2) as srv:
        t = srv.submit_snapshot(s, substructure=True)
        h = srv.wait(t)
        lv, parents, counts = device_tree(h)
        ps, st = classify(parents, counts)
        check_against(h, ps, st)
