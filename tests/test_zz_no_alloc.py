"""The label query that allocates nothing (static staging array) against the
workspace-backed label query, through the C ABI: two calls in a row, the
second with fewer keys, plus keys outside S_L and the size limit."""
import numpy as np
import pytest

from paper_0904_3662_amd import synth

pytestmark = pytest.mark.gpu


def test_static_label_query_matches_the_workspace_query():
    from paper_0904_3662_amd import ahf
    s = synth.subvolume(17, 400000)
    rng = np.random.Generator(np.random.PCG64(71))
    with ahf.Context(0) as ctx:
        h, _ = ahf.build_snapshot(ctx, s)
        assert h.num_levels() >= 3
        for L in range(1, h.num_levels()):
            d = h.level_numpy(L)
            keys = d["cell_key"]
            # cells of S_L, ghost cells of the bricks and keys far away
            ghost = (d["brick_key"][d["brick_cell"] < 0] << np.uint64(3))
            far = rng.integers(0, 1 << (3 * d["bits"]), 1000, dtype=np.uint64)
            pool = np.concatenate([keys, ghost, far]).astype(np.uint64)
            for n in (min(len(pool), 200000), min(len(pool), 777)):  # a call, then a smaller one
                q = pool[rng.integers(0, len(pool), n)]
                want = h.query_label(ctx, L, q)
                got = h.query_label_static(L, q)
                assert np.array_equal(got, want), (L, n)
                inS = np.isin(q, keys)
                assert np.all(want[~inS] == -1) and np.all(want[inS] >= 0)
        assert np.all(h.query_label_static(0, np.arange(5, dtype=np.uint64)) == -1)
        with pytest.raises(ahf.AhfError) as e:
            h.query_label_static(1, np.zeros(262145, np.uint64))
        assert e.value.code == ahf.AHF_ELIMIT
        h.free()
