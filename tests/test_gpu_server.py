"""Serving path (ahf_submit / ahf_poll): continuous batching, admission by
HBM footprint, resident results, label queries.  Every result must be the same
alone and in the mix (builds are deterministic, so bit for bit)."""
import numpy as np
import pytest

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import compare_hierarchy
from tests.helpers import clustered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0904_3662_amd import ahf
    c = ahf.Context(0)
    yield c
    c.close()


def level_arrays(h):
    return [h.level_numpy(L) for L in range(h.num_levels())]


def assert_same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for k, v in x.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, y[k]), k
            else:
                assert v == y[k], k


def subvolumes():
    sizes = [20000, 150000, 60000, 400000, 9000, 1200000, 90000, 30000]
    return [synth.subvolume(100 + i, n) for i, n in enumerate(sizes)]


def test_results_alone_and_in_the_mix_are_identical(ctx):
    from paper_0904_3662_amd import ahf
    subs = subvolumes()
    devs = [ahf.snapshot_to_device(s) for s in subs]
    alone = []
    for s, d in zip(subs, devs):
        print(f"alone {s.name}", flush=True)
        h, _ = ahf.build_snapshot(ctx, s, dev=d)
        alone.append(level_arrays(h))
        h.free()
    with ahf.Server(ctx, n_streams=4) as srv:
        tickets = [srv.submit_snapshot(s, dev=d) for s, d in zip(subs, devs)]
        for t, ref in zip(tickets, alone):
            h = srv.wait(t)
            assert_same(level_arrays(h), ref)
        st = srv.stats()
        assert st["completed"] == len(subs) and st["failed"] == 0
        assert st["resident"] == len(subs)
        for t in tickets:
            tt = srv.times(t)
            assert tt[0] <= tt[1] <= tt[2] <= tt[3]
            srv.release(t)
        assert srv.stats()["resident"] == 0


def test_served_result_matches_the_oracle(ctx):
    from paper_0904_3662_amd import ahf
    p = clustered(41, 20000, n_clumps=5, spread=0.01, g=4, thr=5, max_levels=5)
    levels, order = oracle.build(p)
    with ahf.Server(ctx, n_streams=2) as srv:
        t = srv.submit_snapshot(p)
        h = srv.wait(t)
        compare_hierarchy(h, p.n, levels, order)


def test_label_queries(ctx):
    from paper_0904_3662_amd import ahf
    s = synth.subvolume(7, 300000)
    rng = np.random.Generator(np.random.PCG64(3))
    with ahf.Server(ctx, n_streams=2) as srv:
        t = srv.submit_snapshot(s)
        h = srv.wait(t)
        for L in range(1, h.num_levels()):
            d = h.level_numpy(L)
            idx = rng.choice(len(d["cell_key"]), size=min(500, len(d["cell_key"])), replace=False)
            got = srv.query_label(t, L, d["cell_key"][idx])
            assert np.array_equal(got, d["cell_patch"][idx])
            # the same through the hierarchy entry point
            got2 = h.query_label(ctx, L, d["cell_key"][idx])
            assert np.array_equal(got2, got)
            # cells outside S_L: keys of ghost cells and of empty regions
            bk = d["brick_key"][d["brick_cell"] < 0]
            if len(bk):
                gk = (bk[: min(100, len(bk))] << np.uint64(3))
                assert np.all(srv.query_label(t, L, gk) == -1)
        assert np.all(srv.query_label(t, 0, np.arange(10, dtype=np.uint64)) == -1)


def test_admission_limits_and_errors(ctx):
    from paper_0904_3662_amd import ahf
    s = synth.subvolume(9, 50000)
    dev = ahf.snapshot_to_device(s)
    # a budget too small for the request alone
    with ahf.Server(ctx, n_streams=1, hbm_budget=1 << 20) as srv:
        with pytest.raises(ahf.AhfError) as e:
            srv.submit_snapshot(s, dev=dev)
        assert e.value.code == ahf.AHF_ELIMIT
    # unknown and released tickets
    with ahf.Server(ctx, n_streams=1) as srv:
        with pytest.raises(ahf.AhfError) as e:
            srv.wait(12345)
        assert e.value.code == ahf.AHF_ENOTFOUND
        t = srv.submit_snapshot(s, dev=dev)
        srv.wait(t)
        srv.release(t)
        with pytest.raises(ahf.AhfError) as e:
            srv.poll(t)
        assert e.value.code == ahf.AHF_ENOTFOUND
    # a full queue: one worker busy on a large build, one queue slot
    big = synth.subvolume(10, 4000000)
    bdev = ahf.snapshot_to_device(big)
    with ahf.Server(ctx, n_streams=1, max_queue=1) as srv:
        codes = []
        tickets = []
        for _ in range(4):
            try:
                tickets.append(srv.submit_snapshot(big, dev=bdev))
            except ahf.AhfError as err:
                codes.append(err.code)
        assert ahf.AHF_EBUSY in codes
        for t in tickets:
            srv.wait(t)


def test_lru_eviction_under_a_tight_budget(ctx):
    # results nobody has polled are evicted oldest first; the one polled is
    # held by the client until released
    from paper_0904_3662_amd import ahf
    subs = [synth.subvolume(200 + i, 200000) for i in range(5)]
    devs = [ahf.snapshot_to_device(s) for s in subs]
    with ahf.Server(ctx, n_streams=1) as srv:
        t = srv.submit_snapshot(subs[0], dev=devs[0])
        srv.wait(t)
        r = srv.stats()["bytes_results"]
    g = subs[0].g
    est = 300 * 200000 + 48 * (1 << (3 * g)) + (160 << 20)
    # room for the build in flight and one and a half resident results
    budget = est + (3 * r) // 2
    with ahf.Server(ctx, n_streams=1, hbm_budget=budget) as srv:
        tickets = [srv.submit_snapshot(s, dev=d) for s, d in zip(subs, devs)]
        assert srv.wait(tickets[-1]) is not None
        st = srv.stats()
        assert st["evicted"] >= 1 and st["failed"] == 0, st
        assert st["bytes_peak"] <= budget
        # the newest result is there, the oldest was evicted
        with pytest.raises(ahf.AhfError) as e:
            srv.poll(tickets[0])
        assert e.value.code == ahf.AHF_ENOTFOUND
        srv.release(tickets[-1])
