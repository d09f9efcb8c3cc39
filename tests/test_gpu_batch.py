"""Sub-volumes rebuilt together with one host wait per run (ahf_batch_*):
every sub-volume's hierarchy is bit for bit the one a single build gives, on
every run, with other work between the runs; the oracle agrees with one of
them; rewritten particles are rebuilt; particles that outgrow the level sizes
the batch was made for are reported as AHF_ELIMIT for that sub-volume alone."""
import numpy as np
import pytest

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import compare_hierarchy
from tests.helpers import clustered, uniform

pytestmark = pytest.mark.gpu


def level_arrays(h):
    return [h.level_numpy(L) for L in range(h.num_levels())]


def assert_same(a, b, what):
    """Every array bit for bit; the FP64 level totals to 1e-12 (they are
    summed over per-block partial sums, and a batch's builds, sized ahead,
    launch those sums over more blocks)."""
    assert len(a) == len(b), (what, len(a), len(b))
    for L, (x, y) in enumerate(zip(a, b)):
        for k, v in x.items():
            if isinstance(v, np.ndarray):
                assert v.dtype == y[k].dtype and np.array_equal(v, y[k]), (what, L, k)
            elif k.startswith("total_"):
                assert abs(v - y[k]) <= 1e-12 * abs(y[k]), (what, L, k, v, y[k])
            else:
                assert v == y[k], (what, L, k, v, y[k])


def single(ctx, snap, dev):
    from paper_0904_3662_amd import ahf
    h, _ = ahf.build_snapshot(ctx, snap, dev=dev)
    out = (level_arrays(h), h.order_numpy(snap.n))
    h.free()
    return out


def test_batch_runs_match_single_builds_and_the_oracle():
    import torch
    from paper_0904_3662_amd import ahf
    sizes = [30000, 250000, 12000, 90000, 1000000, 40000]
    snaps = [synth.subvolume(400 + i, n) for i, n in enumerate(sizes)]
    snaps.append(synth.small_mixed(0))
    devs = [ahf.snapshot_to_device(s) for s in snaps]
    levels, order = oracle.build(snaps[-1])
    with ahf.Context(0) as ctx:
        want = [single(ctx, s, d) for s, d in zip(snaps, devs)]
        with ahf.Batch(ctx, snaps, devs, n_chains=3) as b:
            for run in range(3):
                print(f"batch run {run}", flush=True)
                b.run()
                b.wait()
                for i, s in enumerate(snaps):
                    h = b.hierarchy(i)
                    assert b.status(i) == ahf.AHF_OK
                    assert_same(level_arrays(h), want[i][0], (run, i))
                    assert np.array_equal(h.order_numpy(s.n), want[i][1]), (run, i)
                compare_hierarchy(b.hierarchy(len(snaps) - 1), snaps[-1].n, levels, order)
                # other work on the GPU between the runs
                single(ctx, snaps[0], devs[0])
                torch.cuda.synchronize()


def test_rewritten_particles_are_rebuilt_and_overflow_is_reported():
    import torch
    from paper_0904_3662_amd import ahf
    a = uniform(41, 30000, g=4, thr=5, max_levels=5)
    b_ = clustered(42, 30000, n_clumps=6, spread=0.01, g=4, thr=5, max_levels=5)
    snaps = [a, b_]
    devs = [ahf.snapshot_to_device(s) for s in snaps]
    with ahf.Context(0) as ctx:
        with ahf.Batch(ctx, snaps, devs, n_chains=2) as bt:
            bt.run()
            bt.wait()
            # sub-volume 1 translated by one domain cell (same level sizes):
            # the batch rebuilds it from the rewritten arrays
            shift = 1 << (21 - b_.g)
            moved = synth.Snapshot((b_.X + shift) & 0x1fffff, b_.Y, b_.Z, b_.fx, b_.fy, b_.fz,
                                   None, b_.g, b_.dom_ref, b_.ref_ref, b_.max_levels, "moved")
            mdev = ahf.snapshot_to_device(moved)
            devs[1][0].copy_(mdev[0])
            torch.cuda.synchronize()
            bt.run()
            bt.wait()
            ref, _ = ahf.build_snapshot(ctx, moved, dev=mdev)
            assert_same(level_arrays(bt.hierarchy(1)), level_arrays(ref), "moved")
            ref.free()
            levels, order = oracle.build(moved)
            compare_hierarchy(bt.hierarchy(1), moved.n, levels, order)
            # sub-volume 0 becomes clustered: its levels outgrow the recorded
            # sizes, which that sub-volume alone reports
            dense = clustered(43, 30000, n_clumps=2, spread=0.003, frac=0.95, g=4, thr=5,
                              max_levels=5)
            ddev = ahf.snapshot_to_device(dense)
            for k in range(6):
                devs[0][k].copy_(ddev[k])
            torch.cuda.synchronize()
            bt.run()
            with pytest.raises(ahf.AhfError) as e:
                bt.wait()
            assert e.value.code == ahf.AHF_ELIMIT
            assert bt.status(0) == ahf.AHF_ELIMIT and bt.status(1) == ahf.AHF_OK
            with pytest.raises(ahf.AhfError):
                bt.hierarchy(0)
            assert_same(level_arrays(bt.hierarchy(1)), level_arrays_of(ctx, moved, mdev), "again")


def level_arrays_of(ctx, snap, dev):
    return single(ctx, snap, dev)[0]


def test_batch_rejects_what_it_cannot_record():
    from paper_0904_3662_amd import ahf
    p = uniform(44, 5000, g=4, thr=5, max_levels=4)
    p.mass = np.ones(p.n, np.float32)
    with ahf.Context(0) as ctx:
        with pytest.raises(ahf.AhfError) as e:
            ahf.Batch(ctx, [p])
        assert e.value.code == ahf.AHF_EINVAL
        q = uniform(45, 5000, g=4, thr=5, max_levels=4)
        with pytest.raises(ahf.AhfError) as e:
            ahf.Batch(ctx, [q], n_chains=0)
        assert e.value.code == ahf.AHF_EINVAL


@pytest.mark.skip(reason="recording a batch into a HIP graph is switched off: the HIP runtime "
                         "segfaulted in hipStreamEndCapture on the multi-stream recording of "
                         "these builds (the builds themselves ran and checked out eagerly)")
def test_batch_recorded_into_a_graph_matches_single_builds():
    from paper_0904_3662_amd import ahf
    snaps = [synth.subvolume(450 + i, n) for i, n in enumerate([20000, 60000, 5000])]
    devs = [ahf.snapshot_to_device(s) for s in snaps]
    with ahf.Context(0) as ctx:
        want = [single(ctx, s, d) for s, d in zip(snaps, devs)]
        with ahf.Batch(ctx, snaps, devs, n_chains=2, graph=True) as b:
            for run in range(3):
                b.run()
                b.wait()
                for i in range(len(snaps)):
                    assert_same(level_arrays(b.hierarchy(i)), want[i][0], (run, i))


def test_graph_recording_is_reported_as_switched_off():
    from paper_0904_3662_amd import ahf
    q = uniform(46, 5000, g=4, thr=5, max_levels=4)
    with ahf.Context(0) as ctx:
        with pytest.raises(ahf.AhfError) as e:
            ahf.Batch(ctx, [q], graph=True)
        assert e.value.code == ahf.AHF_EINVAL
