"""The C-ABI boundary's memory and request contracts, through ctypes:
allocation callbacks (PyTorch-owned memory, an injected allocation failure),
cancellation of a queued request, results held by the client surviving
eviction, and measured device memory staying inside a server's budget."""
import ctypes as C
import gc
import threading
import time

import numpy as np
import pytest

import oracle
from paper_0904_3662_amd import synth
from tests.gpu_compare import compare_hierarchy
from tests.helpers import clustered

pytestmark = pytest.mark.gpu


class CountingMemory:
    """Allocation callbacks on PyTorch's caching allocator that record every
    allocation and free, and fail the k-th allocation when asked."""

    def __init__(self):
        import torch
        from paper_0904_3662_amd import ahf
        self.raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
        self.raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete
        self.lock = threading.Lock()
        self.live = {}       # pointer -> bytes
        self.n_alloc = 0
        self.n_free = 0
        self.bad_frees = 0
        self.fail_at = None  # 1-based index of the allocation that fails
        self.alloc = ahf.ALLOC_FN(self._alloc)
        self.free = ahf.FREE_FN(self._free)

    def _alloc(self, user, nbytes, stream):
        with self.lock:
            self.n_alloc += 1
            if self.fail_at is not None and self.n_alloc == self.fail_at:
                return None
        p = self.raw_alloc(int(nbytes), int(stream or 0))
        with self.lock:
            self.live[p] = int(nbytes)
        return p

    def _free(self, user, ptr, nbytes, stream):
        with self.lock:
            self.n_free += 1
            if ptr not in self.live or self.live[ptr] != int(nbytes):
                self.bad_frees += 1
                return
            del self.live[ptr]
        self.raw_delete(int(ptr))


def small_case():
    return clustered(61, 30000, n_clumps=5, spread=0.01, g=4, thr=5, max_levels=5)


def test_torch_owned_memory_and_release():
    import torch
    from paper_0904_3662_amd import ahf
    p = small_case()
    levels, order = oracle.build(p)
    dev = ahf.snapshot_to_device(p)
    # objects of earlier tests that only the cycle collector frees would
    # otherwise be freed in the middle of this test
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = ahf.Context(0)  # PyTorch's caching allocator by default
    h, _ = ahf.build_snapshot(ctx, p, dev=dev)
    held = torch.cuda.memory_allocated() - base
    assert held > 0, "the hierarchy and the scratch space are PyTorch allocations"
    compare_hierarchy(h, p.n, levels, order)
    h.free()
    ctx.close()
    assert torch.cuda.memory_allocated() == base


def test_allocation_failure_gives_enomem_and_the_context_recovers():
    from paper_0904_3662_amd import ahf
    p = small_case()
    levels, order = oracle.build(p)
    dev = ahf.snapshot_to_device(p)
    # how many allocations a first build on a fresh context makes
    mem = CountingMemory()
    ctx = ahf.Context(0, memory=mem)
    h, _ = ahf.build_snapshot(ctx, p, dev=dev)
    h.free()
    ctx.close()
    total = mem.n_alloc
    assert total >= 3 and not mem.live and mem.bad_frees == 0
    print(f"a first build makes {total} allocations", flush=True)
    for k in range(1, total + 1):
        mem = CountingMemory()
        mem.fail_at = k
        ctx = ahf.Context(0, memory=mem)
        with pytest.raises(ahf.AhfError) as e:
            ahf.build_snapshot(ctx, p, dev=dev)
        assert e.value.code == ahf.AHF_ENOMEM, (k, e.value)
        assert mem.bad_frees == 0
        # the same context builds the right hierarchy afterwards
        mem.fail_at = None
        h, _ = ahf.build_snapshot(ctx, p, dev=dev)
        compare_hierarchy(h, p.n, levels, order)
        h.free()
        ctx.close()
        # every allocation was given back exactly once
        assert not mem.live, (k, len(mem.live))
        assert mem.n_free == mem.n_alloc - 1 and mem.bad_frees == 0, k


def test_canceled_queued_request():
    from paper_0904_3662_amd import ahf
    rng = np.random.Generator(np.random.PCG64(5))
    n = 8_000_000
    X, fx = synth.quantize(rng.random(n))
    Y, fy = synth.quantize(rng.random(n))
    Z, fz = synth.quantize(rng.random(n))
    big = synth.Snapshot(X, Y, Z, fx, fy, fz, None, 7, 5.0, 5.0, 6, "uniform-8M")
    small = clustered(62, 20000, g=4, thr=5, max_levels=4)
    bdev = ahf.snapshot_to_device(big)
    sdev = ahf.snapshot_to_device(small)
    ctx = ahf.Context(0)
    with ahf.Server(ctx, n_streams=1) as srv:
        a = srv.submit_snapshot(big, dev=bdev)
        b = srv.submit_snapshot(small, dev=sdev)
        c = srv.submit_snapshot(small, dev=sdev)
        srv.release(b)  # still queued behind the 8M build
        with pytest.raises(ahf.AhfError) as e:
            srv.wait(b)
        assert e.value.code == ahf.AHF_ECANCELED
        with pytest.raises(ahf.AhfError) as e:
            srv.poll(b)
        assert e.value.code == ahf.AHF_ECANCELED
        assert srv.wait(a) is not None and srv.wait(c) is not None
        st = srv.stats()
        assert st["completed"] == 2 and st["failed"] == 0
        # releasing the canceled ticket again forgets it
        srv.release(b)
        with pytest.raises(ahf.AhfError) as e:
            srv.poll(b)
        assert e.value.code == ahf.AHF_ENOTFOUND
        srv.release(a)
        srv.release(c)
    ctx.close()


def level_arrays(h):
    return [h.level_numpy(L) for L in range(h.num_levels())]


def device_used():
    from paper_0904_3662_amd import ahf
    hip = ahf._hip_runtime()
    fr, tot = C.c_size_t(), C.c_size_t()
    hip.hipMemGetInfo.argtypes = [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    assert hip.hipMemGetInfo(C.byref(fr), C.byref(tot)) == 0
    return tot.value - fr.value


def test_held_result_survives_eviction_and_device_memory_stays_in_budget():
    import torch
    from paper_0904_3662_amd import ahf
    subs = [synth.subvolume(300 + i, 400000) for i in range(6)]
    devs = [ahf.snapshot_to_device(s) for s in subs]
    # the library's own pool: everything the server holds is visible to
    # hipMemGetInfo (PyTorch's cache would hide what it keeps)
    ctx = ahf.Context(0, memory="pool")
    ref, _ = ahf.build_snapshot(ctx, subs[0], dev=devs[0])
    want = level_arrays(ref)
    ref.free()
    with ahf.Server(ctx, n_streams=1) as srv:
        t = srv.submit_snapshot(subs[0], dev=devs[0])
        srv.wait(t)
        r = srv.stats()["bytes_results"]
    g = subs[0].g
    est = 300 * 400000 + 48 * (1 << (3 * g)) + (160 << 20)
    # room for a build in flight (its estimate covers the worker's workspace
    # and its result) and about two and a half finished results
    budget = est + (5 * r) // 2
    torch.cuda.synchronize()
    base = device_used()
    slack = 64 << 20  # the runtime's own allocations (streams, kernel arguments)
    worst = 0
    with ahf.Server(ctx, n_streams=1, hbm_budget=budget) as srv:
        held = srv.submit_snapshot(subs[0], dev=devs[0])
        h = srv.wait(held)  # the client holds this result from here on
        tickets = []
        for s, d in zip(subs[1:], devs[1:]):
            tickets.append(srv.submit_snapshot(s, dev=d))
            worst = max(worst, device_used() - base)
        while srv.stats()["completed"] + srv.stats()["failed"] < len(subs):
            worst = max(worst, device_used() - base)
            time.sleep(0.001)
        worst = max(worst, device_used() - base)
        st = srv.stats()
        assert st["evicted"] >= 1 and st["failed"] == 0, st
        assert st["bytes_peak"] <= budget, (st, budget)
        assert worst <= budget + slack, (worst, budget)
        # the held result was never evicted and still reads back intact
        assert_same(level_arrays(h), want)
        # the newest result is resident, the oldest unheld one was evicted
        assert srv.poll(tickets[-1]) is not None
        with pytest.raises(ahf.AhfError) as e:
            srv.poll(tickets[0])
        assert e.value.code == ahf.AHF_ENOTFOUND
        srv.release(held)
        srv.release(tickets[-1])
    ctx.close()


def assert_same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for k, v in x.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, y[k]), k
            else:
                assert v == y[k], k


def test_held_results_that_leave_no_room_fail_the_request():
    from paper_0904_3662_amd import ahf
    s = synth.subvolume(320, 300000)
    dev = ahf.snapshot_to_device(s)
    ctx = ahf.Context(0, memory="pool")
    with ahf.Server(ctx, n_streams=1) as srv:
        srv.wait(srv.submit_snapshot(s, dev=dev))
        st = srv.stats()
    g = s.g
    est = 300 * 300000 + 48 * (1 << (3 * g)) + (160 << 20)
    # the budget holds one request, but not a second one beside a held result
    budget = est + st["bytes_results"] // 2
    with ahf.Server(ctx, n_streams=1, hbm_budget=budget) as srv:
        a = srv.submit_snapshot(s, dev=dev)
        assert srv.wait(a) is not None
        b = srv.submit_snapshot(s, dev=dev)
        with pytest.raises(ahf.AhfError) as e:
            srv.wait(b)
        assert e.value.code == ahf.AHF_ELIMIT
        srv.release(a)
        # with the held result released the same request is admitted
        c = srv.submit_snapshot(s, dev=dev)
        assert srv.wait(c) is not None
        srv.release(c)
    ctx.close()
