"""Throughput of the full hierarchy build on one MI355X.

One step = one complete build of the adaptive density hierarchy (Morton keys,
stable sort, per-level counts, refinement flags, TSC deposit, FP64 totals,
grid-tree labels) of the 134M-particle lattice + NFW-halo + subhalo snapshot
(512^3 particles, 256^3 domain grid, threshold 5, up to 12 levels), with the
input already resident in HBM; the 16.8M snapshot (256^3 particles, 128^3
domain grid, up to 10 levels) is measured the same way under its own key.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particles/s through full hierarchy build (1 GPU, % HBM peak); p50/p99 latency"


# the files every kernel of the library is compiled from: a PMC summary holds
# their SHA-256 and is used only while they are unchanged
KERNEL_SRC = [os.path.join(ROOT, "paper_0904_3662_amd", "csrc", f)
              for f in ("ahf_prims.hip", "ahf_levels.hip", "ahf_dev.h", "ahf_internal.h",
                        "ahf_block.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of one kernel from the committed PMC summary
    profiles/pmc_<kernel>_<workload>.txt (FETCH_SIZE and WRITE_SIZE runs scaled
    by a copy kernel of known size), or None when there is none or the kernel
    sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            vals["t"] = float(line.split(":")[1])
        if line.startswith("source_sha256"):
            vals["h"] = line.split(":")[1].strip()
    if "t" not in vals or vals.get("h") != kernel_source_hash():
        return None
    return vals["t"]


def sort_plan(n, key_bits):
    """Index width ib and number q of (key, index) passes of the radix sort:
    q is the first pass count after which the unsorted key bits fit beside
    the index in one 64-bit word."""
    ib = 1
    while ib < 32 and (1 << ib) < n:
        ib += 1
    q = 0
    while key_bits - 8 * q > 64 - ib:
        q += 1
    return ib, q, (key_bits + 7) // 8


def sort_scatter_bytes(n, key_bits):
    """Bytes the scatter kernels of one sort read and write: a (key, index)
    pass reads the 8-byte key (and the 4-byte index after the first pass) and
    writes both, the pass that packs writes one 8-byte word, and every later
    pass reads and writes one word."""
    ib, q, npass = sort_plan(n, key_bits)
    tot = 0
    for p in range(npass):
        if p < q:
            rd = 8 + (4 if p > 0 else 0)
            wr = 8 if p == q - 1 else 12
        else:
            rd, wr = 8, 8
        tot += (rd + wr) * n
    return tot


def algorithmic_bytes(n, levels, sp=24):
    """Bytes the method itself must move per build (inputs read once, one
    read+write of the key/index pairs, the sorted payload written once, and
    per level the particles of S_L read once plus the cell arrays written)."""
    b = n * sp + 24 * n + n * sp
    for d in levels:
        b += d["n_particles"] * sp + d["n_cells"] * 16 + 8 * d["n_bricks"] * 4 + d["n_cells"] * 4
    return b


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "affinity": share}


def sub_cubes(snap, k, count, seed=12345):
    """`count` distinct cubes of k^3 domain cells (drawn at random among the
    (2^g / k)^3 cubes on a grid of k cells), each as the snapshot's particles
    inside it: samples of the same workload at the same density, which the
    oracle refines as deeply as the whole snapshot (only cells at a cube's
    faces see a different neighbourhood)."""
    nc = (1 << snap.g) // k
    sh = 21 - snap.g
    cid = np.zeros(snap.n, np.int64)
    inside = np.ones(snap.n, bool)
    for a in (snap.X, snap.Y, snap.Z):
        c = (a >> sh) // k
        inside &= c < nc
        cid = cid * nc + np.minimum(c, nc - 1)
    cid[~inside] = -1
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.permutation(nc ** 3)[:count]
    return [snap.subset(np.nonzero(cid == j)[0], f"{snap.name}-cube{k}") for j in pick], nc


def cpu_baseline(snap, k, threads, repeats=1):
    """The FP64 oracle (its unchanged source built -O3 -march=native for this
    host) on sub-cubes of the snapshot: once with one thread on one sub-cube
    (median of `repeats` runs), and once with `threads` threads, each running
    the oracle on its own sub-cube at the same time (the oracle is one thread;
    the ctypes call releases the interpreter lock).  Value: the all-thread
    aggregate in particles/s."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build_library(force=True, native=True)
    subs, nc = sub_cubes(snap, k, max(threads, 1))
    one = []
    for r in range(repeats):
        t0 = time.perf_counter()
        lev, _ = oracle.build(subs[0], native=True)
        one.append(time.perf_counter() - t0)
    t1 = float(np.median(one))

    def run(sb):
        oracle.build(sb, native=True)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, subs[:threads]))
    tall = time.perf_counter() - t0
    nall = sum(sb.n for sb in subs[:threads])
    info = host_info()
    frac = f"1/{nc ** 3}"
    return {"value": nall / tall, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} sub-cubes of {k}^3 domain cells ({frac} of the box each, "
                      f"{nall} particles in all) of the {snap.name} snapshot, same grid "
                      f"parameters, one oracle thread per sub-cube, {tall:.1f} s wall",
            "single_thread": {"value": subs[0].n / t1, "seconds": t1, "particles": subs[0].n,
                              "levels": len(lev), "runs": repeats},
            "build": "gcc -O3 -march=native", **info}


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def batched_measure(warmup, chains=(1, 2, 4, 8), servers=(2, 4, 8), runs=3):
    """64 independent periodic sub-volumes with particle counts log-uniform in
    1e4..1e7 (seed 3; halo fraction 10..40%, domain grid ~N^{1/3}/2 clamped to
    32^3..128^3, threshold 5, 10 levels), built three ways: one at a time on
    one stream (sequential), by the server with several workers, and as a
    batch (ahf_batch: one host wait per run) with the builds in several
    chains."""
    import torch
    from paper_0904_3662_amd import ahf, synth
    sizes = synth.subvolume_sizes(3, 64, 4.0, 7.0)
    t0 = time.perf_counter()
    subs = [synth.subvolume(1000 + i, int(n)) for i, n in enumerate(sizes)]
    print(f"# generated 64 sub-volumes, {int(sizes.sum())} particles in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    devs = [ahf.snapshot_to_device(s) for s in subs]
    torch.cuda.synchronize()
    ctx = ahf.Context(0)
    total = int(sizes.sum())
    order = np.argsort(-sizes, kind="stable")  # largest first
    out = {"workload": "64 sub-volumes, N log-uniform 1e4..1e7", "particles": total,
           "sub_volumes": 64}
    # sequential: one stream, one build at a time
    for rep in range(warmup + 1):
        lat = []
        a = time.perf_counter()
        for i in order:
            b = time.perf_counter()
            h, _ = ahf.build_snapshot(ctx, subs[i], dev=devs[i])
            h.free()
            lat.append((time.perf_counter() - b) * 1e3)
        seq = time.perf_counter() - a
    out["sequential"] = {"value": total / seq, "seconds": seq, "p50_ms": _pct(lat, 50),
                         "p99_ms": _pct(lat, 99)}
    print(f"# sequential {seq:.3f} s", file=sys.stderr, flush=True)
    for k in servers:
        with ahf.Server(ctx, n_streams=k) as srv:
            for rep in range(warmup + 1):
                a = time.perf_counter()
                tickets = [srv.submit_snapshot(subs[i], dev=devs[i]) for i in order]
                for t in tickets:
                    srv.wait(t)
                el = time.perf_counter() - a
                lat = []
                for t in tickets:
                    tt = srv.times(t)
                    lat.append(tt[3] - tt[0])
                    srv.release(t)
        out[f"server_{k}"] = {"value": total / el, "seconds": el, "p50_ms": _pct(lat, 50),
                              "p99_ms": _pct(lat, 99)}
        print(f"# server with {k} workers {el:.3f} s", file=sys.stderr, flush=True)
    # a batch: one host wait per run, every sub-volume rebuilt from its arrays
    stream = torch.cuda.current_stream()
    for k in chains:
        a = time.perf_counter()
        bt = ahf.Batch(ctx, [subs[i] for i in order], [devs[i] for i in order], n_chains=k,
                       stream=stream)
        setup = time.perf_counter() - a
        for rep in range(warmup):
            bt.run(stream)
            bt.wait()
        lat = []
        a = time.perf_counter()
        for rep in range(runs):
            b = time.perf_counter()
            bt.run(stream)
            bt.wait()
            lat.append((time.perf_counter() - b) * 1e3)
        el = (time.perf_counter() - a) / runs
        bt.close()
        out[f"batch_{k}"] = {"value": total / el, "seconds": el, "p50_ms": _pct(lat, 50),
                             "p99_ms": _pct(lat, 99), "setup_s": setup}
        print(f"# batch with {k} chains {el:.3f} s per run (set-up {setup:.1f} s)",
              file=sys.stderr, flush=True)
    best = max((out[key]["value"], key) for key in out
               if key.startswith("server_") or key.startswith("batch_"))
    out["value"] = best[0]
    out["best"] = best[1]
    out["speedup_vs_sequential"] = best[0] / out["sequential"]["value"]
    ctx.close()
    return out


def run_batched(args):
    res = batched_measure(args.warmup)
    out = {"metric": "particles/s through full hierarchy build, batched sub-volumes",
           "unit": "particles/s", "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "value": res["value"], "config": {"workload": res["workload"],
                                             "particles": res["particles"],
                                             "sub_volumes": res["sub_volumes"]}}
    out.update({k: v for k, v in res.items() if k not in out and k != "value"})
    print(json.dumps(out), flush=True)


def run_served(args):
    out = served_measure(args.pool, args.requests, args.streams, (0.5, 0.8, 1.2))
    print(json.dumps(out), flush=True)


def served_measure(npool, R, streams, fracs):
    """Poisson stream of sub-volume builds, sizes log-uniform in 1e5..5e7 (seed 4),
    admitted by the server against the HBM budget, results kept resident for
    follow-up label queries; each arrival rate (a fraction of the sequential
    capacity) is run with several streams and with one stream (the
    sequential per-request path)."""
    import torch
    from paper_0904_3662_amd import ahf, synth
    sizes = synth.subvolume_sizes(4, npool, 5.0, float(np.log10(5e7)))
    t0 = time.perf_counter()
    subs = [synth.subvolume(4000 + i, int(n)) for i, n in enumerate(sizes)]
    print(f"# generated a pool of {npool} sub-volumes, {int(sizes.sum())} particles in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    devs = [ahf.snapshot_to_device(s) for s in subs]
    torch.cuda.synchronize()
    ctx = ahf.Context(0)
    rng = np.random.Generator(np.random.PCG64(44))
    pick = rng.integers(0, npool, R)
    # sequential capacity: mean build time over the request mix
    for i in range(npool):
        h, _ = ahf.build_snapshot(ctx, subs[i], dev=devs[i])
        h.free()
    tb = []
    for i in range(npool):
        a = time.perf_counter()
        h, _ = ahf.build_snapshot(ctx, subs[i], dev=devs[i])
        h.free()
        tb.append(time.perf_counter() - a)
    mean_t = float(np.mean(np.asarray(tb)[pick]))
    capacity = 1.0 / mean_t
    out = {"metric": "particles/s through full hierarchy build, served request stream",
           "unit": "particles/s", "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"Poisson stream, {R} requests from a pool of {npool} "
                                  "sub-volumes, N log-uniform 1e5..5e7",
                      "requests": R, "sequential_capacity_req_per_s": capacity},
           "rates": {}}
    for frac in fracs:
        lam = frac * capacity
        gaps = rng.exponential(1.0 / lam, R)
        arrive = np.cumsum(gaps)
        res = {}
        for k in (1, streams):
            with ahf.Server(ctx, n_streams=k) as srv:
                live = []
                lat = []
                queries = 0
                a = time.perf_counter()
                i = 0
                while i < R or live:
                    now = time.perf_counter() - a
                    if i < R and now >= arrive[i]:
                        live.append(srv.submit_snapshot(subs[pick[i]], dev=devs[pick[i]]))
                        i += 1
                        continue
                    still = []
                    for t in live:
                        h = srv.poll(t)
                        if h is None:
                            still.append(t)
                            continue
                        if h.num_levels() > 1:
                            v = h.view(1)
                            keys = np.arange(min(64, v.n_cells), dtype=np.uint64)
                            srv.query_label(t, 1, keys)
                            queries += 1
                        tt = srv.times(t)
                        lat.append(tt[3] - tt[0])
                        srv.release(t)
                    live = still
                    if i < R:
                        wait = arrive[i] - (time.perf_counter() - a)
                        if wait > 0:
                            time.sleep(min(wait, 0.0005))
                    else:
                        time.sleep(0.0002)
                el = time.perf_counter() - a
                parts = int(sizes[pick].sum())
                res[f"streams_{k}"] = {"value": parts / el, "seconds": el,
                                       "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                                       "label_queries": queries,
                                       "bytes_peak": srv.stats()["bytes_peak"]}
            print(f"# rate {frac} x capacity, {k} streams: {el:.2f} s, p99 "
                  f"{res[f'streams_{k}']['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        out["rates"][f"{frac}"] = {"req_per_s": lam, **res}
    r = out["rates"][f"{0.8 if 0.8 in fracs else fracs[0]}"]
    out["value"] = r[f"streams_{streams}"]["value"]
    out["p50_ms"] = r[f"streams_{streams}"]["p50_ms"]
    out["p99_ms"] = r[f"streams_{streams}"]["p99_ms"]
    out["n_streams"] = streams
    ctx.close()
    del devs
    return out


# per-launch algorithmic bytes of the kernels that can be the roofline kernel
# (what the step must move, not what the implementation moves):
#  rs_scatter: one radix pass reads and writes every element (sort_scatter_bytes)
#  gather: the sorted word (8 B) and the payload X,Y,Z,fx,fy,fz (24 B) read,
#          the payload (24 B), the particle index (4 B) and the full key (8 B)
#          written per particle, and the level-0 cell starts (4 B per cell)
#  tile_deposit0/1: the level's particles (24 B each), the cell ranges (8 B per
#          cell of S_L) and the field (4 B per brick cell) -- the per-level
#          deposit terms of the algorithmic byte count
ROOFLINE_KERNELS = ("rs_scatter", "gather", "tile_deposit0", "tile_deposit1")
# what holds each candidate below its HBM roofline, from the counters in profiles/
LIMITER = {
    "rs_scatter": "HBM traffic of the scatter passes",
    "gather": "random 32-byte record reads, each fetching a whole line",
    "tile_deposit0": "latency of dependent loads (ranks, cell ranges, records) and the barrier",
    "tile_deposit1": "latency of dependent loads (ranks, cell ranges, records) and the barrier: "
                     "0.68 of wave cycles waiting, 0.14 issuing VALU",
}


def kernel_alg_bytes(name, n, key_bits, g, lv_info, launches_per_step):
    if name == "rs_scatter":
        return sort_scatter_bytes(n, key_bits) / max(launches_per_step, 1)
    if name == "gather":
        return 68.0 * n + 4.0 * ((1 << (3 * g)) + 1)
    L = 0 if name == "tile_deposit0" else 1
    if L >= len(lv_info):
        return None
    d = lv_info[L]
    return 24.0 * d["n_particles"] + 8.0 * d["n_cells"] + 32.0 * d["n_bricks"]


def measure(ctx, snap, dev, stream, steps, warmup, extras=True):
    """Warm-up builds (the first also records the level sizes, the second the
    per-kernel split with every kernel timed), then `steps` timed builds with
    HIP events only around the roofline kernel, on the stream it runs on."""
    import torch
    from paper_0904_3662_amd import ahf

    def step():
        h, _ = ahf.build_snapshot(ctx, snap, dev=dev, stream=stream)
        return h

    names = ("rs_scatter", "rs_up", "rs_tscan", "keys", "gather", "fix_runs", "fix_long_runs",
             "child_ranges",
             "heavy_chunk", "tile_deposit0", "tile_deposit1", "tile_halo", "patches",
             "combine", "mark", "uf_hook", "uf_cross")
    lv_info = None
    ksplit = {}
    for i in range(max(warmup, 2)):
        if i == 1:
            ctx.profile_only(None)
            ctx.set_profiling(True)
        h = step()
        if i == 0:
            lv_info = [dict(n_particles=v.n_particles, n_cells=v.n_cells, n_bricks=v.n_bricks,
                            n_refined=v.n_refined, n_patches=v.n_patches)
                       for v in (h.view(L) for L in range(h.num_levels()))]
            sort_bits = h.build_info()["sort_key_bits"]
        h.free()
        if i == 1:
            torch.cuda.synchronize()
            ksplit = {nm: ctx.kernel_time(nm) for nm in names}
            ctx.set_profiling(False)
        print(f"# {snap.name}: warmup {i} done", file=sys.stderr, flush=True)
    n = snap.n
    key_bits = sort_bits  # the bits the sort ordered by (it may leave low ones out)
    # the roofline kernel: the one of the candidates with the most time per build
    rk = max(ROOFLINE_KERNELS, key=lambda nm: ksplit.get(nm, (0, 0.0))[1])
    per_step = max(ksplit.get(rk, (1, 0.0))[0], 1)

    ctx.profile_only([rk])
    ctx.set_profiling(True)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = []
    for i in range(steps):
        a = time.perf_counter()
        h = step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
        infos.append(h.build_info())
        h.free()
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    launches, tms = ctx.kernel_time(rk)
    ctx.set_profiling(False)
    print(f"# {snap.name}: {steps} steps in {total:.3f} s", file=sys.stderr, flush=True)

    ms_per_step = total * 1e3 / steps
    avg_ms = tms / max(launches, 1)
    alg = kernel_alg_bytes(rk, n, key_bits, snap.g, lv_info, per_step)
    achieved = alg / (avg_ms * 1e-3) / 1e9 if launches and alg else None
    traffic = measured_traffic(snap.name, rk)
    out = {
        "value": n * steps / total,
        "ms_per_step": ms_per_step,
        "p50_ms": _pct(lat, 50),
        "p99_ms": _pct(lat, 99),
        "end_to_end_hbm_frac": algorithmic_bytes(n, lv_info) / (ms_per_step * 1e-3) /
                               (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "kernel": rk, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_over_algorithmic": None if traffic is None else traffic / alg,
                     "algorithmic_bytes_per_launch": alg, "avg_launch_ms": avg_ms,
                     "launches": launches, "limiter": LIMITER.get(rk)},
        "kernels_ms_per_step": {nm: v[1] for nm, v in ksplit.items()},
        "levels": lv_info,
        # timed builds sized ahead from the context's plan (no host wait per
        # level), and the host waits for level counts per build
        "planned_builds": sum(i["planned"] for i in infos),
        "host_waits_per_build": float(np.mean([i["host_waits"] for i in infos])),
    }
    # the other candidates, from the profiled warm-up build
    others = {}
    for nm in ROOFLINE_KERNELS:
        cnt, t = ksplit.get(nm, (0, 0.0))
        b = kernel_alg_bytes(nm, n, key_bits, snap.g, lv_info, cnt)
        if cnt and b:
            gbs = b / (t / cnt * 1e-3) / 1e9
            others[nm] = {"achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "avg_launch_ms": t / cnt,
                          "algorithmic_bytes_per_launch": b, "launches_per_build": cnt}
    out["kernel_rooflines"] = others
    if not extras:
        return out

    # host/substructure classification of the grid tree (a step after the
    # labels): wall time of the classification call on built hierarchies
    cls = []
    for i in range(3):
        h = step()
        torch.cuda.synchronize()
        a = time.perf_counter()
        h.classify(ctx, stream)
        cls.append((time.perf_counter() - a) * 1e3)
        nstruct = h.structures()["n_structures"]
        h.free()
    # the paper-literal density criterion (refine on the TSC particle number):
    # same workload and thresholds, whole builds timed
    # these builds run on one stream, so the roofline kernel runs there
    # alone: its HIP-event time in builds 2-4 and its own level sizes
    dens = []
    dens_lv = None
    for i in range(4):
        if i == 1:
            ctx.profile_only([rk])
            ctx.set_profiling(True)
        torch.cuda.synchronize()
        a = time.perf_counter()
        h, _ = ahf.build_snapshot(ctx, snap, dev=dev, stream=stream, density_criterion=True)
        torch.cuda.synchronize()
        dens.append((time.perf_counter() - a) * 1e3)
        dens_levels = h.num_levels()
        if i == 0:
            dens_lv = [dict(n_particles=v.n_particles, n_cells=v.n_cells, n_bricks=v.n_bricks)
                       for v in (h.view(L) for L in range(h.num_levels()))]
        h.free()
    alone_n, alone_t = ctx.kernel_time(rk)
    ctx.set_profiling(False)
    alone_b = kernel_alg_bytes(rk, n, key_bits, snap.g, dens_lv, max(alone_n // 3, 1))
    if alone_n and alone_b:
        alone_ms = alone_t / alone_n
        out["roofline"]["alone"] = {
            "what": "the same kernel in the one-stream builds of the density criterion, "
                    "priced on their own level sizes",
            "avg_launch_ms": alone_ms, "launches": alone_n, "algorithmic_bytes_per_launch": alone_b,
            "achieved": alone_b / (alone_ms * 1e-3) / 1e9,
            "frac": alone_b / (alone_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    out["substructure"] = {"ms": float(np.median(cls)), "structures": int(nstruct)}
    # particle collection and unbinding of every structure (needs velocities)
    if snap.vel is not None:
        vel = torch.from_numpy(snap.vel).to("cuda")
        h = step()
        h.classify(ctx, stream)
        hal = []
        for i in range(3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            res = ahf.find_halos(ctx, h, dev, vel, stream=stream, fetch=False)
            torch.cuda.synchronize()
            hal.append((time.perf_counter() - a) * 1e3)
        h.free()
        del vel
        cand = int(res["cand_count"].astype(np.int64).sum())
        out["halos"] = {"ms": float(np.median(hal)), "halos": int(res["n_halos"]),
                        "with_particles": int((res["member_count"] > 0).sum()),
                        "candidates": cand,
                        "members": int(res["member_count"].astype(np.int64).sum()),
                        "max_rounds": int(res["iterations"].max()) if res["n_halos"] else 0,
                        "candidates_per_s": cand / (float(np.median(hal)) * 1e-3)}
        print(f"# {snap.name}: halos {np.median(hal):.2f} ms", file=sys.stderr, flush=True)
    out["density_criterion"] = {"ms_per_build": float(np.median(dens[1:])),
                                "levels_built": int(dens_levels)}
    return out


WORKLOADS = {"134m": ("snapshot_134m", 2), "16m": ("snapshot_16m", 1), "32k": ("small_mixed", 0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true",
                    help="leave the short served stream out of the default line")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched sub-volume measurement of the default line")
    ap.add_argument("--cpu-cube", type=int, default=48,
                    help="sub-cube edge in domain cells for the CPU baseline")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0: the host's share, at most 16)")
    ap.add_argument("--cpu-repeats", type=int, default=1)
    ap.add_argument("--workload", default="134m", choices=sorted(WORKLOADS))
    ap.add_argument("--extra-workload", default="16m", choices=sorted(WORKLOADS) + ["none"],
                    help="a second workload measured the same way, reported under its name")
    ap.add_argument("--mode", default="single", choices=["single", "batched", "served"])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=8)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batched":
        return run_batched(args)
    if args.mode == "served":
        return run_served(args)

    import torch
    from paper_0904_3662_amd import ahf, synth

    def make(w, velocities=False):
        fn, seed = WORKLOADS[w]
        t0 = time.perf_counter()
        sn = getattr(synth, fn)(seed, velocities=velocities)
        print(f"# generated {sn.name}: {sn.n} particles in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        return sn

    snap = make(args.workload, velocities=True)  # velocities for the halo step
    torch.cuda.set_device(0)
    ctx = ahf.Context(0)
    stream = torch.cuda.current_stream()
    dev = ahf.snapshot_to_device(snap)
    torch.cuda.synchronize()
    res = measure(ctx, snap, dev, stream, args.steps, args.warmup)
    del dev
    extra = None
    if args.extra_workload not in ("none", args.workload):
        esnap = make(args.extra_workload)
        edev = ahf.snapshot_to_device(esnap)
        torch.cuda.synchronize()
        extra = measure(ctx, esnap, edev, stream, args.steps, args.warmup, extras=False)
        extra["config"] = {"workload": esnap.name, "particles": esnap.n,
                           "domain_grid": 1 << esnap.g, "threshold": esnap.dom_ref,
                           "max_levels": esnap.max_levels, "levels_built": len(extra["levels"])}
        del edev, esnap
    n = snap.n
    rec = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": snap.name, "particles": n, "domain_grid": 1 << snap.g,
                   "threshold": snap.dom_ref, "max_levels": snap.max_levels,
                   "levels_built": len(res["levels"])},
    }
    rec.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step")})
    if extra is not None:
        rec["workload_" + extra["config"]["workload"]] = extra
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)   # a plain streaming kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = 2 * a.numel() * 4
        del a, b
    ctx.close()
    if not args.no_batched:
        # the batched form: 64 sub-volumes, sequential vs server vs batch
        rec["batched"] = batched_measure(args.warmup, chains=(1, 4), servers=(4,), runs=3)
    if not args.no_served:
        # the served form: a short Poisson stream at 0.8 of the sequential
        # capacity, 4 streams against one
        rec["served"] = served_measure(8, 300, 4, (0.8,))
    if not args.no_cpu_baseline:
        share = host_info()["affinity"]
        threads = args.cpu_threads or min(16, share)
        rec["cpu_baseline"] = cpu_baseline(snap, args.cpu_cube, threads, args.cpu_repeats)
        print("# cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
