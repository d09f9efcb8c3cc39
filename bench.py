"""Throughput of the full hierarchy build on one MI355X.

One step = one complete build of the adaptive density hierarchy (Morton keys,
stable sort, per-level counts, refinement flags, TSC deposit, FP64 totals,
grid-tree labels) of the 16.8M-particle lattice + NFW-halo snapshot (256^3
particles, 128^3 domain grid, threshold 5, up to 10 levels), with the input
already resident in HBM.  Prints one JSON line.
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


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_rs_scatter_lattice-nfw-16.8M.txt")
# the files the scatter kernel is compiled from
SCATTER_SRC = [os.path.join(ROOT, "paper_0904_3662_amd", "csrc", f)
               for f in ("ahf_prims.hip", "ahf_dev.h", "ahf_internal.h")]


def scatter_source_hash():
    h = hashlib.sha256()
    for f in SCATTER_SRC:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per scatter launch from the committed PMC summary (FETCH_SIZE
    and WRITE_SIZE runs scaled by a copy kernel of known size), or None when
    the summary is for another workload or the scatter source has changed
    since the counters were taken."""
    if workload != "lattice-nfw-16.8M" or not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    for line in open(PMC_SUMMARY):
        if line.startswith("rs_scatter_traffic_bytes_per_launch:"):
            vals["t"] = float(line.split(":")[1])
        if line.startswith("source_sha256"):
            vals["h"] = line.split(":")[1].strip()
    if "t" not in vals or vals.get("h") != scatter_source_hash():
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


def cpu_baseline(snap, seconds_target=20.0):
    """The FP64 oracle on a bounded random sample of the same workload."""
    import oracle
    rng = np.random.Generator(np.random.PCG64(12345))
    n = min(snap.n, 1 << 22)  # about 20 s of single-thread oracle work
    idx = np.sort(rng.choice(snap.n, n, replace=False))
    sub = snap.subset(idx, "sample")
    t0 = time.perf_counter()
    oracle.build(sub)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} particles drawn at random (seed 12345) from the 16.8M snapshot, "
                      f"same grid parameters, single-threaded FP64 oracle, {dt:.1f} s"}


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def run_batched(args):
    """64 independent periodic sub-volumes with particle counts log-uniform in
    1e4..1e7 (seed 3; halo fraction 10..40%, domain grid ~N^{1/3}/2 clamped to
    32^3..128^3, threshold 5, 10 levels): the sequential one-stream path against
    the server with several streams building them concurrently."""
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
    out = {"metric": "particles/s through full hierarchy build, batched sub-volumes",
           "unit": "particles/s", "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "64 sub-volumes, N log-uniform 1e4..1e7", "particles": total,
                      "sub_volumes": 64}}
    # sequential: one stream, one build at a time
    for rep in range(args.warmup + 1):
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
    for k in (2, 4, 8):
        with ahf.Server(ctx, n_streams=k) as srv:
            for rep in range(args.warmup + 1):
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
        out[f"streams_{k}"] = {"value": total / el, "seconds": el, "p50_ms": _pct(lat, 50),
                               "p99_ms": _pct(lat, 99)}
        print(f"# {k} streams {el:.3f} s", file=sys.stderr, flush=True)
    best = max((out[f"streams_{k}"]["value"], k) for k in (2, 4, 8))
    out["value"] = best[0]
    out["n_streams"] = best[1]
    out["speedup_vs_sequential"] = best[0] / out["sequential"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


def run_served(args):
    """Poisson stream of sub-volume builds, sizes log-uniform in 1e5..5e7 (seed 4),
    admitted by the server against the HBM budget, results kept resident for
    follow-up label queries; each arrival rate is run with several streams and
    with one stream (the sequential per-request path)."""
    import torch
    from paper_0904_3662_amd import ahf, synth
    npool = args.pool
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
    R = args.requests
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
    for frac in (0.5, 0.8, 1.2):
        lam = frac * capacity
        gaps = rng.exponential(1.0 / lam, R)
        arrive = np.cumsum(gaps)
        res = {}
        for k in (1, args.streams):
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
    r = out["rates"]["0.8"]
    out["value"] = r[f"streams_{args.streams}"]["value"]
    out["p50_ms"] = r[f"streams_{args.streams}"]["p50_ms"]
    out["p99_ms"] = r[f"streams_{args.streams}"]["p99_ms"]
    out["n_streams"] = args.streams
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="16m", choices=["16m", "32k"])
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

    t0 = time.perf_counter()
    snap = synth.snapshot_16m(1) if args.workload == "16m" else synth.small_mixed(0)
    print(f"# generated {snap.name}: {snap.n} particles in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    dev = ahf.snapshot_to_device(snap)
    torch.cuda.synchronize()
    ctx = ahf.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        h, _ = ahf.build_snapshot(ctx, snap, dev=dev, stream=stream)
        return h

    for i in range(args.warmup):
        h = step()
        if i == 0:
            levels = [h.view(L) for L in range(h.num_levels())]
            lv_info = [dict(n_particles=v.n_particles, n_cells=v.n_cells, n_bricks=v.n_bricks,
                            n_refined=v.n_refined, n_patches=v.n_patches) for v in levels]
        h.free()
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    if args.warmup == 0:
        h = step()
        lv_info = [dict(n_particles=h.view(L).n_particles, n_cells=h.view(L).n_cells,
                        n_bricks=h.view(L).n_bricks, n_refined=h.view(L).n_refined,
                        n_patches=h.view(L).n_patches) for L in range(h.num_levels())]
        h.free()

    # timed region: HIP events only around the roofline kernel (the sort
    # scatter), on the build stream; each event recorded between two kernels
    # holds the stream for a few microseconds, so nothing else is timed here
    ctx.profile_only(["rs_scatter"])
    ctx.set_profiling(True)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        h = step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
        h.free()
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    kstats = {"rs_scatter": ctx.kernel_time("rs_scatter")}
    ctx.set_profiling(False)
    print(f"# steps done: {args.steps} in {total:.3f} s", file=sys.stderr, flush=True)

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
    dens = []
    for i in range(4):
        torch.cuda.synchronize()
        a = time.perf_counter()
        h, _ = ahf.build_snapshot(ctx, snap, dev=dev, stream=stream, density_criterion=True)
        torch.cuda.synchronize()
        dens.append((time.perf_counter() - a) * 1e3)
        dens_levels = h.num_levels()
        h.free()

    # per-kernel split from two more builds, untimed, with every kernel timed
    names = ("rs_scatter", "rs_up", "rs_tscan", "keys", "gather", "child_ranges",
             "heavy_chunk", "patches", "combine", "mark", "uf_hook", "uf_cross")
    ctx.profile_only(None)
    ctx.set_profiling(True)
    for i in range(2):
        step().free()
    torch.cuda.synchronize()
    ksplit = {name: ctx.kernel_time(name)[1] / 2 for name in names}
    kstats["gather"] = ctx.kernel_time("gather")
    ctx.set_profiling(False)

    n = snap.n
    ms_per_step = total * 1e3 / args.steps
    value = n * args.steps / total
    launches, tms = kstats["rs_scatter"]
    avg_ms = tms / max(launches, 1)
    alg_bytes_launch = sort_scatter_bytes(n, 3 * (snap.g + snap.max_levels)) / max(launches // args.steps, 1)
    achieved = alg_bytes_launch / (avg_ms * 1e-3) / 1e9 if launches else None
    b_alg = algorithmic_bytes(n, lv_info)
    traffic = measured_traffic(snap.name)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": snap.name, "particles": n, "domain_grid": 1 << snap.g,
                   "threshold": snap.dom_ref, "max_levels": snap.max_levels,
                   "levels_built": len(lv_info)},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "end_to_end_hbm_frac": b_alg / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "kernel": "rs_scatter", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_over_algorithmic":
                         None if traffic is None else traffic / alg_bytes_launch,
                     "avg_launch_ms": avg_ms, "launches": launches},
        # the particle gather, the largest single launch: 8 B word + 32 B record
        # read, 32 B record + 4 B index + 8 B key written per particle (timed
        # in the two builds after the timed region)
        "gather_roofline": None if not kstats["gather"][0] else {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "achieved": 84.0 * n / (kstats["gather"][1] / kstats["gather"][0] * 1e-3) / 1e9,
            "frac": 84.0 * n / (kstats["gather"][1] / kstats["gather"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernels_ms_per_step": ksplit,
        "substructure": {"ms": float(np.median(cls)), "structures": int(nstruct)},
        "density_criterion": {"ms_per_build": float(np.median(dens[1:])),
                              "levels_built": int(dens_levels)},
        "levels": lv_info,
    }
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)   # a plain streaming kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = 2 * a.numel() * 4
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(snap)
    ctx.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
