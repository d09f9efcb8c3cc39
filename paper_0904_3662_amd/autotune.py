"""Autotuner of the build's bin sizes: per size class, the light/heavy cell
thresholds of level 0, level 1 and the deeper levels, the records in flight
per thread on level 1, and the low key digits the sort leaves out
(ahf_ctx_set_tuning).

For each size class a seeded snapshot of the lattice + NFW recipe is built on
the GPU with every candidate tuning (coordinate descent from the library's
defaults: level 1 first, then level 0, the deeper levels, the sort), the median
build time of a few builds decides, and the winners are written as a JSON
table that ahf.Context loads (tuning_gfx950.json beside this file).

    python -m paper_0904_3662_amd.autotune [--out FILE] [--sizes N ...]

Every tuning gives the same hierarchy up to FP32 summation order (the tests
check the oracle's parity for several), so the table only changes speed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning_gfx950.json")

DEFAULTS = dict(heavy_level0=64, heavy_level1=64, heavy_deeper=64, batch_level1=2,
                sort_skip_digits=-1)
CANDIDATES = {
    "level1": [dict(heavy_level1=h, batch_level1=b) for h in (8, 16, 32, 64) for b in (2, 4)],
    "level0": [dict(heavy_level0=h) for h in (16, 32, 48, 64)],
    "deeper": [dict(heavy_deeper=h) for h in (16, 32, 48, 64)],
    "sort": [dict(sort_skip_digits=k) for k in (-1, 0, 1, 2)],
}
# size classes: the tuning of the largest min_n <= n applies
SIZES = [1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 27]


def snapshot_for(n: int):
    from paper_0904_3662_amd import synth
    if n >= 1 << 27:
        return synth.snapshot_134m(2)
    if n == 1 << 24:
        return synth.snapshot_16m(1)
    return synth.scaled_like_16m(1000 + int(np.log2(n)), n)


def time_builds(ctx, snap, dev, tuning, reps):
    import torch
    from paper_0904_3662_amd import ahf
    ctx.set_tuning([(0, tuning)])
    stream = torch.cuda.current_stream()
    for _ in range(2):  # warm-up (the first also teaches the build plan)
        ahf.build_snapshot(ctx, snap, dev=dev, stream=stream)[0].free()
    lat = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        h, _ = ahf.build_snapshot(ctx, snap, dev=dev, stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
        h.free()
    return float(np.median(lat))


def tune_size(ctx, n, reps, log):
    from paper_0904_3662_amd import ahf
    snap = snapshot_for(n)
    dev = ahf.snapshot_to_device(snap)
    best = dict(DEFAULTS)
    best_ms = time_builds(ctx, snap, dev, best, reps)
    log(f"n={snap.n}: defaults {best_ms:.3f} ms")
    for stage in ("level1", "level0", "deeper", "sort"):
        for cand in CANDIDATES[stage]:
            t = dict(best, **cand)
            if t == best:
                continue
            ms = time_builds(ctx, snap, dev, t, reps)
            log(f"n={snap.n}: {stage} {cand} {ms:.3f} ms")
            if ms < best_ms * 0.99:  # a clear gain only
                best, best_ms = t, ms
    del dev
    return dict(best, min_n=int(n), ms=best_ms, particles=int(snap.n))


def load_table(path: str = DEFAULT_TABLE):
    """The tuning table as [(min_n, tuning dict)], or [] without a file."""
    if not os.path.exists(path):
        return []
    with open(path) as f:
        doc = json.load(f)
    keys = ("heavy_level0", "heavy_level1", "heavy_deeper", "batch_level1")
    return [(int(e["min_n"]), dict({k: int(e[k]) for k in keys},
                                   sort_skip_digits=int(e.get("sort_skip_digits", -1))))
            for e in doc["entries"]]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--sizes", type=int, nargs="*", default=SIZES)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    import torch
    from paper_0904_3662_amd import ahf
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    entries = []
    with ahf.Context(0, tuning=None) as ctx:
        for n in args.sizes:
            entries.append(tune_size(ctx, n, args.reps, log))
    doc = {"device": torch.cuda.get_device_name(0), "method": "coordinate descent, median of "
           f"{args.reps} builds per candidate after 2 warm-up builds", "entries": entries}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
