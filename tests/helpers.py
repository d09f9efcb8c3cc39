"""Shared test helpers: tiny hand-made particle sets and comparisons.
Holds no hierarchy arithmetic."""
from __future__ import annotations

import numpy as np

from paper_0904_3662_amd.synth import Snapshot, quantize, small_mixed

Q = 1 << 21


def particles(X, Y, Z, fx=None, fy=None, fz=None, mass=None, g=3, thr=5.0, max_levels=3,
              ref=None, name="hand"):
    X = np.asarray(X, np.uint32); Y = np.asarray(Y, np.uint32); Z = np.asarray(Z, np.uint32)
    n = len(X)
    z = np.zeros(n, np.float32)
    fx = z.copy() if fx is None else np.asarray(fx, np.float32)
    fy = z.copy() if fy is None else np.asarray(fy, np.float32)
    fz = z.copy() if fz is None else np.asarray(fz, np.float32)
    m = None if mass is None else np.asarray(mass, np.float32)
    return Snapshot(X, Y, Z, fx, fy, fz, m, g, float(thr), float(thr if ref is None else ref),
                    max_levels, name)


def from_positions(pos, **kw):
    pos = np.asarray(pos, np.float64)
    X, fx = quantize(pos[:, 0]); Y, fy = quantize(pos[:, 1]); Z, fz = quantize(pos[:, 2])
    return particles(X, Y, Z, fx, fy, fz, **kw)


def uniform(seed, n, **kw):
    rng = np.random.Generator(np.random.PCG64(seed))
    return from_positions(rng.random((n, 3)), **kw)


def clustered(seed, n, n_clumps=3, spread=0.01, frac=0.7, **kw):
    rng = np.random.Generator(np.random.PCG64(seed))
    nc = int(frac * n)
    centres = rng.random((n_clumps, 3))
    which = rng.integers(0, n_clumps, nc)
    pos = np.concatenate([centres[which] + rng.normal(0, spread, (nc, 3)),
                          rng.random((n - nc, 3))])
    return from_positions(pos, **kw)


def small_mixed_scaled(seed=0, n=4096, g=4, max_levels=3):
    """The 32^3 mixed recipe shrunk (random subset) for quick oracle runs."""
    s = small_mixed(seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    idx = np.sort(rng.choice(s.n, n, replace=False))
    t = s.subset(idx, name=f"small-mixed-{n}")
    t.g = g
    t.max_levels = max_levels
    return t


def morton_py(x, y, z, bits):
    """Independent vectorised Morton key (bit 3j+2 = x_j, 3j+1 = y_j, 3j = z_j)."""
    x = np.asarray(x, np.uint64); y = np.asarray(y, np.uint64); z = np.asarray(z, np.uint64)
    k = np.zeros(x.shape, np.uint64)
    for j in range(bits):
        jj = np.uint64(j)
        one = np.uint64(1)
        k |= ((x >> jj) & one) << np.uint64(3 * j + 2)
        k |= ((y >> jj) & one) << np.uint64(3 * j + 1)
        k |= ((z >> jj) & one) << np.uint64(3 * j)
    return k


def demorton_py(k, bits):
    k = np.asarray(k, np.uint64)
    x = np.zeros(k.shape, np.uint64); y = np.zeros(k.shape, np.uint64); z = np.zeros(k.shape, np.uint64)
    one = np.uint64(1)
    for j in range(bits):
        jj = np.uint64(j)
        x |= ((k >> np.uint64(3 * j + 2)) & one) << jj
        y |= ((k >> np.uint64(3 * j + 1)) & one) << jj
        z |= ((k >> np.uint64(3 * j)) & one) << jj
    return x, y, z
