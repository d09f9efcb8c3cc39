"""Seeded synthetic particle snapshots in a periodic unit box.

This module only makes inputs; it holds none of the hierarchy arithmetic and
is shared by the oracle tests, the GPU tests and the benchmark.  The paper's
simulations (its Table 1 set) are not available, so NFW halos on top of a
uniform or Gaussian-perturbed-lattice background stand in for them.

Canonical particle format (what both the oracle and the device library take):
  X, Y, Z : uint32, the integer part of x * 2**21 (21 significant bits)
  fx, fy, fz : float32 in [0, 1), the remaining fraction of x * 2**21
  mass : None (every particle has mass 1) or float32 per particle

Generators:
  quantize                 positions in [0,1) -> (X, f)
  power_law_counts         halo particle budgets from dN/dM ~ M^slope
  nfw_offsets              isotropic offsets following a truncated NFW profile
  plummer_offsets          isotropic offsets following a truncated Plummer sphere
  snapshot                 the general recipe (background + halos [+ subhalos])
  small_mixed / snapshot_16m / snapshot_134m / subvolume   the named workloads
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

QBITS = 21
QSCALE = float(1 << QBITS)


@dataclasses.dataclass
class Snapshot:
    X: np.ndarray
    Y: np.ndarray
    Z: np.ndarray
    fx: np.ndarray
    fy: np.ndarray
    fz: np.ndarray
    mass: np.ndarray | None
    g: int            # domain grid = 2**g cells per axis
    dom_ref: float
    ref_ref: float
    max_levels: int
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)
    vel: np.ndarray | None = None  # (n, 3) float32 velocities, when drawn

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    def params(self, connectivity: int = 26) -> dict:
        return dict(g=self.g, dom_ref=self.dom_ref, ref_ref=self.ref_ref,
                    max_levels=self.max_levels, connectivity=connectivity)

    def subset(self, idx: np.ndarray, name: str | None = None) -> "Snapshot":
        return Snapshot(self.X[idx].copy(), self.Y[idx].copy(), self.Z[idx].copy(),
                        self.fx[idx].copy(), self.fy[idx].copy(), self.fz[idx].copy(),
                        None if self.mass is None else self.mass[idx].copy(),
                        self.g, self.dom_ref, self.ref_ref, self.max_levels,
                        name or self.name + "-subset", dict(self.meta),
                        None if self.vel is None else self.vel[idx].copy())


def quantize(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Unit-box coordinate (any real; wrapped periodically) -> (uint32 X, float32 f)."""
    x = np.asarray(x, dtype=np.float64)
    x = x - np.floor(x)
    s = x * QSCALE
    Xi = np.floor(s)
    Xi = np.clip(Xi, 0, QSCALE - 1)
    f = (s - Xi).astype(np.float32)
    below_one = np.float32(np.nextafter(np.float32(1.0), np.float32(0.0)))
    f = np.minimum(np.maximum(f, np.float32(0.0)), below_one)
    return Xi.astype(np.uint32), f


def power_law_counts(rng: np.random.Generator, k: int, lo: float, hi: float,
                     budget: int, slope: float = -1.9) -> np.ndarray:
    """k halo sizes drawn from dN/dM ~ M^slope on [lo, hi] by inverse CDF, then
    scaled by one common factor so they sum to `budget` exactly (largest-remainder
    rounding, every halo keeps at least one particle)."""
    a = slope + 1.0
    u = rng.random(k)
    m = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    w = m * (budget / m.sum())
    base = np.maximum(np.floor(w).astype(np.int64), 1)
    rest = budget - int(base.sum())
    if rest > 0:
        order = np.argsort(-(w - np.floor(w)), kind="stable")
        base[order[:rest]] += 1
    elif rest < 0:
        order = np.argsort(-base, kind="stable")
        i = 0
        while rest < 0:
            j = order[i % k]
            if base[j] > 1:
                base[j] -= 1
                rest += 1
            i += 1
    return base


CHUNK = 1 << 21


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _pmap(fn, items):
    items = list(items)
    if len(items) <= 1:
        return [fn(it) for it in items]
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        return list(ex.map(fn, items))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)


def _nfw_m(x):
    return np.log1p(x) - x / (1.0 + x)


def _nfw_chunk(rng, c, rs):
    target = rng.random(len(c)) * _nfw_m(c)
    lo = np.zeros(len(c))
    hi = c.copy()
    for _ in range(40):  # 2^-40 of c r_s: far below the 2^-21 quantum
        mid = 0.5 * (lo + hi)
        up = _nfw_m(mid) < target
        np.copyto(lo, mid, where=up)
        np.copyto(hi, mid, where=~up)
    return _isotropic(rng, len(c)) * (0.5 * (lo + hi) * rs)[:, None]


def nfw_offsets(seq: np.random.SeedSequence, counts: np.ndarray, conc: np.ndarray,
                r200: np.ndarray) -> np.ndarray:
    """Offsets for halos with `counts[i]` particles, concentration conc[i] and
    radius r200[i]: radius x*r_s with m(x)/m(c) uniform (m(x) = ln(1+x) -
    x/(1+x)), solved by bisection in float64 on [0, c]; directions isotropic.
    Drawn in fixed chunks, each from its own child stream of `seq`."""
    n = int(counts.sum())
    c = np.repeat(conc.astype(np.float64), counts)
    rs = np.repeat((r200 / conc).astype(np.float64), counts)
    starts = list(range(0, n, CHUNK))
    seqs = seq.spawn(len(starts))
    parts = _pmap(lambda k: _nfw_chunk(np.random.Generator(np.random.PCG64(seqs[k])),
                                       c[starts[k]:starts[k] + CHUNK],
                                       rs[starts[k]:starts[k] + CHUNK]), range(len(starts)))
    return np.concatenate(parts) if parts else np.zeros((0, 3))


def plummer_offsets(rng: np.random.Generator, counts: np.ndarray, a: np.ndarray,
                    r_t: np.ndarray) -> np.ndarray:
    """Plummer spheres with scale a[i] truncated at r_t[i]: enclosed fraction
    u = (r^2/(r^2+a^2))^{3/2}, so r = a / sqrt(u^{-2/3} - 1) with u uniform
    below its value at r_t."""
    n = int(counts.sum())
    aa = np.repeat(a.astype(np.float64), counts)
    rt = np.repeat(r_t.astype(np.float64), counts)
    ut = (rt * rt / (rt * rt + aa * aa)) ** 1.5
    u = rng.random(n) * ut
    u = np.maximum(u, 1e-300)
    r = aa / np.sqrt(np.maximum(u ** (-2.0 / 3.0) - 1.0, 1e-300))
    r = np.minimum(r, rt)
    return _isotropic(rng, n) * r[:, None]


def r200_of(count: np.ndarray, n_total: int) -> np.ndarray:
    """Radius enclosing 200 times the mean particle density of the box."""
    return (3.0 * count / (4.0 * math.pi * 200.0 * n_total)) ** (1.0 / 3.0)


def _lattice_subset(seq, sites: int, k: int) -> np.ndarray:
    """Exactly k distinct lattice sites, each site equally likely: a
    Bernoulli(k/sites) draw per site in fixed chunks, then the surplus or
    shortfall removed or added uniformly at random."""
    starts = list(range(0, sites, 1 << 24))
    seqs = seq.spawn(len(starts) + 1)
    frac = k / float(sites)

    def draw(j):
        r = np.random.Generator(np.random.PCG64(seqs[j]))
        m = min(1 << 24, sites - starts[j])
        return np.nonzero(r.random(m) < frac)[0].astype(np.int64) + starts[j]
    pick = np.concatenate(_pmap(draw, range(len(starts))))
    fix = np.random.Generator(np.random.PCG64(seqs[-1]))
    if len(pick) > k:
        drop = fix.choice(len(pick), len(pick) - k, replace=False)
        keep = np.ones(len(pick), bool)
        keep[drop] = False
        pick = pick[keep]
    elif len(pick) < k:
        chosen = np.zeros(sites, bool)
        chosen[pick] = True
        while len(pick) < k:
            extra = fix.integers(0, sites, 2 * (k - len(pick)) + 16)
            extra = np.unique(extra[~chosen[extra]])
            extra = extra[:k - len(pick)]
            chosen[extra] = True
            pick = np.sort(np.concatenate([pick, extra]))
    return pick


def _quantize_chunks(pos: np.ndarray):
    n = pos.shape[0]
    X = np.empty(n, np.uint32); Y = np.empty(n, np.uint32); Z = np.empty(n, np.uint32)
    fx = np.empty(n, np.float32); fy = np.empty(n, np.float32); fz = np.empty(n, np.float32)

    def q(a):
        sl = slice(a, min(n, a + CHUNK))
        X[sl], fx[sl] = quantize(pos[sl, 0])
        Y[sl], fy[sl] = quantize(pos[sl, 1])
        Z[sl], fz[sl] = quantize(pos[sl, 2])
    _pmap(q, range(0, n, CHUNK))
    return X, Y, Z, fx, fy, fz


def snapshot(seed: int, n: int, *, g: int, thr: float, max_levels: int,
             halo_frac: float, n_halos: int, mass_lo: float, mass_hi: float,
             conc: float | tuple[float, float], lattice_side: int = 0,
             sigma_cells: float = 0.3, n_sub: int = 0,
             sub_frac: tuple[float, float] = (0.01, 0.1), shuffle: bool = True,
             name: str = "", velocities: bool = False) -> Snapshot:
    """Background (uniform if lattice_side == 0, else a random subset of a
    lattice_side^3 lattice perturbed by a Gaussian of sigma_cells * spacing per
    axis) plus `n_halos` NFW halos holding round(halo_frac*n) particles, with
    optional Plummer subhalos inside each host.  Every random draw comes from a
    child stream of SeedSequence(seed) in fixed-size chunks, so the result does
    not depend on the number of threads.

    With velocities, every particle also gets a velocity (units: box length 1,
    particle mass 1, G = 1), drawn from a child stream of its own so that the
    positions are those of the same call without velocities:
      background  isotropic Gaussian, sigma = v0, the circular velocity at r200
                  of a halo of the mean host size;
      host halo   a bulk velocity (Gaussian, sigma = v0) plus an isotropic
                  Gaussian of sigma = 0.6 * sqrt(G M / r200) per axis, except
                  5% of its particles, drawn with 3 times that sigma;
      subhalo     its host's bulk velocity plus a Gaussian of the host's sigma,
                  plus the same internal recipe with its own count and
                  truncation radius."""
    root = np.random.SeedSequence(seed)
    s_bg, s_halo, s_nfw, s_sub, s_shuf = root.spawn(5)
    rng = np.random.Generator(np.random.PCG64(s_halo))
    n_halo_part = int(round(halo_frac * n))
    n_bg = n - n_halo_part
    meta = dict(seed=seed, n=n, n_background=n_bg, n_halo_particles=n_halo_part,
                n_halos=n_halos, lattice_side=lattice_side)
    pos = np.empty((n, 3), np.float64)
    vel = None
    if velocities:
        s_vel = root.spawn(1)[0]  # the sixth child: the first five are unchanged
        vrng = np.random.Generator(np.random.PCG64(s_vel))
        vel = np.empty((n, 3), np.float64)
        mean_host = max(1.0, n_halo_part / max(n_halos, 1))
        v0 = math.sqrt(mean_host / float(r200_of(np.array([mean_host]), n)[0]))
    if lattice_side > 0:
        sites = lattice_side ** 3
        if n_bg > sites:
            raise ValueError("background larger than the lattice")
        s_pick, s_noise = s_bg.spawn(2)
        pick = _lattice_subset(s_pick, sites, n_bg)
        sp = 1.0 / lattice_side
        starts = list(range(0, n_bg, CHUNK))
        seqs = s_noise.spawn(len(starts))

        def lat(j):
            a = starts[j]
            b = min(n_bg, a + CHUNK)
            pk = pick[a:b]
            r = np.random.Generator(np.random.PCG64(seqs[j]))
            pos[a:b, 0] = (pk // (lattice_side * lattice_side)) * sp + 0.5 * sp
            pos[a:b, 1] = ((pk // lattice_side) % lattice_side) * sp + 0.5 * sp
            pos[a:b, 2] = (pk % lattice_side) * sp + 0.5 * sp
            pos[a:b] += r.normal(0.0, sigma_cells * sp, size=(b - a, 3))
        _pmap(lat, range(len(starts)))
    else:
        starts = list(range(0, n_bg, CHUNK))
        seqs = s_bg.spawn(len(starts))

        def uni(j):
            a = starts[j]
            b = min(n_bg, a + CHUNK)
            pos[a:b] = np.random.Generator(np.random.PCG64(seqs[j])).random((b - a, 3))
        _pmap(uni, range(len(starts)))
    if n_halo_part > 0 and n_halos > 0:
        counts = power_law_counts(rng, n_halos, mass_lo, mass_hi, n_halo_part)
        if isinstance(conc, tuple):
            cc = np.exp(rng.uniform(math.log(conc[0]), math.log(conc[1]), n_halos))
        else:
            cc = np.full(n_halos, float(conc))
        centres = rng.random((n_halos, 3))
        if n_sub > 0:
            frac = rng.uniform(sub_frac[0], sub_frac[1], (n_halos, n_sub))
            sub_counts = np.floor(frac * counts[:, None]).astype(np.int64)
            host_counts = counts - sub_counts.sum(axis=1)
            bad = host_counts < 1
            if np.any(bad):
                sub_counts[bad] = 0
                host_counts = counts - sub_counts.sum(axis=1)
        else:
            host_counts = counts
        r200 = r200_of(counts, n)
        a = n_bg
        nh = int(host_counts.sum())
        pos[a:a + nh] = np.repeat(centres, host_counts, axis=0) + nfw_offsets(s_nfw, host_counts, cc, r200)
        if vel is not None:
            vel[:n_bg] = vrng.normal(0.0, v0, size=(n_bg, 3))
            bulk = vrng.normal(0.0, v0, size=(n_halos, 3))
            sig = 0.6 * np.sqrt(counts / r200)
            s_each = np.repeat(sig, host_counts)
            s_each = s_each * np.where(vrng.random(nh) < 0.05, 3.0, 1.0)
            vel[a:a + nh] = (np.repeat(bulk, host_counts, axis=0)
                             + vrng.normal(0.0, 1.0, size=(nh, 3)) * s_each[:, None])
        a += nh
        if n_sub > 0:
            srng = np.random.Generator(np.random.PCG64(s_sub))
            sc = sub_counts.reshape(-1)
            keep = sc > 0
            owner = np.repeat(np.arange(n_halos), n_sub)[keep]
            sc = sc[keep]
            # subhalo centres follow the host's NFW profile inside r200
            sub_centre = centres[owner] + nfw_offsets(
                s_sub.spawn(1)[0], np.ones(len(sc), dtype=np.int64), cc[owner], r200[owner])
            rt = r200_of(sc, n)
            ns = int(sc.sum())
            pos[a:a + ns] = np.repeat(sub_centre, sc, axis=0) + plummer_offsets(srng, sc, rt / 5.0, rt)
            if vel is not None:
                sbulk = bulk[owner] + vrng.normal(0.0, 1.0, size=(len(sc), 3)) * sig[owner, None]
                ssig = 0.6 * np.sqrt(sc / rt)
                s_each = np.repeat(ssig, sc) * np.where(vrng.random(ns) < 0.05, 3.0, 1.0)
                vel[a:a + ns] = (np.repeat(sbulk, sc, axis=0)
                                 + vrng.normal(0.0, 1.0, size=(ns, 3)) * s_each[:, None])
            a += ns
            meta["n_subhalos"] = int(len(sc))
        assert a == n, (a, n)
        meta["halo_count_sum"] = int(counts.sum())
    elif vel is not None:
        vel[:] = vrng.normal(0.0, v0, size=(n, 3))
    if shuffle:
        perm = np.random.Generator(np.random.PCG64(s_shuf)).permutation(n)
        pos = pos[perm]
        if vel is not None:
            vel = vel[perm]
    X, Y, Z, fx, fy, fz = _quantize_chunks(pos)
    return Snapshot(X, Y, Z, fx, fy, fz, None, g, float(thr), float(thr), max_levels,
                    name, meta, None if vel is None else vel.astype(np.float32))


def small_mixed(seed: int = 0, velocities: bool = False) -> Snapshot:
    """32^3 equal-mass particles: 70% uniform, 30% in 8 NFW halos (c = 8,
    sizes from M^-1.9 over 200..4000 rescaled to the budget); 32^3 domain
    grid, threshold 5, at most 4 refinement levels."""
    return snapshot(seed, 32 ** 3, g=5, thr=5.0, max_levels=4, halo_frac=0.3,
                    n_halos=8, mass_lo=200.0, mass_hi=4000.0, conc=8.0,
                    name="small-mixed-32k", velocities=velocities)


def snapshot_16m(seed: int = 1, velocities: bool = False) -> Snapshot:
    """256^3 particles: 80% of a 256^3 lattice perturbed by 0.3 lattice spacing,
    20% in 2000 NFW halos (c log-uniform 4..15, sizes M^-1.9 over 20..2e5);
    128^3 domain grid, threshold 5, at most 10 refinement levels."""
    return snapshot(seed, 1 << 24, g=7, thr=5.0, max_levels=10, halo_frac=0.2,
                    n_halos=2000, mass_lo=20.0, mass_hi=2e5, conc=(4.0, 15.0),
                    lattice_side=256, name="lattice-nfw-16.8M", velocities=velocities)


def snapshot_134m(seed: int = 2, velocities: bool = False) -> Snapshot:
    """512^3 particles: 70% of a 512^3 lattice perturbed by 0.3 spacing, 30% in
    20000 NFW hosts with 5 Plummer subhalos each (0.01..0.1 of the host);
    256^3 domain grid, threshold 5, at most 12 refinement levels."""
    return snapshot(seed, 1 << 27, g=8, thr=5.0, max_levels=12, halo_frac=0.3,
                    n_halos=20000, mass_lo=20.0, mass_hi=2e5, conc=(4.0, 15.0),
                    lattice_side=512, n_sub=5, name="lattice-nfw-sub-134M",
                    velocities=velocities)


def scaled_like_16m(seed: int, n: int, g: int | None = None, max_levels: int = 10,
                    halo_frac: float = 0.2, velocities: bool = False,
                    n_sub: int = 0) -> Snapshot:
    """The 16.8M recipe at another particle count: lattice on ceil(n^{1/3})^3
    sites, 2000*n/2^24 halos (at least 1), domain grid chosen so that a domain
    cell holds about 8 particles (clamped to 32^3..128^3 unless given)."""
    side = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
    while side ** 3 < int(n * (1 - halo_frac)) + 1:
        side += 1
    if g is None:
        g = int(min(7, max(5, round(math.log2(max(n, 1) ** (1.0 / 3.0) / 2.0)))))
    nh = max(1, int(round(2000 * n / float(1 << 24))))
    return snapshot(seed, n, g=g, thr=5.0, max_levels=max_levels, halo_frac=halo_frac,
                    n_halos=nh, mass_lo=20.0, mass_hi=2e5, conc=(4.0, 15.0),
                    lattice_side=side, name=f"lattice-nfw-{n}", velocities=velocities,
                    n_sub=n_sub)


def subvolume_sizes(seed: int, count: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.round(10.0 ** rng.uniform(lo_exp, hi_exp, count)).astype(np.int64)


def subvolume(seed: int, n: int, halo_frac: float | None = None) -> Snapshot:
    """One independent periodic sub-volume of the batched / served workloads:
    the 16.8M recipe at n particles with halo fraction drawn in 10..40% unless
    given, threshold 5, at most 10 levels."""
    if halo_frac is None:
        halo_frac = float(np.random.Generator(np.random.PCG64(seed + 7919)).uniform(0.1, 0.4))
    return scaled_like_16m(seed, int(n), halo_frac=halo_frac)
