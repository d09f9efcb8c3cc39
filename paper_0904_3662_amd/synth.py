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
                        name or self.name + "-subset", dict(self.meta))


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


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)


def _nfw_m(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_offsets(rng: np.random.Generator, counts: np.ndarray, conc: np.ndarray,
                r200: np.ndarray) -> np.ndarray:
    """Offsets for halos with `counts[i]` particles, concentration conc[i] and
    radius r200[i]: radius x*r_s with m(x)/m(c) uniform, solved by bisection in
    float64 on [0, c]; directions isotropic."""
    n = int(counts.sum())
    c = np.repeat(conc.astype(np.float64), counts)
    rs = np.repeat((r200 / conc).astype(np.float64), counts)
    target = rng.random(n) * _nfw_m(c)
    lo = np.zeros(n)
    hi = c.copy()
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        go_up = _nfw_m(mid) < target
        lo = np.where(go_up, mid, lo)
        hi = np.where(go_up, hi, mid)
    r = 0.5 * (lo + hi) * rs
    return _isotropic(rng, n) * r[:, None]


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


def snapshot(seed: int, n: int, *, g: int, thr: float, max_levels: int,
             halo_frac: float, n_halos: int, mass_lo: float, mass_hi: float,
             conc: float | tuple[float, float], lattice_side: int = 0,
             sigma_cells: float = 0.3, n_sub: int = 0,
             sub_frac: tuple[float, float] = (0.01, 0.1), shuffle: bool = True,
             name: str = "") -> Snapshot:
    """Background (uniform if lattice_side == 0, else a random subset of a
    lattice_side^3 lattice perturbed by a Gaussian of sigma_cells * spacing per
    axis) plus `n_halos` NFW halos holding round(halo_frac*n) particles, with
    optional Plummer subhalos inside each host."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_halo_part = int(round(halo_frac * n))
    n_bg = n - n_halo_part
    if lattice_side > 0:
        sites = lattice_side ** 3
        if n_bg > sites:
            raise ValueError("background larger than the lattice")
        pick = rng.choice(sites, size=n_bg, replace=False)
        iz = pick % lattice_side
        iy = (pick // lattice_side) % lattice_side
        ix = pick // (lattice_side * lattice_side)
        sp = 1.0 / lattice_side
        bg = np.stack([ix, iy, iz], axis=1).astype(np.float64) * sp + 0.5 * sp
        bg += rng.normal(0.0, sigma_cells * sp, size=bg.shape)
    else:
        bg = rng.random((n_bg, 3))
    parts = [bg]
    meta = dict(seed=seed, n=n, n_background=n_bg, n_halo_particles=n_halo_part,
                n_halos=n_halos, lattice_side=lattice_side)
    if n_halo_part > 0 and n_halos > 0:
        counts = power_law_counts(rng, n_halos, mass_lo, mass_hi, n_halo_part)
        expect = counts.sum()
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
        host_off = nfw_offsets(rng, host_counts, cc, r200)
        parts.append(np.repeat(centres, host_counts, axis=0) + host_off)
        if n_sub > 0:
            sc = sub_counts.reshape(-1)
            keep = sc > 0
            owner = np.repeat(np.arange(n_halos), n_sub)[keep]
            sc = sc[keep]
            # subhalo centres follow the host's NFW profile inside r200
            sub_centre = centres[owner] + nfw_offsets(
                rng, np.ones(len(sc), dtype=np.int64), cc[owner], r200[owner])
            rt = r200_of(sc, n)
            parts.append(np.repeat(sub_centre, sc, axis=0) +
                         plummer_offsets(rng, sc, rt / 5.0, rt))
            meta["n_subhalos"] = int(len(sc))
        meta["halo_count_sum"] = int(expect)
    pos = np.concatenate(parts, axis=0)
    assert pos.shape[0] == n, (pos.shape, n)
    if shuffle:
        pos = pos[rng.permutation(n)]
    X, fx = quantize(pos[:, 0])
    Y, fy = quantize(pos[:, 1])
    Z, fz = quantize(pos[:, 2])
    return Snapshot(X, Y, Z, fx, fy, fz, None, g, float(thr), float(thr), max_levels,
                    name, meta)


def small_mixed(seed: int = 0) -> Snapshot:
    """32^3 equal-mass particles: 70% uniform, 30% in 8 NFW halos (c = 8,
    sizes from M^-1.9 over 200..4000 rescaled to the budget); 32^3 domain
    grid, threshold 5, at most 4 refinement levels."""
    return snapshot(seed, 32 ** 3, g=5, thr=5.0, max_levels=4, halo_frac=0.3,
                    n_halos=8, mass_lo=200.0, mass_hi=4000.0, conc=8.0,
                    name="small-mixed-32k")


def snapshot_16m(seed: int = 1) -> Snapshot:
    """256^3 particles: 80% of a 256^3 lattice perturbed by 0.3 lattice spacing,
    20% in 2000 NFW halos (c log-uniform 4..15, sizes M^-1.9 over 20..2e5);
    128^3 domain grid, threshold 5, at most 10 refinement levels."""
    return snapshot(seed, 1 << 24, g=7, thr=5.0, max_levels=10, halo_frac=0.2,
                    n_halos=2000, mass_lo=20.0, mass_hi=2e5, conc=(4.0, 15.0),
                    lattice_side=256, name="lattice-nfw-16.8M")


def snapshot_134m(seed: int = 2) -> Snapshot:
    """512^3 particles: 70% of a 512^3 lattice perturbed by 0.3 spacing, 30% in
    20000 NFW hosts with 5 Plummer subhalos each (0.01..0.1 of the host);
    256^3 domain grid, threshold 5, at most 12 refinement levels."""
    return snapshot(seed, 1 << 27, g=8, thr=5.0, max_levels=12, halo_frac=0.3,
                    n_halos=20000, mass_lo=20.0, mass_hi=2e5, conc=(4.0, 15.0),
                    lattice_side=512, n_sub=5, name="lattice-nfw-sub-134M")


def scaled_like_16m(seed: int, n: int, g: int | None = None, max_levels: int = 10,
                    halo_frac: float = 0.2) -> Snapshot:
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
                    lattice_side=side, name=f"lattice-nfw-{n}")


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
