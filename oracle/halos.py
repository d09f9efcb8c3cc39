"""Particle collection and iterative unbinding of the halos of a grid tree --
test infrastructure (oracle): plain FP64 NumPy, one halo at a time.  Only the
tests, the smoke check and the benchmark's CPU baseline use it.

What it computes (Sect. 2.1, the paragraphs after the classification of the
grid tree, and App. A):
- every structure of the classified grid tree is a prospective halo; its
  centre comes from the leaf of its branch (the finest grid on it);
- particles are collected: for a host, everything out to the first
  isodensity contour below the virial overdensity; for a substructure, the
  sphere around its centre with half the distance to its host's centre as
  radius;
- the halo is then considered in isolation and unbound particles are removed
  iteratively: along the radially ordered particles the potential is
  integrated from the spherical Poisson equation, phi(r) = G int_0^r
  M(<r')/r'^2 dr' + phi_0, with phi_0 fixed by phi(infinity) = 0 for a halo
  truncated at r_vir (App. A), and a particle is unbound when its speed
  relative to the halo exceeds the escape speed sqrt(2 |phi|);
- the virial radius is where the mean enclosed density falls to Delta_vir
  times the background density (the equation that defines r_vir).

Readings taken here (the paper leaves them open):
- H1 halos: one per structure of the classification (host structures and
  substructures); its leaf is the patch of its main branch on the deepest
  level that branch reaches;
- H2 centre: the centre of mass of the particles in the cells of the leaf
  patch, with every position taken as the periodic minimum image relative to
  the lower corner of the leaf's smallest-key cell;
- H3 isodensity contours: the boundary of a level-L patch is where the
  particles per level-(L-1) cell reach that level's threshold, a density of
  thr_{L-1} 8^(L-1) 2^(3g) / N times the background; a host collects the
  particles in the cells of its main-branch patch on the deepest level (from
  its start level to its leaf) whose contour is below Delta_vir, or of its
  start patch when none is;
- H4 a substructure collects every particle within half the distance to its
  host's centre (host = the structure it is a substructure of), periodic
  minimum image, distance <= radius, the radius capped by the extent of the
  isolated grid that started the substructure (its start patch): the largest
  distance from the centre to a corner of one of that patch's cells.  (Where
  the background itself refines, the host of a first-level substructure is the
  box-spanning background grid, whose centre can lie anywhere; the paper's
  first collection step takes the particles on a halo's own isolated grids,
  and the cap keeps the sphere on them);
- H5 per iteration: the halo velocity is the mass-weighted mean velocity of
  its current particles; radii are measured from the fixed centre (clamped
  below at half a position quantum); the particles are ordered by radius,
  ties by index; M(<r_k) includes particle k; r_vir is the radius of the last
  particle k whose enclosed mean density M_k / (4/3 pi r_k^3) is at least
  Delta_vir rho_b (no such particle: the halo dissolves); between particle
  radii the enclosed mass is constant, so the integral is a sum of
  M_j (1/r_j - 1/r_{j+1}); beyond r_vir phi = -G M_vir / r;
- H6 a particle is unbound when half its squared speed relative to the halo
  exceeds |phi| (strictly); all unbound particles of an iteration go at once;
  the iteration stops when none goes (at most max_iter iterations);
- H7 the halo's particles are those left within r_vir; M_vir is their mass;
  a halo that dissolves (H5) or has not converged after max_iter iterations
  keeps no particles and has r_vir = M_vir = 0; a leaf patch without mass
  (possible only with a negative threshold) has the centre of its
  smallest-key cell;
- H8 units: box length 1, particle mass 1 (or the given masses), G = 1;
  rho_b = total mass / box volume; Delta_vir = 340 (the value the paper uses
  for its mass functions).
"""
from __future__ import annotations

import math

import numpy as np

QSCALE = float(1 << 21)
HALF_QUANTUM = 0.5 / QSCALE


def positions(p) -> np.ndarray:
    """(n, 3) FP64 positions in box units from the canonical (X, f) form."""
    X = np.stack([p.X, p.Y, p.Z], axis=1).astype(np.float64)
    f = np.stack([p.fx, p.fy, p.fz], axis=1).astype(np.float64)
    return (X + f) / QSCALE


def min_image(d: np.ndarray) -> np.ndarray:
    """Periodic minimum image of displacements in the unit box."""
    return d - np.round(d)


def leaves(patch_struct, n_structs: int):
    """(level, patch) of every structure's leaf: its patch on the deepest level
    (H1)."""
    leaf = [(-1, -1)] * n_structs
    for L in range(1, len(patch_struct)):
        for q, s in enumerate(patch_struct[L]):
            leaf[int(s)] = (L, q)  # deeper levels come later and win
    return leaf


def patch_particles(levels, order, L: int, q: int) -> np.ndarray:
    """Particle indices (ascending) of the cells of patch q of level L."""
    lv = levels[L]
    cells = np.nonzero(lv.cell_patch == q)[0]
    parts = [order[lv.cell_start[c]:lv.cell_start[c] + lv.cell_count[c]] for c in cells]
    if not parts:
        return np.zeros(0, np.int64)
    return np.sort(np.concatenate(parts).astype(np.int64))


def cell_corner(key: int, bits: int) -> np.ndarray:
    """Lower corner, in box units, of the level cell with Morton key `key` at
    `bits` bits per axis (bit 3j+2 = x_j, 3j+1 = y_j, 3j = z_j)."""
    x = y = z = 0
    for j in range(bits):
        x |= ((key >> (3 * j + 2)) & 1) << j
        y |= ((key >> (3 * j + 1)) & 1) << j
        z |= ((key >> (3 * j)) & 1) << j
    return np.array([x, y, z], np.float64) / float(1 << bits)


def centre_of(levels, order, pos, mass, L: int, q: int) -> np.ndarray:
    """H2: centre of mass of the leaf patch's particles, minimum image
    relative to the lower corner of its smallest-key cell."""
    lv = levels[L]
    cells = np.nonzero(lv.cell_patch == q)[0]
    kmin = int(lv.cell_key[cells].min())
    ref = cell_corner(kmin, lv.bits)
    idx = patch_particles(levels, order, L, q)
    d = min_image(pos[idx] - ref)
    w = mass[idx]
    if w.sum() == 0:
        c = ref + 0.5 / float(1 << lv.bits)
    else:
        c = ref + (w[:, None] * d).sum(axis=0) / w.sum()
    return c - np.floor(c)


def patch_extent(levels, L: int, q: int, centre) -> float:
    """H4: the largest distance from the centre to a corner of a cell of
    patch q of level L (per axis the farther of the cell's two faces, periodic
    minimum image)."""
    lv = levels[L]
    h = 1.0 / float(1 << lv.bits)
    ext = 0.0
    for c in np.nonzero(lv.cell_patch == q)[0]:
        lo = cell_corner(int(lv.cell_key[c]), lv.bits)
        a = np.abs(min_image(lo - centre))
        b = np.abs(min_image(lo + h - centre))
        d = np.maximum(a, b)
        ext = max(ext, float(np.sqrt((d * d).sum())))
    return ext


def iso_level(start: int, leaf_level: int, thr_dom: float, thr_ref: float, g: int,
              n_total: float, delta_vir: float) -> int:
    """H3: the deepest level in [start, leaf_level] whose patch boundary lies
    on a contour below delta_vir times the background density (start when
    none does)."""
    best = start
    for L in range(start, leaf_level + 1):
        thr = thr_dom if L - 1 == 0 else thr_ref
        rho = thr * 8.0 ** (L - 1) * 2.0 ** (3 * g) / n_total
        if rho < delta_vir:
            best = L
    return best


def profile(r, m, rho_b, delta_vir=340.0, G=1.0):
    """H5 on particles already ordered by radius: the index v of the last
    particle within r_vir (-1 when the enclosed density never reaches
    delta_vir * rho_b), r_vir, M_vir and phi at every particle (App. A: the
    integral of M(<r')/r'^2 from r to r_vir, plus G M_vir / r_vir, with the
    enclosed mass constant between particle radii; -G M_vir / r beyond)."""
    Mk = np.cumsum(m)
    dens = Mk / (4.0 / 3.0 * math.pi * r ** 3)
    ok = np.nonzero(dens >= delta_vir * rho_b)[0]
    if ok.size == 0:
        return -1, 0.0, 0.0, None
    v = int(ok[-1])
    r_vir, m_vir = float(r[v]), float(Mk[v])
    term = Mk[:v] * (1.0 / r[:v] - 1.0 / r[1:v + 1])
    tail = np.zeros(v + 1)
    tail[:v] = np.cumsum(term[::-1])[::-1]
    phi = np.empty(r.size)
    phi[:v + 1] = -G * (tail + m_vir / r_vir)
    phi[v + 1:] = -G * m_vir / r[v + 1:]
    return v, r_vir, m_vir, phi


def unbind(idx, pos, vel, mass, centre, rho_b, delta_vir=340.0, G=1.0, max_iter=1000):
    """H5-H7: iterative removal of unbound particles from the candidate set
    idx around a fixed centre.  Returns a dict with the members (ascending
    indices within r_vir), r_vir, m_vir, the halo velocity and the number of
    iterations (0 when the candidate set was empty)."""
    alive = np.sort(np.asarray(idx, np.int64))
    out = dict(members=np.zeros(0, np.int64), r_vir=0.0, m_vir=0.0,
               vel=np.zeros(3), iterations=0)
    for it in range(1, max_iter + 1):
        if alive.size == 0:
            return out
        out["iterations"] = it
        m = mass[alive]
        vh = (m[:, None] * vel[alive]).sum(axis=0) / m.sum()
        d = min_image(pos[alive] - centre)
        r = np.maximum(np.sqrt((d * d).sum(axis=1)), HALF_QUANTUM)
        o = np.lexsort((alive, r))  # by radius, ties by particle index
        a, r, m = alive[o], r[o], m[o]
        v, r_vir, m_vir, phi = profile(r, m, rho_b, delta_vir, G)
        if v < 0:  # never dense enough: the halo dissolves
            out.update(members=np.zeros(0, np.int64), vel=vh, r_vir=0.0, m_vir=0.0)
            return out
        dv = vel[a] - vh
        ke = 0.5 * (dv * dv).sum(axis=1)
        gone = ke > np.abs(phi)
        out["vel"] = vh
        if not gone.any():
            keep = np.sort(a[:v + 1])
            out.update(members=keep, r_vir=r_vir, m_vir=float(mass[keep].sum()))
            return out
        alive = np.sort(a[~gone])
    # no convergence within max_iter: no particles
    out.update(members=np.zeros(0, np.int64), r_vir=0.0, m_vir=0.0)
    return out


def halos(p, levels, order, patch_struct, structs, delta_vir=340.0, G=1.0, max_iter=1000):
    """Every structure's halo: centre, collected candidates and the unbinding
    result.  Returns a list (one dict per structure, in structure order)."""
    pos = positions(p)
    n = p.n
    mass = np.ones(n) if p.mass is None else p.mass.astype(np.float64)
    vel = p.vel.astype(np.float64)
    rho_b = float(mass.sum())
    ns = len(structs["host"])
    leaf = leaves(patch_struct, ns)
    centres = np.zeros((ns, 3))
    for s in range(ns):
        L, q = leaf[s]
        centres[s] = centre_of(levels, order, pos, mass, L, q)
    res = []
    for s in range(ns):
        L, q = leaf[s]
        start = int(structs["level"][s])
        if int(structs["depth"][s]) == 0:
            Li = iso_level(start, L, p.dom_ref, p.ref_ref, p.g, float(n), delta_vir)
            qi = int(np.nonzero(patch_struct[Li] == s)[0][0])
            cand = patch_particles(levels, order, Li, qi)
            radius = 0.0
        else:
            h = int(structs["host"][s])
            sep = min_image(centres[s] - centres[h])
            radius = 0.5 * float(np.sqrt((sep * sep).sum()))
            ext = patch_extent(levels, start, int(structs["patch"][s]), centres[s])
            radius = min(radius, ext)
            d = min_image(pos - centres[s])
            cand = np.nonzero((d * d).sum(axis=1) <= radius * radius)[0].astype(np.int64)
        u = unbind(cand, pos, vel, mass, centres[s], rho_b, delta_vir, G, max_iter)
        u.update(struct=s, leaf=leaf[s], centre=centres[s], candidates=cand,
                 radius=radius)
        res.append(u)
    return res
