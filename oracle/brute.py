"""Dense brute force of the adaptive density hierarchy for tiny inputs.

Test infrastructure: pins the C oracle.  Written independently of it:
every level is a dense numpy grid, membership of a particle is a dense mask
lookup, the TSC weight is the textbook distance form W(d) = 3/4 - d^2 for
|d| <= 1/2 and (3/2 - |d|)^2 / 2 for 1/2 <= |d| <= 3/2 (Hockney & Eastwood),
evaluated at the distance from the particle to each cell centre, and the
components are found with a plain breadth-first search on the dense mask.
Only for grids up to ~2^7 cells per axis.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def tsc_distance_weight(d: float) -> float:
    d = abs(d)
    if d <= 0.5:
        return 0.75 - d * d
    if d <= 1.5:
        return 0.5 * (1.5 - d) ** 2
    return 0.0


def _key(x: int, y: int, z: int, bits: int) -> int:
    k = 0
    for j in range(bits):
        k |= ((x >> j) & 1) << (3 * j + 2)
        k |= ((y >> j) & 1) << (3 * j + 1)
        k |= ((z >> j) & 1) << (3 * j)
    return k


def brute(p, g, thr_dom, thr_ref, max_levels, conn=26, density=False):
    """Returns a list of dicts, one per level, with dense arrays indexed [x,y,z]:
    inS, count, flag, mass (numpy float64, zero outside E), number (TSC particle
    number), inE, patch (-1 off S), plus per-patch parents, the smallest key
    of every patch, and per patch its cells, particles and particle mass.  density: refine where the TSC particle number exceeds the
    threshold instead of the count."""
    X = np.asarray(p.X, np.int64); Y = np.asarray(p.Y, np.int64); Z = np.asarray(p.Z, np.int64)
    fx = np.asarray(p.fx, np.float64); fy = np.asarray(p.fy, np.float64)
    fz = np.asarray(p.fz, np.float64)
    mass = np.ones(len(X)) if getattr(p, "mass", None) is None else np.asarray(p.mass, np.float64)
    out = []
    inS = None
    for L in range(max_levels + 1):
        b = g + L
        n = 1 << b
        if L == 0:
            inS = np.ones((n, n, n), bool)
        sh = 21 - b
        cx, cy, cz = X >> sh, Y >> sh, Z >> sh
        # continuous position in units of this level's cells
        px = (X + fx) / float(1 << sh)
        py = (Y + fy) / float(1 << sh)
        pz = (Z + fz) / float(1 << sh)
        count = np.zeros((n, n, n), np.int64)
        inP = inS[cx, cy, cz]
        np.add.at(count, (cx[inP], cy[inP], cz[inP]), 1)
        # particle mass held by each cell (the particles whose cell it is)
        cell_mass = np.zeros((n, n, n))
        np.add.at(cell_mass, (cx[inP], cy[inP], cz[inP]), mass[inP])
        field = np.zeros((n, n, n))
        number = np.zeros((n, n, n))
        for i in np.nonzero(inP)[0]:
            for a in (-1, 0, 1):
                ix = cx[i] + a
                wx = tsc_distance_weight(px[i] - (ix + 0.5))
                for bb in (-1, 0, 1):
                    iy = cy[i] + bb
                    wy = tsc_distance_weight(py[i] - (iy + 0.5))
                    for c in (-1, 0, 1):
                        iz = cz[i] + c
                        wz = tsc_distance_weight(pz[i] - (iz + 0.5))
                        field[ix % n, iy % n, iz % n] += mass[i] * wx * wy * wz
                        number[ix % n, iy % n, iz % n] += wx * wy * wz
        # E = S dilated by one cell, periodic
        inE = np.zeros_like(inS)
        for a in (-1, 0, 1):
            for bb in (-1, 0, 1):
                for c in (-1, 0, 1):
                    inE |= np.roll(inS, (a, bb, c), axis=(0, 1, 2))
        last = (L == max_levels) or (b >= 21)
        thr = thr_dom if L == 0 else thr_ref
        crit = number if density else count
        flag = (crit > thr) & inS & (not last)
        lev = dict(level=L, bits=b, inS=inS.copy(), count=count, flag=flag, mass=field,
                   number=number, inE=inE, n_particles=int(inP.sum()))
        if L >= 1:
            patch = -np.ones((n, n, n), np.int64)
            cells = np.argwhere(inS)
            keys = np.array([_key(int(x), int(y), int(z), b) for x, y, z in cells], np.int64)
            order = np.argsort(keys)
            npatch = 0
            minkeys = []
            for j in order:
                x0, y0, z0 = (int(v) for v in cells[j])
                if patch[x0, y0, z0] >= 0:
                    continue
                patch[x0, y0, z0] = npatch
                q = deque([(x0, y0, z0)])
                while q:
                    x, y, z = q.popleft()
                    for a in (-1, 0, 1):
                        for bb in (-1, 0, 1):
                            for c in (-1, 0, 1):
                                s = abs(a) + abs(bb) + abs(c)
                                if s == 0 or (conn == 6 and s > 1) or (conn == 18 and s > 2):
                                    continue
                                u, v, w = (x + a) % n, (y + bb) % n, (z + c) % n
                                if inS[u, v, w] and patch[u, v, w] < 0:
                                    patch[u, v, w] = npatch
                                    q.append((u, v, w))
                minkeys.append(int(keys[j]))
                npatch += 1
            lev["patch"] = patch
            lev["patch_minkey"] = minkeys
            parents = []
            for pk in minkeys:
                if L == 1:
                    parents.append(-1)
                    continue
                # parent cell coordinates of the patch's smallest cell
                x = y = z = 0
                for j in range(b):
                    x |= ((pk >> (3 * j + 2)) & 1) << j
                    y |= ((pk >> (3 * j + 1)) & 1) << j
                    z |= ((pk >> (3 * j)) & 1) << j
                parents.append(int(out[L - 1]["patch"][x >> 1, y >> 1, z >> 1]))
            lev["patch_parent"] = parents
            # per patch, walking the dense grid cell by cell: cells of S in
            # it, particles inside those cells, and their mass
            ncells = [0] * npatch
            npart = [0] * npatch
            pmass = [0.0] * npatch
            for x, y, z in cells:
                pid = int(patch[x, y, z])
                ncells[pid] += 1
                npart[pid] += int(count[x, y, z])
                pmass[pid] += float(cell_mass[x, y, z])
            lev["patch_ncells"] = ncells
            lev["patch_nparticles"] = npart
            lev["patch_mass"] = pmass
        out.append(lev)
        if not flag.any():
            break
        # children of flagged cells form the next level
        inS = np.repeat(np.repeat(np.repeat(flag, 2, axis=0), 2, axis=1), 2, axis=2)
    return out


def dense_index(key: int, bits: int) -> tuple[int, int, int]:
    x = y = z = 0
    for j in range(bits):
        x |= ((key >> (3 * j + 2)) & 1) << j
        y |= ((key >> (3 * j + 1)) & 1) << j
        z |= ((key >> (3 * j)) & 1) << j
    return x, y, z
