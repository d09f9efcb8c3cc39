"""Classification of the grid tree into host structures and substructures --
test infrastructure (oracle), plain Python loops.

Definition (Sect. 2.1, the paragraphs on the grid tree and on classifying it
into substructure, with the figure that illustrates the classification):
the tree is walked from the coarsest level to the finer ones.  Where a patch
splits into several isolated patches on the next finer level, the one holding
the most particles continues the structure of its parent (the main branch);
every other one starts a new structure, a substructure of the parent's
structure.  The rule applies again inside substructures (sub-substructure).

Readings taken here:
- every level-1 patch is the coarsest grid of its own tree and starts a host
  structure (depth 0, no host): the domain grid is the whole box, not a halo;
- ties in the particle count go to the lower patch id;
- structures are numbered by (start level, start patch id).

Returns, for levels given as the oracle's (or the device's) per-level patch
parents and particle counts, the structure id of every patch and, per
structure, its host structure, start level, start patch and depth.
"""
from __future__ import annotations

import numpy as np


def classify(parents, nparticles):
    """parents[L], nparticles[L]: arrays over the patches of level L (index 0
    is level 0, which has no patches).  Returns (patch_struct, structs) with
    patch_struct[L] an int32 array per level (empty on level 0) and structs a
    dict of int32 arrays host, level, patch, depth."""
    nlev = len(parents)
    patch_struct = [np.zeros(0, np.int32) for _ in range(nlev)]
    host, level, patch, depth = [], [], [], []
    if nlev < 2:
        return patch_struct, dict(host=np.zeros(0, np.int32), level=np.zeros(0, np.int32),
                                  patch=np.zeros(0, np.int32), depth=np.zeros(0, np.int32))
    # level 1: every patch starts a host structure
    n1 = len(parents[1])
    ps = np.zeros(n1, np.int32)
    for p in range(n1):
        ps[p] = len(host)
        host.append(-1)
        level.append(1)
        patch.append(p)
        depth.append(0)
    patch_struct[1] = ps
    for L in range(2, nlev):
        par = [int(q) for q in parents[L]]
        cnt = [int(c) for c in nparticles[L]]
        # the main branch of every parent: most particles, then lowest id
        best = {}
        for p, q in enumerate(par):
            if q not in best or cnt[p] > cnt[best[q]] or (cnt[p] == cnt[best[q]] and p < best[q]):
                best[q] = p
        ps = np.zeros(len(par), np.int32)
        for p, q in enumerate(par):
            parent_struct = int(patch_struct[L - 1][q])
            if best[q] == p:
                ps[p] = parent_struct
            else:
                ps[p] = len(host)
                host.append(parent_struct)
                level.append(L)
                patch.append(p)
                depth.append(depth[parent_struct] + 1)
        patch_struct[L] = ps
    structs = dict(host=np.array(host, np.int32), level=np.array(level, np.int32),
                   patch=np.array(patch, np.int32), depth=np.array(depth, np.int32))
    return patch_struct, structs


def classify_levels(levels):
    """classify() on the oracle's build output (a list of oracle levels)."""
    parents = [np.zeros(0, np.int32)] + [lv.patch_parent for lv in levels[1:]]
    counts = [np.zeros(0, np.uint64)] + [lv.patch_nparticles for lv in levels[1:]]
    return classify(parents, counts)
