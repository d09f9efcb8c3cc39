"""Pins of the substructure classification oracle (grid tree -> host
structures and substructures, Sect. 2.1 and its figure on classifying a grid
tree): hand-made trees with known answers, ties, sub-substructure, and an
independent recursive formulation on trees from real oracle builds."""
import numpy as np
import pytest

import oracle
from oracle.substructure import classify, classify_levels
from tests.helpers import clustered


def tree(*levels):
    """levels: lists of (parent, nparticles) per level 1, 2, ..."""
    parents = [np.zeros(0, np.int32)]
    counts = [np.zeros(0, np.uint64)]
    for lv in levels:
        parents.append(np.array([p for p, _ in lv], np.int32))
        counts.append(np.array([c for _, c in lv], np.uint64))
    return parents, counts


def test_five_isolated_grids_one_host_four_subhalos():
    # one coarse patch splits into five; the one with the most particles
    # continues the host, the other four are subhalos
    ps, st = classify(*tree([(-1, 500)],
                            [(0, 10), (0, 50), (0, 20), (0, 5), (0, 7)]))
    assert list(ps[1]) == [0]
    assert list(ps[2]) == [1, 0, 2, 3, 4]
    assert list(st["host"]) == [-1, 0, 0, 0, 0]
    assert list(st["level"]) == [1, 2, 2, 2, 2]
    assert list(st["patch"]) == [0, 0, 2, 3, 4]
    assert list(st["depth"]) == [0, 1, 1, 1, 1]


def test_tie_goes_to_the_lower_patch_id():
    ps, st = classify(*tree([(-1, 100)], [(0, 30), (0, 30), (0, 30)]))
    assert list(ps[2]) == [0, 1, 2]
    assert list(st["patch"]) == [0, 1, 2]
    assert list(st["level"]) == [1, 2, 2]


def test_sub_substructure_is_recursive():
    # level 1: A; level 2: A splits into B (big, main) and C (sub);
    # level 3: C splits into D (main of C) and E (sub-sub), B continues alone
    ps, st = classify(*tree([(-1, 1000)],
                            [(0, 600), (0, 300)],
                            [(1, 100), (0, 500), (1, 150)]))
    # level-3 patches: 0 -> child of C, 1 -> child of B, 2 -> child of C (largest of C)
    assert list(ps[2]) == [0, 1]
    assert list(ps[3]) == [2, 0, 1]
    assert list(st["host"]) == [-1, 0, 1]
    assert list(st["depth"]) == [0, 1, 2]
    assert list(st["level"]) == [1, 2, 3]
    assert list(st["patch"]) == [0, 1, 0]


def test_several_roots_and_chains():
    ps, st = classify(*tree([(-1, 5), (-1, 9)], [(1, 9)], [(0, 7)]))
    assert list(ps[1]) == [0, 1]
    assert list(ps[2]) == [1]
    assert list(ps[3]) == [1]
    assert list(st["host"]) == [-1, -1]
    assert list(st["depth"]) == [0, 0]


def test_no_patches():
    ps, st = classify(*tree())
    assert len(st["host"]) == 0
    ps, st = classify(*tree([]))
    assert len(st["host"]) == 0 and len(ps[1]) == 0


def recursive_classification(parents, counts):
    """Independent formulation: depth-first walk of each tree, following the
    main child first; structures collected as chains, then renumbered by
    (start level, start patch)."""
    nlev = len(parents)
    children = [dict() for _ in range(nlev)]
    for L in range(2, nlev):
        for p, q in enumerate(parents[L]):
            children[L - 1].setdefault(int(q), []).append(p)
    chains = []  # (start level, start patch, host chain index, depth, members)

    def walk(L, p, chain):
        chain[4].append((L, p))
        kids = children[L].get(p, []) if L < nlev - 1 else []
        if not kids:
            return
        main = sorted(kids, key=lambda c: (-int(counts[L + 1][c]), c))[0]
        walk(L + 1, main, chain)
        for c in kids:
            if c != main:
                sub = [L + 1, c, chain, chain[3] + 1, []]
                chains.append(sub)
                walk(L + 1, c, sub)

    if nlev > 1:
        for p in range(len(parents[1])):
            root = [1, p, None, 0, []]
            chains.append(root)
            walk(1, p, root)
    order = sorted(range(len(chains)), key=lambda i: (chains[i][0], chains[i][1]))
    newid = {id(chains[i]): k for k, i in enumerate(order)}
    ps = [np.full(len(parents[L]), -1, np.int32) for L in range(nlev)]
    host, level, patch, depth = [], [], [], []
    for i in order:
        c = chains[i]
        host.append(-1 if c[2] is None else newid[id(c[2])])
        level.append(c[0]); patch.append(c[1]); depth.append(c[3])
        for (L, p) in c[4]:
            ps[L][p] = newid[id(c)]
    return ps, dict(host=np.array(host), level=np.array(level), patch=np.array(patch),
                    depth=np.array(depth))


@pytest.mark.parametrize("seed,n,g,thr,lmax", [(51, 6000, 3, 3, 6), (52, 20000, 4, 4, 6),
                                               (53, 12000, 3, 2, 7)])
def test_matches_an_independent_recursive_walk(seed, n, g, thr, lmax):
    p = clustered(seed, n, n_clumps=7, spread=0.02, g=g, thr=thr, max_levels=lmax)
    levels, _ = oracle.build(p)
    ps, st = classify_levels(levels)
    parents = [np.zeros(0, np.int32)] + [lv.patch_parent for lv in levels[1:]]
    counts = [np.zeros(0, np.uint64)] + [lv.patch_nparticles for lv in levels[1:]]
    ps2, st2 = recursive_classification(parents, counts)
    assert len(st["host"]) > 1
    for L in range(1, len(levels)):
        assert np.array_equal(ps[L], ps2[L]), L
    for k in ("host", "level", "patch", "depth"):
        assert np.array_equal(st[k], st2[k]), k
    # every structure starts where its id first appears and has one patch per level
    for s in range(len(st["host"])):
        lv0, p0 = int(st["level"][s]), int(st["patch"][s])
        assert ps[lv0][p0] == s
        for L in range(1, len(levels)):
            assert np.count_nonzero(ps[L] == s) <= 1
    # structures = level-1 patches + one per extra child of every split
    extra = 0
    for L in range(2, len(levels)):
        q = levels[L].patch_parent
        extra += len(q) - len(np.unique(q))
    assert len(st["host"]) == len(levels[1].patch_parent) + extra
