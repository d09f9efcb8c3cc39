"""Pins of the halo oracle (particle collection and unbinding, Sect. 2.1 and
App. A) against what the mathematics fixes: the shell theorem written as
point-mass sums, two-body escape in closed form, a removal cascade whose
iterations are counted by hand, the virial radius of a constructed profile,
the isodensity levels of the named workloads, periodic centres."""
import math

import numpy as np
import pytest

import oracle
from oracle import halos as H
from oracle import substructure
from paper_0904_3662_amd import synth

DELTA = 340.0


def shell_phi(r, m, v, G=1.0):
    """Potential of point masses ordered by radius under spherical symmetry,
    halo truncated after particle v: the mass inside a particle's radius acts
    from the centre, every shell outside it (up to v) adds G m_j / r_j."""
    n = len(r)
    phi = np.empty(n)
    m_vir = m[:v + 1].sum()
    for k in range(n):
        if k <= v:
            inner = m[:k + 1].sum() / r[k]
            outer = sum(m[j] / r[j] for j in range(k + 1, v + 1))
            phi[k] = -G * (inner + outer)
        else:
            phi[k] = -G * m_vir / r[k]
    return phi


def test_potential_is_the_shell_theorem():
    rng = np.random.Generator(np.random.PCG64(1))
    for n in (1, 2, 7, 200):
        r = np.sort(rng.uniform(1e-3, 0.02, n))
        m = rng.uniform(0.5, 2.0, n)
        rho_b = 1.0
        v, r_vir, m_vir, phi = H.profile(r, m, rho_b, DELTA)
        dens = np.cumsum(m) / (4.0 / 3.0 * math.pi * r ** 3)
        want_v = int(np.nonzero(dens >= DELTA * rho_b)[0][-1])
        assert v == want_v and r_vir == r[v] and m_vir == pytest.approx(m[:v + 1].sum())
        np.testing.assert_allclose(phi, shell_phi(r, m, v), rtol=1e-12)


def test_virial_radius_of_a_constructed_profile():
    # enclosed density exactly 2, 1.5, 1.0 (= threshold), 0.5 times DELTA*rho_b
    rho_b = 3.0
    r = np.array([0.01, 0.02, 0.03, 0.04])
    target = np.array([2.0, 1.5, 1.0, 0.5]) * DELTA * rho_b
    M = target * 4.0 / 3.0 * math.pi * r ** 3
    m = np.diff(np.concatenate([[0.0], M]))
    assert np.all(m > 0)
    v, r_vir, m_vir, phi = H.profile(r, m * (1 + 1e-12), rho_b, DELTA)
    assert v == 2 and r_vir == 0.03
    v, r_vir, m_vir, phi = H.profile(r, m * (1 - 1e-9), rho_b, DELTA)
    assert v == 1 and r_vir == 0.02
    # never dense enough: no virial radius
    assert H.profile(r, m * 1e-3, rho_b, DELTA)[0] == -1


def two_body(speed, M=1.0e4, r=0.01, m=1e-9):
    """A heavy particle at rest at the centre and a light one at radius r
    moving at `speed`; positions are offsets from the centre."""
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]])
    vel = np.array([[0.0, 0.0, 0.0], [0.0, speed, 0.0]])
    mass = np.array([M, m])
    return pos, vel, mass


def test_two_body_escape_speed():
    M, r, m = 1.0e4, 0.01, 1e-9
    v_esc = math.sqrt(2.0 * (M + m) / r)  # -phi = G (M + m) / r at the outermost particle
    rho_b = 1.0  # enclosed densities are ~1e9: both particles lie within r_vir
    for f, bound in ((0.999999, True), (1.000001, False)):
        pos, vel, mass = two_body(f * v_esc, M, r, m)
        out = H.unbind([0, 1], pos, vel, mass, np.array([0.5, 0.5, 0.5]), rho_b, DELTA)
        assert (1 in out["members"]) == bound, f
        assert 0 in out["members"]
        assert out["iterations"] == (1 if bound else 2)


def test_removal_cascade_takes_two_rounds():
    # a central mass M0; a fast pair (masses M1/2 each, opposite velocities,
    # so the halo velocity stays zero) at r1; a light test particle at r2
    # whose binding needs the pair: G M0 / r2 < v^2 / 2 < G (M0 + M1) / r2
    M0, M1, r1, r2, mt = 1.0e4, 1.0e4, 0.005, 0.01, 1e-12
    c = np.array([0.5, 0.5, 0.5])
    u = 10 * math.sqrt(2.0 * (M0 + M1) / r1)
    vt = math.sqrt(2.0 * (M0 + 0.5 * M1) / r2)
    pos = np.array([c, c + [r1, 0, 0], c - [r1, 0, 0], c + [0, r2, 0]])
    vel = np.array([[0, 0, 0], [0, u, 0], [0, -u, 0], [0, 0, vt]], np.float64)
    mass = np.array([M0, M1 / 2, M1 / 2, mt])
    out = H.unbind([0, 1, 2, 3], pos, vel, mass, c, 1.0, DELTA)
    # round 1 removes the pair, round 2 the test particle, round 3 removes nothing
    assert list(out["members"]) == [0]
    assert out["iterations"] == 3
    assert out["m_vir"] == M0


def test_unbinding_edge_cases():
    c = np.array([0.25, 0.25, 0.25])
    out = H.unbind([], np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), c, 1.0)
    assert out["iterations"] == 0 and out["members"].size == 0
    # a particle exactly at the centre: its radius is clamped to half a quantum
    pos = np.array([c])
    out = H.unbind([0], pos, np.zeros((1, 3)), np.ones(1), c, 1.0)
    assert list(out["members"]) == [0] and out["r_vir"] == H.HALF_QUANTUM
    # a diffuse set never reaches the virial density: the halo dissolves
    rng = np.random.Generator(np.random.PCG64(3))
    pos = rng.random((50, 3))
    out = H.unbind(np.arange(50), pos, np.zeros((50, 3)), np.ones(50), c, 50.0)
    assert out["members"].size == 0 and out["r_vir"] == 0.0 and out["m_vir"] == 0.0
    # not converged within max_iter: no particles either (the cascade needs 3)
    M0, M1, r1, r2, mt = 1.0e4, 1.0e4, 0.005, 0.01, 1e-12
    u = 10 * math.sqrt(2.0 * (M0 + M1) / r1)
    vt = math.sqrt(2.0 * (M0 + 0.5 * M1) / r2)
    pos = np.array([c, c + [r1, 0, 0], c - [r1, 0, 0], c + [0, r2, 0]])
    vel = np.array([[0, 0, 0], [0, u, 0], [0, -u, 0], [0, 0, vt]], np.float64)
    out = H.unbind([0, 1, 2, 3], pos, vel, np.array([M0, M1 / 2, M1 / 2, mt]), c, 1.0,
                   max_iter=2)
    assert out["members"].size == 0 and out["iterations"] == 2 and out["r_vir"] == 0.0


def test_isodensity_levels_of_the_workloads():
    # 16.8M: 2^21 domain cells, 2^24 particles, threshold 5: contours at
    # 0.625, 5, 40, 320, 2560 times the background on levels 1..5
    assert H.iso_level(1, 9, 5.0, 5.0, 7, 2.0 ** 24, DELTA) == 4
    assert H.iso_level(1, 3, 5.0, 5.0, 7, 2.0 ** 24, DELTA) == 3
    assert H.iso_level(2, 9, 5.0, 5.0, 7, 2.0 ** 24, 4.0) == 2  # none below 4: the start
    assert H.iso_level(1, 9, 5.0, 5.0, 7, 2.0 ** 24, 321.0) == 4
    assert H.iso_level(1, 9, 5.0, 5.0, 7, 2.0 ** 24, 319.0) == 3


def test_cell_corner_matches_the_morton_definition():
    for bits in (1, 5, 9):
        rng = np.random.Generator(np.random.PCG64(bits))
        for _ in range(20):
            x, y, z = (int(v) for v in rng.integers(0, 1 << bits, 3))
            key = oracle.morton(x, y, z, bits)
            np.testing.assert_array_equal(H.cell_corner(key, bits),
                                          np.array([x, y, z]) / float(1 << bits))


def test_leaf_is_the_deepest_patch_of_the_structure():
    ps = [np.zeros(0, np.int32), np.array([0, 1], np.int32), np.array([0, 2, 1], np.int32),
          np.array([2, 0], np.int32)]
    assert H.leaves(ps, 3) == [(3, 1), (2, 2), (3, 0)]


def clump_snapshot(centre, n_clump=3000, n_bg=20000, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = np.concatenate([np.asarray(centre) + rng.normal(0, 0.004, (n_clump, 3)),
                          rng.random((n_bg, 3))]) % 1.0
    X, fx = synth.quantize(pts[:, 0])
    Y, fy = synth.quantize(pts[:, 1])
    Z, fz = synth.quantize(pts[:, 2])
    return synth.Snapshot(X, Y, Z, fx, fy, fz, None, 5, 5.0, 5.0, 5, "clump")


@pytest.mark.parametrize("centre", [(0.31, 0.62, 0.18), (0.999, 0.0005, 0.5)])
def test_centre_of_the_leaf_is_its_periodic_mean(centre):
    p = clump_snapshot(centre)
    levels, order = oracle.build(p)
    ps, st = substructure.classify([lv.patch_parent for lv in levels],
                                   [lv.patch_nparticles for lv in levels])
    leaf = H.leaves(ps, len(st["host"]))
    pos = H.positions(p)
    # the biggest structure is the clump
    s = int(np.argmax([levels[1].patch_nparticles[q] for q in range(levels[1].n_patches)]))
    s = int(ps[1][s])
    L, q = leaf[s]
    c = H.centre_of(levels, order, pos, np.ones(p.n), L, q)
    idx = H.patch_particles(levels, order, L, q)
    # brute force: unwrap around the true clump centre, plain mean
    d = pos[idx] - np.asarray(centre)
    d -= np.round(d)
    want = (np.asarray(centre) + d.mean(axis=0)) % 1.0
    np.testing.assert_allclose(H.min_image(c - want), 0.0, atol=1e-12)
    assert np.linalg.norm(H.min_image(c - np.asarray(centre))) < 0.004


def test_full_run_invariants():
    p = synth.small_mixed(0, velocities=True)
    levels, order = oracle.build(p)
    ps, st = substructure.classify([lv.patch_parent for lv in levels],
                                   [lv.patch_nparticles for lv in levels])
    res = H.halos(p, levels, order, ps, st)
    assert len(res) == len(st["host"]) > 0
    pos = H.positions(p)
    kept = 0
    for h in res:
        mem, cand = h["members"], h["candidates"]
        assert np.all(np.isin(mem, cand)) and np.all(np.diff(mem) > 0)
        if mem.size:
            kept += 1
            d = H.min_image(pos[mem] - h["centre"])
            r = np.maximum(np.sqrt((d * d).sum(axis=1)), H.HALF_QUANTUM)
            assert r.max() <= h["r_vir"] and h["m_vir"] == mem.size
            assert h["m_vir"] / (4.0 / 3.0 * math.pi * h["r_vir"] ** 3) >= DELTA * p.n
        if st["depth"][h["struct"]] > 0:
            d = H.min_image(pos[cand] - h["centre"])
            assert np.all((d * d).sum(axis=1) <= h["radius"] ** 2)
    assert kept >= 5  # the eight NFW halos mostly survive their unbinding


def test_patch_extent_is_the_farthest_cell_corner():
    # a one-cell patch around its own centre: half the cell's diagonal
    p = clump_snapshot((0.3, 0.3, 0.3))
    levels, order = oracle.build(p)
    lv = levels[2]
    q = int(lv.cell_patch[0])
    cells = np.nonzero(lv.cell_patch == q)[0]
    h = 1.0 / (1 << lv.bits)
    corners = []
    for c in cells:
        lo = H.cell_corner(int(lv.cell_key[c]), lv.bits)
        for dx in (0, h):
            for dy in (0, h):
                for dz in (0, h):
                    corners.append(lo + [dx, dy, dz])
    centre = np.array([0.301, 0.299, 0.3005])
    d = H.min_image(np.array(corners) - centre)
    want = float(np.sqrt((d * d).sum(axis=1)).max())
    assert H.patch_extent(levels, 2, q, centre) == pytest.approx(want, rel=1e-15)
