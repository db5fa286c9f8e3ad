"""Pins of the whole oracle FMM: exactness where every pair is near, convergence
to the O(N^2) direct sum with p, invariants (linearity, mirror symmetry,
per-tree vs merged summation, nearest-field antisymmetry), the adaptive time
stepping life cycle (Alg. 1/2) and the input checks."""
import numpy as np
import pytest

import oracle
from synth import cell_masses, plummer, shuffle_order, unigrid, mirror_x
from synth.hierarchy import Hierarchy, build_graded, refine_sphere


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _direct_leaves(h, m):
    leaf = h.leaf_mask()
    x = h.centres()
    return oracle.direct(x[leaf], m[leaf], x[leaf])


@pytest.mark.parametrize("level", [1, 2])
def test_all_pairs_near_equals_direct(level):
    """2^3 and 4^3 grids: every pair is in the near field, so FMM == direct sum."""
    h = unigrid(level)
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    pd, ad = _direct_leaves(h, m)
    for p in (1, 4, 8):
        phi, acc = oracle.Oracle(h, p).solve_all(m)
        np.testing.assert_allclose(phi, pd, rtol=1e-13)
        np.testing.assert_allclose(acc, ad, rtol=1e-12, atol=1e-13 * np.abs(ad).max())


@pytest.mark.parametrize("level", [3, 4])
def test_unigrid_error_falls_with_order(level):
    h = unigrid(level)
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    pd, ad = _direct_leaves(h, m)
    ea = []
    for p in (2, 4, 6, 8):
        phi, acc = oracle.Oracle(h, p).solve_all(m)
        ea.append(_rel(acc, ad))
        assert _rel(phi, pd) < 2e-3
    assert all(b < 0.5 * a for a, b in zip(ea, ea[1:]))
    assert ea[-1] < 1e-4


def test_unigrid_32_full_size_against_direct():
    """The 32^3 unigrid (Plummer a = 0.1, 1% noise, seed 1) at full size against the
    O(N^2) direct sum over all 32,768 cells.  The paper prints no error for this
    setting, so the values are recorded rather than pinned: relative L2 force error
    2.35e-3 and potential error 1.6e-4 at p = 4, 4.1e-4 and 2.6e-5 at p = 6."""
    h = unigrid(5)
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    pd, ad = _direct_leaves(h, m)
    phi4, acc4 = oracle.Oracle(h, 4).solve_all(m)
    phi6, acc6 = oracle.Oracle(h, 6).solve_all(m)
    e4, e6 = _rel(acc4, ad), _rel(acc6, ad)
    assert 2.0e-3 < e4 < 2.7e-3 and 1.3e-4 < _rel(phi4, pd) < 1.9e-4
    assert 3.4e-4 < e6 < 4.8e-4 and e6 < 0.25 * e4 and _rel(phi6, pd) < 0.25 * _rel(phi4, pd)


def _amr(lmin=4, radii=None):
    radii = radii or {4: 0.25, 5: 0.12}
    return build_graded(lmin, lmin + len(radii), refine_sphere((0.5, 0.5, 0.5), radii))


def test_amr_error_falls_with_order():
    h = _amr(3, {3: 0.3, 4: 0.2, 5: 0.1})
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 3)
    leaf = h.leaf_mask()
    pd, ad = _direct_leaves(h, m)
    ea = []
    for p in (2, 4, 6):
        phi, acc = oracle.Oracle(h, p).solve_all(m)
        ea.append(_rel(acc[leaf], ad))
    assert all(b < 0.5 * a for a, b in zip(ea, ea[1:]))
    assert ea[-1] < 5e-4


def test_per_tree_equals_merged_and_chain():
    """Alg. 3/4 applied tree by tree equals one merged multipole per source (linearity),
    and the P2M + M2M chain equals the multipole definition."""
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 4)
    o = oracle.Oracle(h, 5)
    phi, acc = o.solve_all(m)
    o.set_merged_all(True)
    phi2, acc2 = o.solve_all(m)
    leaf = h.leaf_mask()
    assert np.abs(phi2[leaf] - phi[leaf]).max() <= 1e-13 * np.abs(phi[leaf]).max()
    assert np.abs(acc2[leaf] - acc[leaf]).max() <= 1e-13 * np.abs(acc[leaf]).max()
    for j in range(h.levelmin, h.levelmax + 1):
        assert o.chain_check(j) < 1e-13


def test_linearity_and_refined_masses_ignored():
    h = _amr()
    rng = np.random.default_rng(1)
    m1 = rng.uniform(0, 1, h.total)
    m2 = rng.uniform(0, 1, h.total)
    o = oracle.Oracle(h, 4)
    p1, a1 = o.solve_all(m1)
    p2, a2 = o.solve_all(m2)
    p3, a3 = o.solve_all(m1 + 2.5 * m2)
    leaf = h.leaf_mask()
    np.testing.assert_allclose(p3[leaf], p1[leaf] + 2.5 * p2[leaf], rtol=1e-12)
    np.testing.assert_allclose(a3[leaf], a1[leaf] + 2.5 * a2[leaf], rtol=1e-10,
                               atol=1e-12 * np.abs(a3).max())
    m4 = m1.copy()
    m4[~leaf] = 1e6
    p4, a4 = o.solve_all(m4)
    np.testing.assert_array_equal(p4[leaf], p1[leaf])


def test_mirror_symmetry():
    """x -> 1 - x maps the dyadic geometry onto itself: phi is mirrored, a_x flips."""
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1, (0.45, 0.55, 0.5)), 0.01, 5)
    phi, acc = oracle.Oracle(h, 4).solve_all(m)
    hm = mirror_x(h)
    phim, accm = oracle.Oracle(hm, 4).solve_all(m)
    leaf = h.leaf_mask()
    np.testing.assert_allclose(phim[leaf], phi[leaf], rtol=1e-12)
    np.testing.assert_allclose(accm[leaf, 0], -acc[leaf, 0], rtol=1e-9, atol=1e-12 * np.abs(acc).max())
    np.testing.assert_allclose(accm[leaf, 1:], acc[leaf, 1:], rtol=1e-9, atol=1e-12 * np.abs(acc).max())


def test_caller_order_does_not_matter():
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 6)
    phi, acc = oracle.Oracle(h, 4).solve_all(m)
    hs = shuffle_order(h, 99)
    lut = {(int(l),) + tuple(int(v) for v in c): i for i, (l, c) in enumerate(zip(h.level_of(), h.flat_ijk()))}
    perm = np.array([lut[(int(l),) + tuple(int(v) for v in c)] for l, c in zip(hs.level_of(), hs.flat_ijk())])
    phis, accs = oracle.Oracle(hs, 4).solve_all(m[perm])
    leaf = hs.leaf_mask()
    np.testing.assert_allclose(phis[leaf], phi[perm][leaf], rtol=1e-12)
    np.testing.assert_allclose(accs[leaf], acc[perm][leaf], rtol=1e-9, atol=1e-12 * np.abs(acc).max())


def _nearest_pair(h):
    """A coarse leaf c and a fine leaf f in c's nearest field (f a child of a refined
    cell touching c); returns flat indices."""
    lev = h.level_of()
    ijk = h.flat_ijk()
    ref = h.flat_refined()
    index = {(int(l),) + tuple(int(v) for v in c): i for i, (l, c) in enumerate(zip(lev, ijk))}
    for i in range(h.total):
        l = int(lev[i])
        if ref[i] or l == h.levelmax:
            continue
        c = ijk[i]
        for d in np.ndindex(3, 3, 3):
            n = tuple(int(c[k] + d[k] - 1) for k in range(3))
            j = index.get((l,) + n)
            if j is None or not ref[j]:
                continue
            f = index[(l + 1, 2 * n[0], 2 * n[1], 2 * n[2])]
            return i, f
    raise AssertionError("no coarse-fine nearest pair")


def test_nearest_pair_forces_are_exactly_antisymmetric():
    """Sec. 3.2: the nearest field makes coarse-fine pairs act by mutual P2P."""
    h = _amr()
    ci, fi = _nearest_pair(h)
    m = np.zeros(h.total)
    m[ci], m[fi] = 0.7, 0.3
    phi, acc = oracle.Oracle(h, 6).solve_all(m)
    mom = m[ci] * acc[ci] + m[fi] * acc[fi]
    assert np.linalg.norm(mom) <= 1e-14 * m[ci] * np.linalg.norm(acc[ci])
    # the pair force is the exact point-mass force
    x = h.centres()
    R = x[ci] - x[fi]
    np.testing.assert_allclose(acc[ci], -m[fi] * R / np.linalg.norm(R) ** 3, rtol=1e-13)


def test_far_pair_is_not_symmetric():
    """Pairs coupled through multipoles do not conserve momentum exactly (Sec. 4)."""
    h = unigrid(4)
    m = np.zeros(h.total)
    ijk = h.flat_ijk()
    # two cells far apart and not related by a symmetry of the grid
    i = int(np.nonzero(np.all(ijk == (1, 2, 0), axis=1))[0][0])
    j = int(np.nonzero(np.all(ijk == (12, 9, 14), axis=1))[0][0])
    m[i], m[j] = 1.0, 1.0
    phi, acc = oracle.Oracle(h, 4).solve_all(m)
    mom = np.linalg.norm(acc[i] + acc[j])
    assert mom > 1e-10 * np.linalg.norm(acc[i])
    assert mom < 1e-2 * np.linalg.norm(acc[i])


def test_unigrid_near_only_momentum_is_zero():
    h = unigrid(2)
    m = cell_masses(h, plummer(1.0, 0.2, (0.4, 0.6, 0.5)), 0.01, 2)
    phi, acc = oracle.Oracle(h, 4).solve_all(m)
    tot = (m[:, None] * acc).sum(0)
    assert np.abs(tot).max() < 1e-13 * np.abs(m[:, None] * acc).sum()


def test_ats_stale_trees_equal_mixed_mass_solve():
    """Alg. 1/2: Solve(l, 1) with stale coarse trees equals a synchronous solve on the
    mixed mass field (coarse levels at their rebuild masses, fine levels fresh)."""
    h = _amr(3, {3: 0.3, 4: 0.2})
    rng = np.random.default_rng(8)
    m_old = cell_masses(h, plummer(1.0, 0.1), 0.01, 1)
    m_new = m_old * (1 + 0.05 * rng.uniform(-1, 1, h.total))
    lev = h.level_of()
    o = oracle.Oracle(h, 4)
    N = h.total
    phi = np.zeros(N)
    acc = np.zeros((N, 3))
    o.solve(3, 1, m_old, phi, acc)               # base step: rebuild all from m_old
    o.solve(4, 2, m_new, phi, acc)               # second half sub-cycle: rebuild trees >= 4
    mixed = np.where(lev >= 4, m_new, m_old)
    ref = oracle.Oracle(h, 4)
    pr, ar = ref.solve_all(mixed)
    sel = (lev == 4) & h.leaf_mask()
    np.testing.assert_allclose(phi[sel], pr[sel], rtol=1e-12)
    np.testing.assert_allclose(acc[sel], ar[sel], rtol=1e-9, atol=1e-12 * np.abs(ar).max())
    # icount = 1 keeps every tree stale: the fresh masses are not seen
    o.solve(5, 1, m_new * 3.0, phi, acc)
    sel5 = (lev == 5) & h.leaf_mask()
    np.testing.assert_allclose(phi[sel5], pr[sel5], rtol=1e-12)


def _single_chain(levelmin=3, depth=2):
    """levelmin complete; one refined cell per level below it (never graded for depth >= 2)."""
    n0 = 1 << levelmin
    g = np.arange(n0)
    ijk = [np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)]
    ref = [np.zeros(n0 ** 3, np.uint8)]
    c = np.array([n0 // 2] * 3)
    ref[0][np.nonzero(np.all(ijk[0] == c, axis=1))[0][0]] = 1
    for d in range(depth):
        ch = np.array([2 * c + np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1]) for o in range(8)], np.int32)
        r = np.zeros(8, np.uint8)
        if d + 1 < depth:
            r[0] = 1
        ijk.append(ch)
        ref.append(r)
        c = ch[0]
    return Hierarchy(levelmin, levelmin + depth, ijk, ref)


def test_input_checks():
    ok = _single_chain(3, 1)
    oracle.Oracle(ok, 4)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.Oracle(_single_chain(3, 2), 4)
    assert ei.value.code == -2
    h = _amr(3, {3: 0.3, 4: 0.2})
    inc = Hierarchy(h.levelmin, h.levelmax, [h.ijk[0], h.ijk[1][1:], h.ijk[2]],
                    [h.refined[0], h.refined[1][1:], h.refined[2]])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.Oracle(inc, 4)
    assert ei.value.code == -3
