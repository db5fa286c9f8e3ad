"""Particle-mesh pieces on the CPU.

- The library's hierarchy that tracks particles (afmm_particle_hierarchy_create,
  C++) against ``synth.build_graded`` with the same refinement predicate
  (numpy): identical cells and flags per level (the library emits each level in
  Morton order, checked here, the numpy builder in (i, j, k) order), and graded
  by the independent checker.
- The time loop skips rebuilding that hierarchy while no particle's cloud
  cells change: whenever the cloud cells of two position sets agree, the
  library builds identical hierarchies from them (positions on and a few ulps
  around cell boundaries, a power-of-two and another box size).
- Pins of the oracle's cloud-in-cell: mass conservation, a particle at a cell
  centre, exact interpolation of linear fields, and the transpose relation
  between deposition and interpolation.
"""
import numpy as np
import pytest

from oracle import pm as opm
from paper_2607_19489_amd.pm import ParticleHierarchy, ParticleMesh, binary_initial
from synth.hierarchy import build_graded, check_graded


def _morton(ijk):
    key = np.zeros(ijk.shape[0], dtype=np.int64)
    for b in range(21):
        for d in range(3):
            key |= ((ijk[:, d].astype(np.int64) >> b) & 1) << (3 * b + d)
    return key


def _same(a, b):
    """Same levels, same cells with the same refined flags on every level; the
    library's levels in strictly increasing Morton order."""
    assert a.levelmin == b.levelmin and a.levelmax == b.levelmax
    assert np.array_equal(np.asarray(a.ncell), np.asarray(b.ncell))
    off = np.concatenate([[0], np.cumsum(np.asarray(a.ncell))])
    for i in range(len(off) - 1):
        ia, ra = a.flat_ijk()[off[i]:off[i + 1]], a.flat_refined()[off[i]:off[i + 1]]
        ib, rb = b.flat_ijk()[off[i]:off[i + 1]], b.flat_refined()[off[i]:off[i + 1]]
        assert np.all(np.diff(_morton(ia)) > 0)
        oa, ob = np.lexsort(ia.T[::-1]), np.lexsort(ib.T[::-1])
        assert np.array_equal(ia[oa], ib[ob]) and np.array_equal(ra[oa], rb[ob])


@pytest.mark.parametrize("lmin,lmax", [(3, 3), (3, 5), (4, 6), (2, 6)])
@pytest.mark.parametrize("nexpand", [0, 1, 2])
def test_particle_hierarchy_equals_python_builder(lmin, lmax, nexpand):
    rng = np.random.default_rng(100 * lmin + 10 * lmax + nexpand)
    for npart in (1, 2, 5):
        pos = rng.uniform(0.05, 0.95, size=(npart, 3))
        nat = ParticleHierarchy(pos, lmin, lmax, nexpand)
        ref = build_graded(lmin, lmax, opm.particle_refinement(pos, nexpand))
        _same(nat, ref)
        assert check_graded(ref) is None


def test_binary_hierarchy_keeps_particles_on_the_finest_level():
    pos, vel, m, omega = binary_initial()
    for lmax in (6, 7, 8):
        h = ParticleHierarchy(pos, 6, lmax, 2)
        assert h.levelmax == lmax
        index = opm._index(h)
        for x in pos:
            for c, w in opm.cloud(x, lmax):
                n = index[(lmax, *c)]
                assert h.flat_refined()[n] == 0


def test_particle_hierarchy_rejects_particles_outside_the_box():
    import paper_2607_19489_amd as A
    with pytest.raises(A.AfmmError):
        ParticleHierarchy(np.array([[0.5, 0.5, 1.2]]), 3, 4)


def _unigrid(level):
    from synth import unigrid
    return unigrid(level)


def test_cic_conserves_mass_and_hits_centres():
    h = _unigrid(4)
    rng = np.random.default_rng(1)
    pos = rng.uniform(0.1, 0.9, size=(20, 3))
    pm = rng.uniform(0.5, 2.0, size=20)
    m = opm.deposit(h, 4, pos, pm)
    assert abs(m.sum() - pm.sum()) <= 1e-13 * pm.sum()
    assert np.all(m >= 0)
    # a particle on a cell centre puts all its mass in that cell
    c = np.array([[5.5, 7.5, 9.5]]) / 16
    m1 = opm.deposit(h, 4, c, [3.0])
    idx = opm._index(h)
    assert m1[idx[(4, 5, 7, 9)]] == 3.0 and np.count_nonzero(m1) == 1


def test_cic_interpolates_linear_fields_exactly_and_is_the_transpose_of_deposit():
    h = _unigrid(4)
    x = (h.flat_ijk().astype(np.float64) + 0.5) / 16
    a, b = np.array([0.3, -1.7, 2.2]), 0.45
    f = x @ a + b
    rng = np.random.default_rng(2)
    pos = rng.uniform(0.1, 0.9, size=(30, 3))
    fp = opm.interpolate(h, 4, pos, f)
    assert np.allclose(fp, pos @ a + b, rtol=0, atol=1e-13)
    # <deposit(m), g> = <m, interpolate(g)> for any cell field g
    g = rng.standard_normal(h.total)
    pm = rng.uniform(0.5, 2.0, size=30)
    lhs = float(np.dot(opm.deposit(h, 4, pos, pm), g))
    rhs = float(np.dot(pm, opm.interpolate(h, 4, pos, g)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_binary_initial_is_a_circular_orbit():
    pos, vel, m, omega = binary_initial(gm=0.01, sep=0.15)
    d = pos[0] - pos[1]
    assert abs(np.linalg.norm(d) - 0.15) < 1e-15
    # centripetal acceleration omega^2 r equals the mutual attraction G m / d^2
    r = 0.075
    assert abs(omega ** 2 * r - 0.01 / 0.15 ** 2) < 1e-14
    assert np.allclose(m[0] * vel[0] + m[1] * vel[1], 0.0)
    # the period is about 2.58, so t = 8 is about three orbits
    assert 3.0 < 8.0 * omega / (2 * np.pi) < 3.2


@pytest.mark.parametrize("boxlen", [1.0, 2.7])
def test_equal_cloud_cells_give_the_same_hierarchy(boxlen):
    class Box:  # the attributes ParticleMesh._cloud_cells reads
        levelmin, levelmax = 3, 6
    Box.boxlen = boxlen
    cloud_cells = lambda pos: ParticleMesh._cloud_cells(Box, pos)
    rng = np.random.default_rng(17)
    checked = changed = 0
    for _ in range(60):
        # a particle placed on a cloud boundary of a random level, then nudged
        # by a few ulps either way; a second particle elsewhere
        l = int(rng.integers(Box.levelmin, Box.levelmax))
        k = rng.integers(2, (1 << l) - 3, size=3)
        x = (k + 0.5) * boxlen / (1 << l)
        base = np.array([x, rng.uniform(0.1, 0.9, 3) * boxlen])
        for ulps in (-3, -1, 0, 1, 3):
            pos = base.copy()
            pos[0] = x + ulps * np.spacing(x)
            for ref in (base, pos):
                if np.array_equal(cloud_cells(ref), cloud_cells(pos)):
                    ha = ParticleHierarchy(ref, Box.levelmin, Box.levelmax, 1, boxlen)
                    hb = ParticleHierarchy(pos, Box.levelmin, Box.levelmax, 1, boxlen)
                    assert hb.same_as(ha)
                    checked += 1
                else:
                    changed += 1
    assert checked > 100 and changed > 20
