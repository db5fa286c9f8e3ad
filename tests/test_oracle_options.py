"""Pins of the oracle's two model options.

- The paper's expansion setting (Sec. 2: local expansions to order p with
  multipoles only up to the quadrupole at p = 3), read as multipoles truncated
  at order p - 1 in every M2L and M2P (reading R1).  Forces only ever use
  multipoles of order <= p - 1, so the cap must leave them untouched; it must
  change the potential exactly where order-p moments exist.
- The optional self-potential term (reading R11): a leaf's own mass treated as
  a uniform cube adds -G m C / h to its potential, C the integral of 1/|r| over
  the unit cube about its centre.

None of these checks reuses the oracle's own formulas: the constant is pinned
to its closed form, the self term to the exact potential of a uniform cube
(prism formula), the cap to symmetry and to convergence against the direct sum.
"""
import numpy as np
import pytest

import oracle
from synth import cell_masses, plummer, unigrid
from synth.hierarchy import build_graded, refine_sphere


def _amr():
    return build_graded(3, 5, refine_sphere((0.5, 0.5, 0.5), {3: 0.3, 4: 0.2}))


def test_self_constant_closed_form():
    # integral of 1/|r| over [-1/2, 1/2]^3 = 3 ln(2 + sqrt 3) - pi/2
    exact = 3.0 * np.log(2.0 + np.sqrt(3.0)) - np.pi / 2.0
    assert abs(oracle.self_constant() - exact) <= 1e-13 * exact


def _prism_potential(pts, lo, hi):
    """Integral of 1/|r - x| over the box [lo, hi] at points x (closed form of the
    uniform rectangular prism: sum over the 8 corners of
    xy ln(z + r) + yz ln(x + r) + zx ln(y + r) - x^2/2 atan(yz / xr) - ...)."""
    def U(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return (x * y * np.log(z + r) + y * z * np.log(x + r) + z * x * np.log(y + r)
                - 0.5 * x * x * np.arctan(y * z / (x * r)) - 0.5 * y * y * np.arctan(z * x / (y * r))
                - 0.5 * z * z * np.arctan(x * y / (z * r)))
    out = np.zeros(pts.shape[0])
    for i, x in enumerate((lo[0] - pts[:, 0], hi[0] - pts[:, 0])):
        for j, y in enumerate((lo[1] - pts[:, 1], hi[1] - pts[:, 1])):
            for k, z in enumerate((lo[2] - pts[:, 2], hi[2] - pts[:, 2])):
                out += (-1.0) ** (3 - i - j - k) * U(x, y, z)
    return out


def test_prism_formula_itself():
    c = np.array([[0.5, 0.5, 0.5]])
    assert abs(_prism_potential(c, (0, 0, 0), (1, 1, 1))[0] - (3 * np.log(2 + np.sqrt(3)) - np.pi / 2)) < 1e-12
    # a far point: the potential of the unit cube is nearly that of a point mass
    far = np.array([[40.5, 0.5, 0.5]])
    assert abs(_prism_potential(far, (0, 0, 0), (1, 1, 1))[0] * 40.0 - 1.0) < 1e-4


def test_self_potential_reproduces_a_uniform_cube():
    """Uniform density filling the box: the exact potential at every cell centre
    is -G times the prism integral.  Cell-centred point masses miss each cell's
    own contribution; the self term restores it, leaving only the small
    higher-moment error of the neighbouring cubes (a cube's quadrupole is zero)."""
    lev = 4
    h = unigrid(lev)
    n = 1 << lev
    m = np.full(h.total, 1.0 / h.total)
    x = (h.flat_ijk().astype(np.float64) + 0.5) / n
    exact = -_prism_potential(x, (0, 0, 0), (1, 1, 1))
    errs = {}
    for self_pot in (False, True):
        phi, acc = oracle.Oracle(h, 6, self_potential=self_pot).solve_all(m)
        errs[self_pot] = np.abs(phi - exact).max() / np.abs(exact).max()
        if self_pot:
            phi0, acc0 = oracle.Oracle(h, 6).solve_all(m)
            assert np.array_equal(acc, acc0)  # the self term is potential only
    assert errs[True] < 1e-3, errs
    assert errs[True] < 0.1 * errs[False], errs


def test_self_potential_uses_each_leaf_level():
    """On AMR the term scales as m / h of the leaf's own level."""
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 7)
    p0, a0 = oracle.Oracle(h, 4).solve_all(m)
    p1, a1 = oracle.Oracle(h, 4, self_potential=True).solve_all(m)
    leaf = h.leaf_mask()
    hl = 1.0 / (1 << h.level_of())
    d = (p1 - p0)[leaf]
    want = -(3 * np.log(2 + np.sqrt(3)) - np.pi / 2) * m[leaf] / hl[leaf]
    assert np.allclose(d, want, rtol=1e-12, atol=0)
    assert np.array_equal(a0, a1)


@pytest.mark.parametrize("p", [2, 3, 5, 6])
def test_quad_cap_keeps_forces_changes_potential(p):
    h = _amr()
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 11)
    pu, au = oracle.Oracle(h, p).solve_all(m)
    pc, ac = oracle.Oracle(h, p, quad_cap=True).solve_all(m)
    leaf = h.leaf_mask()
    assert np.array_equal(au[leaf], ac[leaf])
    dphi = np.linalg.norm(pc[leaf] - pu[leaf]) / np.linalg.norm(pu[leaf])
    assert dphi > 1e-9, dphi


def test_quad_cap_is_inert_when_order_p_moments_vanish():
    """Uniform masses on a unigrid: every FMM cell holds a cube of equal masses,
    mirror-symmetric about its centre, so all odd moments vanish; at p = 3 the
    capped order is odd and the cap changes nothing.  At p = 4 the dropped
    order-4 moments (the cube's hexadecapole, the first non-isotropic moment of
    a cube) do change the potential."""
    h = unigrid(4)
    m = np.full(h.total, 1.0 / h.total)
    pu, _ = oracle.Oracle(h, 3).solve_all(m)
    pc, _ = oracle.Oracle(h, 3, quad_cap=True).solve_all(m)
    assert np.linalg.norm(pc - pu) <= 1e-14 * np.linalg.norm(pu)
    p4u, _ = oracle.Oracle(h, 4).solve_all(m)
    p4c, _ = oracle.Oracle(h, 4, quad_cap=True).solve_all(m)
    assert np.linalg.norm(p4c - p4u) > 1e-9 * np.linalg.norm(p4u)


def test_quad_cap_potential_converges_to_direct_sum():
    h = unigrid(4)
    m = cell_masses(h, plummer(1.0, 0.1), 0.01, 3)
    x = (h.flat_ijk().astype(np.float64) + 0.5) / 16
    pd, _ = oracle.direct(x, m, x)
    errs = []
    for p in (2, 4, 6, 8):
        pc, _ = oracle.Oracle(h, p, quad_cap=True).solve_all(m)
        errs.append(np.linalg.norm(pc - pd) / np.linalg.norm(pd))
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
