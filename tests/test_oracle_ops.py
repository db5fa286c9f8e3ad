"""Pins of the oracle's translation steps (Sec. 2: Eqs. eqn:multipole, eq:M2M_general,
eq:M2L, eq:L2L) against definitions, exact polynomial identities and the
classical multipole truncation bound."""
import math

import numpy as np
import pytest
import sympy as sp

import oracle


def _cloud(rng, n, c, w):
    x = c + rng.uniform(-w, w, size=(n, 3))
    m = rng.uniform(0.1, 1.0, size=n)
    return x, m


def test_multipole_monopole_dipole_and_parity():
    rng = np.random.default_rng(0)
    c = np.array([0.3, 0.4, 0.5])
    x, m = _cloud(rng, 50, c, 0.1)
    M = oracle.multipole(4, x, m, c)
    mi = oracle.multi_index(4)
    assert M[0] == pytest.approx(m.sum(), rel=1e-14)
    for k in range(3):
        e = [0, 0, 0]
        e[k] = 1
        idx = int(np.nonzero(np.all(mi == e, axis=1))[0][0])
        assert M[idx] == pytest.approx(np.sum(m * (x[:, k] - c[k])), rel=1e-13)
    # a mass distribution symmetric under x -> 2c - x has no odd moments
    xs = np.concatenate([x, 2 * c - x])
    ms = np.concatenate([m, m])
    Ms = oracle.multipole(6, xs, ms, c)
    odd = oracle.multi_index(6).sum(1) % 2 == 1
    assert np.max(np.abs(Ms[odd])) < 1e-15 * ms.sum()


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_m2m_is_exact_and_composes(p):
    rng = np.random.default_rng(p)
    c1 = np.array([0.5, 0.5, 0.5])
    x, m = _cloud(rng, 40, c1, 0.05)
    M1 = oracle.multipole(p, x, m, c1)
    c2 = c1 + np.array([0.05, -0.025, 0.0125])
    c3 = c2 + np.array([-0.1, 0.05, 0.025])
    M2 = oracle.m2m(p, c2 - c1, M1)
    direct2 = oracle.multipole(p, x, m, c2)
    np.testing.assert_allclose(M2, direct2, rtol=1e-11, atol=1e-14 * np.abs(direct2).max())
    M3 = oracle.m2m(p, c3 - c2, M2)
    M3b = oracle.m2m(p, c3 - c1, M1)
    np.testing.assert_allclose(M3, M3b, rtol=1e-11, atol=1e-14 * np.abs(M3b).max())


def _poly_taylor(p, coeffs, mi, c):
    """Exact Taylor coefficients d^b phi(c) of phi = sum coeffs * x^k, |b| <= p."""
    x, y, z = sp.symbols("x y z")
    phi = sum(sp.Rational(int(cf), 7) * x ** int(a) * y ** int(b) * z ** int(cc)
              for cf, (a, b, cc) in zip(coeffs, mi))
    pt = {x: sp.Rational(c[0]), y: sp.Rational(c[1]), z: sp.Rational(c[2])}
    out = []
    for a, b, cc in mi:
        e = sp.diff(phi, x, int(a), y, int(b), z, int(cc)) if a + b + cc else phi
        out.append(float(e.subs(pt)))
    return phi, np.array(out), (x, y, z)


@pytest.mark.parametrize("p", [3, 5])
def test_l2l_and_l2p_exact_on_polynomials(p):
    rng = np.random.default_rng(11)
    mi = oracle.multi_index(p)
    coeffs = rng.integers(-9, 10, size=mi.shape[0])
    c = (sp.Rational(1, 4), sp.Rational(-1, 8), sp.Rational(3, 8))
    c2 = (sp.Rational(5, 16), sp.Rational(1, 16), sp.Rational(1, 4))
    phi, L, (x, y, z) = _poly_taylor(p, coeffs, mi, c)
    _, L2exact, _ = _poly_taylor(p, coeffs, mi, c2)
    a = np.array([float(c2[k] - c[k]) for k in range(3)])
    L2 = oracle.l2l(p, a, L)
    np.testing.assert_allclose(L2, L2exact, rtol=1e-12, atol=1e-12 * np.abs(L2exact).max())
    u = np.array([0.03, -0.02, 0.05])
    out = oracle.l2p(p, u, L)
    pt = {x: c[0] + sp.Rational(3, 100), y: c[1] - sp.Rational(2, 100), z: c[2] + sp.Rational(5, 100)}
    assert out[0] == pytest.approx(float(phi.subs(pt)), rel=1e-12)
    for k, s in enumerate((x, y, z)):
        assert out[1 + k] == pytest.approx(-float(sp.diff(phi, s).subs(pt)), rel=1e-11, abs=1e-12)


def test_m2p_obeys_point_source_bound_and_converges():
    """|phi_M2P - phi_exact| <= sum m/|R| * t^(p+1)/(1-t), t = max|v|/|R|."""
    rng = np.random.default_rng(5)
    c = np.zeros(3)
    x, m = _cloud(rng, 30, c, 0.125)
    vmax = np.max(np.linalg.norm(x - c, axis=1))
    dirs = rng.normal(size=(20, 3))
    pts = dirs / np.linalg.norm(dirs, axis=1)[:, None] * rng.uniform(0.6, 1.2, size=(20, 1))
    errs = []
    for p in range(1, 10):
        M = oracle.multipole(p, x, m, c)
        worst = 0.0
        for R in pts:
            out = oracle.m2p(p, R, M)
            ex, ea = oracle.direct(x, m, R[None, :])
            t = vmax / np.linalg.norm(R)
            bound = m.sum() / np.linalg.norm(R) * t ** (p + 1) / (1 - t)
            err = abs(out[0] - ex[0])
            assert err <= bound * (1 + 1e-9) + 1e-15
            worst = max(worst, err / abs(ex[0]))
            assert np.linalg.norm(out[1:] - ea[0]) / np.linalg.norm(ea[0]) < 20 * t ** p
        errs.append(worst)
    # the truncation error decays geometrically with the order
    assert all(errs[i + 2] < errs[i] for i in range(len(errs) - 2))
    assert errs[-1] < 1e-3 * errs[0]


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_m2l_then_l2p_at_centre_equals_m2p(p):
    """The total-degree truncation makes L_0 and -L_{e_i} the M2P potential and force exactly."""
    rng = np.random.default_rng(2)
    c = np.zeros(3)
    x, m = _cloud(rng, 20, c, 0.1)
    M = oracle.multipole(p, x, m, c)
    R = np.array([0.8, -0.35, 0.4])
    L = oracle.m2l(p, R, M)
    a = oracle.l2p(p, np.zeros(3), L)
    b = oracle.m2p(p, R, M)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-16)


def test_m2l_l2p_converges_to_exact():
    rng = np.random.default_rng(9)
    c = np.zeros(3)
    x, m = _cloud(rng, 25, c, 0.125)
    R = np.array([0.75, 0.375, -0.25])
    u = np.array([0.1, -0.05, 0.08])
    ex, ea = oracle.direct(x, m, (R + u)[None, :])
    errs = []
    for p in range(2, 10):
        M = oracle.multipole(p, x, m, c)
        out = oracle.l2p(p, u, oracle.m2l(p, R, M))
        errs.append(np.linalg.norm(out[1:] - ea[0]) / np.linalg.norm(ea[0]))
    assert errs[-1] < 1e-5
    assert all(b < a for a, b in zip(errs, errs[1:]))
