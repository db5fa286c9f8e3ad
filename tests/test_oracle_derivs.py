"""Pins of the oracle's derivative tables D_g(R) = d^g(-1/|R|).

The oracle evaluates exact integer numerator polynomials; these tests pin it to
(1) sympy's symbolic differentiation at rational points, (2) the Legendre
generating function of 1/|R - d| order by order (scipy's Legendre polynomials),
(3) Laplace's equation and (4) homogeneity of degree -1-|g|.
"""
import math

import numpy as np
import pytest
import sympy as sp
from scipy.special import eval_legendre

import oracle


def _mi(p):
    return oracle.multi_index(p)


@pytest.mark.parametrize("R", [(3, -2, 5), (1, 1, 1), (-7, 2, 1), (2, 0, -3)])
def test_derivs_match_sympy(R):
    p = 8
    x, y, z = sp.symbols("x y z", real=True)
    g = -1 / sp.sqrt(x * x + y * y + z * z)
    mi = _mi(p)
    D = oracle.derivs(p, np.array(R, dtype=float) / 4.0)
    pt = {x: sp.Rational(R[0], 4), y: sp.Rational(R[1], 4), z: sp.Rational(R[2], 4)}
    exact = np.zeros(len(mi))
    for k, (a, b, c) in enumerate(mi):
        key = (int(a), int(b), int(c))
        expr = sp.diff(g, x, key[0], y, key[1], z, key[2]) if sum(key) else g
        exact[k] = float(sp.N(expr.subs(pt), 30))
    deg = mi.sum(1)
    for n in range(p + 1):
        sel = deg == n
        scale = np.max(np.abs(exact[sel]))
        np.testing.assert_allclose(D[sel], exact[sel], rtol=1e-12, atol=1e-13 * scale)


def test_legendre_generating_function():
    """sum_{|g|=n} (-1)^n d^g/g! D_g(R) = -|d|^n P_n(cos t)/|R|^(n+1) for every n."""
    rng = np.random.default_rng(7)
    p = 9
    mi = _mi(p)
    deg = mi.sum(1)
    fact = np.array([math.factorial(a) * math.factorial(b) * math.factorial(c) for a, b, c in mi])
    for _ in range(20):
        R = rng.normal(size=3) * 2
        d = rng.normal(size=3)
        D = oracle.derivs(p, R)
        r, dn = np.linalg.norm(R), np.linalg.norm(d)
        cost = R @ d / (r * dn)
        mono = np.prod(d[None, :] ** mi, axis=1)
        for n in range(p + 1):
            sel = deg == n
            lhs = np.sum((-1) ** n * mono[sel] / fact[sel] * D[sel])
            rhs = -dn ** n * eval_legendre(n, cost) / r ** (n + 1)
            assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-13 * dn ** n / r ** (n + 1))


def test_laplace_and_homogeneity():
    rng = np.random.default_rng(3)
    p = 9
    mi = [tuple(int(v) for v in r) for r in _mi(p)]
    idx = {m: i for i, m in enumerate(mi)}
    for _ in range(10):
        R = rng.uniform(-3, 3, size=3) + np.array([4.0, 0, 0])
        D = oracle.derivs(p, R)
        for m in mi:
            if sum(m) + 2 > p:
                continue
            lap = sum(D[idx[(m[0] + 2 * (k == 0), m[1] + 2 * (k == 1), m[2] + 2 * (k == 2))]] for k in range(3))
            assert abs(lap) <= 1e-11 * max(1.0, np.max(np.abs(D)))
        s = 0.37
        Ds = oracle.derivs(p, s * R)
        for k, m in enumerate(mi):
            assert Ds[k] == pytest.approx(s ** (-1 - sum(m)) * D[k], rel=1e-12)


def test_low_order_closed_forms():
    R = np.array([0.3, -1.1, 0.7])
    r = np.linalg.norm(R)
    D = oracle.derivs(2, R)
    mi = [tuple(int(v) for v in a) for a in _mi(2)]
    idx = {m: i for i, m in enumerate(mi)}
    assert D[idx[(0, 0, 0)]] == pytest.approx(-1 / r)
    for k in range(3):
        e = tuple(int(k == j) for j in range(3))
        assert D[idx[e]] == pytest.approx(R[k] / r ** 3)
    assert D[idx[(2, 0, 0)]] == pytest.approx(-(3 * R[0] ** 2 - r * r) / r ** 5)
    assert D[idx[(1, 1, 0)]] == pytest.approx(-3 * R[0] * R[1] / r ** 5)
