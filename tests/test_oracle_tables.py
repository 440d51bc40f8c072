"""Pins of the oracle's 1D tables: closed forms, exactness, and high-precision roots."""
import mpmath
import numpy as np
import pytest

from oracle.tables import gll_nodes, gauss, lagrange_values, lagrange_derivs
from golden_fixtures import read_table

FX = read_table("gll_gauss_closed_forms.txt")


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_forms(p):
    np.testing.assert_allclose(gll_nodes(p), FX[("gll", p)], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [5, 6, 7, 8])
def test_gll_roots_high_precision(p):
    # interior nodes are roots of P_p'(2t-1): check against mpmath's root at 40 digits
    mpmath.mp.dps = 40
    xi = gll_nodes(p)
    dP = lambda s: mpmath.diff(lambda u: mpmath.legendre(p, u), s)
    for t in xi[1:-1]:
        root = mpmath.findroot(dP, 2 * t - 1)
        assert abs(float((root + 1) / 2) - t) < 2e-16
    np.testing.assert_allclose(xi + xi[::-1], 1.0, atol=1e-15)
    assert xi[0] == 0.0 and xi[-1] == 1.0


@pytest.mark.parametrize("q", [2, 3])
def test_gauss_closed_forms(q):
    z, w = gauss(q)
    np.testing.assert_allclose(z, FX[("gauss_points", q)], atol=1e-15)
    np.testing.assert_allclose(w, FX[("gauss_weights", q)], atol=1e-15)


@pytest.mark.parametrize("q", range(1, 10))
def test_gauss_exact_on_monomials(q):
    z, w = gauss(q)
    for k in range(2 * q):
        assert abs(np.sum(w * z ** k) - 1.0 / (k + 1)) < 5e-16
    # and not exact one degree higher (it is a q-point Gauss rule, not more)
    assert abs(np.sum(w * z ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-13


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_basis_properties(p):
    xi = gll_nodes(p)
    np.testing.assert_allclose(lagrange_values(xi, xi), np.eye(p + 1), atol=1e-14)
    t = np.linspace(-0.1, 1.1, 37)
    np.testing.assert_allclose(lagrange_values(xi, t).sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(lagrange_derivs(xi, t).sum(1), 0.0, atol=1e-10)
    # exact differentiation of t^k, k <= p
    Dv = lagrange_derivs(xi, t)
    for k in range(p + 1):
        expect = k * t ** (k - 1) if k > 0 else 0 * t
        np.testing.assert_allclose(Dv @ xi ** k, expect, atol=1e-11)


@pytest.mark.parametrize("p", [2, 4, 7])
def test_lagrange_derivative_vs_mpmath(p):
    # derivative of the Lagrange polynomial computed in 40-digit arithmetic by numerical differentiation
    mpmath.mp.dps = 40
    xi = gll_nodes(p)
    z, _ = gauss(p + 1)
    Dv = lagrange_derivs(xi, z)
    xs = [mpmath.mpf(float(v)) for v in xi]
    for a in range(p + 1):
        la = lambda t, a=a: mpmath.fprod([(t - xs[b]) / (xs[a] - xs[b]) for b in range(p + 1) if b != a])
        for k, zk in enumerate(z):
            assert abs(float(mpmath.diff(la, mpmath.mpf(float(zk)))) - Dv[k, a]) < 1e-13 * max(1, abs(Dv[k, a]))
