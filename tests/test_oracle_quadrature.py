"""Pins of the oracle's 1D rules and Lagrange tables against closed forms and library routines."""
import json
import math
import os

import numpy as np
import pytest

from oracle.quadrature import gauss_rule, gll_rule, lagrange_deriv_table, lagrange_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quadrature_closed_forms.json")


def _ev(s):
    return eval(s, {"sqrt": math.sqrt})


@pytest.mark.parametrize("family", ["gauss", "gll"])
def test_closed_forms(family):
    data = json.load(open(GOLDEN))[family]
    for n, ref in data.items():
        n = int(n)
        x, w = gauss_rule(n) if family == "gauss" else gll_rule(n)
        np.testing.assert_allclose(x, [_ev(s) for s in ref["nodes"]], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(s) for s in ref["weights"]], rtol=1e-14)


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_matches_library_routine(q):
    x, w = gauss_rule(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, xr, atol=2e-15)
    np.testing.assert_allclose(w, wr, rtol=1e-13)


@pytest.mark.parametrize("n", range(1, 11))
def test_exactness_degrees(n):
    # Gauss with n points: exact to degree 2n-1; GLL of degree n (n+1 points): exact to 2n-1.
    for x, w in (gauss_rule(n), gll_rule(n)):
        assert abs(w.sum() - 2.0) < 1e-14
        for d in range(0, 2 * n):
            exact = 0.0 if d % 2 else 2.0 / (d + 1)
            assert abs(np.sum(w * x ** d) - exact) < 1e-13, (n, d)
        d = 2 * n  # first degree that is not integrated exactly
        exact = 2.0 / (d + 1)
        assert abs(np.sum(w * x ** d) - exact) > 1e-8


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_identities(p):
    xn, _ = gll_rule(p)
    pts = np.linspace(-1, 1, 17)
    phi = lagrange_table(xn, xn)
    np.testing.assert_allclose(phi, np.eye(p + 1), atol=1e-14)
    phi = lagrange_table(xn, pts)
    dphi = lagrange_deriv_table(xn, pts)
    np.testing.assert_allclose(phi.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(dphi.sum(axis=1), 0.0, atol=1e-11)
    # the interpolant of x^m, m <= p, is x^m itself, and so is its derivative
    for m in range(0, p + 1):
        np.testing.assert_allclose(phi @ xn ** m, pts ** m, atol=1e-13)
        dm = m * pts ** (m - 1) if m > 0 else np.zeros_like(pts)
        np.testing.assert_allclose(dphi @ xn ** m, dm, atol=1e-11)
