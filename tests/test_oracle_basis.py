"""Pins of the oracle's 1D rules against textbook facts (not against the oracle itself)."""
import numpy as np
import pytest

from oracle import basis


def test_gll_closed_forms():
    # Closed forms of the Gauss-Lobatto points on [-1, 1], mapped to [0, 1].
    np.testing.assert_allclose(basis.gll_points(1), [0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(basis.gll_points(2), [0.0, 0.5, 1.0], atol=1e-15)
    r3 = 1.0 / np.sqrt(5.0)
    np.testing.assert_allclose(basis.gll_points(3), 0.5 * (1 + np.array([-1, -r3, r3, 1])), atol=1e-15)
    r4 = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(basis.gll_points(4), 0.5 * (1 + np.array([-1, -r4, 0, r4, 1])), atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_are_roots_of_legendre_derivative(p):
    x = basis.gll_points(p)
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x + x[::-1], 1.0, atol=1e-14)
    if p > 1:
        _, dP = basis.legendre(p, 2 * x[1:-1] - 1)
        assert np.max(np.abs(dP)) < 1e-11


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exactness(n):
    x, w = basis.gauss_rule(n)
    for k in range(2 * n):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
    # first inexact monomial: the textbook remainder on [0, 1] is (n!)^4 / ((2n+1) ((2n)!)^2)
    from math import factorial
    rem = factorial(n) ** 4 / ((2 * n + 1) * factorial(2 * n) ** 2)
    err = 1.0 / (2 * n + 1) - np.dot(w, x ** (2 * n))
    assert abs(err - rem) < 1e-14 + 1e-6 * rem


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_properties(p):
    nodes = basis.gll_points(p)
    np.testing.assert_allclose(basis.lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-13)
    x = np.linspace(0, 1, 17)
    L = basis.lagrange_values(nodes, x)
    dL = basis.lagrange_derivatives(nodes, x)
    np.testing.assert_allclose(L.sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(dL.sum(axis=1), 0.0, atol=1e-10)
    for m in range(p + 1):
        np.testing.assert_allclose(L @ nodes ** m, x ** m, atol=1e-12)
        np.testing.assert_allclose(dL @ nodes ** m, m * x ** max(m - 1, 0) if m else 0 * x, atol=1e-10)
