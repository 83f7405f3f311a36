"""Pins for oracle.basis: closed-form GLL / Gauss rules and Lagrange properties."""
import math

import numpy as np
import pytest

from oracle import basis


def test_gll_closed_forms():
    x, w = basis.gll_nodes_weights(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = basis.gll_nodes_weights(3)
    r = 1 / math.sqrt(5)
    assert np.allclose(x, [-1, -r, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = basis.gll_nodes_weights(4)
    r = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


def test_gauss_closed_forms():
    x, w = basis.gauss_points_weights(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)]) and np.allclose(w, [1, 1])
    x, w = basis.gauss_points_weights(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_quadrature_exactness(p):
    xg, wg = basis.gll_nodes_weights(p)
    for d in range(2 * p):                # GLL exact to degree 2p - 1
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.dot(wg, xg ** d) - exact) < 1e-13
    nq = p + 1
    xq, wq = basis.gauss_points_weights(nq)
    for d in range(2 * nq):               # Gauss exact to degree 2 nq - 1
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.dot(wq, xq ** d) - exact) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8, 9])
def test_lagrange_properties(p):
    xg, _ = basis.gll_nodes_weights(p)
    assert np.allclose(basis.lagrange_values(xg, xg), np.eye(p + 1), atol=1e-14)
    x = np.linspace(-1, 1, 37)
    V = basis.lagrange_values(xg, x)
    D = basis.lagrange_derivatives(xg, x)
    assert np.allclose(V.sum(1), 1.0, atol=1e-13)
    assert np.allclose(D.sum(1), 0.0, atol=1e-11)
    for d in range(p + 1):            # interpolation / derivative exact on degree <= p
        assert np.allclose(V @ xg ** d, x ** d, atol=1e-12)
        dd = d * x ** (d - 1) if d else np.zeros_like(x)
        assert np.allclose(D @ xg ** d, dd, atol=1e-10)


def test_derivative_matches_finite_difference():
    xg, _ = basis.gll_nodes_weights(5)
    x = np.array([-0.7, 0.1, 0.55])
    h = 1e-6
    fd = (basis.lagrange_values(xg, x + h) - basis.lagrange_values(xg, x - h)) / (2 * h)
    assert np.allclose(basis.lagrange_derivatives(xg, x), fd, atol=1e-7)
