"""1D tables of the spectral finite-element basis (oracle; test infrastructure).

Sec. 2.2 (eqn FEdiscr): the basis is C0 Lagrange interpolation on the
Gauss-Lobatto-Legendre (GLL) points of degree p = FEOrder, n_p = p + 1 nodes
per direction.  Sec. 3.1 (eqn cellIntegrals): integrals use an n_q-point
Gauss-Legendre rule per direction.

Everything here is the textbook definition written out:
  * GLL nodes: -1, +1 and the roots of P'_p;   weights 2 / (p (p+1) P_p(x_i)^2)
  * Gauss nodes and weights: numpy's Legendre-Gauss routine
  * l_i(x) = prod_{j != i} (x - x_j) / (x_i - x_j)   (product formula)
  * l_i'(x) by the product rule (the *direct* derivative, not a collocation
    derivative).

Pins (tests/test_oracle_basis.py): closed-form GLL nodes/weights for p = 2, 3, 4,
Kronecker-delta property, partition of unity, exactness of interpolation and
differentiation on polynomials of degree <= p, exactness of both quadratures
on polynomials of the degree they are supposed to integrate.
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gll_nodes_weights(p):
    """GLL nodes (ascending) and weights for polynomial degree p >= 1."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    Pp = _leg.Legendre.basis(p)
    dP = Pp.deriv()
    x = np.empty(p + 1)
    x[0], x[-1] = -1.0, 1.0
    if p > 1:
        inner = np.sort(dP.roots().real)
        d2P = dP.deriv()
        for _ in range(4):                      # Newton polish of P'_p roots
            inner = inner - dP(inner) / d2P(inner)
        x[1:-1] = inner
    w = 2.0 / (p * (p + 1) * Pp(x) ** 2)
    return x, w


def gauss_points_weights(nq):
    """Gauss-Legendre points (ascending) and weights on [-1, 1]."""
    x, w = _leg.leggauss(nq)
    return np.asarray(x, float), np.asarray(w, float)


def lagrange_values(nodes, x):
    """V[a, i] = l_i(x_a) for the Lagrange polynomials on ``nodes``."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[a, i] = l_i'(x_a), product rule applied to the product formula."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


def tables_1d(p, nq):
    """(GLL nodes, GLL weights, Gauss points, Gauss weights, N1, dN1).

    N1[q, i] = l_i(xi_q), dN1[q, i] = l_i'(xi_q) at the Gauss points: the
    1D shape-function values and direct derivatives (n_q x n_p).
    """
    xg, wg = gll_nodes_weights(p)
    xq, wq = gauss_points_weights(nq)
    return xg, wg, xq, wq, lagrange_values(xg, xq), lagrange_derivatives(xg, xq)
