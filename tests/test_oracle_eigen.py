"""Pins for oracle.eigen: Chebyshev closed forms, the Alg. 4 identity, Lanczos, RR."""
import numpy as np
import scipy.linalg as sla

from oracle import eigen
from oracle import operator as op
from oracle.mesh import Mesh


def _cheb(n, t):
    t = np.asarray(t, float)
    out = np.empty_like(t)
    a = np.abs(t) <= 1
    out[a] = np.cos(n * np.arccos(t[a]))
    b = t > 1
    out[b] = np.cosh(n * np.arccosh(t[b]))
    c = t < -1
    out[c] = (-1) ** n * np.cosh(n * np.arccosh(-t[c]))
    return out


def test_plain_filter_closed_form():
    a = np.linspace(-3.0, 10.0, 14)
    lmin, lT, lmax, deg = -3.2, 2.0, 10.5, 17
    X = np.eye(len(a))
    Y = eigen.cheb_filter_plain(lambda V: a[:, None] * V, X, deg, lmin, lmax, lT)
    e, c = (lmax - lT) / 2, (lmax + lT) / 2
    want = _cheb(deg, (a - c) / e) / _cheb(deg, np.array([(lmin - c) / e]))[0]
    assert np.allclose(np.diag(Y), want, rtol=1e-12, atol=1e-14)
    assert np.abs(Y - np.diag(np.diag(Y))).max() == 0.0


def test_residual_filter_equals_plain_filter_when_M_is_D():
    rng = np.random.default_rng(0)
    n, k = 50, 6
    A = rng.standard_normal((n, n))
    H = A + A.T + np.diag(np.arange(n, dtype=float))
    Dv = rng.uniform(0.5, 2.0, n)
    w = sla.eigvalsh(H, np.diag(Dv))
    X = rng.standard_normal((n, k))
    lam = rng.uniform(w[0], w[k], k)
    lmin, lmax, lT = w[0] - 0.1, w[-1] + 0.1, w[k + 4]
    Hop = lambda V: H @ V
    Dop = lambda V: Dv[:, None] * V
    Z1 = eigen.cheb_filter_residual(Hop, Dop, 1.0 / Dv, X, lam, 12, lmin, lmax, lT)
    Z2 = eigen.cheb_filter_plain(lambda V: (H @ V) / Dv[:, None], X, 12, lmin, lmax, lT)
    assert np.linalg.norm(Z1 - Z2) < 1e-12 * np.linalg.norm(Z2)


def test_lanczos_brackets_spectrum():
    rng = np.random.default_rng(1)
    d = np.sort(rng.uniform(-1, 5, 200))
    Dv = rng.uniform(0.5, 2.0, 200)
    H = np.diag(d * Dv)                           # D^-1 H has eigenvalues d
    theta, beta = eigen.lanczos_bounds(lambda V: H @ V, Dv, rng.standard_normal(200), 10)
    assert theta.max() <= d.max() + 1e-12 and theta.min() >= d.min() - 1e-12
    assert theta.max() + abs(beta) >= d.max()


def test_rayleigh_ritz_exact_on_invariant_subspace():
    rng = np.random.default_rng(2)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = A + A.conj().T
    Dv = rng.uniform(0.5, 2.0, n)
    w, V = sla.eigh(H, np.diag(Dv))
    Y = V[:, :5] @ (rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5)))
    lam, X = eigen.rayleigh_ritz(lambda B: H @ B, lambda B: Dv[:, None] * B, Y)
    assert np.allclose(lam, w[:5], atol=1e-10)


def test_chfsi_converges_to_generalized_eigenvalues():
    m = Mesh(np.eye(3) * 8.0, (3, 3, 3), 3, 4, kpoint=(0.1, 0.2, -0.1))
    rng = np.random.default_rng(5)
    nq = m.E * m.nq ** 3
    H = op.assemble_H(m, -np.abs(rng.standard_normal(nq)))
    Dv = op.lumped_mass(m)
    want = sla.eigvalsh(H.toarray(), np.diag(Dv))[:12]
    X0 = rng.standard_normal((m.m, 16)) + 1j * rng.standard_normal((m.m, 16))
    lam, X, _ = eigen.chfsi(lambda V: H @ V, Dv, X0, rng.standard_normal(m.m), m.volume,
                            outer=12, degree=20)
    assert np.abs(lam[:12] - want).max() < 1e-9


def test_chfsi_with_consistent_mass_converges_to_eigh_H_M():
    """Alg. 4 with the consistent M in the residual and Rayleigh-Ritz, D^-1 in
    the recurrence, reaches the eigenvalues of H u = eps M u."""
    m = Mesh(np.eye(3) * 8.0, (3, 3, 3), 3, 4, kpoint=(0.1, 0.2, -0.1))
    rng = np.random.default_rng(6)
    nq = m.E * m.nq ** 3
    H = op.assemble_H(m, -np.abs(rng.standard_normal(nq)))
    M = op.assemble_M(m)
    Dv = op.lumped_mass(m)
    want = sla.eigvalsh(H.toarray(), M.toarray())[:12]
    lumped = sla.eigvalsh(H.toarray(), np.diag(Dv))[:12]
    assert np.abs(want - lumped).max() > 1e-4          # the two problems differ
    X0 = rng.standard_normal((m.m, 16)) + 1j * rng.standard_normal((m.m, 16))
    lam, X, _ = eigen.chfsi(lambda V: H @ V, Dv, X0, rng.standard_normal(m.m), m.volume,
                            outer=14, degree=20, Mop=lambda V: M @ V)
    assert np.abs(lam[:12] - want).max() < 1e-9
