"""Pins for the nonlocal projector matrix (eqn Vnonloc) and projector functions."""
import numpy as np
import pytest
from scipy import integrate

from oracle import operator as op
from oracle import projectors as pj
from oracle.mesh import Mesh


def _radial_s_integral(sigma, rc):
    f = lambda r: 4 * np.pi * r * r * np.exp(-r * r / (2 * sigma * sigma)) * (1 - r * r / (rc * rc)) ** 2
    return integrate.quad(f, 0.0, rc, epsabs=1e-14, epsrel=1e-13)[0]


def test_s_projector_integral_converges_to_radial_integral():
    rc, sigma = 3.0, 1.0
    want = _radial_s_integral(sigma, rc)
    R = np.array([[4.3, 3.9, 4.1]])
    errs = []
    for N in (4, 8):
        m = Mesh(np.eye(3) * 10.0, (N, N, N), 5, 6)
        P, h = op.projector_matrix(m, R, [dict(atom=0, l=0, m=0, sigma=sigma, rc=rc, h=1.0)])
        errs.append(abs(P.sum() - want) / want)        # sum_I F_I = int chi (partition of unity)
    # the radial factor is only C^1 at r_c, which limits the rate to about h^3
    assert errs[1] < 1e-6 and errs[1] < errs[0] / 6


@pytest.mark.parametrize("l,mm", [(1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (2, 2), (2, 3)])
def test_odd_and_traceless_projectors_integrate_to_zero(l, mm):
    # atom on a mesh vertex: the mesh and the Gauss points are symmetric about it
    m = Mesh(np.eye(3) * 8.0, (4, 4, 4), 4, 5)
    R = np.array([[4.0, 4.0, 4.0]])
    P, _ = op.projector_matrix(m, R, [dict(atom=0, l=l, m=mm, sigma=1.0, rc=3.0, h=1.0)])
    P0, _ = op.projector_matrix(m, R, [dict(atom=0, l=0, m=0, sigma=1.0, rc=3.0, h=1.0)])
    assert abs(P.sum()) < 1e-13 * abs(P0.sum())


def test_lattice_translation_covariance():
    k = np.array([0.4, -0.3, 0.2])
    A = np.array([[7.0, 0, 0], [1.0, 6.5, 0], [0.5, 0.3, 7.5]])
    m = Mesh(A, (3, 3, 3), 3, 4, kpoint=k)
    R = np.array([1.3, 5.2, 2.2])
    pr = [dict(atom=0, l=1, m=2, sigma=1.0, rc=3.0, h=0.7), dict(atom=0, l=2, m=3, sigma=1.0, rc=3.0, h=-0.4)]
    P1, h = op.projector_matrix(m, R[None], pr)
    P1b, _ = op.projector_matrix(m, R[None], pr, images=2)
    assert np.abs((P1b - P1).toarray()).max() < 1e-15       # 27 images are complete
    P2, _ = op.projector_matrix(m, (R + A[1])[None], pr, images=2)
    phase = np.exp(-1j * (k @ A[1]))
    assert np.abs(P2.toarray() - phase * P1.toarray()).max() < 1e-13 * np.abs(P1.toarray()).max()
    H1, H2 = op.nonlocal_dense(P1, h), op.nonlocal_dense(P2, h)
    assert np.abs(H1 - H2).max() < 1e-13 * np.abs(H1).max()


def test_rank_and_sign_structure():
    m = Mesh(np.eye(3) * 8.0, (3, 3, 3), 3, 4, kpoint=(0.2, 0.1, 0.0))
    rng = np.random.default_rng(0)
    R = rng.uniform(0, 8, (2, 3))
    pr = [dict(atom=a, l=l, m=mm, sigma=1.0, rc=3.0, h=1.0) for a in range(2) for l, mm in [(0, 0), (1, 0), (1, 1)]]
    P, h = op.projector_matrix(m, R, pr)
    Hn = op.nonlocal_dense(P, h)
    assert np.linalg.matrix_rank(Hn, tol=1e-10 * np.abs(Hn).max()) == len(pr)
    assert np.abs(Hn - Hn.conj().T).max() < 1e-14 * np.abs(Hn).max()
    x = rng.standard_normal(m.m) + 1j * rng.standard_normal(m.m)
    Pd = P.toarray()
    assert abs(x.conj() @ Hn @ x - np.sum(np.abs(Pd.conj().T @ x) ** 2)) < 1e-10 * np.abs(x.conj() @ Hn @ x)
    # a vector orthogonal to every projector column is annihilated
    Q, _ = np.linalg.qr(Pd)
    y = x - Q @ (Q.conj().T @ x)
    assert np.abs(Hn @ y).max() < 1e-12 * np.abs(Hn @ x).max()


def test_chi_form():
    r = np.array([[0.3, -0.4, 1.2], [2.9, 0.1, 0.0], [3.1, 0.0, 0.0]])
    rho2 = np.sum(r * r, 1)
    rad = np.exp(-rho2 / 2.0) * (1 - rho2 / 9.0) ** 2
    rad[2] = 0.0
    assert np.allclose(pj.chi(0, 0, r, 1.0, 3.0), rad)
    assert np.allclose(pj.chi(1, 1, r, 1.0, 3.0), r[:, 1] * rad)
    assert np.allclose(pj.chi(2, 4, r, 1.0, 3.0), (3 * r[:, 2] ** 2 - rho2) * rad)
