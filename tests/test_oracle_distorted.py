"""Pins for oracle.distorted (cells with a Jacobian per quadrature point)."""
import numpy as np
import pytest

from oracle import distorted as dm
from oracle import operator as op
from oracle.mesh import Mesh
from paper_2512_08571_amd import inputs

LAT = np.array([[6.0, 0.0, 0.0], [0.4, 6.5, 0.0], [0.2, -0.3, 7.0]])


def _pair(amp, p=2, N=(3, 3, 4), k=(0.0, 0.0, 0.0), seed=3):
    vd = inputs.vertex_displacement(N, LAT, amp, seed)
    return dm.DistortedMesh(LAT, N, p, p + 1, vd, kpoint=k), Mesh(LAT, N, p, p + 1, kpoint=k)


def test_zero_displacement_is_the_affine_oracle():
    d, a = _pair(0.0, p=2, k=(0.2, -0.1, 0.3))
    rng = np.random.default_rng(0)
    nq = a.E * a.nq ** 3
    vl, vg = rng.standard_normal(nq), rng.standard_normal((nq, 3))
    assert np.abs(d.quad_points() - a.quad_points()).max() < 1e-12
    Hd, Ha = dm.assemble_H(d, vl, vg).toarray(), op.assemble_H(a, vl, vg).toarray()
    assert np.abs(Hd - Ha).max() < 1e-12 * np.abs(Ha).max()
    assert np.abs(dm.assemble_M(d).toarray() - op.assemble_M(a).toarray()).max() < 1e-14
    assert np.abs(dm.lumped_mass(d) - op.lumped_mass(a)).max() < 1e-14
    pos = np.array([[1.0, 2.0, 3.0]])
    projs = [dict(atom=0, l=1, m=mm, sigma=0.6, rc=1.8, h=0.5) for mm in range(3)]
    Pd, _ = dm.projector_matrix(d, pos, projs)
    Pa, _ = op.projector_matrix(a, pos, projs)
    assert np.abs((Pd - Pa).toarray()).max() < 1e-13


@pytest.mark.parametrize("p", [2, 4])
def test_volumes_and_mass_sums(p):
    d, a = _pair(0.15, p=p)
    vol = abs(np.linalg.det(LAT))
    cv = dm.cell_volumes(d)
    assert abs(cv.sum() - vol) < 1e-11 * vol
    assert np.std(cv) > 1e-3 * cv.mean()                  # the cells really differ
    Me = dm.mass_elements(d)
    assert np.abs(Me.sum(axis=(1, 2)) - cv).max() < 1e-12 * cv.max()
    assert abs(dm.lumped_mass(d).sum() - vol) < 1e-11 * vol


@pytest.mark.parametrize("p", [2, 3, 5])
def test_kinetic_patch_test_and_constants(p):
    """T 1 = 0 everywhere; for a physical linear function u = g.x (taken at the
    nodes' unwrapped positions) the kinetic rows of nodes whose surrounding
    cells all lie off the periodic seam vanish: int grad N_I = 0 exactly."""
    N = (4, 4, 4)
    d, _ = _pair(0.15, p=p, N=N, seed=7)
    nq = d.E * d.nq ** 3
    T = dm.assemble_H(d, np.zeros(nq)).toarray()
    assert np.abs(T @ np.ones(d.m)).max() < 1e-11 * np.abs(T).max()
    g = np.array([0.7, -1.3, 0.4])
    cells = np.arange(d.E)
    Te = dm.element_matrices(d, np.zeros(nq), None, cells)
    ue = d.node_points(cells) @ g                                         # [E, n_p^3]
    r = np.zeros(d.m)
    np.add.at(r, d.cell_dofs().reshape(-1), np.einsum("cij,cj->ci", Te, ue).reshape(-1))
    # nodes with global index strictly inside 1 .. N p - 1 along every axis:
    # all their cells see the same (unwrapped) positions
    idx = np.arange(d.m)
    gc = [idx % d.M[0], (idx // d.M[0]) % d.M[1], idx // (d.M[0] * d.M[1])]
    inner = np.all([(gc[k] > 0) for k in range(3)], axis=0)
    assert inner.sum() > 0
    assert np.abs(r[inner]).max() < 1e-11 * np.abs(Te).max() * np.abs(ue).max()
    # and a physical quadratic is not in the kernel (the test can fail)
    ue2 = (d.node_points(cells) @ g) ** 2
    r2 = np.zeros(d.m)
    np.add.at(r2, d.cell_dofs().reshape(-1), np.einsum("cij,cj->ci", Te, ue2).reshape(-1))
    assert np.abs(r2[inner]).max() > 1e-3


def test_hermitian_and_bloch_antisymmetry():
    k = (0.25, -0.2, 0.15)
    d, _ = _pair(0.12, p=3, k=k)
    rng = np.random.default_rng(2)
    nq = d.E * d.nq ** 3
    H = dm.assemble_H(d, rng.standard_normal(nq), rng.standard_normal((nq, 3))).toarray()
    assert np.abs(H - H.conj().T).max() < 1e-12 * np.abs(H).max()
    H0 = dm.assemble_H(dm.DistortedMesh(LAT, d.N, 3, 4, d.vdisp), np.zeros(nq)).toarray()
    Hk = dm.assemble_H(d, np.zeros(nq)).toarray()
    K = (Hk - H0 - 0.5 * float(np.dot(k, k)) * dm.assemble_M(d).toarray()) * 1j
    assert np.abs(K.imag).max() < 1e-12 and np.abs(K + K.T).max() < 1e-12
    assert np.abs(K @ np.ones(d.m)).max() < 1e-12
