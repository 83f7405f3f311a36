"""Dirichlet (non- and semi-periodic) axes on the GPU.

With homogeneous Dirichlet faces the discrete operator is the open mesh's
operator restricted to the nodes off those faces (the oracle's
``dirichlet_dofs``); the library numbers exactly those nodes.  Checked:
H X (local + projectors, real and complex, both quadrature rules, odd cell
counts) to 1e-12 relative, a brute-force H I, the consistent mass M X, and
the ChFSI driver converging to eigh(H, D) of the restricted matrices.
"""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")
from oracle import operator as op  # noqa: E402
from oracle.mesh import Mesh as OMesh  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _case(periodic, N=(3, 4, 3), p=3, nq=None, natoms=2, pset="spd", nvec=6, seed=61, kscale=0.2):
    k = tuple(kscale * (d + 1) if periodic[d] else 0.0 for d in range(3))
    s = inputs.make_custom(np.diag([7.5, 8.0, 7.0]), N, p, p + 1 if nq is None else nq, kpoint=k, nvec=nvec,
                           seed=seed, natoms=natoms, pset=pset, rc=3.0)
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, periodic=periodic)
    idx = om.dirichlet_dofs()
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors) if s.projectors else (None, None)
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0, periodic=periodic)
    m.set_potential(vl, vg)
    if s.projectors:
        m.set_projectors(inputs.positions_array(s), s.projectors)
    assert m.ndofs == len(idx)
    H = op.assemble_H(om, vl, vg)[idx][:, idx]
    Pr = P[idx] if P is not None else None
    return s, om, idx, m, H, Pr, h


def _apply(m, X, prec="f64"):
    Xd = to_dev(X)
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, prec)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("periodic,p,nq,kscale", [
    ((False, False, False), 3, None, 0.0), ((True, True, False), 3, None, 0.2), ((True, False, True), 5, None, 0.1),
    ((False, True, False), 4, None, 0.3), ((True, True, False), 3, 6, 0.2), ((False, False, False), 2, 5, 0.0)])
def test_dirichlet_hx_matches_restricted_oracle(periodic, p, nq, kscale):
    s, om, idx, m, H, Pr, h = _case(periodic, p=p, nq=nq, kscale=kscale)
    X = inputs.make_vectors(s, ndofs=len(idx))
    want = op.apply_sparse(H, X, Pr, h)
    assert rel(_apply(m, X), want) < TOL


def test_dirichlet_odd_cells_brute_force_and_mass():
    s, om, idx, m, H, Pr, h = _case((False, True, False), N=(3, 5, 3), p=2, natoms=1, pset="sp", kscale=0.15)
    Hd = H.toarray() + (op.nonlocal_dense(Pr, h) if Pr is not None else 0)
    I = np.eye(len(idx), dtype=complex if s.is_complex else float)
    assert rel(_apply(m, I), Hd) < TOL
    M = op.assemble_M(om)[idx][:, idx]
    X = inputs.make_vectors(s, ndofs=len(idx))
    Xd = to_dev(X)
    Yd = torch.empty_like(Xd)
    m.apply_mass(Xd, Yd)
    torch.cuda.synchronize()
    assert rel(Yd.cpu().numpy(), M @ X) < TOL


def test_dirichlet_chfsi_converges_to_restricted_eigenproblem():
    s, om, idx, m, H, Pr, h = _case((True, True, False), N=(3, 3, 3), p=3, natoms=1, pset="sp", nvec=8,
                                    kscale=0.0)
    Dr = op.lumped_mass(om)[idx]
    assert np.abs(m.lumped_mass() - Dr).max() < 1e-14 * Dr.max()
    X0 = inputs.make_vectors(s, ndofs=len(idx))
    v0 = inputs.lanczos_start(s, ndofs=len(idx))
    lam, _ = m.chfsi(to_dev(X0), to_dev(v0), outer=12, degree=20, inner="f64")
    Hd = H.toarray() + (op.nonlocal_dense(Pr, h) if Pr is not None else 0)
    want = sla.eigvalsh(Hd, np.diag(Dr))[:5]
    assert np.abs(lam[:5] - want).max() < 1e-8
