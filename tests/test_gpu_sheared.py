"""General parallelepiped boxes (off-diagonal J, one affine map per cell).

The kinetic metric 1/2 J^-1 J^-T then has off-diagonal entries: the kernel
stages the three reference gradients of a cell in LDS and adds the coupling
terms to each direction's flux.  Checked against the oracle's assembled
operator (direct, not collocation, derivatives on the same mesh): FP64 H X
to 1e-12 for real and complex fields, both quadrature rules and a Dirichlet
axis, a brute-force H I, FP32 close to FP64, batched = separate bit for bit,
and the ChFSI driver converging to eigh(H, D).
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
SHEARED = np.array([[6.0, 0.0, 0.0], [1.5, 5.0, 0.0], [0.7, -0.9, 7.0]])


def _case(k=(0, 0, 0), p=3, nq=None, periodic=(True, True, True), N=(3, 4, 3), natoms=2, pset="spd", nvec=6,
          seed=71):
    A = SHEARED.copy()
    if not periodic[2]:
        A[2] = [0.0, 0.0, 7.0]
    s = inputs.make_custom(A, N, p, p + 1 if nq is None else nq, kpoint=k, nvec=nvec, seed=seed, natoms=natoms,
                           pset=pset, rc=2.0)
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, periodic=periodic)
    idx = om.dirichlet_dofs()
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors) if s.projectors else (None, None)
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0, periodic=periodic)
    m.set_potential(vl, vg)
    if s.projectors:
        m.set_projectors(inputs.positions_array(s), s.projectors)
    H = op.assemble_H(om, vl, vg)[idx][:, idx]
    return s, om, idx, m, H, (P[idx] if P is not None else None), h


def _apply(m, X, prec="f64"):
    Xd = to_dev(X)
    if prec == "f32":
        Xd = Xd.to(torch.complex64 if Xd.is_complex() else torch.float32)
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, prec)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("k,p,nq,periodic", [
    ((0, 0, 0), 3, None, (True, True, True)), ((0.3, -0.2, 0.1), 4, None, (True, True, True)),
    ((0.2, 0.1, 0.3), 3, 6, (True, True, True)), ((0.2, 0.1, 0.0), 3, None, (True, True, False)),
    ((0.0, 0.0, 0.0), 6, None, (True, True, True))])
def test_sheared_hx_matches_oracle(k, p, nq, periodic):
    s, om, idx, m, H, Pr, h = _case(k, p, nq, periodic, N=(3, 2, 3) if p > 5 else (3, 4, 3))
    X = inputs.make_vectors(s, ndofs=len(idx))
    want = op.apply_sparse(H, X, Pr, h)
    assert rel(_apply(m, X), want) < TOL


def test_sheared_brute_force_fp32_and_batch():
    s, om, idx, m, H, Pr, h = _case((0.25, 0.1, -0.2), 2, None, N=(2, 3, 2), natoms=1, pset="sp")
    Hd = H.toarray() + op.nonlocal_dense(Pr, h)
    assert rel(_apply(m, np.eye(len(idx), dtype=complex)), Hd) < TOL
    X = inputs.make_vectors(s, ndofs=len(idx))
    y64 = _apply(m, X)
    assert rel(_apply(m, X, "f32"), y64) < 2e-5
    # a sheared and an orthorhombic system of one class in one batched launch
    s2 = inputs.make_custom(np.diag([5.0, 6.0, 5.5]), (2, 3, 2), 2, 3, kpoint=(0.1, 0.2, 0.0), nvec=6, seed=72)
    m2 = fehx.Mesh(s2.lattice, s2.ncell, s2.degree, s2.nq, s2.kpoint, device=0)
    pts2 = m2.quad_points()
    m2.set_potential(inputs.eval_vloc(s2, pts2), inputs.eval_vgga(s2, pts2))
    X2 = inputs.make_vectors(s2)
    Xs = [to_dev(X), to_dev(X2)]
    Ys = [torch.full_like(x, 4.0) for x in Xs]
    fehx.batch_apply([m, m2], Xs, Ys)
    torch.cuda.synchronize()
    assert np.array_equal(Ys[0].cpu().numpy(), y64)
    assert np.array_equal(Ys[1].cpu().numpy(), _apply(m2, X2))


def test_sheared_chfsi_converges():
    s, om, idx, m, H, Pr, h = _case((0, 0, 0), 3, None, N=(3, 3, 3), natoms=1, pset="sp", nvec=8)
    Dr = op.lumped_mass(om)[idx]
    X0 = inputs.make_vectors(s, ndofs=len(idx))
    v0 = inputs.lanczos_start(s, ndofs=len(idx))
    lam, _ = m.chfsi(to_dev(X0), to_dev(v0), outer=12, degree=20, inner="f64")
    Hd = H.toarray() + op.nonlocal_dense(Pr, h)
    want = sla.eigvalsh(Hd, np.diag(Dr))[:5]
    assert np.abs(lam[:5] - want).max() < 1e-8
