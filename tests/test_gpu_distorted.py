"""Distorted (trilinear, non-affine) cells on the GPU against the oracle with a
Jacobian per quadrature point (oracle.distorted): H X in FP64 to 1e-12 and
FP32 to 2e-5 for several (p, n_q, k, GGA, projector) cases on a sheared
lattice with a seeded periodic vertex displacement; M X; and the converged
FP64 eigensolver against scipy's eigh(H, D) of the oracle's matrices."""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")
from oracle import distorted as dm  # noqa: E402
from oracle import eigen  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu
LAT = np.array([[7.0, 0.0, 0.0], [0.6, 7.5, 0.0], [0.3, -0.4, 8.0]])


def _case(p, nq, k, natoms, pset, N=(3, 3, 4), amp=0.15, seed=5, nvec=6):
    s = inputs.make_custom(LAT, N, p, nq, kpoint=k, nvec=nvec, seed=seed, natoms=natoms, pset=pset, rc=2.5)
    vd = inputs.vertex_displacement(N, LAT, amp, seed + 100)
    om = dm.DistortedMesh(LAT, N, p, nq, vd, kpoint=k)
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    m = fehx.Mesh(LAT, N, p, nq, k, device=0)
    m.set_geometry(vd)
    assert np.abs(m.quad_points() - pts).max() < 1e-12
    m.set_potential(vl, vg)
    P = h = None
    if natoms:
        P, h = dm.projector_matrix(om, inputs.positions_array(s), s.projectors)
        m.set_projectors(inputs.positions_array(s), s.projectors)
    H = dm.assemble_H(om, vl, vg)
    return s, om, m, H, P, h


def _hx(H, P, h, X):
    Y = H @ X
    if P is not None:
        Y = Y + P @ (h[:, None] * (P.conj().T @ X))
    return Y


@pytest.mark.parametrize("p,dq,k,natoms,pset", [(2, 1, (0, 0, 0), 0, "s"), (3, 1, (0.25, -0.1, 0.2), 2, "sp"),
                                                (4, 1, (0, 0, 0), 1, "spd"), (3, 3, (0.1, 0.2, -0.15), 1, "sp"),
                                                (5, 1, (0.2, 0.0, 0.1), 1, "sp")])
def test_distorted_hx(p, dq, k, natoms, pset):
    s, om, m, H, P, h = _case(p, p + dq, k, natoms, pset)
    X = inputs.make_vectors(s)
    want = _hx(H, P, h, X)
    Xd = to_dev(X)
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, "f64")
    torch.cuda.synchronize()
    assert rel(Yd.cpu().numpy(), want) < 1e-12
    dt = torch.complex64 if np.iscomplexobj(X) else torch.float32
    X32 = Xd.to(dt)
    Y32 = torch.empty_like(X32)
    m.apply(X32, Y32, "f32")
    torch.cuda.synchronize()
    assert rel(Y32.cpu().numpy().astype(X.dtype), want) < 2e-5
    # the consistent mass matrix with the same per-point weights
    Md = torch.empty_like(Xd)
    m.apply_mass(Xd, Md, "f64")
    torch.cuda.synchronize()
    assert rel(Md.cpu().numpy(), dm.assemble_M(om) @ X) < 1e-12
    assert np.abs(m.lumped_mass() - dm.lumped_mass(om)).max() < 1e-13 * dm.lumped_mass(om).max()


def test_distorted_eigensolver_converges_to_eigh():
    s, om, m, H, P, h = _case(3, 4, (0.0, 0.0, 0.0), 1, "sp", N=(3, 3, 3), nvec=8)
    Dv = dm.lumped_mass(om)
    Hd = H.toarray() + (P @ (h[:, None] * P.conj().T.toarray()))
    want = sla.eigh(0.5 * (Hd + Hd.conj().T), np.diag(Dv), eigvals_only=True)[:6]
    X = to_dev(inputs.make_vectors(s))
    lam, _ = m.chfsi(X, to_dev(inputs.lanczos_start(s)), outer=12, degree=20, inner="f64")
    assert np.abs(lam[:6] - want).max() < 1e-8
    # and the oracle's own driver agrees on the same procedure
    lam_o, _, _ = eigen.chfsi(lambda V: _hx(H, P, h, V), Dv, inputs.make_vectors(s), inputs.lanczos_start(s),
                              om.volume, outer=12, degree=20)
    assert np.abs(lam - lam_o).max() < 1e-8
