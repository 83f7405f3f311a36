"""Distorted (non-affine) hexahedral cells (oracle; test infrastructure).

Sec. 3.1 / eqn cellIntegrals with the Jacobian evaluated at every quadrature
point: the cells of a periodic box whose vertices are displaced.  Each cell is
the trilinear image of the reference cube [-1, 1]^3 through its eight corner
vertices, so J(xi) = dx/dxi varies inside the cell and every cell integral
becomes sum_Q (.) w_Q det J(xi_Q), with physical gradients J(xi_Q)^-T grad_xi.
The FE space is the same tensor-product GLL basis in the reference
coordinates; the map is the Q1 (trilinear) one.

Conventions: vertex (i, j, k) of the N0 x N1 x N2 periodic vertex grid sits
at (i/N0) a_0 + (j/N1) a_1 + (k/N2) a_2 + vdisp[i + N0 (j + N1 k)]; corner
(a, b, c) in {0, 1}^3 of cell (c0, c1, c2) is vertex (c0 + a, c1 + b, c2 + c)
taken modulo the grid (its unwrapped lattice position plus the displacement of
the wrapped vertex), corner index a + 2 b + 4 c.

Everything below restates the integrals of oracle.operator (eqn Hloc /
HlocIntegral, eqn Vnonloc) with per-point geometry, written out directly: no
sum factorisation, direct derivatives of the Lagrange basis.

Pins (tests/test_oracle_distorted.py): zero displacement reproduces the affine
oracle; cell volumes equal a 4-point Gauss integral of det J and sum to the
box volume, as do the consistent and the lumped mass; T 1 = 0; the
element-level patch test (a physical linear function gives zero kinetic rows
at every node, since int grad N_I = 0 around an interior node); K
antisymmetric and H Hermitian.
"""
import numpy as np
import scipy.sparse as sp

from .basis import gauss_points_weights, lagrange_derivatives, lagrange_values
from .mesh import Mesh
from .projectors import bloch_chi

CORNERS = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)])   # index a + 2b + 4c


def trilinear(xi):
    """phi[n, 8] and dphi[n, 8, 3] of the eight corner shape functions at xi [n, 3]."""
    xi = np.atleast_2d(xi)
    s = 2.0 * CORNERS - 1.0                                   # corner signs
    f = 0.5 * (1.0 + xi[:, None, :] * s[None, :, :])          # [n, 8, 3] per-axis factors
    phi = np.prod(f, axis=2)
    dphi = np.empty(f.shape)
    for d in range(3):
        others = [e for e in range(3) if e != d]
        dphi[:, :, d] = 0.5 * s[None, :, d] * f[:, :, others[0]] * f[:, :, others[1]]
    return phi, dphi


class DistortedMesh(Mesh):
    """Periodic mesh whose cell vertices are displaced by vdisp [N0 N1 N2, 3]."""

    distorted = True

    def __init__(self, lattice, ncell, degree, nq, vdisp, kpoint=(0.0, 0.0, 0.0)):
        super().__init__(lattice, ncell, degree, nq, kpoint)
        self.vdisp = np.asarray(vdisp, float).reshape(int(np.prod(self.N)), 3)

    def corners(self, cells):
        """Corner positions [nc, 8, 3] of the given cells."""
        cc = self.cell_coords(np.atleast_1d(cells))
        out = np.empty((len(cc), 8, 3))
        for ci, off in enumerate(CORNERS):
            g = cc + off[None, :]
            x = (g / self.N[None, :]) @ self.A
            v = (g[:, 0] % self.N[0]) + self.N[0] * ((g[:, 1] % self.N[1]) + self.N[1] * (g[:, 2] % self.N[2]))
            out[:, ci] = x + self.vdisp[v]
        return out

    def geometry(self, cells, xi):
        """Physical points x [nc, n, 3] and Jacobians J [nc, n, 3, 3]
        (J[..., a, d] = dx_a / dxi_d) at reference points xi [n, 3]."""
        X = self.corners(cells)
        phi, dphi = trilinear(xi)
        return np.einsum("np,cpa->cna", phi, X), np.einsum("npd,cpa->cnad", dphi, X)

    def ref_quad(self):
        """Reference quadrature points [n_q^3, 3] (Q = q1 + n_q (q2 + n_q q3)) and weights."""
        q, w = self.xq, self.wq
        ref = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
        W = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
        return ref, W

    def quad_points(self):
        ref, _ = self.ref_quad()
        x, _ = self.geometry(np.arange(self.E), ref)
        return x.reshape(-1, 3)

    def node_points(self, cells):
        """Physical positions of the cells' nodes [nc, n_p^3, 3] (I = i + n_p (j + n_p k))."""
        g = self.gll
        ref = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
        return self.geometry(cells, ref)[0]


def cell_point_tables(mesh, cells):
    """N3 [Q, I], physical gradients dN [nc, a, Q, I], weights W [nc, Q] = w_Q det J(xi_Q)."""
    N1 = lagrange_values(mesh.gll, mesh.xq)
    D1 = lagrange_derivatives(mesh.gll, mesh.xq)
    nq, npp = mesh.nq, mesh.np_

    def kron3(a, b, c):
        return np.einsum("ai,bj,ck->cbakji", a, b, c).reshape(nq ** 3, npp ** 3)

    N3 = kron3(N1, N1, N1)
    dref = np.stack([kron3(D1, N1, N1), kron3(N1, D1, N1), kron3(N1, N1, D1)])
    ref, wref = mesh.ref_quad()
    _, J = mesh.geometry(cells, ref)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                                   # [nc, Q, d, a]
    dN = np.einsum("cqda,dqi->caqi", Jinv, dref)
    return N3, dN, wref[None, :] * det


def element_matrices(mesh, vloc, vgga=None, cells=None):
    """H^(e) = T + L + G - i K for the given cells with per-point geometry."""
    cells = np.arange(mesh.E) if cells is None else np.atleast_1d(cells)
    N3, dN, W = cell_point_tables(mesh, cells)
    nq3 = mesh.nq ** 3
    VL = np.asarray(vloc, float).reshape(mesh.E, nq3)[cells] + 0.5 * float(mesh.k @ mesh.k)
    T = 0.5 * sum(np.matmul(dN[:, a].transpose(0, 2, 1) * W[:, None, :], dN[:, a]) for a in range(3))
    He = T + np.matmul(N3.T[None, :, :] * (VL * W)[:, None, :], N3)
    if vgga is not None:
        VG = np.asarray(vgga, float).reshape(mesh.E, nq3, 3)[cells] * W[:, :, None]
        g = sum(np.matmul(dN[:, a].transpose(0, 2, 1) * VG[:, None, :, a], N3) for a in range(3))
        He = He + g + g.transpose(0, 2, 1)
    if np.any(mesh.k != 0.0):
        K = sum(mesh.k[a] * np.matmul((N3.T[None, :, :] * W[:, None, :]), dN[:, a]) for a in range(3))
        He = He - 1j * K
    return He


def mass_elements(mesh, cells=None):
    cells = np.arange(mesh.E) if cells is None else np.atleast_1d(cells)
    N3, _, W = cell_point_tables(mesh, cells)
    return np.matmul(N3.T[None, :, :] * W[:, None, :], N3)


def assemble(mesh, blocks):
    dofs = mesh.cell_dofs()
    npp3 = mesh.np_ ** 3
    rows = np.repeat(dofs, npp3, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, npp3)).reshape(-1)
    return sp.coo_matrix((blocks.reshape(-1), (rows, cols)), shape=(mesh.m, mesh.m)).tocsr()


def assemble_H(mesh, vloc, vgga=None):
    return assemble(mesh, element_matrices(mesh, vloc, vgga))


def assemble_M(mesh):
    return assemble(mesh, mass_elements(mesh))


def lumped_mass(mesh):
    """D_II = sum over cells containing I of w^GLL_i w^GLL_j w^GLL_k det J(node I)."""
    g = mesh.gll
    ref = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    w = mesh.gllw
    wl = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
    _, J = mesh.geometry(np.arange(mesh.E), ref)
    D = np.zeros(mesh.m)
    np.add.at(D, mesh.cell_dofs().reshape(-1), (wl[None, :] * np.linalg.det(J)).reshape(-1))
    return D


def cell_volumes(mesh, n=4):
    """int over each cell of det J, by an n-point Gauss rule per axis."""
    x, w = gauss_points_weights(n)
    ref = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
    _, J = mesh.geometry(np.arange(mesh.E), ref)
    return np.linalg.det(J) @ W


def projector_matrix(mesh, positions, projectors):
    """Sparse P (m x n_s) of eqn Vnonloc on the distorted cells (every cell
    integrated; the integrand vanishes outside the projector supports)."""
    N3, _, W = cell_point_tables(mesh, np.arange(mesh.E))
    ref, _ = mesh.ref_quad()
    pts, _ = mesh.geometry(np.arange(mesh.E), ref)
    dtype = complex if np.any(mesh.k != 0.0) else float
    pos = np.asarray(positions, float).reshape(-1, 3)
    dofs = mesh.cell_dofs().reshape(-1)
    rows, cols, vals, h = [], [], [], np.zeros(len(projectors))
    for s, pr in enumerate(projectors):
        chi = bloch_chi(pr["l"], pr["m"], pts, pos[pr["atom"]], mesh.A, mesh.k, pr["sigma"], pr["rc"], 1,
                        mesh.periodic)
        cellcols = np.einsum("cq,qi->ci", chi * W, N3).reshape(-1)
        keep = cellcols != 0
        rows.append(dofs[keep])
        cols.append(np.full(int(keep.sum()), s))
        vals.append(cellcols[keep].astype(dtype))
        h[s] = pr["h"]
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.m, len(projectors))).tocsr()
    return P, h
