"""The FE-discretised Kohn-Sham operator by its definition (oracle; test infrastructure).

Eqn Hloc / HlocIntegral (Sec. 2.2, 3.1):
    T_IJ = 1/2 int grad N_I . grad N_J
    L_IJ = int V^L N_I N_J,         V^L = V_eff + |k|^2 / 2   (eqn Vloc)
    G_IJ = int V^G . (grad N_I N_J + N_I grad N_J)
    K_IJ = int k . (N_I grad N_J)
    H_loc = T + L + G - i K,        M_IJ = int N_I N_J
Eqn cellIntegrals: every integral becomes sum_Q (.) w_Q det J on the n_q^3
Gauss rule of each cell.  Eqn HX: the global matrix is sum_e Q^(e)T H^(e) Q^(e)
(with the periodic wrap as the constraint).  Eqn Vnonloc:
    H_nloc = sum_a sum_s F_s h_s F_s^*,
    F_{I,s} = int sum_r exp(-i k.(x - L_r)) chi_s(x, R_a + L_r) N_I(x) dx.
Sec. 5.3 (R-ChFSI): D is the diagonal mass from the GLL rule on the nodes.

Here the cell matrices are built by explicit 3D quadrature with the 3D shape
functions and their direct physical gradients J^-T grad_xi N: no sum
factorisation and no collocation derivative (those are what the library
does).  Three ways to apply H: assembled sparse product, the cell-matrix (CM)
route of the paper's baseline (dense H^(e) per cell, gather / multiply /
scatter), and single rows (for sampling outputs of meshes too large to
assemble).

Pins (tests/test_oracle_operator.py, test_oracle_nonlocal.py): polynomial
exactness of T, M, L, G, K on single cells against closed-form integrals,
mass sums, T 1 = 0 and K antisymmetry on periodic meshes, constant V^G giving
G = 0, free-electron spectra that are exact Kronecker sums of 1D spectra and
converge to |k + G|^2 / 2, Hermiticity, the three application routes agreeing.
"""
import numpy as np
import scipy.sparse as sp

from .basis import lagrange_values, lagrange_derivatives
from .projectors import bloch_chi


# --- 3D tables on one cell --------------------------------------------------
def cell_tables(mesh):
    """N3[Q, I], physical gradients dN[a, Q, I], and weights W[Q] = w_Q det J."""
    N1 = lagrange_values(mesh.gll, mesh.xq)          # [nq, np]
    D1 = lagrange_derivatives(mesh.gll, mesh.xq)     # [nq, np]
    nq, npp = mesh.nq, mesh.np_

    def kron3(a, b, c):   # a along xi_0 (q1, i), b along xi_1, c along xi_2
        return np.einsum("ai,bj,ck->cbakji", a, b, c).reshape(nq ** 3, npp ** 3)

    N3 = kron3(N1, N1, N1)
    dref = np.stack([kron3(D1, N1, N1), kron3(N1, D1, N1), kron3(N1, N1, D1)])
    # grad_x = J^-T grad_xi :  (grad_x N)_a = sum_d Jinv[d, a] d/dxi_d N
    dphys = np.einsum("da,dqi->aqi", mesh.Jinv, dref)
    return N3, dphys, mesh.quad_weights()


def _is_complex(mesh):
    return bool(np.any(mesh.k != 0.0))


def element_matrices(mesh, vloc, vgga=None, cells=None, tables=None):
    """H^(e) for the requested cells (all if None): [nc, n_p^3, n_p^3].

    vloc: V_eff at all quadrature points [E n_q^3] (|k|^2/2 added here);
    vgga: the GGA vector field V^G at all quadrature points [E n_q^3, 3] or None.
    """
    N3, dN, W = tables if tables is not None else cell_tables(mesh)
    nq3 = mesh.nq ** 3
    if cells is None:
        cells = np.arange(mesh.E)
    cells = np.atleast_1d(cells)
    VL = np.asarray(vloc, float).reshape(mesh.E, nq3)[cells] + 0.5 * float(mesh.k @ mesh.k)
    T = 0.5 * sum((dN[a] * W[:, None]).T @ dN[a] for a in range(3))
    He = T[None, :, :] + np.matmul(N3.T[None, :, :] * (VL * W[None, :])[:, None, :], N3)
    if vgga is not None:
        VG = np.asarray(vgga, float).reshape(mesh.E, nq3, 3)[cells] * W[None, :, None]
        g = sum(np.matmul(dN[a].T[None, :, :] * VG[:, None, :, a], N3) for a in range(3))
        He = He + g + g.transpose(0, 2, 1)
    if _is_complex(mesh):
        K = sum(mesh.k[a] * ((N3 * W[:, None]).T @ dN[a]) for a in range(3))
        He = He - 1j * K[None, :, :]
    return He


def element_rows(mesh, vloc, vgga, cells, locs, tables=None):
    """Row ``locs[n]`` of H^(e) for cell ``cells[n]``: [n, n_p^3] (same integrals)."""
    N3, dN, W = tables if tables is not None else cell_tables(mesh)
    nq3 = mesh.nq ** 3
    cells = np.atleast_1d(cells)
    locs = np.atleast_1d(locs)
    VL = np.asarray(vloc, float).reshape(mesh.E, nq3)[cells] + 0.5 * float(mesh.k @ mesh.k)
    nI = N3[:, locs].T * W[None, :]                      # N_I(x_Q) w_Q det J  [n, nq3]
    dI = [dN[a][:, locs].T * W[None, :] for a in range(3)]
    rows = 0.5 * sum(dI[a] @ dN[a] for a in range(3)) + (nI * VL) @ N3
    if vgga is not None:
        VG = np.asarray(vgga, float).reshape(mesh.E, nq3, 3)[cells]
        for a in range(3):
            rows = rows + (dI[a] * VG[:, :, a]) @ N3 + (nI * VG[:, :, a]) @ dN[a]
    if _is_complex(mesh):
        rows = rows - 1j * sum(mesh.k[a] * (nI @ dN[a]) for a in range(3))
    return rows


def mass_element(mesh, tables=None):
    N3, _, W = tables if tables is not None else cell_tables(mesh)
    return (N3 * W[:, None]).T @ N3


def _assemble(mesh, blocks):
    dofs = mesh.cell_dofs()
    npp3 = mesh.np_ ** 3
    rows = np.repeat(dofs, npp3, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, npp3)).reshape(-1)
    if blocks.ndim == 2:
        blocks = np.broadcast_to(blocks, (mesh.E,) + blocks.shape)
    return sp.coo_matrix((blocks.reshape(-1), (rows, cols)),
                         shape=(mesh.m, mesh.m)).tocsr()


def assemble_H(mesh, vloc, vgga=None):
    """Global H_loc = sum_e Q^T H^(e) Q as CSR (duplicates summed)."""
    return _assemble(mesh, element_matrices(mesh, vloc, vgga))


def assemble_M(mesh):
    return _assemble(mesh, mass_element(mesh))


def lumped_mass(mesh):
    """D_II = sum over cells containing I of w^GLL_i w^GLL_j w^GLL_k det J."""
    w = mesh.gllw
    dloc = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1) * mesh.detJ
    D = np.zeros(mesh.m)
    np.add.at(D, mesh.cell_dofs().reshape(-1), np.tile(dloc, mesh.E))
    return D


# --- nonlocal ----------------------------------------------------------------
def support_cells(mesh, R, rc, images=1):
    """Cells whose bounding sphere meets a ball of radius rc around any image of R."""
    centres = mesh.cell_origin(np.arange(mesh.E)) + mesh.J @ np.ones(3)
    # circumradius of the cell: the longest of |J s| over corner sign patterns s
    radius = max(np.linalg.norm(mesh.J @ np.array(s, float))
                 for s in ((1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1)))
    keep = np.zeros(mesh.E, bool)
    rr = [np.arange(-images, images + 1) if mesh.periodic[d] else np.zeros(1, int) for d in range(3)]
    for r in np.array(np.meshgrid(*rr)).T.reshape(-1, 3):
        d = np.linalg.norm(centres - (R + r @ mesh.A), axis=1)
        keep |= d < rc + radius + 1e-9
    return np.nonzero(keep)[0]


def projector_matrix(mesh, positions, projectors, tables=None, images=1):
    """Sparse P (m x n_s) with P[:, s] = F_{., s} of eqn Vnonloc, and h[s].

    ``projectors`` is a sequence of dicts with keys atom, l, m, sigma, rc, h.
    Only cells that can meet the support of the projector are integrated
    (outside them the integrand is identically zero).
    """
    N3, _, W = tables if tables is not None else cell_tables(mesh)
    ns = len(projectors)
    dtype = complex if _is_complex(mesh) else float
    pos = np.asarray(positions, float).reshape(-1, 3)
    rows, cols, vals_all = [], [], []
    h = np.zeros(ns)
    for s, pr in enumerate(projectors):
        R = pos[pr["atom"]]
        cells = support_cells(mesh, R, pr["rc"], images)
        pts = quad_points_of(mesh, cells)                                  # [nc, nq3, 3]
        vals = bloch_chi(pr["l"], pr["m"], pts, R, mesh.A, mesh.k, pr["sigma"], pr["rc"], images, mesh.periodic)
        cellcols = (vals * W[None, :]) @ N3                                # [nc, np3]
        rows.append(mesh.cell_dofs(cells).reshape(-1))
        cols.append(np.full(cellcols.size, s))
        vals_all.append(cellcols.reshape(-1).astype(dtype))
        h[s] = pr["h"]
    if ns == 0:
        return sp.csr_matrix((mesh.m, 0), dtype=dtype), h
    P = sp.coo_matrix((np.concatenate(vals_all), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.m, ns)).tocsr()
    P.eliminate_zeros()
    return P, h


def quad_points_of(mesh, cells):
    """Physical quadrature points of the given cells: [nc, n_q^3, 3]."""
    q = mesh.xq
    ref = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    return mesh.cell_origin(np.atleast_1d(cells))[:, None, :] + (ref + 1.0) @ mesh.J.T


def nonlocal_dense(P, h):
    Pd = P.toarray() if sp.issparse(P) else P
    return (Pd * h[None, :]) @ Pd.conj().T


# --- applications of H -------------------------------------------------------
def apply_sparse(Hloc, X, P=None, h=None):
    """Y = H_loc X + P diag(h) P^H X (assembled sparse route)."""
    Y = Hloc @ X
    if P is not None and P.shape[1]:
        Y = Y + P @ (h[:, None] * (P.conj().T @ X))
    return Y


def apply_cm(mesh, vloc, vgga, X, P=None, h=None, cells=None, He=None):
    """Cell-matrix route: Y = sum_e Q^T (H^(e) (Q X)) (+ nonlocal if P given).

    With ``cells`` only those cells' local contributions are summed (the
    nonlocal term is then left out).
    """
    if cells is None:
        cells = np.arange(mesh.E)
    cells = np.atleast_1d(cells)
    if He is None:
        He = element_matrices(mesh, vloc, vgga, cells)
    dofs = mesh.cell_dofs(cells)
    Xe = X[dofs]                                  # [nc, np3, nv]
    Ye = He @ Xe
    Y = np.zeros(X.shape, dtype=np.result_type(He, X))
    np.add.at(Y, dofs.reshape(-1), Ye.reshape(-1, X.shape[1]))
    if P is not None and P.shape[1] and len(cells) == mesh.E:
        Y = Y + P @ (h[:, None] * (P.conj().T @ X))
    return Y


def cm_operator(mesh, vloc, vgga, P=None, h=None, batch=512):
    """The cell-matrix route as an operator on blocks, for meshes whose full
    gathered block does not fit in memory: the same Y = sum_e Q^T (H^(e) (Q X))
    (+ P diag(h) P^H X) as apply_cm, taken over batches of cells.  Q^T is a
    sparse 0/1 matrix (one entry per (cell, local node)), so the scatter-add
    is a sparse product.  H^(e) of every cell is built once, here."""
    He = element_matrices(mesh, vloc, vgga)
    dofs = mesh.cell_dofs()
    npp3 = dofs.shape[1]
    rows_all = dofs.reshape(-1)
    Qt = sp.csr_matrix((np.ones(rows_all.size), (rows_all, np.arange(rows_all.size))),
                       shape=(mesh.m, rows_all.size))

    def Hop(X):
        X = np.asarray(X)
        Y = np.zeros(X.shape, dtype=np.result_type(He, X))
        for c0 in range(0, mesh.E, batch):
            c1 = min(c0 + batch, mesh.E)
            Ye = He[c0:c1] @ X[dofs[c0:c1]]                         # [nc, np3, nv]
            Y += Qt[:, c0 * npp3:c1 * npp3] @ Ye.reshape(-1, X.shape[1])
        if P is not None and P.shape[1]:
            Y += P @ (h[:, None] * (P.conj().T @ X))
        return Y

    return Hop


def apply_rows(mesh, vloc, vgga, X, rows, P=None, h=None, tables=None):
    """(H X)[rows, :] from the rows of the cell matrices that touch each node."""
    tables = tables if tables is not None else cell_tables(mesh)
    rows = np.atleast_1d(rows)
    cplx = _is_complex(mesh) or np.iscomplexobj(X)
    out = np.zeros((len(rows), X.shape[1]), dtype=complex if cplx else float)
    for r, dof in enumerate(rows):
        pairs = mesh.node_cells(int(dof))
        cells = np.array([c for c, _ in pairs])
        locs = np.array([i for _, i in pairs])
        hrows = element_rows(mesh, vloc, vgga, cells, locs, tables)   # [nc, np3]
        dofs = mesh.cell_dofs(cells)
        out[r] = np.einsum("cj,cjv->v", hrows, X[dofs])
    if P is not None and P.shape[1]:
        out = out + P[rows] @ (h[:, None] * (P.conj().T @ X))
    return out
