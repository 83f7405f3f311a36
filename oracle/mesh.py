"""Structured hexahedral mesh of a parallelepiped box (oracle; test infrastructure).

Sec. 3.1: the domain is split into E hexahedral cells; every cell is an affine
image of the reference cube [-1, 1]^3 (meshes made by subdividing a
parallelepiped), so the Jacobian J and det J are constant per cell.

Conventions (shared with the library only through its documented C-ABI, not
through code):
  * ``lattice`` rows are the box vectors a_0, a_1, a_2 (bohr).
  * cell (c0, c1, c2), flat id c = c0 + N0 (c1 + N1 c2).
  * reference -> physical:  x = x_c + J (xi + 1),  J[:, d] = a_d / (2 N_d),
    x_c = sum_d (c_d / N_d) a_d.
  * local node (i, j, k), i along xi_0, flat I = i + n_p (j + n_p k).
  * global node index along axis d: g_d = c_d p + i_d, wrapped mod N_d p when
    the axis is periodic (the wrap *is* the periodic constraint C of eqn HX);
    an open axis has N_d p + 1 nodes.  DoF id = g_0 + M_0 (g_1 + M_1 g_2).
  * quadrature point (q1, q2, q3), flat Q = q1 + n_q (q2 + n_q q3); the
    global point list is cell-major: index c n_q^3 + Q.

Pins (tests/test_oracle_mesh.py): brute-force node coordinates (nodes shared by
neighbouring cells coincide physically), multiplicity counts 1/2/4/8 and the
unique-DoF count, cell volumes summing to |det A|.
"""
import numpy as np

from .basis import gll_nodes_weights, gauss_points_weights


class Mesh:
    def __init__(self, lattice, ncell, degree, nq, kpoint=(0.0, 0.0, 0.0),
                 periodic=(True, True, True)):
        self.A = np.asarray(lattice, dtype=float).reshape(3, 3)
        self.N = np.asarray(ncell, dtype=int).reshape(3)
        self.p = int(degree)
        self.np_ = self.p + 1
        self.nq = int(nq)
        self.k = np.asarray(kpoint, dtype=float).reshape(3)
        self.periodic = tuple(bool(v) for v in periodic)
        if self.nq < self.np_:
            raise ValueError("quadrature needs n_q >= n_p")
        self.E = int(np.prod(self.N))
        self.M = np.array([self.N[d] * self.p + (0 if self.periodic[d] else 1)
                           for d in range(3)])
        self.m = int(np.prod(self.M))
        # J[:, d] = a_d / (2 N_d)
        self.J = (self.A / (2.0 * self.N[:, None])).T
        self.detJ = float(np.linalg.det(self.J))
        if self.detJ <= 0.0:
            raise ValueError("lattice must be right-handed (det A > 0)")
        self.Jinv = np.linalg.inv(self.J)
        self.gll, self.gllw = gll_nodes_weights(self.p)
        self.xq, self.wq = gauss_points_weights(self.nq)

    # --- cells -----------------------------------------------------------
    def cell_coords(self, c):
        c = np.asarray(c)
        return np.stack([c % self.N[0], (c // self.N[0]) % self.N[1],
                         c // (self.N[0] * self.N[1])], axis=-1)

    def cell_origin(self, c):
        cc = self.cell_coords(c)
        return (cc / self.N) @ self.A

    # --- the cell -> DoF map Q^(e) --------------------------------------
    def cell_dofs(self, c=None):
        """dofs[c, I] for I = i + n_p (j + n_p k); all cells if c is None."""
        if c is None:
            c = np.arange(self.E)
        c = np.atleast_1d(np.asarray(c))
        cc = self.cell_coords(c)                         # [nc, 3]
        loc = np.arange(self.np_)
        g = []
        for d in range(3):
            gd = cc[:, d, None] * self.p + loc[None, :]  # [nc, np]
            if self.periodic[d]:
                gd = gd % self.M[d]
            g.append(gd)
        dof = (g[0][:, None, None, :]
               + self.M[0] * (g[1][:, None, :, None]
                              + self.M[1] * g[2][:, :, None, None]))
        return dof.reshape(len(c), self.np_ ** 3)

    def node_cells(self, dof):
        """All (cell, local index) pairs whose node maps to global ``dof``."""
        g = [dof % self.M[0], (dof // self.M[0]) % self.M[1],
             dof // (self.M[0] * self.M[1])]
        per_axis = []
        for d in range(3):
            opts = []
            for cd in range(self.N[d]):
                i = g[d] - cd * self.p
                if self.periodic[d]:
                    # node g lies in cell cd if g - cd p (mod M) is in [0, p]
                    i = i % self.M[d]
                if 0 <= i <= self.p:
                    opts.append((cd, i))
            per_axis.append(opts)
        out = []
        for c0, i in per_axis[0]:
            for c1, j in per_axis[1]:
                for c2, k in per_axis[2]:
                    c = c0 + self.N[0] * (c1 + self.N[1] * c2)
                    out.append((c, i + self.np_ * (j + self.np_ * k)))
        return out

    def dirichlet_dofs(self):
        """Nodes off every face normal to an open axis, in DoF order.

        Homogeneous Dirichlet conditions on the open axes fix the face nodes at
        zero (constraint C of eqn HX), so the Dirichlet operator is the open
        mesh's operator restricted to these rows and columns.
        """
        idx = np.arange(self.m)
        g = [idx % self.M[0], (idx // self.M[0]) % self.M[1], idx // (self.M[0] * self.M[1])]
        keep = np.ones(self.m, bool)
        for d in range(3):
            if not self.periodic[d]:
                keep &= (g[d] > 0) & (g[d] < self.M[d] - 1)
        return np.nonzero(keep)[0]

    # --- geometry --------------------------------------------------------
    def node_coords(self):
        """Physical coordinates of every DoF (periodic image inside the box)."""
        gl = self.gll
        idx = np.arange(self.m)
        g = [idx % self.M[0], (idx // self.M[0]) % self.M[1],
             idx // (self.M[0] * self.M[1])]
        frac = []
        for d in range(3):
            cd = np.minimum(g[d] // self.p, self.N[d] - 1)
            loc = g[d] - cd * self.p
            frac.append((cd + (gl[loc] + 1.0) / 2.0) / self.N[d])
        x = np.stack(frac, axis=-1) @ self.A
        return x

    def quad_points(self):
        """Physical quadrature points, cell-major: [E * n_q^3, 3]."""
        q = self.xq
        ref = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1)  # [q1,q2,q3,3]
        ref = ref.transpose(2, 1, 0, 3).reshape(-1, 3)   # Q = q1 + nq(q2 + nq q3)
        xc = self.cell_origin(np.arange(self.E))          # [E, 3]
        pts = xc[:, None, :] + (ref + 1.0) @ self.J.T     # x = x_c + J (xi + 1)
        return pts.reshape(-1, 3)

    def quad_weights(self):
        """w_q1 w_q2 w_q3 det J for one cell, flat Q order."""
        w = self.wq
        W = w[None, None, :] * w[None, :, None] * w[:, None, None]   # [q3,q2,q1]
        return W.reshape(-1) * self.detJ

    @property
    def volume(self):
        return abs(float(np.linalg.det(self.A)))

    @property
    def cell_volume(self):
        return 8.0 * abs(self.detJ)
