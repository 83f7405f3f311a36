"""Pins for oracle.mesh: brute-force geometry and the cell-to-DoF map."""
import numpy as np
import pytest

from oracle.mesh import Mesh

SHEARED = np.array([[6.0, 0.0, 0.0], [1.5, 5.0, 0.0], [0.7, -0.9, 7.0]])


@pytest.mark.parametrize("N,p", [((3, 2, 4), 2), ((2, 3, 2), 4), ((4, 4, 4), 1)])
def test_shared_nodes_coincide(N, p):
    m = Mesh(SHEARED, N, p, p + 1)
    xn = m.node_coords()
    dofs = m.cell_dofs()
    ref = m.gll
    loc = np.stack(np.meshgrid(ref, ref, ref, indexing="ij"), -1).transpose(2, 1, 0, 3).reshape(-1, 3)
    Ainv = np.linalg.inv(m.A)
    for c in range(m.E):
        x = m.cell_origin(c) + (loc + 1.0) @ m.J.T
        d = (x - xn[dofs[c]]) @ Ainv                 # difference in box units
        assert np.allclose(d, np.round(d), atol=1e-12)


@pytest.mark.parametrize("N,p", [((3, 3, 3), 3), ((2, 4, 3), 2), ((4, 4, 4), 4)])
def test_multiplicity_and_counts(N, p):
    m = Mesh(np.eye(3) * 5.0, N, p, p + 1)
    counts = np.bincount(m.cell_dofs().reshape(-1), minlength=m.m)
    E = m.E
    assert m.m == np.prod(np.array(N) * p)
    assert sorted(set(counts.tolist())) == [1, 2, 4, 8]
    assert (counts == 8).sum() == E
    assert (counts == 4).sum() == 3 * (p - 1) * E
    assert (counts == 2).sum() == 3 * (p - 1) ** 2 * E
    assert (counts == 1).sum() == (p - 1) ** 3 * E


def test_node_cells_inverse_of_cell_dofs():
    m = Mesh(SHEARED, (3, 2, 2), 3, 4)
    dofs = m.cell_dofs()
    rng = np.random.default_rng(0)
    for dof in rng.integers(0, m.m, 40):
        pairs = m.node_cells(int(dof))
        assert all(dofs[c, I] == dof for c, I in pairs)
        assert len(pairs) == (dofs == dof).sum()


def test_volume_and_quadrature_points():
    m = Mesh(SHEARED, (2, 3, 2), 3, 5)
    assert abs(m.quad_weights().sum() * m.E - m.volume) < 1e-12 * m.volume
    f = m.quad_points() @ np.linalg.inv(m.A)
    assert f.min() > 0 and f.max() < 1
    # every cell holds exactly its own points
    cell_of = np.floor(f * m.N).astype(int)
    cid = cell_of[:, 0] + m.N[0] * (cell_of[:, 1] + m.N[1] * cell_of[:, 2])
    assert np.array_equal(cid, np.repeat(np.arange(m.E), m.nq ** 3))
