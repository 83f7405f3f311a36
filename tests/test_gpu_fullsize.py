"""GPU parity at the benchmark sizes, in the launch configuration bench.py times.

mid     : 16^3 cells, degree 6, 256 real vectors, GGA, 32 atoms x 4 projectors;
          all 256 columns, sampled output rows (cell corners, edges, faces,
          interiors, rows inside projector supports), against oracle rows.
complex : 24^3 cells, degree 7, Bloch k, 512 complex vectors, 128 atoms x 9
          projectors; 16 seeded columns tiled to the full 512-column block
          (H X is column-independent), sampled rows of every column.
Tolerance 1e-12 relative to the largest entry of the sampled oracle rows.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import operator as op  # noqa: E402
from oracle.mesh import Mesh as OMesh  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _rows(om, rng, extra=()):
    p = om.p
    pick = [0, p - 1 if p > 1 else 0, p, p + 1, om.M[0] * p + p // 2,
            (om.M[0] * om.M[1]) * p + om.M[0] * p + p, om.m - 1]
    pick += list(rng.integers(0, om.m, 24)) + list(extra)
    return np.unique(np.array(pick) % om.m)


def _setup(s):
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint)
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    m.set_potential(vl, vg)
    m.set_projectors(inputs.positions_array(s), s.projectors)
    P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors)
    return om, vl, vg, m, P, h


def test_mid_full_size():
    s = inputs.make_system("mid")
    om, vl, vg, m, P, h = _setup(s)
    X = inputs.make_vectors(s)
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, "f64")
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    supp = P.tocoo().row
    rows = _rows(om, rng, extra=rng.choice(supp, 8))
    got = Yd[torch.from_numpy(rows).to("cuda:0")].cpu().numpy()
    want = op.apply_rows(om, vl, vg, X, rows, P, h)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < TOL, err


def test_complex_full_size():
    """Expected rows come from tests/golden/complex_rows.npz (written by the
    oracle-only script tests/golden/make_complex_rows.py)."""
    import os
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "complex_rows.npz"))
    rows, want = gold["rows"], gold["y"]
    s = inputs.make_system("complex")
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    pts = m.quad_points()
    m.set_potential(inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts))
    m.set_projectors(inputs.positions_array(s), s.projectors)
    base = inputs.make_vectors(s, cols=range(16))
    Xd = torch.from_numpy(base).to("cuda:0").repeat(1, s.nvec // 16).contiguous()
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, "f64")
    torch.cuda.synchronize()
    del Xd
    got = Yd[torch.from_numpy(rows).to("cuda:0")].cpu().numpy()          # [rows, 512]
    err = np.abs(got - np.tile(want, (1, s.nvec // 16))).max() / np.abs(want).max()
    assert err < TOL, err
