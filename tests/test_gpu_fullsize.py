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


@pytest.fixture(scope="module")
def mid():
    s = inputs.make_system("mid")
    om, vl, vg, m, P, h = _setup(s)
    X = inputs.make_vectors(s)
    rng = np.random.default_rng(5)
    rows = _rows(om, rng, extra=rng.choice(P.tocoo().row, 8))
    want = op.apply_rows(om, vl, vg, X, rows, P, h)
    return s, om, vl, vg, m, P, h, X, rows, want


def _sampled(Yd, rows):
    return Yd[torch.from_numpy(rows).to(Yd.device)].cpu().numpy()


def test_mid_full_size(mid):
    """Every FP64 vector tile the kernel has at n_p = 7 (4, 8, 16) and the
    autotuned one (the instance bench.py times) against the oracle rows."""
    s, om, vl, vg, m, P, h, X, rows, want = mid
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.empty_like(Xd)
    best, times = m.autotune("f64", s.nvec, kind=0, reps=1)
    tiles = sorted(t for t, ms in times.items() if ms > 0)
    assert best in tiles and set(tiles) >= {4, 8, 16}
    for vt in tiles + [best]:
        m.set_tile("f64", vt)
        Yd.fill_(float("nan"))
        m.apply(Xd, Yd, "f64")
        torch.cuda.synchronize()
        err = np.abs(_sampled(Yd, rows) - want).max() / np.abs(want).max()
        print(f"mid f64 tile {vt}{' (autotuned)' if vt == best else ''}: rel err {err:.2e}")
        assert err < TOL, (vt, err)
    m.set_tile("f64", 0)


def _round_bf16(X):
    """X rounded to bfloat16 (nearest even), as float64 (input of the BF16 path)."""
    f = np.ascontiguousarray(X, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mid_low_precision_tiles(mid, prec):
    """FP32 and BF16 H X at the Mid size for every vector tile (8, 16, 32),
    sampled rows against the oracle applied to the same (rounded) input.
    FP32: 2e-5 of the largest entry.  BF16 (float arithmetic, bfloat16 output):
    the output rounding, 2^-8 of the largest entry."""
    s, om, vl, vg, m, P, h, X, rows, want = mid
    if prec == "f32":
        Xin, tol = X.astype(np.float32).astype(np.float64), 2e-5
        Xd = torch.from_numpy(X).to("cuda:0").float()
        ref = want if np.array_equal(Xin, X) else op.apply_rows(om, vl, vg, Xin, rows, P, h)
    else:
        Xin, tol = _round_bf16(X), 2.0 ** -8
        Xd = torch.from_numpy(X).to("cuda:0").to(torch.bfloat16)
        ref = op.apply_rows(om, vl, vg, Xin, rows, P, h)
    Yd = torch.empty_like(Xd)
    for vt in (8, 16, 32):
        m.set_tile(prec, vt)
        Yd.fill_(float("nan"))
        m.apply(Xd, Yd, prec)
        torch.cuda.synchronize()
        got = _sampled(Yd.double(), rows)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"mid {prec} tile {vt}: rel err {err:.2e}")
        assert err < tol, (vt, err)
    m.set_tile(prec, 0)


def test_mid_filter_steps_per_tile():
    """The filter's operator (D^-1 applied at the gather, the recurrence
    update after it) at the Mid size: a degree-3 pass on 32 seeded columns of
    the filter workload, per inner precision and every filter-step tile,
    against the oracle's Alg. 4 with the cell-matrix operator.  FP64 1e-10,
    FP32 1e-5, BF16 2e-2 of the largest entry."""
    from oracle import eigen
    s = inputs.make_system("filter")
    om, vl, vg, m, P, h = _setup(s)
    X = inputs.make_vectors(s, cols=range(32))
    Hop = op.cm_operator(om, vl, vg, P, h, batch=512)
    Dv = op.lumped_mass(om)
    lam = np.linspace(-1.5, 0.5, 32)
    lmin, lT, lmax = -2.0, 0.8, 120.0
    want = eigen.cheb_filter_residual(Hop, lambda V: Dv[:, None] * V, 1.0 / Dv, X, lam, 3, lmin, lmax, lT)
    lam_d = torch.from_numpy(lam).to("cuda:0")
    X0 = torch.from_numpy(X).to("cuda:0")
    for prec, tiles, tol in (("f64", (4, 8, 16), 1e-10), ("f32", (8, 16, 32), 1e-5), ("bf16", (8, 16, 32), 2e-2)):
        for vt in tiles:
            m.set_tile(prec, vt, kind=1)
            Xf = X0.clone()
            m.cheb_filter(Xf, lam_d, 3, lmin, lT, lmax, inner=prec)
            torch.cuda.synchronize()
            err = np.abs(Xf.cpu().numpy() - want).max() / np.abs(want).max()
            print(f"mid filter step {prec} tile {vt}: rel err {err:.2e}")
            assert err < tol, (prec, vt, err)
        m.set_tile(prec, 0, kind=1)


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
