"""Batched persistent launches and launch-shape tuning.

* fe_batch_apply over systems of different sizes, degrees and real/complex
  type equals separate fe_apply_H calls bit for bit (the same per-item
  arithmetic runs in the batched kernel), and one system against the oracle
  (1e-12 relative);
* more systems of one class than one launch carries (8) are split correctly;
* every vector tile gives bit-identical results (lanes are independent), and
  the autotuner keeps a valid tile without changing results.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import operator as op  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import lib_side, oracle_side, rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _sys(n, p, k, nvec, seed, natoms=1):
    L = np.diag([1.25 * n[0], 1.25 * n[1], 1.25 * n[2]])
    return inputs.make_custom(L, n, p, p + 1, kpoint=k, nvec=nvec, seed=seed, natoms=natoms, pset="sp", rc=1.5)


SYSTEMS = [_sys((4, 3, 5), 4, (0, 0, 0), 24, 31), _sys((3, 3, 3), 4, (0, 0, 0), 7, 32),
           _sys((4, 4, 3), 3, (0.2, 0.0, 0.1), 10, 33), _sys((5, 4, 4), 4, (0, 0, 0), 33, 34),
           _sys((3, 4, 3), 3, (0.1, 0.3, 0.0), 5, 35)]


def _setup(s):
    pts_mesh = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=0)
    pts = pts_mesh.quad_points()
    m = pts_mesh
    m.set_potential(inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts))
    if s.projectors:
        m.set_projectors(inputs.positions_array(s), s.projectors)
    return m


def test_batch_equals_separate_and_oracle():
    ms = [_setup(s) for s in SYSTEMS]
    Xs = [to_dev(inputs.make_vectors(s)) for s in SYSTEMS]
    Ys_sep = []
    for m, X in zip(ms, Xs):
        Y = torch.empty_like(X)
        m.apply(X, Y)
        Ys_sep.append(Y)
    Ys = [torch.full_like(X, 3.0) for X in Xs]
    fehx.batch_apply(ms, Xs, Ys)
    torch.cuda.synchronize()
    for a, b in zip(Ys, Ys_sep):
        assert torch.equal(a, b)
    s = SYSTEMS[2]
    om, vl, vg, P, h = oracle_side(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), inputs.make_vectors(s), P, h)
    assert rel(Ys[2].cpu().numpy(), want) < 1e-12


def test_batch_of_more_systems_than_one_launch_carries():
    systems = [_sys((3, 3, 3 + (i % 3)), 3, (0, 0, 0), 4 + i, 40 + i, natoms=0) for i in range(11)]
    ms = [_setup(s) for s in systems]
    Xs = [to_dev(inputs.make_vectors(s)) for s in systems]
    Ys = [torch.empty_like(X) for X in Xs]
    fehx.batch_apply(ms, Xs, Ys)
    for m, X, Yb in zip(ms, Xs, Ys):
        Y = torch.empty_like(X)
        m.apply(X, Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yb)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_every_tile_gives_identical_results(prec):
    s = SYSTEMS[3]
    m = _setup(s)
    X = to_dev(inputs.make_vectors(s))
    if prec == "f32":
        X = X.float()
    if prec == "bf16":
        X = X.to(torch.bfloat16)
    outs = []
    for vt in ((4, 8, 10, 16) if prec == "f64" else (8, 16, 32)):
        m.set_tile(prec, vt)
        assert m.get_tile(prec) == vt
        Y = torch.empty_like(X)
        m.apply(X, Y, prec)
        torch.cuda.synchronize()
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(Y, outs[0])


def test_autotune_keeps_a_valid_tile():
    s = SYSTEMS[0]
    m = _setup(s)
    X = to_dev(inputs.make_vectors(s))
    Y0 = torch.empty_like(X)
    m.apply(X, Y0)
    for kind in (0, 1):
        best, times = m.autotune("f64", s.nvec, kind=kind, reps=2)
        assert best in (2, 4, 8, 10, 16) and times[best] > 0
        assert m.get_tile("f64", kind) == best
    Y1 = torch.empty_like(X)
    m.apply(X, Y1)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)


def _mp_grid(L, q=2):
    """Monkhorst-Pack grid: k = sum_i u_i b_i, u = (2r - q - 1) / 2q, b_i = 2 pi / L_i."""
    u = [(2 * r - q - 1) / (2.0 * q) for r in range(1, q + 1)]
    return [tuple(2 * np.pi * np.array([a, b, c]) / np.diag(L)) for a in u for b in u for c in u]


def test_kpoint_grid_in_one_batch():
    """A 2x2x2 Monkhorst-Pack grid of one system: the eight k-point operators
    in one batched launch per colour phase equal separate applications bit
    for bit and the oracle (1e-12); H(-k) conj(X) = conj(H(k) X)."""
    base = inputs.make_custom(np.diag([6.0, 6.5, 7.0]), (3, 3, 4), 4, 5, kpoint=(0.1, 0.1, 0.1), nvec=6,
                              seed=41, natoms=2, pset="spd", rc=2.0)
    ks = _mp_grid(base.lattice)
    systems = [inputs.make_custom(base.lattice, base.ncell, base.degree, base.nq, kpoint=k, nvec=6, seed=41,
                                  natoms=2, pset="spd", rc=2.0) for k in ks]
    ms = [_setup(s) for s in systems]
    X = inputs.make_vectors(systems[0])
    Xs = [to_dev(X) for _ in ms]
    Ys = [torch.full_like(x, 2.0) for x in Xs]
    fehx.batch_apply(ms, Xs, Ys)
    torch.cuda.synchronize()
    for m, x, y in zip(ms, Xs, Ys):
        y1 = torch.empty_like(x)
        m.apply(x, y1)
        torch.cuda.synchronize()
        assert torch.equal(y, y1)
    for i in (0, 5):
        om, vl, vg, P, h = oracle_side(systems[i])
        want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
        assert rel(Ys[i].cpu().numpy(), want) < 1e-12
    # k and -k are both on the grid: H(-k) conj(X) = conj(H(k) X)
    j = [np.allclose(np.array(ks[i]), -np.array(ks[0])) for i in range(len(ks))].index(True)
    yc = torch.empty_like(Xs[0])
    ms[j].apply(to_dev(X.conj()), yc)
    torch.cuda.synchronize()
    assert rel(yc.cpu().numpy(), Ys[0].cpu().numpy().conj()) < 1e-13


def test_set_tile_refuses_blocks_that_do_not_fit():
    """At n_p = 8 an FP64 block of 16 lanes needs more than 160 KB of LDS and
    two lanes are offered only where four do not fit: both are refused, the
    ten-lane tile is taken."""
    m = _setup(_sys((3, 3, 3), 7, (0, 0, 0), 4, 77, natoms=0))
    for vt in (2, 16):
        with pytest.raises(fehx.FeError):
            m.set_tile("f64", vt)
    m.set_tile("f64", 10)
    assert m.get_tile("f64") == 10
    m.set_tile("f64", 0)
