"""A filter pass captured as a HIP graph replays the eager pass bit for bit.

The graph is replayed several times with the program's own eager work (block
copies, an unrelated operator application) and synchronisations in between;
every replay is compared with the eager fe_cheb_filter result, and the FP64
result with the oracle's Alg. 4 (1e-10 relative).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import eigen  # noqa: E402
from oracle import operator as op  # noqa: E402
from paper_2512_08571_amd import inputs  # noqa: E402

from gpu_common import lib_side, oracle_side, rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    s = inputs.make_custom(np.diag([7.5, 8.0, 7.0]), (3, 4, 3), 3, 4, kpoint=(0.3, -0.2, 0.1), nvec=8,
                           seed=21, natoms=2, pset="spd", rc=3.0)
    om, vl, vg, P, h = oracle_side(s)
    H = op.assemble_H(om, vl, vg)
    Hop = lambda V: op.apply_sparse(H, V, P, h)
    Dv = op.lumped_mass(om)
    X = inputs.make_vectors(s)
    theta, beta = eigen.lanczos_bounds(Hop, Dv, inputs.lanczos_start(s), 10)
    lam, _ = eigen.rayleigh_ritz(Hop, lambda V: Dv[:, None] * V, X)
    bounds = (theta.min(), lam.max() + 0.1, theta.max() + abs(beta))
    return s, Hop, Dv, X, lam, bounds, lib_side(s, vl, vg)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_graph_replays_equal_eager(case, prec):
    s, Hop, Dv, X, lam, (lmin, lT, lmax), m = case
    lam_d = torch.from_numpy(lam).cuda()
    X0 = to_dev(X)
    Xe = X0.clone()
    m.cheb_filter(Xe, lam_d, 9, lmin, lT, lmax, inner=prec)
    torch.cuda.synchronize()
    if prec == "f64":
        want = eigen.cheb_filter_residual(Hop, lambda V: Dv[:, None] * V, 1.0 / Dv, X, lam, 9, lmin, lmax, lT)
        assert rel(Xe.cpu().numpy(), want) < 1e-10
    Xg = torch.empty_like(X0)
    g = m.filter_graph(Xg, lam_d, 9, lmin, lT, lmax, inner=prec)
    other_in, other_out = X0.clone(), torch.empty_like(X0)
    for rep in range(4):
        Xg.copy_(X0)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(Xg, Xe), f"replay {rep}"
        m.apply(other_in, other_out)          # unrelated eager work between replays
        torch.cuda.synchronize()
    g.close()


def test_live_graph_keeps_its_workspaces():
    """A live graph holds the addresses of the mesh's filter and projector
    workspaces, so no call may free or move them while it exists.  Real mesh
    with 972 DoFs x 8 vectors (7776 elements, not a multiple of 64): an FP32
    pass would need a larger shared R_X block than the FP64 graph's, and a
    16-vector H X a larger projector workspace; both return FE_ESTATE, and a
    replay afterwards still equals the eager FP64 pass bit for bit.  After the
    graph is destroyed the FP32 pass runs."""
    from paper_2512_08571_amd import fehx
    s = inputs.make_custom(np.diag([7.5, 8.0, 7.0]), (3, 4, 3), 3, 4, kpoint=(0.0, 0.0, 0.0), nvec=8,
                           seed=22, natoms=2, pset="spd", rc=3.0)
    om, vl, vg, P, h = oracle_side(s)
    H = op.assemble_H(om, vl, vg)
    Hop = lambda V: op.apply_sparse(H, V, P, h)
    Dv = op.lumped_mass(om)
    X = inputs.make_vectors(s)
    assert (om.m * X.shape[1]) % 64 != 0
    theta, beta = eigen.lanczos_bounds(Hop, Dv, inputs.lanczos_start(s), 10)
    lam, _ = eigen.rayleigh_ritz(Hop, lambda V: Dv[:, None] * V, X)
    lmin, lT, lmax = theta.min(), lam.max() + 0.1, theta.max() + abs(beta)
    m = lib_side(s, vl, vg)
    lam_d = torch.from_numpy(lam).cuda()
    X0 = to_dev(X)
    Xe = X0.clone()
    m.cheb_filter(Xe, lam_d, 9, lmin, lT, lmax, inner="f64")
    torch.cuda.synchronize()
    Xg = torch.empty_like(X0)
    g = m.filter_graph(Xg, lam_d, 9, lmin, lT, lmax, inner="f64")
    X1 = X0.clone()
    with pytest.raises(fehx.FeError) as e:
        m.cheb_filter(X1, lam_d, 9, lmin, lT, lmax, inner="f32")
    assert e.value.code == -4
    wide = torch.from_numpy(np.tile(X, (1, 2))).cuda()
    with pytest.raises(fehx.FeError) as e:
        m.apply(wide, torch.empty_like(wide))
    assert e.value.code == -4
    with pytest.raises(fehx.FeError) as e:
        m.set_projectors(inputs.positions_array(s), s.projectors)
    assert e.value.code == -4
    Xg.copy_(X0)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(Xg, Xe)
    g.close()
    m.cheb_filter(X1, lam_d, 9, lmin, lT, lmax, inner="f32")
    torch.cuda.synchronize()
    assert rel(X1.cpu().numpy(), Xe.cpu().numpy()) < 1e-4
