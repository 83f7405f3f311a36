"""GPU parity of the eigensolver entry points (Alg. 3 / Alg. 4 with M = D)
against the CPU oracle on the same seeded inputs.

  fe_cheb_filter   vs oracle.eigen.cheb_filter_residual  (FP64 inner: 1e-10 rel)
  fe_lanczos       vs oracle.eigen.lanczos_bounds        (1e-9 of the spectral range)
  fe_rayleigh_ritz vs oracle.eigen.rayleigh_ritz         (Ritz values 1e-10 rel;
                   the rotated block is checked by the properties every correct
                   answer has: X^H H X = diag(ritz), X^H D X = I); also a block
                   inside a wider buffer on 972 DoFs (a remainder DoF chunk in
                   the Gram products) and the error for a rank-deficient block
  fe_chfsi         vs oracle.eigen.chfsi                 (FP64: 1e-9 Ha; FP32 / BF16
                   inner filter steps: the precision gate of 1e-5 Ha)
The filter's tolerance: the recurrence of degree p multiplies rounding errors by
at most p times the condition of the scaled filter, far below 1e-10 here.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import eigen  # noqa: E402
from oracle import operator as op  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import lib_side, oracle_side, rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _systems():
    real = inputs.make_system("tiny")
    cplx = inputs.make_custom(np.diag([7.5, 8.0, 7.0]), (3, 4, 3), 3, 4, kpoint=(0.3, -0.2, 0.1), nvec=8,
                              seed=21, natoms=2, pset="spd", rc=3.0)
    return {"tiny-real": real, "small-complex-spd": cplx}


SYS = _systems()


@pytest.fixture(scope="module", params=sorted(SYS))
def case(request):
    s = SYS[request.param]
    om, vl, vg, P, h = oracle_side(s)
    H = op.assemble_H(om, vl, vg)
    Hop = lambda V: op.apply_sparse(H, V, P, h)
    Dv = op.lumped_mass(om)
    return s, om, Hop, Dv, lib_side(s, vl, vg)


def _bounds(s, Hop, Dv, X):
    theta, beta = eigen.lanczos_bounds(Hop, Dv, inputs.lanczos_start(s), 10)
    lam, _ = eigen.rayleigh_ritz(Hop, lambda V: Dv[:, None] * V, X)
    return lam, theta.min(), lam.max() + 0.1, theta.max() + abs(beta)


@pytest.mark.parametrize("degree", [2, 12])
def test_filter_fp64_matches_oracle(case, degree):
    s, om, Hop, Dv, m = case
    X = inputs.make_vectors(s)
    lam, lmin, lT, lmax = _bounds(s, Hop, Dv, X)
    want = eigen.cheb_filter_residual(Hop, lambda V: Dv[:, None] * V, 1.0 / Dv, X, lam, degree, lmin, lmax, lT)
    Xd = to_dev(X)
    m.cheb_filter(Xd, torch.from_numpy(lam).cuda(), degree, lmin, lT, lmax, inner="f64")
    torch.cuda.synchronize()
    got = Xd.cpu().numpy()
    assert rel(got, want) < 1e-10
    for j in range(X.shape[1]):
        assert rel(got[:, j], want[:, j]) < 1e-10


def test_filter_low_precision_close(case):
    s, om, Hop, Dv, m = case
    X = inputs.make_vectors(s)
    lam, lmin, lT, lmax = _bounds(s, Hop, Dv, X)
    want = eigen.cheb_filter_residual(Hop, lambda V: Dv[:, None] * V, 1.0 / Dv, X, lam, 12, lmin, lmax, lT)
    for prec, tol in (("f32", 1e-4), ("bf16", 5e-2)):
        Xd = to_dev(X)
        m.cheb_filter(Xd, torch.from_numpy(lam).cuda(), 12, lmin, lT, lmax, inner=prec)
        torch.cuda.synchronize()
        assert rel(Xd.cpu().numpy(), want) < tol, prec


def test_lanczos_matches_oracle(case):
    s, om, Hop, Dv, m = case
    v0 = inputs.lanczos_start(s)
    theta_o, beta_o = eigen.lanczos_bounds(Hop, Dv, v0, 10)
    theta, beta = m.lanczos(to_dev(v0), 10)
    span = theta_o.max() - theta_o.min()
    assert np.abs(np.sort(theta) - np.sort(theta_o)).max() < 1e-9 * span
    assert abs(abs(beta) - abs(beta_o)) < 1e-9 * span


def test_rayleigh_ritz_matches_oracle(case):
    s, om, Hop, Dv, m = case
    X = inputs.make_vectors(s)
    lam_o, _ = eigen.rayleigh_ritz(Hop, lambda V: Dv[:, None] * V, X)
    Xd = to_dev(X)
    ritz = torch.empty(X.shape[1], dtype=torch.float64, device="cuda:0")
    m.rayleigh_ritz(Xd, ritz)
    torch.cuda.synchronize()
    lam = ritz.cpu().numpy()
    scale = np.abs(lam_o).max()
    assert np.abs(lam - lam_o).max() < 1e-10 * scale
    V = Xd.cpu().numpy()
    G = V.conj().T @ Hop(V)
    S = V.conj().T @ (Dv[:, None] * V)
    assert np.abs(S - np.eye(len(lam))).max() < 1e-10
    assert np.abs(G - np.diag(lam)).max() < 1e-10 * scale
    # the rotated block spans the same space as the input block
    Q, _ = np.linalg.qr(X)
    assert np.linalg.norm(V - Q @ (Q.conj().T @ V)) < 1e-10 * np.linalg.norm(V)


def test_filter_workspace_layout_switch(case):
    """FP32 passes keep the FP64 residual inside the R_X block, FP64 and BF16
    passes in a slot of its own: alternating precisions on one mesh reuses
    and regrows the same workspaces, and every pass must give what a pass on
    a fresh layout gives (FP32 bit for bit, FP64 against the oracle)."""
    s, om, Hop, Dv, m = case
    X = inputs.make_vectors(s)
    lam, lmin, lT, lmax = _bounds(s, Hop, Dv, X)
    want = eigen.cheb_filter_residual(Hop, lambda V: Dv[:, None] * V, 1.0 / Dv, X, lam, 8, lmin, lmax, lT)
    lam_d = torch.from_numpy(lam).cuda()

    def run(prec):
        Xd = to_dev(X)
        m.cheb_filter(Xd, lam_d, 8, lmin, lT, lmax, inner=prec)
        torch.cuda.synchronize()
        return Xd.cpu().numpy()

    first = run("f32")
    assert rel(first, want) < 1e-4
    assert rel(run("f64"), want) < 1e-10
    assert rel(run("bf16"), want) < 5e-2
    assert np.array_equal(run("f32"), first)
    assert rel(run("f64"), want) < 1e-10


@pytest.mark.parametrize("kpoint", [(0.0, 0.0, 0.0), (0.2, -0.1, 0.3)])
def test_rayleigh_ritz_padded_block_ragged_dof_chunks(kpoint):
    """972 DoFs: the Gram matrices' DoF split leaves a remainder chunk (972 =
    64 x 15 + 12); the block sits in a wider buffer (ldx = nvec + 3) whose
    padding columns must come back untouched."""
    s = inputs.make_custom(np.diag([7.5, 8.0, 7.0]), (3, 4, 3), 3, 4, kpoint=kpoint, nvec=6, seed=23,
                           natoms=1, pset="sp", rc=3.0)
    om, vl, vg, P, h = oracle_side(s)
    H = op.assemble_H(om, vl, vg)
    Hop = lambda V: op.apply_sparse(H, V, P, h)
    Dv = op.lumped_mass(om)
    m = lib_side(s, vl, vg)
    assert m.ndofs == 972
    X = inputs.make_vectors(s)
    lam_o, _ = eigen.rayleigh_ritz(Hop, lambda V: Dv[:, None] * V, X)
    nv = X.shape[1]
    Xw = torch.full((m.ndofs, nv + 3), 7.0, dtype=to_dev(X).dtype, device="cuda:0")
    Xw[:, :nv] = to_dev(X)
    ritz = torch.empty(nv, dtype=torch.float64, device="cuda:0")
    m.rayleigh_ritz(Xw[:, :nv], ritz)
    torch.cuda.synchronize()
    lam = ritz.cpu().numpy()
    assert np.abs(lam - lam_o).max() < 1e-10 * np.abs(lam_o).max()
    W = Xw.cpu().numpy()
    assert np.all(W[:, nv:] == 7.0)
    V = W[:, :nv]
    assert np.abs(V.conj().T @ (Dv[:, None] * V) - np.eye(nv)).max() < 1e-10


def test_rayleigh_ritz_rank_deficient_block_is_an_error(case):
    """A zero column makes Y^H D Y singular with an exactly zero pivot."""
    s, om, Hop, Dv, m = case
    X = inputs.make_vectors(s)
    X[:, 2] = 0
    Xd = to_dev(X)
    ritz = torch.empty(X.shape[1], dtype=torch.float64, device="cuda:0")
    with pytest.raises(fehx.FeError) as e:
        m.rayleigh_ritz(Xd, ritz)
    assert e.value.code == -3 and "positive definite" in str(e.value)


def _oracle_chfsi(s, Hop, Dv, outer, degree):
    X0 = inputs.make_vectors(s)
    lam, X, log = eigen.chfsi(Hop, Dv, X0, inputs.lanczos_start(s), s.volume, outer=outer, degree=degree)
    return lam, log


def test_chfsi_fp64_matches_oracle(case):
    s, om, Hop, Dv, m = case
    lam_o, log = _oracle_chfsi(s, Hop, Dv, 3, 20)
    Xd = to_dev(inputs.make_vectors(s))
    lam, bounds = m.chfsi(Xd, to_dev(inputs.lanczos_start(s)), outer=3, degree=20, inner="f64")
    for it, b in enumerate(log):
        assert np.allclose(bounds[it], [b["lmin"], b["lT"], b["lmax"]], rtol=1e-9, atol=1e-9)
    assert np.abs(lam - lam_o).max() < 1e-9


@pytest.mark.parametrize("prec,degree,outer", [("f32", 40, 3), ("bf16", 40, 3), ("bf16", 16, 6)])
def test_precision_gate(case, prec, degree, outer):
    """Low-precision inner filter steps against the FP64 oracle running the same
    procedure from the same seeds: the lowest 75% of the block (the rest is the
    unconverged buffer) within 1e-5 Ha, at the filter workload's degree 40 x 3
    passes and at degree 16 x 6.  BF16 steps keep the recurrence state in FP32
    and take BF16 hi/lo operands on the matrix cores."""
    s, om, Hop, Dv, m = case
    lam_o, _ = _oracle_chfsi(s, Hop, Dv, outer, degree)
    Xd = to_dev(inputs.make_vectors(s))
    lam, _ = m.chfsi(Xd, to_dev(inputs.lanczos_start(s)), outer=outer, degree=degree, inner=prec)
    k = (3 * len(lam)) // 4
    err = np.abs(lam - lam_o)
    print(f"{prec} degree {degree} x {outer}: max |dlambda| lowest {k} = {err[:k].max():.3e} Ha, all = {err.max():.3e}")
    assert err[:k].max() < 1e-5
