"""GPU parity of the HIP H.X path against the CPU oracle (FP64: 1e-12 relative).

Inputs are the seeded arrays of paper_2512_08571_amd.inputs, identical on both
sides.  Tolerance: the two sides sum the same terms in different orders, so
agreement to a few ulps of the largest entry is expected; 1e-12 relative to
the largest |Y| entry is the bar (per column as well).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import operator as op  # noqa: E402
from oracle.mesh import Mesh as OMesh  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import lib_side, oracle_side, rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _apply(m, X, prec="f64", dtype=None):
    Xd = to_dev(X, dtype)
    Yd = torch.empty_like(Xd)
    m.apply(Xd, Yd, prec)
    torch.cuda.synchronize()
    return Yd


@pytest.fixture(scope="module")
def tiny():
    s = inputs.make_system("tiny")
    om, vl, vg, P, h = oracle_side(s)
    return s, om, vl, vg, lib_side(s, vl, vg)


def test_index_map_is_bit_exact(tiny):
    s, om, _, _, m = tiny
    assert np.array_equal(m.cell_dofs(), om.cell_dofs().astype(np.int32))
    assert m.ndofs == om.m == 4096


def test_quad_points_and_lumped_mass(tiny):
    s, om, _, _, m = tiny
    assert np.abs(m.quad_points() - om.quad_points()).max() < 1e-13
    assert rel(m.lumped_mass(), op.lumped_mass(om)) < 1e-14


def test_tiny_hx_matches_assembled_operator(tiny):
    s, om, vl, vg, m = tiny
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X)
    got = _apply(m, X).cpu().numpy()
    assert rel(got, want) < TOL
    for j in range(X.shape[1]):
        assert rel(got[:, j], want[:, j]) < TOL


def test_tiny_brute_force_full_matrix(tiny):
    s, om, vl, vg, m = tiny
    H = op.assemble_H(om, vl, vg).toarray()
    got = _apply(m, np.eye(om.m)).cpu().numpy()          # column j = H e_j
    assert rel(got, H) < TOL


def _small(k, natoms, pset, gga=True, N=(3, 4, 3), p=3, nvec=6, seed=11, nq=None):
    L = np.diag([7.5, 8.0, 7.0])
    return inputs.make_custom(L, N, p, p + 1 if nq is None else nq, kpoint=k, nvec=nvec, seed=seed,
                              natoms=natoms, pset=pset, rc=3.0, gga=gga)


@pytest.mark.parametrize("k,natoms,pset,p", [((0, 0, 0), 0, "s", 2), ((0, 0, 0), 3, "sp", 3),
                                             ((0.3, -0.2, 0.1), 2, "spd", 3), ((0.2, 0.1, 0.4), 2, "spd", 5),
                                             ((0.0, 0.0, 0.0), 2, "spd", 8)])
def test_small_full_operator(k, natoms, pset, p):
    s = _small(k, natoms, pset, p=p, N=(3, 2, 3) if p > 5 else (3, 4, 3))
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    got = _apply(m, X).cpu().numpy()
    assert rel(got, want) < TOL


def test_tiny_nonlocal_brute_force():
    s = _small((0.25, 0.1, 0.0), 2, "spd", N=(2, 3, 2), p=3)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    H = op.assemble_H(om, vl, vg).toarray() + op.nonlocal_dense(P, h)
    got = _apply(m, np.eye(om.m, dtype=complex)).cpu().numpy()
    assert rel(got, H) < TOL


def test_hermitian_deterministic_and_column_independent():
    s = _small((0.3, -0.2, 0.1), 2, "spd", nvec=8)
    om, vl, vg, P, h = oracle_side(s, with_P=False)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    Y1 = _apply(m, X).cpu().numpy()
    Y2 = _apply(m, X).cpu().numpy()
    assert np.array_equal(Y1, Y2)                                     # bitwise replay
    G = X.conj().T @ Y1
    assert np.abs(G - G.conj().T).max() < 1e-12 * np.abs(G).max()    # X^H H X Hermitian
    Ys = _apply(m, X[:, [5, 1, 6]]).cpu().numpy()
    assert np.array_equal(Ys, Y1[:, [5, 1, 6]])


def test_odd_cell_counts_use_three_colours():
    s = _small((0.1, 0.0, -0.2), 1, "sp", N=(3, 5, 2), p=2)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    assert rel(_apply(m, X).cpu().numpy(), want) < TOL


def test_ragged_vector_counts():
    s = _small((0, 0, 0), 1, "sp", nvec=21)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    for n in (1, 7, 21):
        assert rel(_apply(m, X[:, :n]).cpu().numpy(), want[:, :n]) < TOL
    # blocks wider than nvec and views whose rows start off any vector alignment
    Xw = to_dev(np.concatenate([np.zeros((om.m, 3)), X], axis=1))
    Yw = torch.full_like(Xw, 7.0)
    for off, n in ((3, 21), (3, 16), (1, 8)):
        Yw.fill_(7.0)
        m.apply(Xw[:, off:], Yw[:, off:], nvec=n)
        torch.cuda.synchronize()
        got = Yw.cpu().numpy()
        ref = np.concatenate([np.zeros((om.m, 3)), X], axis=1)[:, off:off + n]
        assert rel(got[:, off:off + n], op.apply_sparse(op.assemble_H(om, vl, vg), ref, P, h)) < TOL
        assert np.all(got[:, :off] == 7.0) and np.all(got[:, off + n:] == 7.0)   # nothing outside the block


def test_low_precision_close_to_fp64():
    s = _small((0.3, -0.2, 0.1), 2, "spd", nvec=16)
    om, vl, vg, P, h = oracle_side(s, with_P=False)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    y64 = _apply(m, X).cpu().numpy()
    y32 = _apply(m, X.astype(np.complex64), "f32").cpu().numpy()
    assert rel(y32, y64) < 2e-5
    xb = torch.view_as_real(to_dev(X)).to(torch.bfloat16).contiguous()
    yb = torch.empty_like(xb)
    m.apply(xb, yb, "bf16")
    torch.cuda.synchronize()
    ybf = torch.view_as_complex(yb.float().contiguous()).cpu().numpy()
    assert rel(ybf, y64) < 5e-2


def _brick_and_overflow_rows(m, s, pmax=64):
    """Support rows the nonlocal update takes in node bricks (8^3, else 4^3,
    of at most pmax projectors) and rows it leaves to the global-W kernel."""
    rows, cols, _ = m.projector_entries()
    M = [n * s.degree for n in s.ncell]
    x, y, z = rows % M[0], (rows // M[0]) % M[1], rows // (M[0] * M[1])
    todo = np.ones(len(rows), bool)
    inb = 0
    for h in (8, 4):
        key = ((z // h) * 1000 + y // h) * 1000 + x // h
        pair = np.unique(key[todo].astype(np.int64) * 100000 + cols[todo])
        bk, cnt = np.unique(pair // 100000, return_counts=True)
        acc = np.isin(key, bk[cnt <= pmax]) & todo
        inb += len(np.unique(rows[acc]))
        todo &= ~acc
    return inb, len(np.unique(rows[todo]))


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.1, 0.2, -0.1)])
def test_crowded_projectors_brick_and_overflow_rows(k):
    """Eight spd atoms in a small cell: some node bricks touch more than 64
    projectors, so both nonlocal update kernels write rows of Y."""
    N = (4, 4, 4)
    s = inputs.make_custom(np.diag([10.0, 32.0 / 3.0, 28.0 / 3.0]), N, 3, 4, kpoint=k, nvec=12, seed=12,
                           natoms=8, pset="spd", rc=3.0)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    inb, over = _brick_and_overflow_rows(m, s)
    assert inb > 0 and over > 0
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    assert rel(_apply(m, X).cpu().numpy(), want) < TOL
    dt = np.complex64 if np.iscomplexobj(X) else np.float32
    assert rel(_apply(m, X.astype(dt), "f32").cpu().numpy(), want) < 2e-5


@pytest.mark.parametrize("k,nvec", [((0, 0, 0), 77), ((0.2, -0.1, 0.3), 45)])
def test_projector_update_ragged_lane_tiles_in_a_wider_buffer(k, nvec):
    """The FP64 projector update runs on the matrix cores over 64-lane tiles
    (a ragged last tile here: 77 real or 90 complex lanes) and over 16-row
    tiles of each node brick; crowded atoms give bricks of up to 64
    projectors.  The block sits in a wider buffer (ld = nvec + 3) whose
    padding columns must come back untouched, and a second application
    must give the same Y bit for bit."""
    s = inputs.make_custom(np.diag([10.0, 32.0 / 3.0, 28.0 / 3.0]), (4, 4, 4), 3, 4, kpoint=k, nvec=nvec,
                           seed=14, natoms=8, pset="spd", rc=3.0)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    Xd = to_dev(X)
    Xw = torch.full((m.ndofs, nvec + 3), 7.0, dtype=Xd.dtype, device="cuda:0")
    Xw[:, :nvec] = Xd
    Yw = torch.full_like(Xw, -3.0)
    m.apply(Xw[:, :nvec], Yw[:, :nvec], "f64")
    torch.cuda.synchronize()
    Y1 = Yw.cpu().numpy()
    assert rel(Y1[:, :nvec], want) < TOL
    for j in range(nvec):
        assert rel(Y1[:, j], want[:, j]) < TOL
    assert np.all(Y1[:, nvec:] == -3.0)
    m.apply(Xw[:, :nvec], Yw[:, :nvec], "f64")
    torch.cuda.synchronize()
    assert np.array_equal(Yw.cpu().numpy(), Y1)


@pytest.mark.parametrize("k,natoms,pset,p", [((0, 0, 0), 2, "sp", 2), ((0.3, -0.2, 0.1), 2, "spd", 3),
                                             ((0.2, 0.1, 0.4), 1, "sp", 5), ((0.0, 0.0, 0.0), 1, "s", 6),
                                             ((0.1, -0.3, 0.2), 1, "sp", 8)])
def test_accurate_quadrature_full_operator(k, natoms, pset, p):
    """The n_q = n_p + 2 rule (nine-pass kernel) against the oracle built with
    the same rule."""
    s = _small(k, natoms, pset, p=p, N=(3, 2, 3) if p > 5 else (3, 4, 3), nq=p + 3)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    assert rel(_apply(m, X).cpu().numpy(), want) < TOL
    dt = np.complex64 if np.iscomplexobj(X) else np.float32
    assert rel(_apply(m, X.astype(dt), "f32").cpu().numpy(), want) < 2e-5
    if p == 8:   # n_q = 11: the tuner keeps only the FP32 tiles whose LDS block fits
        best, times = m.autotune("f32", X.shape[1], reps=1)
        assert best in times and len(times) >= 1
        assert rel(_apply(m, X.astype(dt), "f32").cpu().numpy(), want) < 2e-5


def test_accurate_quadrature_brute_force_and_low_precision():
    s = _small((0.25, 0.1, 0.0), 1, "sp", N=(2, 3, 2), p=3, nq=6)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    H = op.assemble_H(om, vl, vg).toarray() + op.nonlocal_dense(P, h)
    got = _apply(m, np.eye(om.m, dtype=complex)).cpu().numpy()
    assert rel(got, H) < TOL
    X = inputs.make_vectors(s)
    y64 = _apply(m, X).cpu().numpy()
    assert rel(y64, H @ X) < TOL
    assert rel(_apply(m, X.astype(np.complex64), "f32").cpu().numpy(), y64) < 2e-5
    xb = torch.view_as_real(to_dev(X)).to(torch.bfloat16).contiguous()
    yb = torch.empty_like(xb)
    m.apply(xb, yb, "bf16")
    torch.cuda.synchronize()
    assert rel(torch.view_as_complex(yb.float().contiguous()).cpu().numpy(), y64) < 5e-2


@pytest.mark.parametrize("k,natoms,pset,p", [((0, 0, 0), 2, "sp", 2), ((0.3, -0.2, 0.1), 2, "spd", 3),
                                             ((0.2, 0.1, 0.4), 1, "sp", 6), ((0.1, -0.3, 0.2), 1, "sp", 8)])
def test_quadrature_np_plus_3_full_operator(k, natoms, pset, p):
    """n_q = n_p + 3 (the rule of the paper's quadrature-cost remark; at p = 8,
    n_q = 12, only the two-lane FP64 tile fits the LDS) against the oracle
    built with the same rule; FP32 to 2e-5; BF16 blocks are refused."""
    from paper_2512_08571_amd import fehx
    s = _small(k, natoms, pset, p=p, N=(3, 2, 3) if p > 5 else (3, 4, 3), nq=p + 4)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    assert rel(_apply(m, X).cpu().numpy(), want) < TOL
    if p == 8:
        best, times = m.autotune("f64", X.shape[1], reps=1)
        assert best == 2 and times[2] > 0 and all(times[v] < 0 for v in (4, 8, 16))
        assert rel(_apply(m, X).cpu().numpy(), want) < TOL
    dt = np.complex64 if np.iscomplexobj(X) else np.float32
    assert rel(_apply(m, X.astype(dt), "f32").cpu().numpy(), want) < 2e-5
    xb = to_dev(X.real.astype(np.float32)).to(torch.bfloat16) if not np.iscomplexobj(X) else \
        torch.view_as_real(to_dev(X)).to(torch.bfloat16).contiguous()
    with pytest.raises(fehx.FeError) as e:
        m.apply(xb, torch.empty_like(xb), "bf16")
    assert e.value.code == -5


@pytest.mark.parametrize("k,p", [((0, 0, 0), 4), ((0.3, -0.2, 0.1), 4), ((0, 0, 0), 6), ((0.2, 0.1, 0.4), 6),
                                 ((0, 0, 0), 7), ((0.1, 0.2, -0.3), 7)])
def test_every_fp64_tile_against_the_oracle(k, p):
    """Every FP64 tile that fits at n_q = n_p (the ten-lane tile included),
    real and complex, on the line-gather path (n_p 5, 7, real 8) and the
    staged path (complex n_p = 8): each against the assembled oracle, and all
    bit-identical."""
    s = _small(k, 2, "spd", p=p, N=(3, 2, 3) if p > 5 else (3, 4, 3), nvec=12)
    om, vl, vg, P, h = oracle_side(s)
    m = lib_side(s, vl, vg)
    X = inputs.make_vectors(s)
    want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
    _, times = m.autotune("f64", s.nvec, kind=0, reps=1)
    tiles = sorted(t for t, ms in times.items() if ms > 0)   # the tiles whose block fits the LDS
    assert {4, 8, 10} <= set(tiles), times
    outs = []
    for vt in tiles:
        m.set_tile("f64", vt)
        Y = _apply(m, X)
        torch.cuda.synchronize()
        assert rel(Y.cpu().numpy(), want) < TOL, vt
        outs.append(Y)
    for Y in outs[1:]:
        assert torch.equal(Y, outs[0])
    m.set_tile("f64", 0)
