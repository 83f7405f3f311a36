"""Pins for oracle.operator against closed forms, invariants and special cases."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis
from oracle import operator as op
from oracle.mesh import Mesh

SHEARED = np.array([[3.0, 0.0, 0.0], [0.8, 2.5, 0.0], [0.4, -0.6, 3.5]])


# ---- polynomial exactness on one open (non-periodic) sheared cell -------
def _poly(rng, deg):
    """Random polynomial of total degree <= deg in physical x: (coef, exps)."""
    exps = [e for e in itertools.product(range(deg + 1), repeat=3) if sum(e) <= deg]
    return rng.standard_normal(len(exps)), np.array(exps)


def _peval(pc, x):
    c, e = pc
    return np.prod(x[:, None, :] ** e[None, :, :], axis=2) @ c


def _pgrad(pc, x):
    c, e = pc
    g = np.zeros((len(x), 3))
    for a in range(3):
        ea = e.copy()
        fac = ea[:, a].astype(float)
        ea[:, a] = np.maximum(ea[:, a] - 1, 0)
        g[:, a] = np.prod(x[:, None, :] ** ea[None, :, :], axis=2) @ (c * fac)
    return g


def _exact_integral(mesh, f, n=14):
    """int over the single cell of f(x) by an n^3 Gauss rule (exact for these polynomials)."""
    xq, wq = basis.gauss_points_weights(n)
    ref = np.stack(np.meshgrid(xq, xq, xq, indexing="ij"), -1).reshape(-1, 3)
    w = np.einsum("i,j,k->ijk", wq, wq, wq).reshape(-1)
    x = (ref + 1.0) @ mesh.J.T
    return np.sum(w * f(x)) * mesh.detJ


@pytest.mark.parametrize("p", [2, 3, 4])
def test_cell_matrices_integrate_polynomials(p):
    rng = np.random.default_rng(p)
    k = np.array([0.3, -0.2, 0.5])
    m = Mesh(SHEARED, (1, 1, 1), p, p + 1, kpoint=k, periodic=(False, False, False))
    xn = m.node_coords()
    u, v = _poly(rng, p), _poly(rng, p)
    U, V = _peval(u, xn), _peval(v, xn)
    # linear potential and linear GGA field: integrands of degree <= 2p+1 per variable
    a0, a1 = rng.standard_normal(), rng.standard_normal(3)
    B0, B1 = rng.standard_normal(3), rng.standard_normal((3, 3))
    xq = m.quad_points()
    vloc = a0 + xq @ a1
    vg = B0[None, :] + xq @ B1.T
    He = op.element_matrices(m, vloc, vg)[0]
    dofs = m.cell_dofs()[0]
    got = U[dofs] @ He @ V[dofs]

    def integrand(x):
        gu, gv = _pgrad(u, x), _pgrad(v, x)
        uu, vv = _peval(u, x), _peval(v, x)
        VL = a0 + x @ a1 + 0.5 * k @ k
        VG = B0[None, :] + x @ B1.T
        kin = 0.5 * np.sum(gu * gv, 1)
        gga = np.sum(VG * (gu * vv[:, None] + uu[:, None] * gv), 1)
        return kin + VL * uu * vv + gga - 1j * (uu * (gv @ k))

    want = _exact_integral(m, integrand)
    assert abs(got - want) < 1e-11 * max(1.0, abs(want))
    Me = op.mass_element(m)
    want_m = _exact_integral(m, lambda x: _peval(u, x) * _peval(v, x))
    assert abs(U[dofs] @ Me @ V[dofs] - want_m) < 1e-12 * max(1.0, abs(want_m))


def test_element_rows_match_element_matrices():
    m = Mesh(SHEARED, (2, 2, 2), 3, 4, kpoint=(0.2, 0.1, -0.3))
    rng = np.random.default_rng(1)
    vl = rng.standard_normal(m.E * 64)
    vg = rng.standard_normal((m.E * 64, 3))
    He = op.element_matrices(m, vl, vg, [1, 6])
    rows = op.element_rows(m, vl, vg, [1, 6], [7, 50])
    assert np.abs(He[0, 7] - rows[0]).max() < 1e-14
    assert np.abs(He[1, 50] - rows[1]).max() < 1e-14


# ---- periodic invariants ---------------------------------------------------
def _periodic(k=(0.0, 0.0, 0.0), p=3, N=(3, 2, 3), lat=SHEARED):
    return Mesh(lat, N, p, p + 1, kpoint=k)


def test_periodic_invariants():
    m = _periodic(k=(0.3, -0.4, 0.25))
    nq = m.E * m.nq ** 3
    one = np.ones(m.m)
    Mm = op.assemble_M(m)
    assert abs(one @ Mm @ one - m.volume) < 1e-12 * m.volume
    assert abs(op.lumped_mass(m).sum() - m.volume) < 1e-12 * m.volume
    assert np.all(sla.eigvalsh(Mm.toarray()) > 0)
    # T 1 = 0;  with V = 0 and no GGA:  H = T + |k|^2/2 M - i K
    Hk = op.assemble_H(m, np.zeros(nq)).toarray()
    K = (Hk - (op.assemble_H(_periodic(p=3), np.zeros(nq)).toarray()
               + 0.5 * (m.k @ m.k) * Mm.toarray())) * 1j
    T = op.assemble_H(_periodic(p=3), np.zeros(nq)).toarray()
    assert np.abs(T @ one).max() < 1e-12
    assert np.abs(K + K.T).max() < 1e-12           # K antisymmetric
    assert np.abs(K @ one).max() < 1e-12
    assert np.abs(K.imag).max() < 1e-12
    # constant V^L = c gives L = c M;  constant V^G gives G = 0
    m0 = _periodic()
    c = 0.7
    HL = op.assemble_H(m0, np.full(nq, c)).toarray() - T
    assert np.abs(HL - c * Mm.toarray()).max() < 1e-12
    HG = op.assemble_H(m0, np.zeros(nq), np.tile([0.3, -1.1, 0.5], (nq, 1))).toarray() - T
    assert np.abs(HG).max() < 1e-12


def test_hermitian_with_all_terms():
    m = _periodic(k=(0.21, 0.13, -0.4))
    rng = np.random.default_rng(3)
    nq = m.E * m.nq ** 3
    H = op.assemble_H(m, rng.standard_normal(nq), rng.standard_normal((nq, 3))).toarray()
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()


# ---- free electrons: Kronecker-sum exactness and convergence ----------------
def _fe_1d(L, N, p, k):
    """1D periodic FE matrices assembled directly: kinetic, mass, N N' and GLL-lumped mass."""
    xg, wg = basis.gll_nodes_weights(p)
    xq, wq = basis.gauss_points_weights(p + 1)
    Nv = basis.lagrange_values(xg, xq)
    Dv = basis.lagrange_derivatives(xg, xq)
    h = L / N
    jac = h / 2.0
    m = N * p
    K1 = np.zeros((m, m)); M1 = np.zeros((m, m)); C1 = np.zeros((m, m)); D1 = np.zeros(m)
    for c in range(N):
        idx = (c * p + np.arange(p + 1)) % m
        dphys = Dv / jac
        K1[np.ix_(idx, idx)] += (dphys * wq[:, None]).T @ dphys * jac
        M1[np.ix_(idx, idx)] += (Nv * wq[:, None]).T @ Nv * jac
        C1[np.ix_(idx, idx)] += (Nv * wq[:, None]).T @ dphys * jac
        np.add.at(D1, idx, wg * jac)
    return 0.5 * K1 + 0.5 * k * k * M1 - 1j * k * C1, M1, np.diag(D1)


def test_free_electron_kronecker_sum():
    """With V = 0 the consistent-mass GHEP is a Kronecker sum of 1D problems.

    (With the lumped D it is not: H keeps consistent 1D masses in the
    transverse directions, so only the consistent M gives exact separation.)
    """
    L, N, p = 6.0, 3, 3
    k = np.array([0.31, -0.17, 0.05])
    m = Mesh(np.eye(3) * L, (N, N, N), p, p + 1, kpoint=k)
    H = op.assemble_H(m, np.zeros(m.E * m.nq ** 3)).toarray()
    B = op.assemble_M(m).toarray()
    lam3 = sla.eigvalsh(H, B)
    mus = []
    for d in range(3):
        h1, M1, D1 = _fe_1d(L, N, p, k[d])
        mus.append(sla.eigvalsh(h1, M1))
    want = np.sort(np.add.outer(np.add.outer(mus[0], mus[1]), mus[2]).reshape(-1))
    assert np.abs(np.sort(lam3) - want).max() < 1e-10


def test_free_electron_1d_convergence_and_degeneracy():
    L, p, k = 8.0, 2, 0.2
    exact = np.sort([0.5 * (k + 2 * np.pi * n / L) ** 2 for n in range(-2, 3)])
    errs = []
    for N in (8, 16):
        h1, M1, _ = _fe_1d(L, N, p, k)
        lam = sla.eigvalsh(h1, M1)[:5]
        errs.append(np.abs(lam - exact))
    assert errs[0][0] < 1e-13          # the constant Bloch state is represented exactly
    rate = errs[0][1:] / errs[1][1:]
    assert np.all(np.abs(rate / 2 ** (2 * p) - 1.0) < 0.2)
    # 3D Gamma point, L = 8: 0 (x1), (2 pi/8)^2/2 (x6), 2x (x12), 3x (x8)
    m = Mesh(np.eye(3) * L, (4, 4, 4), 4, 5)
    H = op.assemble_H(m, np.zeros(m.E * 125)).toarray()
    lam = sla.eigvalsh(H, op.assemble_M(m).toarray())[:27]
    e1 = 0.5 * (2 * np.pi / L) ** 2
    want = np.array([0] + [e1] * 6 + [2 * e1] * 12 + [3 * e1] * 8)
    assert np.abs(lam - want).max() < 2e-4


# ---- the three application routes agree -----------------------------------
def test_apply_routes_agree():
    m = _periodic(k=(0.1, 0.3, -0.2), p=2, N=(3, 3, 2))
    rng = np.random.default_rng(7)
    nq = m.E * m.nq ** 3
    vl, vg = rng.standard_normal(nq), rng.standard_normal((nq, 3))
    X = rng.standard_normal((m.m, 3)) + 1j * rng.standard_normal((m.m, 3))
    Hs = op.assemble_H(m, vl, vg)
    ys = op.apply_sparse(Hs, X)
    yc = op.apply_cm(m, vl, vg, X)
    rows = rng.integers(0, m.m, 25)
    yr = op.apply_rows(m, vl, vg, X, rows)
    assert np.abs(ys - yc).max() < 1e-13 * np.abs(ys).max()
    assert np.abs(ys[rows] - yr).max() < 1e-13 * np.abs(ys).max()


@pytest.mark.parametrize("periodic,L", [((False, False, False), (4.0, 5.0, 6.0)), ((True, True, False), (3.0, 3.5, 5.0))])
def test_dirichlet_restriction_lowest_eigenvalues(periodic, L):
    """Homogeneous Dirichlet faces (the open mesh restricted to interior
    nodes): the lowest eigenvalues of T u = eps M u approach the continuum
    box values 1/2 pi^2 sum_d (n_d / L_d)^2 (n_d >= 1 on Dirichlet axes, the
    plane-wave values (2 pi j / L)^2 / 2 on periodic ones) at spectral rate."""
    m = Mesh(np.diag(L), (3, 3, 3), 6, 7, periodic=periodic)
    idx = m.dirichlet_dofs()
    assert len(idx) == np.prod([m.N[d] * m.p + (0 if periodic[d] else -1) for d in range(3)])
    T = op.assemble_H(m, np.zeros(m.E * m.nq ** 3))[idx][:, idx].toarray()
    M = op.assemble_M(m)[idx][:, idx].toarray()
    got = sla.eigvalsh(T, M)[:4]
    vals = []
    for a in range(0, 4):
        for b in range(0, 4):
            for c in range(0, 4):
                e = 0.0
                for d, n in enumerate((a, b, c)):
                    if periodic[d]:
                        # plane waves cos/sin pairs: each j > 0 twice
                        e += 0.5 * (2 * np.pi * ((n + 1) // 2) / L[d]) ** 2
                    else:
                        e += 0.5 * (np.pi * (n + 1) / L[d]) ** 2
                vals.append(e)
    want = np.sort(vals)[:4]
    assert np.abs(got - want).max() < 1e-6 * want.max()


# ---- the lumped mass D (Sec. 5.3: the mass under the GLL rule on the nodes) --
def test_lumped_mass_closed_form_p4():
    """At p = 4 the 1D GLL weights are 1/10, 49/90, 32/45, 49/90, 1/10.  On a
    periodic orthorhombic mesh a node with g_d = 0 (mod p) along axis d is a
    cell-boundary node shared by the two cells along d (1D factor 2/10); any
    other node sits at local index g_d mod p of one cell (factor w_{g_d mod p}).
    So D at node g is det J times the product of the three 1D factors."""
    L, N = (5.0, 6.0, 7.0), (3, 2, 3)
    m = Mesh(np.diag(L), N, 4, 5)
    D = op.lumped_mass(m)
    w1 = {0: 2.0 / 10.0, 1: 49.0 / 90.0, 2: 32.0 / 45.0, 3: 49.0 / 90.0}
    detJ = np.prod([L[d] / (2.0 * N[d]) for d in range(3)])
    idx = np.arange(m.m)
    g = [idx % m.M[0], (idx // m.M[0]) % m.M[1], idx // (m.M[0] * m.M[1])]
    want = detJ * np.prod([np.vectorize(w1.get)(g[d] % 4) for d in range(3)], axis=0)
    assert np.abs(D - want).max() < 1e-14 * want.max()
    # spot values named in closed form: a cell corner and a cell centre
    corner = 0
    centre = 2 + m.M[0] * (2 + m.M[1] * 2)
    assert abs(D[corner] - 8 * (1 / 10) ** 3 * detJ) < 1e-15 * detJ
    assert abs(D[centre] - (32 / 45) ** 3 * detJ) < 1e-15 * detJ


@pytest.mark.parametrize("p", [2, 4, 6])
def test_lumped_mass_is_gll_quadrature_mass(p):
    """D equals the mass matrix assembled with the n_p-point GLL rule: the
    shape functions evaluated at the GLL points (product formula) times the
    GLL weights and det J, assembled over the cells.  That matrix is diagonal
    because l_i(x_j) = delta_ij; its diagonal must be D (sheared periodic box)."""
    m = Mesh(SHEARED, (3, 2, 2), p, p + 1)
    xg, wg = basis.gll_nodes_weights(p)
    N1 = basis.lagrange_values(xg, xg)                          # [point, node]
    N3 = np.einsum("ai,bj,ck->cbakji", N1, N1, N1).reshape((p + 1) ** 3, (p + 1) ** 3)
    W = np.einsum("a,b,c->cba", wg, wg, wg).reshape(-1) * m.detJ
    Me = (N3 * W[:, None]).T @ N3
    Mg = op._assemble(m, Me).toarray()
    D = op.lumped_mass(m)
    assert np.abs(Mg - np.diag(np.diag(Mg))).max() < 1e-13 * D.max()
    assert np.abs(np.diag(Mg) - D).max() < 1e-13 * D.max()


@pytest.mark.parametrize("p", [2, 3, 5])
def test_lumped_mass_integrates_polynomials(p):
    """The n_p-point GLL rule integrates polynomials of degree <= 2p - 1 per
    variable exactly, so on one open (sheared) cell sum_I D_I f(x_I) equals
    int f for every such f; a Gauss weight or a misplaced node breaks it."""
    rng = np.random.default_rng(10 + p)
    m = Mesh(SHEARED, (1, 1, 1), p, p + 1, periodic=(False, False, False))
    D = op.lumped_mass(m)
    xn = m.node_coords()
    deg = 2 * p - 1
    exps = np.array([e for e in itertools.product(range(deg + 1), repeat=3) if sum(e) <= deg])
    c = rng.standard_normal(len(exps))
    f = lambda x: np.prod(x[:, None, :] ** exps[None, :, :], axis=2) @ c
    want = _exact_integral(m, f, n=p + 2)
    assert abs(D @ f(xn) - want) < 1e-11 * max(1.0, abs(want))


def test_cm_operator_batches_equal_assembled():
    """The batched cell-matrix operator (sparse scatter) against the assembled
    sparse product, with every term and projectors, batches that split the
    cells unevenly."""
    m = _periodic(k=(0.1, 0.3, -0.2), p=2, N=(3, 3, 2))
    rng = np.random.default_rng(17)
    nq = m.E * m.nq ** 3
    vl, vg = rng.standard_normal(nq), rng.standard_normal((nq, 3))
    pos = rng.uniform(0, 1, (2, 3)) @ m.A
    projs = [dict(atom=a, l=1, m=mm, sigma=0.5, rc=1.4, h=0.7 - 0.3 * mm) for a in range(2) for mm in range(3)]
    P, h = op.projector_matrix(m, pos, projs)
    X = rng.standard_normal((m.m, 3)) + 1j * rng.standard_normal((m.m, 3))
    want = op.apply_sparse(op.assemble_H(m, vl, vg), X, P, h)
    got = op.cm_operator(m, vl, vg, P, h, batch=5)(X)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
