"""Seeded synthetic inputs for the FE Kohn-Sham H.X workloads.

This module only draws random numbers and evaluates the synthetic input
fields at points it is given; it holds none of the finite-element method
(no basis, quadrature, mesh map or operator).  The same arrays feed the CPU
oracle and the library, so both sides see identical inputs.

Workloads (sizes in bohr / Hartree):

* ``tiny``    periodic cube L = 8, 4^3 cells, degree 4, 5 Gauss points, Gamma
              point; V_eff = 4 Gaussians (depth U[-2, -0.5], width 1) at
              U[0, L)^3 centres; 8 vectors U[-1, 1].
* ``mid``     periodic cube L = 20, 16^3 cells, degree 6, 7 Gauss points,
              Gamma point, real; V_eff = one Gaussian per atom; GGA field
              V^G (three smooth positive periodic components); 32 atoms with
              4 projectors (s, p), cutoff 3 bohr, couplings U[-1, 1];
              256 vectors U[-1, 1].
* ``complex`` periodic cube L = 28, 24^3 cells, degree 7, 8 Gauss points,
              k = (0.25, 0.1, 0) 2 pi / L; fields as ``mid``; 128 atoms with
              9 projectors (s, p, d), cutoff 3.5; 512 complex vectors with
              independent U[-1, 1] real and imaginary parts.
* ``filter``  the ``mid`` mesh and operator, 512 vectors (start block and
              Lanczos start vector from their own seed).

Draw order for every system: atom / Gaussian centres, then depths and
couplings, then field coefficients; vectors come from per-column generators
so that any column subset can be drawn without drawing the rest.
"""
import itertools
import math
from dataclasses import dataclass, field

import numpy as np

SEEDS = {"tiny": 0, "mid": 1, "complex": 2, "filter": 3}

# real solid harmonics per angular momentum: (l, m) pairs, m = 0 .. 2l
PROJ_SETS = {"s": [(0, 0)],
             "sp": [(0, 0), (1, 0), (1, 1), (1, 2)],
             "spd": [(0, 0), (1, 0), (1, 1), (1, 2),
                     (2, 0), (2, 1), (2, 2), (2, 3), (2, 4)]}


@dataclass
class System:
    name: str
    lattice: np.ndarray              # rows are the box vectors
    ncell: tuple
    degree: int
    nq: int
    kpoint: np.ndarray
    nvec: int
    seed: int
    centres: np.ndarray              # Gaussian centres of V_eff
    depths: np.ndarray
    width: float = 1.0
    gga_coef: np.ndarray = None      # [3 comps, 26 wavevectors, 2] or None
    atoms: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    projectors: list = field(default_factory=list)   # dicts atom,l,m,sigma,rc,h

    @property
    def is_complex(self):
        return bool(np.any(self.kpoint != 0.0))

    @property
    def ndofs(self):
        return int(np.prod([n * self.degree for n in self.ncell]))

    @property
    def volume(self):
        return abs(float(np.linalg.det(self.lattice)))


_WAVEVECTORS = np.array([n for n in itertools.product((-1, 0, 1), repeat=3) if any(n)], float)


def _gga_coefficients(rng):
    return rng.standard_normal((3, len(_WAVEVECTORS), 2))


def _projectors(rng, natoms, pset, rc):
    lm = PROJ_SETS[pset]
    h = rng.uniform(-1.0, 1.0, (natoms, len(lm)))
    out = []
    for a in range(natoms):
        for s, (l, m) in enumerate(lm):
            out.append(dict(atom=a, l=l, m=m, sigma=rc / 3.0, rc=rc, h=float(h[a, s])))
    return out


def make_system(name, seed=None):
    """The named workload; ``seed`` overrides its default seed."""
    seed = SEEDS[name] if seed is None else seed
    rng = np.random.default_rng(seed)
    if name == "tiny":
        L = 8.0
        centres = rng.uniform(0.0, L, (4, 3))
        depths = rng.uniform(-2.0, -0.5, 4)
        return System(name, np.eye(3) * L, (4, 4, 4), 4, 5, np.zeros(3), 8, seed,
                      centres, depths)
    if name in ("mid", "filter"):
        rng = np.random.default_rng(SEEDS["mid"] if seed == SEEDS.get(name) else seed)
        L = 20.0
        atoms = rng.uniform(0.0, L, (32, 3))
        depths = rng.uniform(-2.0, -0.5, 32)
        projs = _projectors(rng, 32, "sp", 3.0)
        gga = _gga_coefficients(rng)
        nvec = 256 if name == "mid" else 512
        return System(name, np.eye(3) * L, (16, 16, 16), 6, 7, np.zeros(3), nvec, seed,
                      atoms.copy(), depths, 1.0, gga, atoms, projs)
    if name == "complex":
        L = 28.0
        atoms = rng.uniform(0.0, L, (128, 3))
        depths = rng.uniform(-2.0, -0.5, 128)
        projs = _projectors(rng, 128, "spd", 3.5)
        gga = _gga_coefficients(rng)
        k = np.array([0.25, 0.1, 0.0]) * 2.0 * np.pi / L
        return System(name, np.eye(3) * L, (24, 24, 24), 7, 8, k, 512, seed,
                      atoms.copy(), depths, 1.0, gga, atoms, projs)
    raise KeyError(name)


def make_custom(lattice, ncell, degree, nq, kpoint=(0, 0, 0), nvec=8, seed=0,
                ngauss=4, natoms=0, pset="sp", rc=3.0, gga=True, name="custom"):
    """A small system of the same recipe (for parity cases and serving requests)."""
    rng = np.random.default_rng(seed)
    A = np.asarray(lattice, float).reshape(3, 3)
    nat = max(natoms, 0)
    atoms = rng.uniform(0.0, 1.0, (nat, 3)) @ A
    centres = atoms.copy() if nat else rng.uniform(0.0, 1.0, (ngauss, 3)) @ A
    depths = rng.uniform(-2.0, -0.5, len(centres))
    projs = _projectors(rng, nat, pset, rc) if nat else []
    coef = _gga_coefficients(rng) if gga else None
    return System(name, A, tuple(int(n) for n in ncell), int(degree), int(nq),
                  np.asarray(kpoint, float), int(nvec), seed, centres, depths, 1.0,
                  coef, atoms, projs)


# --- field evaluation at given points --------------------------------------
def _min_spacing(A):
    """Smallest distance between opposite faces of the box."""
    vol = abs(np.linalg.det(A))
    return min(vol / np.linalg.norm(np.cross(A[(i + 1) % 3], A[(i + 2) % 3])) for i in range(3))


def eval_vloc(sysm, points, chunk=1 << 20):
    """V_eff(x) = sum_c d_c sum_r exp(-|x - c - L_r|^2 / (2 w^2)), r in {-1,0,1}^3.

    When every box face pair is more than 20 w apart only the minimum image
    is summed: the other images add less than exp(-50) relative, below
    double-precision resolution.
    """
    A = np.asarray(sysm.lattice, float)
    pts = np.asarray(points, float).reshape(-1, 3)
    out = np.zeros(len(pts))
    w2 = 2.0 * sysm.width ** 2
    full = _min_spacing(A) < 20.0 * sysm.width
    Ainv = np.linalg.inv(A)
    images = np.array(list(itertools.product((-1, 0, 1), repeat=3)), float) @ A
    for s in range(0, len(pts), chunk):
        x = pts[s:s + chunk]
        acc = np.zeros(len(x))
        for c, d in zip(sysm.centres, sysm.depths):
            disp = x - c
            if full:
                for Lr in images:
                    r = disp - Lr
                    acc += d * np.exp(-np.einsum("ij,ij->i", r, r) / w2)
            else:
                f = disp @ Ainv
                r = (f - np.round(f)) @ A
                acc += d * np.exp(-np.einsum("ij,ij->i", r, r) / w2)
        out[s:s + chunk] = acc
    return out


def eval_vgga(sysm, points, chunk=1 << 20):
    """V^G_d(x) = 0.1 exp(s_d(x)), s_d = 0.5 / sqrt(26) sum_n (a cos + b sin)(2 pi n.f).

    f are the fractional coordinates of x; n runs over {-1,0,1}^3 minus 0.
    Returns [npoints, 3] or None when the system has no GGA term.
    """
    if sysm.gga_coef is None:
        return None
    A = np.asarray(sysm.lattice, float)
    pts = np.asarray(points, float).reshape(-1, 3)
    Ainv = np.linalg.inv(A)
    out = np.zeros((len(pts), 3))
    coef = sysm.gga_coef
    for s in range(0, len(pts), chunk):
        f = pts[s:s + chunk] @ Ainv
        ph = 2.0 * np.pi * (f @ _WAVEVECTORS.T)              # [n, 26]
        c, sn = np.cos(ph), np.sin(ph)
        for d in range(3):
            sd = (c @ coef[d, :, 0] + sn @ coef[d, :, 1]) * (0.5 / math.sqrt(26.0))
            out[s:s + chunk, d] = 0.1 * np.exp(sd)
    return out


def positions_array(sysm):
    return np.ascontiguousarray(np.asarray(sysm.atoms, float).reshape(-1, 3))


# --- vectors ----------------------------------------------------------------
def make_vectors(sysm, cols=None, seed_offset=0, ndofs=None):
    """X[:, j] ~ U[-1, 1] (complex: independent real and imaginary parts).

    Column j comes from its own generator keyed by (seed, j), so a subset of
    columns is drawn without the rest.  Returns a C-contiguous [m, ncols] array.
    """
    m = sysm.ndofs if ndofs is None else ndofs
    cols = range(sysm.nvec) if cols is None else cols
    cols = list(cols)
    dt = complex if sysm.is_complex else float
    X = np.empty((m, len(cols)), dtype=dt)
    for t, j in enumerate(cols):
        rng = np.random.default_rng([sysm.seed, 1000 + seed_offset, int(j)])
        if sysm.is_complex:
            X[:, t] = rng.uniform(-1.0, 1.0, m) + 1j * rng.uniform(-1.0, 1.0, m)
        else:
            X[:, t] = rng.uniform(-1.0, 1.0, m)
    return X


def lanczos_start(sysm, seed_offset=0, ndofs=None):
    m = sysm.ndofs if ndofs is None else ndofs
    rng = np.random.default_rng([sysm.seed, 2000 + seed_offset])
    v = rng.uniform(-1.0, 1.0, m)
    if sysm.is_complex:
        v = v + 1j * rng.uniform(-1.0, 1.0, m)
    return v


# --- serving stream ------------------------------------------------------------
SERVE_SEED0 = 100


def make_serving_stream(run=0, n=64):
    """The request stream of the serving workload: n random periodic systems.

    Cubic meshes of 6..20 cells per axis with h = 1.25 bohr (L = 1.25 N),
    degree p in {5, 6, 7, 8} (n_q = p + 1), nvec log-uniform in 32..512,
    8..64 atoms with s+p (4 projectors, r_c = 3) or s+p+d (9 projectors,
    r_c = 3.5) and couplings U[-1, 1]; half the systems real (Gamma point),
    half complex with k = u 2 pi / L, u ~ U[-0.5, 0.5]^3.  Seeded by
    SERVE_SEED0 + run; every system also carries its own seed for its fields
    and vectors.
    """
    rng = np.random.default_rng(SERVE_SEED0 + run)
    out = []
    for i in range(n):
        N = int(rng.integers(6, 21))
        p = int(rng.choice([5, 6, 7, 8]))
        nvec = int(np.exp(rng.uniform(np.log(32), np.log(512))) + 0.5)
        natoms = int(rng.integers(8, 65))
        spd = bool(rng.integers(0, 2))
        cplx = bool(rng.integers(0, 2))
        L = 1.25 * N
        k = rng.uniform(-0.5, 0.5, 3) * 2.0 * np.pi / L if cplx else np.zeros(3)
        seed = int(rng.integers(0, 2 ** 31))
        out.append(make_custom(np.eye(3) * L, (N, N, N), p, p + 1, kpoint=k, nvec=nvec, seed=seed,
                               natoms=natoms, pset="spd" if spd else "sp", rc=3.5 if spd else 3.0,
                               name=f"serve{run}_{i}"))
    return out


def eval_serving_fields(sysm, points):
    """Cheap smooth periodic fields for the serving stream (O(points)).

    V_eff(x) = -1 + sum_d 0.5 a_d cos(2 pi x_d / L_d + phi_d) and
    V^G_d(x) = 0.1 exp(0.5 b_d sin(2 pi x_d / L_d + psi_d)), with a, b ~ U[0.5, 1]
    and phases U[0, 2 pi) from the system's seed: the scheduling workload only
    needs fields of the right structure, and the Gaussian sums of the other
    workloads cost minutes on the largest serving meshes.
    """
    rng = np.random.default_rng([sysm.seed, 77])
    a, b = rng.uniform(0.5, 1.0, 3), rng.uniform(0.5, 1.0, 3)
    phi, psi = rng.uniform(0, 2 * np.pi, 3), rng.uniform(0, 2 * np.pi, 3)
    Ld = np.diag(sysm.lattice)
    t = 2.0 * np.pi * np.asarray(points) / Ld[None, :]
    v = -1.0 + 0.5 * (a[None, :] * np.cos(t + phi[None, :])).sum(axis=1)
    g = 0.1 * np.exp(0.5 * b[None, :] * np.sin(t + psi[None, :]))
    return v, g


def vertex_displacement(ncell, lattice, amp, seed):
    """A seeded smooth periodic displacement of the cell vertices, [N0 N1 N2, 3]
    in vertex order i + N0 (j + N1 k): amp times the cell size times a sum of
    the 26 lowest Fourier modes (n in {-1, 0, 1}^3 without 0) with N(0, 1)
    cosine and sine amplitudes per component, over sqrt(26).  The cells stay
    well shaped for amp up to about 0.2."""
    N = np.asarray(ncell)
    A = np.asarray(lattice, float)
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(N[0]), np.arange(N[1]), np.arange(N[2]), indexing="ij"), -1)
    g = g.transpose(2, 1, 0, 3).reshape(-1, 3) / N[None, :]
    h = np.min(np.linalg.norm(A, axis=1) / N)
    out = np.zeros((len(g), 3))
    for n in itertools.product((-1, 0, 1), repeat=3):
        if n == (0, 0, 0):
            continue
        ph = 2.0 * np.pi * g @ np.array(n, float)
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        out += np.cos(ph)[:, None] * a[None, :] + np.sin(ph)[:, None] * b[None, :]
    return amp * h * out / np.sqrt(26.0)
