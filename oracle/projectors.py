"""Analytic nonlocal projector functions (oracle; test infrastructure).

Eqn Vnonloc / eq nlps: the nonlocal term is built from compactly supported
atom-centred projectors chi_{lpm}(x, R_a + L_r) and coupling constants h.  The
paper leaves the radial form to the pseudopotential; the reading used here is

    chi_{lm}(r) = S_lm(r) * exp(-rho^2 / (2 sigma^2)) * (1 - rho^2 / r_c^2)^2,
                  rho = |r| < r_c,   zero outside,

with the unnormalised real solid harmonics S_lm indexed m = 0 .. 2l:
    l = 0: 1
    l = 1: x, y, z
    l = 2: xy, yz, zx, x^2 - y^2, 3 z^2 - rho^2
The image sum over r in {-1, 0, 1}^3 and the Bloch factor
exp(-i k.(x - L_r)) follow eqn Vnonloc.

Pins (tests/test_oracle_nonlocal.py): the s-projector integral against a 1D
radial quadrature, the symmetric vanishing of p- and d-integrals, the lattice
translation covariance P(R + L) = exp(-i k.L) P(R).
"""
import itertools

import numpy as np


def solid_harmonic(l, m, r):
    x, y, z = r[..., 0], r[..., 1], r[..., 2]
    if l == 0 and m == 0:
        return np.ones_like(x)
    if l == 1:
        return (x, y, z)[m]
    if l == 2:
        rho2 = x * x + y * y + z * z
        return (x * y, y * z, z * x, x * x - y * y, 3.0 * z * z - rho2)[m]
    raise ValueError("only l <= 2 projectors are defined")


def chi(l, m, r, sigma, rc):
    """chi_{lm}(r) for displacement vectors r[..., 3]."""
    rho2 = np.sum(r * r, axis=-1)
    inside = rho2 < rc * rc
    radial = np.where(inside,
                      np.exp(-rho2 / (2.0 * sigma * sigma)) * (1.0 - rho2 / (rc * rc)) ** 2,
                      0.0)
    return solid_harmonic(l, m, r) * radial


def bloch_chi(l, m, x, R, A, k, sigma, rc, images=1, periodic=(True, True, True)):
    """sum_r chi(x - R - L_r) exp(-i k.(x - L_r)) over r in {-images..images}^3.

    The lattice translations L_r exist only along periodic axes: r_d = 0 on an
    open axis.

    With the atom inside the box and r_c below half the smallest face spacing
    the default 27 images hold every nonzero term for points in the box.
    Returns a complex array for k != 0, a real array for k == 0.
    """
    k = np.asarray(k, float)
    cplx = bool(np.any(k != 0.0))
    out = np.zeros(x.shape[:-1], dtype=complex if cplx else float)
    rngs = [range(-images, images + 1) if periodic[d] else range(0, 1) for d in range(3)]
    lo = x.reshape(-1, 3).min(axis=0)
    hi = x.reshape(-1, 3).max(axis=0)
    for r in itertools.product(*rngs):
        L = np.asarray(r, float) @ A
        c = R + L
        # chi vanishes beyond r_c: an image farther than r_c from the points'
        # bounding box contributes exactly zero and is skipped
        if np.linalg.norm(np.maximum(np.maximum(lo - c, c - hi), 0.0)) >= rc:
            continue
        val = chi(l, m, x - R - L, sigma, rc)
        if cplx:
            out = out + val * np.exp(-1j * ((x - L) @ k))
        else:
            out = out + val
    return out
