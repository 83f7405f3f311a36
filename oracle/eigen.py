"""Eigensolver pieces around H.X (oracle; test infrastructure, float64/complex128).

Alg. 4 (R-ChFSI filter for H X = M X Lambda): the residual form of the scaled
Chebyshev filter, exactly in the paper's order and notation:
    e = (lmax - lT)/2, c = (lmax + lT)/2, sigma = e / (lmin - c), sigma1 = sigma,
    gamma = 2 / sigma1
    Y = H X - M X Lambda;   R_X = 0;   R_Y = (sigma1/e) Y
    Lambda_X = I;  Lambda_Y = (sigma1/e)(Lambda - c I)
    for k = 2..p:
        sigma2 = 1 / (gamma - sigma)
        R_X = (2 sigma2/e)[(H D^-1 - c I) R_Y + Y Lambda_Y] - sigma sigma2 R_X
        Lambda_X = (2 sigma2/e) Lambda_Y (Lambda - c I) - sigma sigma2 Lambda_X
        swap(R_X, R_Y); swap(Lambda_X, Lambda_Y); sigma = sigma2
    return D^-1 R_Y + X Lambda_Y
Alg. 3: Rayleigh-Ritz on the filtered block, (Y^H H Y) E = (Y^H M Y) E Lambda.

Readings (where the paper is silent): M is taken as the GLL-lumped D inside
the filter driver; the spectral bounds come from a 10-step Lanczos run on
D^-1/2 H D^-1/2 with full reorthogonalisation (lmax = largest Ritz value +
|last beta|); the first pass uses lmin = smallest Lanczos Ritz value and
lT = lmin + free-electron Fermi level of n_v states, later passes use the
smallest / largest Ritz value of the previous Rayleigh-Ritz step.

Pins (tests/test_oracle_eigen.py): the plain scaled filter on a diagonal
matrix equals the closed-form ratio of Chebyshev polynomials (cos/cosh);
with M = D, Alg. 4 equals the plain filter applied to D^-1 H (exact algebra);
Lanczos extreme Ritz values bracket the spectrum of a known matrix; the
converged driver reproduces scipy's generalized eigenvalues, for M = D and
for the consistent mass matrix M.
"""
import numpy as np
import scipy.linalg as sla


def cheb_filter_residual(Hop, Mop, Dinv, X, lam, degree, lmin, lmax, lT):
    """Alg. 4.  Hop/Mop: callables on blocks; Dinv: diagonal of D^-1 (vector)."""
    e = (lmax - lT) / 2.0
    c = (lmax + lT) / 2.0
    sigma = e / (lmin - c)
    sigma1 = sigma
    gamma = 2.0 / sigma1
    lam = np.asarray(lam, float)
    Y = Hop(X) - Mop(X) * lam[None, :]
    RX = np.zeros_like(Y)
    RY = (sigma1 / e) * Y
    LX = np.ones_like(lam)
    LY = (sigma1 / e) * (lam - c)
    for _ in range(2, degree + 1):
        sigma2 = 1.0 / (gamma - sigma)
        Z = Dinv[:, None] * RY
        RX = (2.0 * sigma2 / e) * (Hop(Z) - c * RY + Y * LY[None, :]) - sigma * sigma2 * RX
        LX = (2.0 * sigma2 / e) * LY * (lam - c) - sigma * sigma2 * LX
        RX, RY = RY, RX
        LX, LY = LY, LX
        sigma = sigma2
    return Dinv[:, None] * RY + X * LY[None, :]


def cheb_filter_plain(Aop, X, degree, lmin, lmax, lT):
    """The standard scaled three-term Chebyshev filter on the operator Aop."""
    e = (lmax - lT) / 2.0
    c = (lmax + lT) / 2.0
    sigma = e / (lmin - c)
    sigma1 = sigma
    gamma = 2.0 / sigma1
    X0 = X
    X1 = (sigma1 / e) * (Aop(X) - c * X)
    for _ in range(2, degree + 1):
        sigma2 = 1.0 / (gamma - sigma)
        X2 = (2.0 * sigma2 / e) * (Aop(X1) - c * X1) - sigma * sigma2 * X0
        X0, X1 = X1, X2
        sigma = sigma2
    return X1


def rayleigh_ritz(Hop, Mop, Y):
    """Alg. 3: solve (Y^H H Y) E = (Y^H M Y) E Lambda; return (Lambda, Y E)."""
    Hp = Y.conj().T @ Hop(Y)
    Sp = Y.conj().T @ Mop(Y)
    Hp = 0.5 * (Hp + Hp.conj().T)
    Sp = 0.5 * (Sp + Sp.conj().T)
    lam, E = sla.eigh(Hp, Sp)
    return lam, Y @ E


def lanczos_bounds(Hop, Dvec, v0, steps=10):
    """Ritz values and last beta of Lanczos on D^-1/2 H D^-1/2 (full reorth)."""
    s = 1.0 / np.sqrt(Dvec)
    A = lambda v: s * Hop((s * v)[:, None])[:, 0]
    q = v0 / np.linalg.norm(v0)
    Q = [q]
    alphas, betas = [], []
    beta_prev, q_prev = 0.0, np.zeros_like(q)
    for _ in range(steps):
        w = A(q) - beta_prev * q_prev
        alpha = np.vdot(q, w).real
        w = w - alpha * q
        Qm = np.stack(Q, axis=1)
        w = w - Qm @ (Qm.conj().T @ w)
        beta = np.linalg.norm(w)
        alphas.append(alpha)
        betas.append(beta)
        q_prev, q = q, w / beta
        beta_prev = beta
        Q.append(q)
    T = np.diag(alphas) + np.diag(betas[:-1], 1) + np.diag(betas[:-1], -1)
    theta = np.linalg.eigvalsh(T)
    return theta, betas[-1]


def fermi_free_electron(volume, nvec):
    """Energy below which a free electron gas in the box has nvec states."""
    return 0.5 * (6.0 * np.pi ** 2 * nvec / volume) ** (2.0 / 3.0)


def chfsi(Hop, Dvec, X0, v0, volume, outer=3, degree=40, lanczos_steps=10, Mop=None):
    """Alg. 3 with the Alg. 4 filter; returns (Ritz values, X, log).

    M is the lumped D unless Mop (the consistent mass, on blocks) is given:
    then the residual and the Rayleigh-Ritz step use M while the filter's
    approximate inverse stays D^-1, as Alg. 4 prescribes.  The bounds come
    from Lanczos on D^-1/2 H D^-1/2 either way.
    """
    Dop = lambda V: Dvec[:, None] * V
    Mop = Dop if Mop is None else Mop
    Dinv = 1.0 / Dvec
    theta, beta = lanczos_bounds(Hop, Dvec, v0, lanczos_steps)
    lmax = theta.max() + abs(beta)
    lam, X = rayleigh_ritz(Hop, Mop, X0)
    lmin = theta.min()
    lT = lmin + fermi_free_electron(volume, X0.shape[1])
    log = []
    for it in range(outer):
        if it > 0:
            lmin, lT = lam.min(), lam.max()
        Y = cheb_filter_residual(Hop, Mop, Dinv, X, lam, degree, lmin, lmax, lT)
        lam, X = rayleigh_ritz(Hop, Mop, Y)
        log.append(dict(lmin=lmin, lT=lT, lmax=lmax))
    return lam, X, log
