// Host construction of the 1D spectral-element tables.
//
// Sec. 2.2 (eqn FEdiscr): C0 Lagrange basis on the GLL points of degree p.
// Eqn cellIntegrals: n_q-point Gauss-Legendre rule per direction.
// Sec. 3.2 (eqn refact): N^1D[q][i] = l_i(xi_q) and the collocation
// derivative Dtilde^1D[q][r] = d/dxi Ltilde_r(xi_q), Ltilde_r being the
// Lagrange polynomial of degree n_q - 1 on the Gauss points, so that
// D^1D = Dtilde^1D N^1D exactly when n_p <= n_q.
// The even-odd packing (Sec. 4.2, used for the contraction counts of
// eqn flopRealMF) relies on N^1D being centro-symmetric and Dtilde^1D
// centro-antisymmetric, which holds because both point sets are symmetric.
#include <cmath>
#include <stdexcept>

#include "fe_internal.h"

namespace fehx {

namespace {

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1) * std::pow(x, n + 1);
}

void gauss_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));   // Chebyshev-like guess
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, z, P, dP);
      double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double P, dP;
    legendre(n, z, P, dP);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

// GLL: -1, +1 and the roots of P_p'; the roots of P_p' are found by Newton
// on q(x) = P_p'(x), with q'(x) from the Legendre ODE.
void gll_rule(int p, std::vector<double> &x, std::vector<double> &w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    // initial guess from the Chebyshev-Gauss-Lobatto points
    double z = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, z, P, dP);
      // (1 - x^2) P'' - 2 x P' + p(p+1) P = 0
      double d2P = (2.0 * z * dP - p * (p + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    legendre(p, x[i], P, dP);
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

// Barycentric weights of a node set.
std::vector<double> bary(const std::vector<double> &z) {
  int n = (int)z.size();
  std::vector<double> b(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (j != i) b[i] /= (z[i] - z[j]);
  return b;
}

}  // namespace

Tables1D make_tables(int p, int nq) {
  Tables1D t;
  t.p = p;
  t.np = p + 1;
  t.nq = nq;
  gll_rule(p, t.gll, t.gllw);
  gauss_rule(nq, t.xq, t.wq);
  // N[q][i] = l_i(xq): barycentric form of the Lagrange basis on GLL nodes
  std::vector<double> bg = bary(t.gll);
  t.N.assign((size_t)nq * t.np, 0.0);
  for (int q = 0; q < nq; ++q) {
    double x = t.xq[q];
    int hit = -1;
    for (int i = 0; i < t.np; ++i)
      if (std::fabs(x - t.gll[i]) < 1e-15) hit = i;   // e.g. xi = 0 in both rules
    if (hit >= 0) {
      for (int i = 0; i < t.np; ++i) t.N[q * t.np + i] = (i == hit) ? 1.0 : 0.0;
      continue;
    }
    double denom = 0.0;
    std::vector<double> tmp(t.np);
    for (int i = 0; i < t.np; ++i) {
      tmp[i] = bg[i] / (x - t.gll[i]);
      denom += tmp[i];
    }
    for (int i = 0; i < t.np; ++i) t.N[q * t.np + i] = tmp[i] / denom;
  }
  // collocation derivative on the Gauss points
  std::vector<double> bq = bary(t.xq);
  t.Dt.assign((size_t)nq * nq, 0.0);
  for (int q = 0; q < nq; ++q) {
    double diag = 0.0;
    for (int r = 0; r < nq; ++r) {
      if (r == q) continue;
      double v = (bq[r] / bq[q]) / (t.xq[q] - t.xq[r]);
      t.Dt[q * nq + r] = v;
      diag -= v;
    }
    t.Dt[q * nq + q] = diag;
  }
  return t;
}

std::vector<double> eo_pack(const std::vector<double> &A, int nout, int nin, int sym) {
  const int CO = (nout + 1) / 2, CI = (nin + 1) / 2, HI = nin / 2;
  std::vector<double> out((size_t)CO * (CI + HI), 0.0);
  for (int q = 0; q < nout; ++q)
    for (int i = 0; i < nin; ++i) {
      double a = A[q * nin + i], b = A[(nout - 1 - q) * nin + (nin - 1 - i)];
      if (!std::isfinite(a) || !(std::fabs(a - sym * b) <= 1e-11 * (1.0 + std::fabs(a))))
        throw std::runtime_error("1D table lacks the even-odd symmetry");
    }
  for (int q = 0; q < CO; ++q) {
    double *E = &out[(size_t)q * (CI + HI)];
    double *O = E + CI;
    for (int i = 0; i < HI; ++i) {
      E[i] = 0.5 * (A[q * nin + i] + A[q * nin + nin - 1 - i]);
      O[i] = 0.5 * (A[q * nin + i] - A[q * nin + nin - 1 - i]);
    }
    if (nin & 1) E[HI] = A[q * nin + HI];
  }
  return out;
}

}  // namespace fehx
