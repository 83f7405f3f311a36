// C-ABI entry points of libfehx: mesh set-up, coefficient fields, nonlocal
// projectors and the operator application (include/fe_hx.h documents each).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <stdexcept>
#include <unordered_map>

#include "fe_internal.h"

namespace fehx {

static thread_local std::string g_last_error;

fe_status set_error(fe_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

fe_status Mesh::dev_alloc(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return FE_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return set_error(FE_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  owned.emplace_back(*p, bytes);
  footprint += (int64_t)bytes;
  return FE_OK;
}

void Mesh::dev_free_all() {
  for (auto &pb : owned) hipFree(pb.first);
  owned.clear();
  footprint = 0;
  for (int i = 0; i < NWS; ++i)
    if (ws[i]) { hipFree(ws[i]); ws[i] = nullptr; ws_bytes[i] = 0; }
  if (nl_W) { hipFree(nl_W); nl_W = nullptr; }
}

fe_status ensure_workspace(Mesh *m, int slot, int64_t bytes) {
  if (m->ws_bytes[slot] >= bytes) return FE_OK;
  const bool filter_slot = slot <= 4 || slot == 8 || slot == 9;   // the slots a filter pass uses
  if (m->ws[slot] && filter_slot && m->graphs > 0)
    return set_error(FE_ESTATE, "a captured filter graph holds this mesh's workspace; destroy it before a call that "
                                "needs a larger one");
  if (m->ws[slot]) { hipFree(m->ws[slot]); m->footprint -= m->ws_bytes[slot]; m->ws[slot] = nullptr; m->ws_bytes[slot] = 0; }
  hipError_t e = hipMalloc(&m->ws[slot], (size_t)bytes);
  if (e != hipSuccess) { m->ws[slot] = nullptr; return set_error(FE_ENOMEM, "filter workspace allocation failed"); }
  m->ws_bytes[slot] = bytes;
  m->footprint += bytes;
  return FE_OK;
}

namespace {

template <typename T>
fe_status upload(Mesh *m, T **dst, const std::vector<T> &src) {
  if (m->host_only) { *dst = nullptr; return FE_OK; }
  void *p = nullptr;
  fe_status st = m->dev_alloc(&p, src.size() * sizeof(T));
  if (st) return st;
  if (!src.empty()) FE_HIP_TRY(hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = (T *)p;
  return FE_OK;
}

template <typename T>
void release(Mesh *m, T *&p) {
  if (!p) return;
  for (auto it = m->owned.begin(); it != m->owned.end(); ++it)
    if (it->first == (void *)p) {
      m->footprint -= (int64_t)it->second;
      m->owned.erase(it);
      break;
    }
  hipFree(p);
  p = nullptr;
}

std::vector<float> to_f32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }

int colour_of(int c, int n) { return ((n & 1) && c == n - 1) ? 2 : (c & 1); }

template <typename M3> double det3(const M3 &a) {
  return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
         a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}
template <typename M3> void inv3(const M3 &a, double out[3][3]) {
  const double d = det3(a);
  out[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / d;
  out[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / d;
  out[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / d;
  out[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / d;
  out[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / d;
  out[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / d;
  out[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / d;
  out[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / d;
  out[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / d;
}

// Cell origin and quadrature point coordinates.
void cell_origin(const Mesh *m, int64_t c, double x[3]) {
  int c0 = (int)(c % m->N[0]), c1 = (int)((c / m->N[0]) % m->N[1]), c2 = (int)(c / ((int64_t)m->N[0] * m->N[1]));
  const int cc[3] = {c0, c1, c2};
  for (int a = 0; a < 3; ++a) {
    x[a] = 0;
    for (int d = 0; d < 3; ++d) x[a] += (double)cc[d] / m->N[d] * m->desc.lattice[d][a];
  }
}

// Corner (a, b, c) (index a + 2 b + 4 c) of cell cell of a distorted mesh:
// the unwrapped lattice position of vertex (c0 + a, c1 + b, c2 + c) plus the
// displacement of the periodic vertex it wraps to.
void cell_corners(const Mesh *m, int64_t c, double X[8][3]) {
  const int cc[3] = {(int)(c % m->N[0]), (int)((c / m->N[0]) % m->N[1]), (int)(c / ((int64_t)m->N[0] * m->N[1]))};
  for (int k = 0; k < 8; ++k) {
    const int g[3] = {cc[0] + (k & 1), cc[1] + ((k >> 1) & 1), cc[2] + ((k >> 2) & 1)};
    const int64_t v = (g[0] % m->N[0]) + (int64_t)m->N[0] * ((g[1] % m->N[1]) + (int64_t)m->N[1] * (g[2] % m->N[2]));
    for (int a = 0; a < 3; ++a) {
      double x = 0.0;
      for (int d = 0; d < 3; ++d) x += (double)g[d] / m->N[d] * m->desc.lattice[d][a];
      X[k][a] = x + (m->distorted ? m->vdisp[3 * v + a] : 0.0);
    }
  }
}

// x(xi) and the Jacobian J[a][d] = dx_a / dxi_d of cell c at the reference
// point xi: the affine map x_c + J (xi + 1), or for a distorted mesh the
// trilinear map through the cell's corners (Sec. 3.1, a Jacobian per point).
void point_geometry(const Mesh *m, int64_t c, const double xi[3], double x[3], double J[3][3]) {
  if (!m->distorted) {
    double xc[3];
    cell_origin(m, c, xc);
    for (int a = 0; a < 3; ++a) {
      x[a] = xc[a] + m->J[a][0] * (xi[0] + 1.0) + m->J[a][1] * (xi[1] + 1.0) + m->J[a][2] * (xi[2] + 1.0);
      for (int d = 0; d < 3; ++d) J[a][d] = m->J[a][d];
    }
    return;
  }
  double X[8][3];
  cell_corners(m, c, X);
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    for (int d = 0; d < 3; ++d) J[a][d] = 0.0;
  }
  for (int k = 0; k < 8; ++k) {
    double f[3], s[3];
    for (int d = 0; d < 3; ++d) {
      s[d] = ((k >> d) & 1) ? 1.0 : -1.0;
      f[d] = 0.5 * (1.0 + s[d] * xi[d]);
    }
    const double phi = f[0] * f[1] * f[2];
    const double dphi[3] = {0.5 * s[0] * f[1] * f[2], 0.5 * s[1] * f[0] * f[2], 0.5 * s[2] * f[0] * f[1]};
    for (int a = 0; a < 3; ++a) {
      x[a] += phi * X[k][a];
      for (int d = 0; d < 3; ++d) J[a][d] += dphi[d] * X[k][a];
    }
  }
}

void quad_point(const Mesh *m, int64_t c, int q1, int q2, int q3, double x[3], double *wdet = nullptr) {
  const double xi[3] = {m->t1.xq[q1], m->t1.xq[q2], m->t1.xq[q3]};
  double J[3][3];
  point_geometry(m, c, xi, x, J);
  if (wdet) *wdet = m->t1.wq[q1] * m->t1.wq[q2] * m->t1.wq[q3] * det3(J);
}

// The weighted coefficient blocks of cell c ([m->ncoef][n_q^3], layout of
// NCOEF_GEN) from the fields at its quadrature points (vloc [n_q^3] or null
// for zero, vgga [n_q^3][3] or null).
void cell_coefficients(const Mesh *m, int64_t c, const double *vloc, const double *vgga, double *out) {
  const int nq = m->nq, nq3 = nq * nq * nq;
  const double *k = m->desc.kpoint;
  for (int q3 = 0; q3 < nq; ++q3)
    for (int q2 = 0; q2 < nq; ++q2)
      for (int q1 = 0; q1 < nq; ++q1) {
        const int Q = (q3 * nq + q2) * nq + q1;
        const double xi[3] = {m->t1.xq[q1], m->t1.xq[q2], m->t1.xq[q3]};
        double x[3], J[3][3], Ji[3][3];
        point_geometry(m, c, xi, x, J);
        const double w = m->t1.wq[q1] * m->t1.wq[q2] * m->t1.wq[q3] * det3(J);
        inv3(J, Ji);
        out[Q] = ((vloc ? vloc[Q] : 0.0) + m->k2half) * w;
        for (int s = 0; s < 3; ++s) {
          // reference-frame GGA coefficient sum_a (J^-1)_{s a} V^G_a (reading C-2)
          double v = 0.0;
          if (vgga)
            for (int a = 0; a < 3; ++a) v += Ji[s][a] * vgga[3 * Q + a];
          out[(1 + s) * nq3 + Q] = v * w;
        }
        if (m->ncoef < NCOEF_GEN) continue;
        const int pr[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
        for (int t = 0; t < 6; ++t) {
          double g = 0.0;
          for (int a = 0; a < 3; ++a) g += Ji[pr[t][0]][a] * Ji[pr[t][1]][a];
          out[(4 + t) * nq3 + Q] = 0.5 * g * w;
        }
        for (int s = 0; s < 3; ++s) {
          double kap = 0.0;
          for (int a = 0; a < 3; ++a) kap += Ji[s][a] * k[a];
          out[(10 + s) * nq3 + Q] = kap * w;
        }
      }
}

// DoF of node (i, j, k) of cell c, or -1 for a node on a Dirichlet face:
// periodic axes wrap g = c p + i modulo N p; Dirichlet axes number the
// interior nodes 0 < g < N p as g - 1.
int64_t dof_of(const Mesh *m, int64_t c, int i, int j, int k) {
  const int cc[3] = {(int)(c % m->N[0]), (int)((c / m->N[0]) % m->N[1]), (int)(c / ((int64_t)m->N[0] * m->N[1]))};
  const int loc[3] = {i, j, k};
  int g[3];
  for (int d = 0; d < 3; ++d) {
    g[d] = cc[d] * m->p + loc[d];
    if (m->desc.periodic[d]) {
      g[d] %= m->Mn[d];
    } else {
      g[d] -= 1;
      if (g[d] < 0 || g[d] >= m->Mn[d]) return -1;
    }
  }
  return g[0] + (int64_t)m->Mn[0] * (g[1] + (int64_t)m->Mn[1] * g[2]);
}

// real solid harmonics times the radial cut-off Gaussian (fe_projector doc)
double chi_value(int l, int mm, const double r[3], double sigma, double rc) {
  const double rho2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  if (rho2 >= rc * rc) return 0.0;
  const double u = 1.0 - rho2 / (rc * rc);
  const double rad = std::exp(-rho2 / (2.0 * sigma * sigma)) * u * u;
  double s = 1.0;
  if (l == 1) s = r[mm];
  else if (l == 2) {
    switch (mm) {
      case 0: s = r[0] * r[1]; break;
      case 1: s = r[1] * r[2]; break;
      case 2: s = r[2] * r[0]; break;
      case 3: s = r[0] * r[0] - r[1] * r[1]; break;
      default: s = 3.0 * r[2] * r[2] - rho2; break;
    }
  }
  return s * rad;
}

}  // namespace

// Every device array that depends on the cell geometry: the mass-operator
// coefficients (one shared block, or one per cell on the general-metric
// path), the lumped mass D and its inverse, and the operator coefficients of
// a zero potential.  Replaces what an earlier call made.
fe_status build_geometry(Mesh *m) {
  const int np = m->np, nq = m->nq, nq3 = nq * nq * nq;
  m->ncoef = m->offd ? NCOEF_GEN : 4;
  release(m, m->coefM64); release(m, m->coefM32); release(m, m->dmass); release(m, m->dinv);
  release(m, m->coef64); release(m, m->coef32);
  fe_status st;
  // the consistent mass: w_Q det J(xi_Q) in block 0, the other blocks zero
  const int64_t ncm = m->distorted ? m->E : 1;
  std::vector<double> coefM((size_t)ncm * m->ncoef * nq3, 0.0);
  for (int64_t c = 0; c < ncm; ++c) {
    for (int q3 = 0; q3 < nq; ++q3)
      for (int q2 = 0; q2 < nq; ++q2)
        for (int q1 = 0; q1 < nq; ++q1) {
          double x[3], w;
          quad_point(m, c, q1, q2, q3, x, &w);
          coefM[(size_t)c * m->ncoef * nq3 + (q3 * nq + q2) * nq + q1] = w;
        }
  }
  m->coefM_cell = m->distorted ? (int64_t)m->ncoef * nq3 : 0;
  if ((st = upload(m, &m->coefM64, coefM))) return st;
  if ((st = upload(m, &m->coefM32, to_f32(coefM)))) return st;
  // lumped mass D: the GLL rule on the nodes, det J at each node (Sec. 5.3)
  m->h_dmass.assign((size_t)m->m, 0.0);
  for (int64_t c = 0; c < m->E; ++c)
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i) {
          const int64_t g = dof_of(m, c, i, j, k);
          if (g < 0) continue;
          double dj = m->detJ;
          if (m->distorted) {
            const double xi[3] = {m->t1.gll[i], m->t1.gll[j], m->t1.gll[k]};
            double x[3], J[3][3];
            point_geometry(m, c, xi, x, J);
            dj = det3(J);
          }
          m->h_dmass[g] += m->t1.gllw[i] * m->t1.gllw[j] * m->t1.gllw[k] * dj;
        }
  std::vector<double> dinv(m->h_dmass.size());
  for (size_t i = 0; i < dinv.size(); ++i) dinv[i] = 1.0 / m->h_dmass[i];
  if ((st = upload(m, &m->dmass, m->h_dmass))) return st;
  if ((st = upload(m, &m->dinv, dinv))) return st;
  // zero potential: (0 + |k|^2/2) w det J, no GGA, the metric and Bloch blocks
  std::vector<double> coef((size_t)m->E * m->ncoef * nq3, 0.0);
  for (int64_t c = 0; c < m->E; ++c) cell_coefficients(m, c, nullptr, nullptr, &coef[(size_t)c * m->ncoef * nq3]);
  if ((st = upload(m, &m->coef64, coef))) return st;
  if ((st = upload(m, &m->coef32, to_f32(coef)))) return st;
  m->has_gga = false;
  return FE_OK;
}

fe_status check_mesh(fe_mesh_t m) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  return FE_OK;
}

}  // namespace fehx

using namespace fehx;

extern "C" {

int32_t fe_abi_version(void) { return 2; }
const char *fe_last_error(void) { return g_last_error.c_str(); }

fe_status fe_mesh_create(const fe_mesh_desc *desc, fe_mesh_t *out) {
  if (!out) return set_error(FE_EINVAL, "NULL output handle");
  *out = nullptr;
  if (!desc) return set_error(FE_EINVAL, "NULL descriptor");
  const fe_mesh_desc &d = *desc;
  for (int a = 0; a < 3; ++a) {
    if (d.ncell[a] < 1) return set_error(FE_EINVAL, "ncell must be positive");
    if (d.ncell[a] < 2) return set_error(FE_EUNSUPPORTED, "ncell >= 2 per axis is required");
    if (!d.periodic[a] &&
        std::fabs(d.kpoint[0] * d.lattice[a][0] + d.kpoint[1] * d.lattice[a][1] + d.kpoint[2] * d.lattice[a][2]) > 1e-14)
      return set_error(FE_EINVAL, "the k-point must vanish along a Dirichlet (non-periodic) axis (k . a_d = 0)");
  }
  if (d.degree < 1) return set_error(FE_EINVAL, "degree must be >= 1");
  if (d.nq < d.degree + 1) return set_error(FE_EINVAL, "n_q must be >= degree + 1");
  if (d.degree < 2 || d.degree > 8) return set_error(FE_EUNSUPPORTED, "degree must be in 2..8");
  if (d.nq != d.degree + 1 && d.nq != d.degree + 3 && d.nq != d.degree + 4)
    return set_error(FE_EUNSUPPORTED, "this build has kernels for n_q = n_p, n_p + 2 and n_p + 3 (n_p = degree + 1)");
  const double detA = det3(d.lattice);
  if (!(detA > 0)) return set_error(FE_EINVAL, "lattice must be right-handed (det > 0)");
  const bool host_only = d.device < 0;
  if (!host_only) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return set_error(FE_EDEVICE, "no HIP device");
    if (d.device >= ndev) return set_error(FE_EINVAL, "device ordinal out of range");
  }

  fe_mesh_s *m = new (std::nothrow) fe_mesh_s();
  if (!m) return set_error(FE_ENOMEM, "host allocation failed");
  m->desc = d;
  m->device = d.device;
  m->host_only = host_only;
  if (!host_only && hipSetDevice(m->device) != hipSuccess) { delete m; return set_error(FE_EDEVICE, "hipSetDevice failed"); }
  m->p = d.degree;
  m->np = d.degree + 1;
  m->nq = d.nq;
  for (int a = 0; a < 3; ++a) {
    m->N[a] = d.ncell[a];
    m->Mn[a] = d.ncell[a] * d.degree - (d.periodic[a] ? 0 : 1);
  }
  m->E = (int64_t)m->N[0] * m->N[1] * m->N[2];
  m->m = (int64_t)m->Mn[0] * m->Mn[1] * m->Mn[2];
  const double kk = d.kpoint[0] * d.kpoint[0] + d.kpoint[1] * d.kpoint[1] + d.kpoint[2] * d.kpoint[2];
  m->cplx = d.is_complex || kk > 0.0;
  // J[:, d] = a_d / (2 N_d) (Sec. 3.1: one affine map per cell)
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) m->J[a][b] = d.lattice[b][a] / (2.0 * m->N[b]);
  m->detJ = det3(m->J);
  inv3(m->J, m->Jinv);
  for (int s = 0; s < 3; ++s) {
    // kinetic metric 1/2 (J^-1 J^-T)_ss and Bloch vector in the reference frame
    m->gdiag[s] = 0.0;
    m->kap[s] = 0.0;
    for (int a = 0; a < 3; ++a) {
      m->gdiag[s] += 0.5 * m->Jinv[s][a] * m->Jinv[s][a];
      m->kap[s] += m->Jinv[s][a] * d.kpoint[a];
    }
  }
  m->k2half = 0.5 * kk;
  fe_status st = FE_OK;
  try {
    m->t1 = make_tables(m->p, m->nq);
    const int np = m->np, nq = m->nq;
    // the four 1D matrices of Alg. 2 in even-odd packed form
    std::vector<double> NT((size_t)np * nq), DT((size_t)nq * nq);
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < np; ++i) NT[i * nq + q] = m->t1.N[q * np + i];
    for (int q = 0; q < nq; ++q)
      for (int r = 0; r < nq; ++r) DT[r * nq + q] = m->t1.Dt[q * nq + r];
    TabLayout L = tab_layout(np, nq);
    std::vector<double> tab(L.total);
    auto put = [&](int off, const std::vector<double> &v) { std::copy(v.begin(), v.end(), tab.begin() + off); };
    put(L.n_off, eo_pack(m->t1.N, nq, np, +1));
    put(L.nt_off, eo_pack(NT, np, nq, +1));
    put(L.d_off, eo_pack(m->t1.Dt, nq, nq, -1));
    put(L.dt_off, eo_pack(DT, nq, nq, -1));
    // w_Q det J = (w_a w_b)(w_i det J) for a line along direction D through
    // (a, b): the pair product per line, the per-point factor with g and kappa
    for (int D = 0; D < 3; ++D)
      for (int i = 0; i < nq; ++i) {
        tab[L.gw_off + D * nq + i] = m->gdiag[D] * m->t1.wq[i] * m->detJ;
        tab[L.kw_off + D * nq + i] = m->kap[D] * m->t1.wq[i] * m->detJ;
      }
    {
      double gmax = 0.0, omax = 0.0;
      for (int a2 = 0; a2 < 3; ++a2)
        for (int b = 0; b < 3; ++b) {
          double g = 0.0;
          for (int c2 = 0; c2 < 3; ++c2) g += 0.5 * m->Jinv[a2][c2] * m->Jinv[b][c2];
          gmax = std::max(gmax, std::fabs(g));
          if (a2 != b) omax = std::max(omax, std::fabs(g));
        }
      m->offd = m->offd_affine = omax > 1e-14 * gmax;
    }
    std::vector<double> wq((size_t)nq * nq);
    for (int b = 0; b < nq; ++b)
      for (int a2 = 0; a2 < nq; ++a2) wq[b * nq + a2] = m->t1.wq[a2] * m->t1.wq[b];
    if ((st = upload(m, &m->tab64, tab))) throw std::runtime_error("upload");
    if ((st = upload(m, &m->tab32, to_f32(tab)))) throw std::runtime_error("upload");
    // the four 1D matrices in full, zero padded to 8 x 8, rows = outputs:
    // N [q][i], N^T [i][q], Dtilde [q][r], Dtilde^T [r][q]
    std::vector<float> mx(4 * 64, 0.0f);
    for (int q = 0; q < nq && q < 8; ++q)
      for (int i = 0; i < np && i < 8; ++i) {
        mx[0 * 64 + q * 8 + i] = (float)m->t1.N[q * np + i];
        mx[1 * 64 + i * 8 + q] = (float)m->t1.N[q * np + i];
      }
    for (int q = 0; q < nq && q < 8; ++q)
      for (int r = 0; r < nq && r < 8; ++r) {
        mx[2 * 64 + q * 8 + r] = (float)m->t1.Dt[q * nq + r];
        mx[3 * 64 + r * 8 + q] = (float)m->t1.Dt[q * nq + r];
      }
    if ((st = upload(m, &m->tabmx, mx))) throw std::runtime_error("upload");
    if ((st = upload(m, &m->wq64, wq))) throw std::runtime_error("upload");
    if ((st = upload(m, &m->wq32, to_f32(wq)))) throw std::runtime_error("upload");
    // the consistent mass M = sum_e N3^T (w det J) N3: the same tables with the
    // kinetic and Bloch factors zeroed, and one coefficient block w det J
    std::vector<double> tabM(tab);
    for (int i = L.gw_off; i < L.total; ++i) tabM[i] = 0.0;
    if ((st = upload(m, &m->tabM64, tabM))) throw std::runtime_error("upload");
    if ((st = upload(m, &m->tabM32, to_f32(tabM)))) throw std::runtime_error("upload");
    if ((st = build_geometry(m))) throw std::runtime_error("geometry");
    // column colouring: phase (a, b) holds columns with colour a along a_0, b along a_1
    m->ncolx = (m->N[0] & 1) ? 3 : 2;
    m->ncoly = (m->N[1] & 1) ? 3 : 2;
    m->nphase = m->ncolx * m->ncoly;
    std::vector<int> cols;
    m->phase_off.assign(m->nphase + 1, 0);
    for (int b = 0; b < m->ncoly; ++b)
      for (int a = 0; a < m->ncolx; ++a) {
        const int ph = a + m->ncolx * b;
        m->phase_off[ph] = (int)(cols.size() / 2);
        for (int cy = 0; cy < m->N[1]; ++cy)
          for (int cx = 0; cx < m->N[0]; ++cx)
            if (colour_of(cx, m->N[0]) == a && colour_of(cy, m->N[1]) == b) {
              cols.push_back(cx);
              cols.push_back(cy);
            }
      }
    m->phase_off[m->nphase] = (int)(cols.size() / 2);
    if ((st = upload(m, &m->cols, cols))) throw std::runtime_error("upload");
  } catch (const std::exception &e) {
    m->dev_free_all();
    delete m;
    if (st == FE_OK) st = set_error(FE_EINVAL, e.what());
    return st;
  }
  *out = m;
  return FE_OK;
}

fe_status fe_mesh_destroy(fe_mesh_t mesh) {
  if (!mesh) return set_error(FE_EINVAL, "NULL mesh handle");
  if (mesh->graphs > 0) return set_error(FE_ESTATE, "destroy the mesh's filter graphs first");
  if (!mesh->host_only) {
    hipSetDevice(mesh->device);
    hipDeviceSynchronize();
    if (mesh->ev_fork) hipEventDestroy(mesh->ev_fork);
    if (mesh->ev_join) hipEventDestroy(mesh->ev_join);
    if (mesh->side) hipStreamDestroy(mesh->side);
    mesh->dev_free_all();
  }
  delete mesh;
  return FE_OK;
}

fe_status fe_mesh_query(fe_mesh_t m, int64_t *ndofs, int64_t *ncells, int64_t *nq3, int64_t *footprint) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (ndofs) *ndofs = m->m;
  if (ncells) *ncells = m->E;
  if (nq3) *nq3 = (int64_t)m->nq * m->nq * m->nq;
  if (footprint) *footprint = m->footprint;
  return FE_OK;
}

fe_status fe_mesh_cell_dofs(fe_mesh_t m, int64_t first, int64_t count, int32_t *dofs) {
  if (!m || !dofs) return set_error(FE_EINVAL, "NULL argument");
  if (first < 0 || count < 0 || first + count > m->E) return set_error(FE_EINVAL, "cell range out of bounds");
  const int np = m->np;
  for (int64_t c = first; c < first + count; ++c)
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < np; ++j)
        for (int i = 0; i < np; ++i)
          dofs[(c - first) * np * np * np + (k * np + j) * np + i] = (int32_t)dof_of(m, c, i, j, k);
  return FE_OK;
}

fe_status fe_mesh_quad_points(fe_mesh_t m, double *xyz) {
  if (!m || !xyz) return set_error(FE_EINVAL, "NULL argument");
  const int nq = m->nq;
  for (int64_t c = 0; c < m->E; ++c)
    for (int q3 = 0; q3 < nq; ++q3)
      for (int q2 = 0; q2 < nq; ++q2)
        for (int q1 = 0; q1 < nq; ++q1) {
          double *x = xyz + 3 * (c * nq * nq * nq + (q3 * nq + q2) * nq + q1);
          quad_point(m, c, q1, q2, q3, x);
        }
  return FE_OK;
}

fe_status fe_mesh_lumped_mass(fe_mesh_t m, double *dd) {
  if (!m || !dd) return set_error(FE_EINVAL, "NULL argument");
  std::memcpy(dd, m->h_dmass.data(), m->h_dmass.size() * sizeof(double));
  return FE_OK;
}

fe_status fe_mesh_set_geometry(fe_mesh_t m, const double *vdisp) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (m->graphs > 0) return set_error(FE_ESTATE, "a captured filter graph uses the mesh's data; destroy it first");
  if (vdisp)
    for (int d = 0; d < 3; ++d)
      if (!m->desc.periodic[d]) return set_error(FE_EUNSUPPORTED, "distorted cells need a periodic box");
  if (!m->host_only) {
    if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
    FE_HIP_TRY(hipDeviceSynchronize());
  }
  const std::vector<double> old = m->vdisp;
  const bool old_dist = m->distorted;
  if (vdisp) {
    m->vdisp.assign(vdisp, vdisp + 3 * m->E);
    m->distorted = true;
  } else {
    m->vdisp.clear();
    m->distorted = false;
  }
  // every quadrature point and every node must keep det J > 0
  if (m->distorted) {
    const int nq = m->nq, np = m->np;
    bool ok = true;
    for (int64_t c = 0; c < m->E && ok; ++c)
      for (int pass = 0; pass < 2 && ok; ++pass) {
        const int n = pass ? np : nq;
        const double *xs = pass ? m->t1.gll.data() : m->t1.xq.data();
        for (int i3 = 0; i3 < n && ok; ++i3)
          for (int i2 = 0; i2 < n && ok; ++i2)
            for (int i1 = 0; i1 < n && ok; ++i1) {
              const double xi[3] = {xs[i1], xs[i2], xs[i3]};
              double x[3], J[3][3];
              point_geometry(m, c, xi, x, J);
              ok = det3(J) > 0.0;
            }
      }
    if (!ok) {
      m->vdisp = old;
      m->distorted = old_dist;
      return set_error(FE_EINVAL, "the displacement folds a cell (det J <= 0 at a quadrature point or node)");
    }
  }
  m->offd = m->distorted || m->offd_affine;
  fe_status st = fe_set_projectors(m, 0, nullptr, 0, nullptr);   // they depend on the geometry
  if (st) return st;
  return build_geometry(m);
}

fe_status fe_set_potential(fe_mesh_t m, const double *vloc, const double *vgga) {
  if (!m || !vloc) return set_error(FE_EINVAL, "NULL argument");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0) holds no operator data");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  FE_HIP_TRY(hipDeviceSynchronize());
  const int nq = m->nq, nq3 = nq * nq * nq;
  std::vector<double> coef((size_t)m->E * m->ncoef * nq3, 0.0);
  for (int64_t c = 0; c < m->E; ++c)
    cell_coefficients(m, c, vloc + c * nq3, vgga ? vgga + 3 * c * nq3 : nullptr, &coef[(size_t)c * m->ncoef * nq3]);
  FE_HIP_TRY(hipMemcpy(m->coef64, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<float> c32 = to_f32(coef);
  FE_HIP_TRY(hipMemcpy(m->coef32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
  m->has_gga = vgga != nullptr;
  return FE_OK;
}

fe_status fe_set_projectors(fe_mesh_t m, int32_t natoms, const double *pos, int32_t nproj,
                            const fe_projector *proj) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (natoms < 0 || nproj < 0) return set_error(FE_EINVAL, "negative count");
  if (nproj > 0 && (!pos || !proj)) return set_error(FE_EINVAL, "NULL projector arrays");
  if (m->graphs > 0) return set_error(FE_ESTATE, "a captured filter graph uses the projector data; destroy it first");
  if (!m->host_only) {
    if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
    FE_HIP_TRY(hipDeviceSynchronize());
  }
  // release any previous projector data
  release(m, m->nl_atom_off); release(m, m->nl_atom_nodes); release(m, m->nl_atom_proj);
  release(m, m->nl_F64); release(m, m->nl_F32); release(m, m->nl_rows); release(m, m->nl_rowptr);
  release(m, m->nl_colidx); release(m, m->nl_val64); release(m, m->nl_val32); release(m, m->nl_h);
  release(m, m->nl_chunk_atom); release(m, m->nl_chunk_n0); release(m, m->nl_chunk_order); release(m, m->nl_atom_chunk0); release(m, m->nl_proj_atom);
  release(m, m->nl_b_row0); release(m, m->nl_b_p0); release(m, m->nl_b_proj); release(m, m->nl_b_rows);
  release(m, m->nl_b_rowptr); release(m, m->nl_b_lcol); release(m, m->nl_b_val32);
  release(m, m->nl_b_A64); release(m, m->nl_b_aoff); release(m, m->nl_b_k);
  m->nl_nbrick = 0; m->nl_bmaxp = 0; m->nl_b_kmax = 0;
  m->nl_nchunks = 0;
  m->natoms = 0; m->ns = 0; m->nl_nrows = 0; m->nl_nnz = 0; m->nl_nsup = 0; m->nl_maxproj = 0;
  m->h_rows.clear(); m->h_rowptr.assign(1, 0); m->h_colidx.clear(); m->h_val.clear();
  if (nproj == 0) return FE_OK;

  // smallest spacing between opposite faces of the box: det A / |a_b x a_c|
  double Lmin = 1e300;
  {
    const auto &A = m->desc.lattice;
    const double vol = det3(A);
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c2 = (a + 2) % 3;
      const double cx = A[b][1] * A[c2][2] - A[b][2] * A[c2][1];
      const double cy = A[b][2] * A[c2][0] - A[b][0] * A[c2][2];
      const double cz = A[b][0] * A[c2][1] - A[b][1] * A[c2][0];
      Lmin = std::min(Lmin, vol / std::sqrt(cx * cx + cy * cy + cz * cz));
    }
  }
  for (int s = 0; s < nproj; ++s) {
    const fe_projector &pr = proj[s];
    if (pr.atom < 0 || pr.atom >= natoms) return set_error(FE_EINVAL, "projector atom index out of range");
    if (pr.l < 0 || pr.l > 2 || pr.m < 0 || pr.m > 2 * pr.l) return set_error(FE_EUNSUPPORTED, "projector (l, m) not in the l <= 2 table");
    if (!(pr.rc > 0) || !(pr.sigma > 0)) return set_error(FE_EINVAL, "projector rc and sigma must be positive");
    if (pr.rc >= 0.5 * Lmin) return set_error(FE_EUNSUPPORTED, "projector cutoff must be below half the box width");
    if (s > 0 && proj[s].atom < proj[s - 1].atom) return set_error(FE_EINVAL, "projectors must be grouped by atom in ascending order");
  }
  const bool cplx = m->cplx;
  const int C = cplx ? 2 : 1;
  const int np = m->np, nq = m->nq, np3 = np * np * np, nq3 = nq * nq * nq;
  std::vector<int> proj_off(natoms + 1, 0);
  for (int s = 0; s < nproj; ++s) proj_off[proj[s].atom + 1]++;
  for (int a = 0; a < natoms; ++a) proj_off[a + 1] += proj_off[a];
  int maxp = 0;
  for (int a = 0; a < natoms; ++a) maxp = std::max(maxp, proj_off[a + 1] - proj_off[a]);

  double Ainv[3][3];
  inv3(m->desc.lattice, Ainv);   // fractional coordinates f = x A^-1 (rows of A are a_d)
  // per cell: the corners' centre and the radius of the sphere around it
  // holding them (a trilinear cell lies in its corners' convex hull)
  std::vector<double> ccen((size_t)m->E * 3), crad((size_t)m->E);
  for (int64_t c = 0; c < m->E; ++c) {
    double X[8][3];
    cell_corners(m, c, X);
    double cen[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
    for (int kk = 0; kk < 8; ++kk)
      for (int d = 0; d < 3; ++d) cen[d] += 0.125 * X[kk][d];
    for (int kk = 0; kk < 8; ++kk) {
      double q = 0.0;
      for (int d = 0; d < 3; ++d) q += (X[kk][d] - cen[d]) * (X[kk][d] - cen[d]);
      r2 = std::max(r2, q);
    }
    for (int d = 0; d < 3; ++d) ccen[3 * c + d] = cen[d];
    crad[c] = std::sqrt(r2);
  }
  const double *k = m->desc.kpoint;

  std::vector<int> atom_off(1, 0), atom_nodes;
  std::vector<double> Fblk;                       // [support node][maxp][C]
  struct Ent { int64_t node; int s; double re, im; };
  std::vector<Ent> ents;
  std::vector<double> cq((size_t)nq3 * maxp * C), t1v, t2v, cellF((size_t)np3 * maxp * C);
  for (int a = 0; a < natoms; ++a) {
    const int s0 = proj_off[a], na = proj_off[a + 1] - s0;
    // the atom wrapped into the box along periodic axes (fractional coordinates)
    double f[3], R[3];
    for (int d = 0; d < 3; ++d) {
      f[d] = pos[3 * a] * Ainv[0][d] + pos[3 * a + 1] * Ainv[1][d] + pos[3 * a + 2] * Ainv[2][d];
      if (m->desc.periodic[d]) f[d] -= std::floor(f[d]);
    }
    for (int d = 0; d < 3; ++d)
      R[d] = f[0] * m->desc.lattice[0][d] + f[1] * m->desc.lattice[1][d] + f[2] * m->desc.lattice[2][d];
    double rcmax = 0;
    for (int s = 0; s < na; ++s) rcmax = std::max(rcmax, proj[s0 + s].rc);
    std::unordered_map<int64_t, int> local;   // node -> row in this atom's block
    std::vector<int64_t> order;
    std::vector<double> blk;
    if (na == 0) { atom_off.push_back((int)atom_nodes.size()); continue; }
    for (int64_t c = 0; c < m->E; ++c) {
      const double *cen = &ccen[3 * c];
      const double rad = crad[c];
      // images of the atom that can reach this cell
      int imgs[27][3];
      int nimg = 0;
      for (int r0 = -1; r0 <= 1; ++r0)
        for (int r1 = -1; r1 <= 1; ++r1)
          for (int r2 = -1; r2 <= 1; ++r2) {
            const int rr[3] = {r0, r1, r2};
            // images only along periodic axes
            if ((r0 && !m->desc.periodic[0]) || (r1 && !m->desc.periodic[1]) || (r2 && !m->desc.periodic[2])) continue;
            double d2 = 0;
            for (int d = 0; d < 3; ++d) {
              const double dx = cen[d] - R[d] - (rr[0] * m->desc.lattice[0][d] + rr[1] * m->desc.lattice[1][d] +
                                                 rr[2] * m->desc.lattice[2][d]);
              d2 += dx * dx;
            }
            if (d2 < (rcmax + rad + 1e-9) * (rcmax + rad + 1e-9)) {
              imgs[nimg][0] = r0; imgs[nimg][1] = r1; imgs[nimg][2] = r2; ++nimg;
            }
          }
      if (nimg == 0) continue;
      // c_s(Q) = sum_r chi_s(x_Q - R - L_r) exp(-i k.(x_Q - L_r)) w_Q det J
      bool any = false;
      std::fill(cq.begin(), cq.end(), 0.0);
      for (int q3 = 0; q3 < nq; ++q3)
        for (int q2 = 0; q2 < nq; ++q2)
          for (int q1 = 0; q1 < nq; ++q1) {
            const int Q = (q3 * nq + q2) * nq + q1;
            double x[3], wQ;
            quad_point(m, c, q1, q2, q3, x, &wQ);
            for (int ii = 0; ii < nimg; ++ii) {
              double Lr[3], r[3];
              for (int d = 0; d < 3; ++d) {
                Lr[d] = imgs[ii][0] * m->desc.lattice[0][d] + imgs[ii][1] * m->desc.lattice[1][d] +
                        imgs[ii][2] * m->desc.lattice[2][d];
                r[d] = x[d] - R[d] - Lr[d];
              }
              double ph_re = 1.0, ph_im = 0.0;
              if (cplx) {
                const double th = -(k[0] * (x[0] - Lr[0]) + k[1] * (x[1] - Lr[1]) + k[2] * (x[2] - Lr[2]));
                ph_re = std::cos(th);
                ph_im = std::sin(th);
              }
              for (int s = 0; s < na; ++s) {
                const fe_projector &pr = proj[s0 + s];
                const double v = chi_value(pr.l, pr.m, r, pr.sigma, pr.rc);
                if (v == 0.0) continue;
                any = true;
                cq[((size_t)Q * maxp + s) * C] += v * ph_re * wQ;
                if (cplx) cq[((size_t)Q * maxp + s) * C + 1] += v * ph_im * wQ;
              }
            }
          }
      if (!any) continue;
      // cell-level F^(a,e)[I][s] = sum_Q N3[Q][I] c_s(Q): three transposed 1D sweeps
      const int M = maxp * C;
      // sweep q1 -> i : [q3][q2][q1] -> [q3][q2][i]
      t1v.assign((size_t)nq * nq * np * M, 0.0);
      for (int q3 = 0; q3 < nq; ++q3)
        for (int q2 = 0; q2 < nq; ++q2)
          for (int i = 0; i < np; ++i)
            for (int q1 = 0; q1 < nq; ++q1) {
              const double nv = m->t1.N[q1 * np + i];
              const double *src = &cq[(((size_t)q3 * nq + q2) * nq + q1) * M];
              double *dst = &t1v[(((size_t)q3 * nq + q2) * np + i) * M];
              for (int e = 0; e < M; ++e) dst[e] += nv * src[e];
            }
      t2v.assign((size_t)nq * np * np * M, 0.0);
      for (int q3 = 0; q3 < nq; ++q3)
        for (int j = 0; j < np; ++j)
          for (int q2 = 0; q2 < nq; ++q2) {
            const double nv = m->t1.N[q2 * np + j];
            for (int i = 0; i < np; ++i) {
              const double *src = &t1v[(((size_t)q3 * nq + q2) * np + i) * M];
              double *dst = &t2v[(((size_t)q3 * np + j) * np + i) * M];
              for (int e = 0; e < M; ++e) dst[e] += nv * src[e];
            }
          }
      std::fill(cellF.begin(), cellF.end(), 0.0);
      for (int kk2 = 0; kk2 < np; ++kk2)
        for (int q3 = 0; q3 < nq; ++q3) {
          const double nv = m->t1.N[q3 * np + kk2];
          for (int jj = 0; jj < np * np; ++jj) {
            const double *src = &t2v[((size_t)q3 * np * np + jj) * M];
            double *dst = &cellF[((size_t)kk2 * np * np + jj) * M];
            for (int e = 0; e < M; ++e) dst[e] += nv * src[e];
          }
        }
      for (int kk2 = 0; kk2 < np; ++kk2)
        for (int j = 0; j < np; ++j)
          for (int i = 0; i < np; ++i) {
            const int64_t g = dof_of(m, c, i, j, kk2);
            if (g < 0) continue;                      // Dirichlet face: no DoF
            auto it = local.find(g);
            int row;
            if (it == local.end()) {
              row = (int)order.size();
              local.emplace(g, row);
              order.push_back(g);
              blk.resize(order.size() * M, 0.0);
            } else {
              row = it->second;
            }
            const double *src = &cellF[((size_t)(kk2 * np + j) * np + i) * M];
            for (int e = 0; e < M; ++e) blk[(size_t)row * M + e] += src[e];
          }
    }
    // sort this atom's support nodes for ordered memory access
    std::vector<int> perm(order.size());
    std::iota(perm.begin(), perm.end(), 0);
    std::sort(perm.begin(), perm.end(), [&](int x, int y) { return order[x] < order[y]; });
    for (int r : perm) {
      atom_nodes.push_back((int)order[r]);
      for (int e = 0; e < maxp * C; ++e) Fblk.push_back(blk[(size_t)r * maxp * C + e]);
      for (int s = 0; s < na; ++s) {
        const double re = blk[((size_t)r * maxp + s) * C];
        const double im = cplx ? blk[((size_t)r * maxp + s) * C + 1] : 0.0;
        if (re != 0.0 || im != 0.0) ents.push_back({order[r], s0 + s, re, im});
      }
    }
    atom_off.push_back((int)atom_nodes.size());
  }
  // node-CSR of P
  std::sort(ents.begin(), ents.end(), [](const Ent &x, const Ent &y) {
    return x.node != y.node ? x.node < y.node : x.s < y.s; });
  std::vector<int> rows, rowptr(1, 0), colidx;
  std::vector<double> val;
  for (size_t e = 0; e < ents.size(); ++e) {
    if (rows.empty() || rows.back() != (int)ents[e].node) {
      if (!rows.empty()) rowptr.push_back((int)colidx.size());
      rows.push_back((int)ents[e].node);
    }
    colidx.push_back(ents[e].s);
    val.push_back(ents[e].re);
    if (cplx) val.push_back(ents[e].im);
  }
  rowptr.push_back((int)colidx.size());
  if (rows.empty()) rowptr.assign(1, 0);
  std::vector<double> hv(nproj);
  std::vector<int> proj_atom(nproj);
  for (int s = 0; s < nproj; ++s) { hv[s] = proj[s].h; proj_atom[s] = proj[s].atom; }
  // node chunks of each atom's support list for the W reduction
  std::vector<int> chunk_atom, chunk_n0, atom_chunk0(1, 0);
  for (int a = 0; a < natoms; ++a) {
    for (int n0 = atom_off[a]; n0 < atom_off[a + 1]; n0 += NL_CHUNK) {
      chunk_atom.push_back(a);
      chunk_n0.push_back(n0);
    }
    atom_chunk0.push_back((int)chunk_atom.size());
  }
  // Execution order of the chunks: by the node in the middle of each chunk, so
  // that chunks of different atoms covering one region run close in time and
  // the X rows they share are read again from the caches instead of HBM.
  // (The partials keep their per-atom order, so the sums are unchanged.)
  std::vector<int> chunk_order(chunk_atom.size());
  {
    std::vector<std::pair<int, int>> key(chunk_atom.size());
    for (size_t c = 0; c < chunk_atom.size(); ++c) {
      const int a = chunk_atom[c], n0 = chunk_n0[c];
      const int mid = std::min(n0 + NL_CHUNK / 2, atom_off[a + 1] - 1);
      key[c] = {atom_nodes[mid], (int)c};
    }
    std::sort(key.begin(), key.end());
    for (size_t c = 0; c < key.size(); ++c) chunk_order[c] = key[c].second;
  }
  // Brick partition of the rows for the LDS-staged update: rows grouped by
  // 8^3-node bricks of the node grid, a brick split into its eight 4^3
  // sub-bricks when it touches more than NL_BPMAX projectors; rows of a
  // sub-brick that still touches more stay in the global-W CSR.
  std::vector<int> b_row0(1, 0), b_p0(1, 0), b_proj, b_rows, b_rowptr(1, 0), b_lcol;
  std::vector<double> b_val;
  std::vector<int> o_rows, o_rowptr(1, 0), o_col;
  std::vector<double> o_val;
  int bmaxp = 0;
  {
    const int64_t M0 = m->Mn[0], M1 = m->Mn[1];
    auto coord = [&](int r, int d) -> int64_t {
      const int64_t g = rows[r];
      return d == 0 ? g % M0 : (d == 1 ? (g / M0) % M1 : g / (M0 * M1));
    };
    std::vector<int> cols_tmp;
    auto distinct_cols = [&](const std::vector<int> &rl) {
      cols_tmp.clear();
      for (int r : rl)
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) cols_tmp.push_back(colidx[e]);
      std::sort(cols_tmp.begin(), cols_tmp.end());
      cols_tmp.erase(std::unique(cols_tmp.begin(), cols_tmp.end()), cols_tmp.end());
      return (int)cols_tmp.size();
    };
    auto brick = [&](const std::vector<int> &rl) {   // cols_tmp: the brick's projectors
      bmaxp = std::max(bmaxp, (int)cols_tmp.size());
      for (int c : cols_tmp) b_proj.push_back(c);
      for (int r : rl) {
        b_rows.push_back(rows[r]);
        int k = 0;
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e, ++k) {
          b_lcol.push_back((int)(std::lower_bound(cols_tmp.begin(), cols_tmp.end(), colidx[e]) - cols_tmp.begin()));
          for (int c = 0; c < C; ++c) b_val.push_back(val[(size_t)e * C + c]);
        }
        for (; k % 8; ++k) {
          b_lcol.push_back(0);
          for (int c = 0; c < C; ++c) b_val.push_back(0.0);
        }
        b_rowptr.push_back((int)b_lcol.size() / 4);
      }
      b_row0.push_back((int)b_rows.size());
      b_p0.push_back((int)b_proj.size());
    };
    auto overflow = [&](const std::vector<int> &rl) {
      for (int r : rl) {
        o_rows.push_back(rows[r]);
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          o_col.push_back(colidx[e]);
          for (int c = 0; c < C; ++c) o_val.push_back(val[(size_t)e * C + c]);
        }
        o_rowptr.push_back((int)o_col.size());
      }
    };
    std::map<int64_t, std::vector<int>> bricks;
    const int64_t nbx = (M0 + 7) / 8, nby = (M1 + 7) / 8;
    for (int r = 0; r < (int)rows.size(); ++r)
      bricks[(coord(r, 2) / 8 * nby + coord(r, 1) / 8) * nbx + coord(r, 0) / 8].push_back(r);
    for (auto &kv : bricks) {
      if (distinct_cols(kv.second) <= NL_BPMAX) { brick(kv.second); continue; }
      std::vector<int> sub[8];
      for (int r : kv.second)
        sub[((coord(r, 0) / 4) & 1) | (((coord(r, 1) / 4) & 1) << 1) | (((coord(r, 2) / 4) & 1) << 2)].push_back(r);
      for (int k = 0; k < 8; ++k) {
        if (sub[k].empty()) continue;
        if (distinct_cols(sub[k]) <= NL_BPMAX) brick(sub[k]);
        else overflow(sub[k]);
      }
    }
  }
  // the same bricks as dense blocks for the FP64 matrix-core update: brick b
  // holds rows x K_b values, K_b = C P_b rounded up to 4, entry (row, C p + c)
  std::vector<double> b_A;
  std::vector<int64_t> b_aoff;
  std::vector<int> b_k;
  int b_kmax = 0;
  for (size_t b = 0; !m->host_only && b + 1 < b_row0.size(); ++b) {   // host-only meshes upload nothing
    const int K = (C * (b_p0[b + 1] - b_p0[b]) + 3) / 4 * 4;
    b_kmax = std::max(b_kmax, K);
    b_k.push_back(K);
    b_aoff.push_back((int64_t)b_A.size());
    const size_t base = b_A.size();
    b_A.resize(base + (size_t)(b_row0[b + 1] - b_row0[b]) * K, 0.0);
    for (int r = b_row0[b]; r < b_row0[b + 1]; ++r)
      for (int g = b_rowptr[r] * 4; g < b_rowptr[r + 1] * 4; ++g)   // padding entries add zero
        for (int c = 0; c < C; ++c)
          b_A[base + (size_t)(r - b_row0[b]) * K + C * b_lcol[g] + c] += b_val[(size_t)g * C + c];
  }
  fe_status st;
  if ((st = upload(m, &m->nl_atom_off, atom_off))) return st;
  if ((st = upload(m, &m->nl_atom_nodes, atom_nodes))) return st;
  if ((st = upload(m, &m->nl_atom_proj, proj_off))) return st;
  if ((st = upload(m, &m->nl_F64, Fblk))) return st;
  if ((st = upload(m, &m->nl_F32, to_f32(Fblk)))) return st;
  if ((st = upload(m, &m->nl_rows, o_rows))) return st;
  if ((st = upload(m, &m->nl_rowptr, o_rowptr))) return st;
  if ((st = upload(m, &m->nl_colidx, o_col))) return st;
  if ((st = upload(m, &m->nl_val64, o_val))) return st;
  if ((st = upload(m, &m->nl_val32, to_f32(o_val)))) return st;
  if ((st = upload(m, &m->nl_b_row0, b_row0))) return st;
  if ((st = upload(m, &m->nl_b_p0, b_p0))) return st;
  if ((st = upload(m, &m->nl_b_proj, b_proj))) return st;
  if ((st = upload(m, &m->nl_b_rows, b_rows))) return st;
  if ((st = upload(m, &m->nl_b_rowptr, b_rowptr))) return st;
  if ((st = upload(m, &m->nl_b_lcol, b_lcol))) return st;
  if ((st = upload(m, &m->nl_b_val32, to_f32(b_val)))) return st;
  if ((st = upload(m, &m->nl_b_A64, b_A))) return st;
  if ((st = upload(m, &m->nl_b_aoff, b_aoff))) return st;
  if ((st = upload(m, &m->nl_b_k, b_k))) return st;
  m->nl_b_kmax = b_kmax;
  m->nl_nbrick = (int)b_row0.size() - 1;
  m->nl_bmaxp = bmaxp;
  if ((st = upload(m, &m->nl_h, hv))) return st;
  if ((st = upload(m, &m->nl_chunk_atom, chunk_atom))) return st;
  if ((st = upload(m, &m->nl_chunk_n0, chunk_n0))) return st;
  if ((st = upload(m, &m->nl_chunk_order, chunk_order))) return st;
  if ((st = upload(m, &m->nl_atom_chunk0, atom_chunk0))) return st;
  if ((st = upload(m, &m->nl_proj_atom, proj_atom))) return st;
  m->nl_nchunks = (int)chunk_atom.size();
  m->natoms = natoms;
  m->ns = nproj;
  m->nl_maxproj = maxp;
  m->nl_nsup = (int64_t)atom_nodes.size();
  m->nl_nrows = (int64_t)o_rows.size();
  m->nl_nnz = (int64_t)o_col.size();
  m->h_h = hv;
  m->h_atom_off = atom_off;
  m->h_atom_proj = proj_off;
  m->h_rows = rows;
  m->h_rowptr = rowptr;
  m->h_colidx = colidx;
  m->h_val = val;
  return FE_OK;
}

fe_status fe_projector_entries(fe_mesh_t m, int64_t *nnz, int32_t *rows, int32_t *cols, double *vals) {
  if (!m || !nnz) return set_error(FE_EINVAL, "NULL argument");
  *nnz = (int64_t)m->h_colidx.size();
  if (!rows && !cols && !vals) return FE_OK;
  if (!rows || !cols || !vals) return set_error(FE_EINVAL, "rows, cols and vals must all be given");
  const int C = m->cplx ? 2 : 1;
  for (size_t r = 0; r + 1 < m->h_rowptr.size(); ++r)
    for (int e = m->h_rowptr[r]; e < m->h_rowptr[r + 1]; ++e) {
      rows[e] = m->h_rows[r];
      cols[e] = m->h_colidx[e];
      for (int q = 0; q < C; ++q) vals[(size_t)e * C + q] = m->h_val[(size_t)e * C + q];
    }
  return FE_OK;
}

fe_status fe_apply_H(fe_mesh_t m, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t nvec,
                     int32_t prec, void *stream) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (nvec < 0) return set_error(FE_EINVAL, "nvec must be >= 0");
  if (nvec == 0) return FE_OK;
  if (!X || !Y) return set_error(FE_EINVAL, "NULL vector block");
  if (ldx < nvec || ldy < nvec) return set_error(FE_EINVAL, "leading dimension smaller than nvec");
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16) return set_error(FE_EINVAL, "unknown precision");
  if (blocks_overlap(X, ldx, Y, ldy, m->m, nvec, block_elem_bytes(prec, m->cplx)))
    return set_error(FE_EINVAL, "X and Y must not overlap");
  const int C = m->cplx ? 2 : 1;
  if (nvec * C > (1 << 30)) return set_error(FE_EINVAL, "nvec too large");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0) cannot apply H");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  LocalLaunch L;
  L.X = X; L.Y = Y; L.ldx = ldx * C; L.ldy = ldy * C; L.nlanes = (int)(nvec * C); L.prec = prec;
  L.vt = m->vt_pref[prec][0];
  return apply_with_nonlocal(m, L, prec, nullptr, 1.0, s);
}

fe_status fe_apply_M(fe_mesh_t m, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t nvec, int32_t prec,
                     void *stream) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (nvec < 0) return set_error(FE_EINVAL, "nvec must be >= 0");
  if (nvec == 0) return FE_OK;
  if (!X || !Y) return set_error(FE_EINVAL, "NULL vector block");
  if (ldx < nvec || ldy < nvec) return set_error(FE_EINVAL, "leading dimension smaller than nvec");
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16) return set_error(FE_EINVAL, "unknown precision");
  if (blocks_overlap(X, ldx, Y, ldy, m->m, nvec, block_elem_bytes(prec, m->cplx)))
    return set_error(FE_EINVAL, "X and Y must not overlap");
  const int C = m->cplx ? 2 : 1;
  if (nvec * C > (1 << 30)) return set_error(FE_EINVAL, "nvec too large");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0) cannot apply M");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  LocalLaunch L;
  L.X = X; L.Y = Y; L.ldx = ldx * C; L.ldy = ldy * C; L.nlanes = (int)(nvec * C); L.prec = prec;
  L.vt = m->vt_pref[prec][0];
  L.mass = true;
  return launch_local(m, L, (hipStream_t)stream);
}

fe_status fe_set_mass(fe_mesh_t m, int32_t kind) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh handle");
  if (kind != FE_MASS_LUMPED && kind != FE_MASS_CONSISTENT) return set_error(FE_EINVAL, "unknown mass kind");
  m->mass_kind = kind;
  return FE_OK;
}

fe_status fe_batch_apply(int32_t n, const fe_mesh_t *meshes, const void *const *X, const int64_t *ldx,
                         void *const *Y, const int64_t *ldy, const int64_t *nvec, int32_t prec, void *stream) {
  if (n <= 0) return FE_OK;
  if (!meshes || !X || !ldx || !Y || !ldy || !nvec) return set_error(FE_EINVAL, "NULL argument");
  if (prec < FE_F64 || prec > FE_BF16) return set_error(FE_EINVAL, "unknown precision");
  for (int i = 0; i < n; ++i) {
    fe_mesh_t m = meshes[i];
    if (!m || !X[i] || !Y[i]) return set_error(FE_EINVAL, "NULL mesh or block in the batch");
    if (m->host_only) return set_error(FE_ESTATE, "host-only mesh in the batch");
    if (nvec[i] <= 0 || ldx[i] < nvec[i] || ldy[i] < nvec[i]) return set_error(FE_EINVAL, "bad nvec / ld in the batch");
    if (blocks_overlap(X[i], ldx[i], Y[i], ldy[i], m->m, nvec[i], block_elem_bytes(prec, m->cplx)))
      return set_error(FE_EINVAL, "input and output blocks must not overlap");
    if (m->device != meshes[0]->device) return set_error(FE_EINVAL, "all meshes of a batch must be on one device");
    for (int j = 0; j < i; ++j)
      if (meshes[j] == m) return set_error(FE_EINVAL, "a mesh may appear only once in a batch (its workspaces are shared)");
  }
  if (hipSetDevice(meshes[0]->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  // projector reductions of every system (FP32 / BF16: on the meshes' second
  // streams), the batched local launches, then the projector updates
  for (int i = 0; i < n; ++i) {
    const int C = meshes[i]->cplx ? 2 : 1;
    fe_status st = fehx::nonlocal_reduce(meshes[i], X[i], ldx[i] * C, (int)(nvec[i] * C), prec, nullptr, s);
    if (st) return st;
  }
  // group by launch class, keeping the caller's order inside a class
  std::vector<int> done(n, 0);
  for (int i = 0; i < n; ++i) {
    if (done[i]) continue;
    std::vector<fehx::Mesh *> ms;
    std::vector<fehx::LocalLaunch> Ls;
    for (int j = i; j < n; ++j) {
      fe_mesh_t a = meshes[i], b = meshes[j];
      if (done[j] || b->np != a->np || b->nq != a->nq || b->cplx != a->cplx ||
          b->vt_pref[prec][0] != a->vt_pref[prec][0])
        continue;
      const int C = b->cplx ? 2 : 1;
      fehx::LocalLaunch L;
      L.X = X[j]; L.Y = Y[j]; L.ldx = ldx[j] * C; L.ldy = ldy[j] * C; L.nlanes = (int)(nvec[j] * C);
      L.prec = prec; L.vt = b->vt_pref[prec][0];
      ms.push_back(b);
      Ls.push_back(L);
      done[j] = 1;
    }
    // A system whose every colour phase has at least two blocks per CU
    // fills the device on its own; when all of a class do, separate launches
    // (same per-item arithmetic) beat the persistent batch, whose blocks
    // stride over all systems' work lists.
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ms[0]->device) != hipSuccess || cus <= 0)
      cus = 256;
    bool all_large = true;
    for (size_t j = 0; j < ms.size(); ++j) {
      const int vt = Ls[j].vt ? Ls[j].vt : (prec == FE_F64 ? 8 : 16);
      const int64_t tiles = (Ls[j].nlanes + vt - 1) / vt;
      int minc = INT32_MAX;
      for (int ph = 0; ph < ms[j]->nphase; ++ph)
        minc = std::min(minc, ms[j]->phase_off[ph + 1] - ms[j]->phase_off[ph]);
      if ((int64_t)minc * tiles < 2LL * cus) all_large = false;
    }
    if (all_large && ms.size() > 1) {
      for (size_t j = 0; j < ms.size(); ++j) {
        fe_status st = fehx::launch_local(ms[j], Ls[j], s);
        if (st) return st;
      }
      continue;
    }
    fehx::LocalBatch B;
    B.ms = ms.data();
    B.Ls = Ls.data();
    B.n = (int)ms.size();
    B.persistent = true;
    fe_status st = fehx::launch_local_batch(B, s);
    if (st) return st;
  }
  for (int i = 0; i < n; ++i) {
    const int C = meshes[i]->cplx ? 2 : 1;
    fe_status st = fehx::nonlocal_update(meshes[i], Y[i], ldy[i] * C, (int)(nvec[i] * C), prec, 1.0, s);
    if (st) return st;
  }
  return FE_OK;
}

}  // extern "C"
