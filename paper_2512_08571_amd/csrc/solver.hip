// Eigensolver pieces around H.X: the residual Chebyshev filter (Alg. 4),
// Lanczos spectral bounds and the Rayleigh-Ritz step (Alg. 3), with M the
// lumped D or the consistent mass matrix.
//
// Filter data flow (Alg. 4; D^-1 is always the lumped inverse):
//   Y   = H X  (FP64), then one streaming pass forms Y - M X Lambda,
//         R_Y = (sigma1/e) Y, Ylp = Y in the block precision, R_X = 0
//   (block precision: FP64 for FP64 steps, FP32 for FP32 and for BF16 steps,
//    whose operator alone takes BF16 operands on the matrix cores)
//   step k: T = H D^-1 R_Y  (local + nonlocal operator on R_Y, D^-1 applied
//           at the gather), then one streaming pass
//           R_X <- a T - a c R_Y + a Lambda_Y Ylp - sigma sigma2 R_X;
//           the two blocks swap roles
//   X   = D^-1 R_Y + X Lambda_Y                     FP64
// The update is a separate streaming pass rather than folded into the
// operator's stores: the folded form raised the operator kernel's register
// use (and so lowered its occupancy) by more than the pass costs.
// The per-vector scalars Lambda_X, Lambda_Y obey a recurrence independent of
// the vectors; a one-thread-per-vector kernel tabulates Lambda_Y for every
// step from the device-resident Ritz values, so a pass never waits on the
// host and can be captured in a graph.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>

#include "fe_internal.h"

namespace fehx {

template <typename TS> struct VCvt;
template <> struct VCvt<double> {
  static __device__ double ld(const double *p, int64_t i) { return p[i]; }
  static __device__ void st(double *p, int64_t i, double v) { p[i] = v; }
};
template <> struct VCvt<float> {
  static __device__ double ld(const float *p, int64_t i) { return p[i]; }
  static __device__ void st(float *p, int64_t i, double v) { p[i] = (float)v; }
};

// Y <- Y - M X Lambda (Y = H X on entry, FP64 [m][lanes]; M X = D X, or the
// given consistent-mass product MX [m][lanes]); R_Y = s Y, Ylp = Y (when the
// inner precision differs), R_X = 0 (unless RX is null: then R_X overlaps Y
// and is cleared afterwards).  Rows over blocks, lanes over threads.
template <typename TS>
__global__ void k_filter_init(double *__restrict__ Y, const double *__restrict__ X, int64_t ldx,
                              const double *__restrict__ MX, int64_t m, int lanes, int cplx,
                              const double *__restrict__ dmass, const double *__restrict__ lam, double s,
                              TS *__restrict__ RY, TS *__restrict__ Ylp, TS *__restrict__ RX) {
  for (int64_t g = blockIdx.x; g < m; g += gridDim.x) {
    const double d = dmass[g];
    for (int v = threadIdx.x; v < lanes; v += blockDim.x) {
      const int64_t t = g * lanes + v;
      const double mx = MX ? MX[t] : d * X[g * ldx + v];
      const double y = Y[t] - lam[cplx ? (v >> 1) : v] * mx;
      Y[t] = y;
      VCvt<TS>::st(RY, t, s * y);
      if (Ylp) VCvt<TS>::st(Ylp, t, y);
      if (RX) VCvt<TS>::st(RX, t, 0.0);
    }
  }
}

// x[0..n) = 0
template <typename T>
__global__ void k_zero(T *__restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

// R_X <- a T - ac R_Y + a Lambda_Y Ylp - s2 R_X  (all [m][lanes], inner precision)
template <typename TS>
__global__ void k_filter_combine(const TS *__restrict__ T, const TS *__restrict__ RY, const TS *__restrict__ Ylp,
                                 TS *__restrict__ RX, int64_t m, int lanes, int cplx, const double *__restrict__ lamk,
                                 double a, double ac, double s2) {
  for (int64_t g = blockIdx.x; g < m; g += gridDim.x) {
    for (int v = threadIdx.x; v < lanes; v += blockDim.x) {
      const int64_t t = g * lanes + v;
      const double ly = lamk[cplx ? (v >> 1) : v];
      double r = a * VCvt<TS>::ld(T, t) - ac * VCvt<TS>::ld(RY, t) + a * ly * VCvt<TS>::ld(Ylp, t);
      if (s2 != 0.0) r -= s2 * VCvt<TS>::ld(RX, t);
      VCvt<TS>::st(RX, t, r);
    }
  }
}

// Four adjacent lanes of a [m][lanes] block as one access (lanes a multiple
// of 4, so a group stays inside its row; the blocks are 256-byte aligned)
template <typename TS> struct V4;
template <> struct V4<double> {
  static __device__ void ld(const double *p, int64_t i, double v[4]) {
    const double2 a = *(const double2 *)(p + i), b = *(const double2 *)(p + i + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  static __device__ void st(double *p, int64_t i, const double v[4]) {
    *(double2 *)(p + i) = make_double2(v[0], v[1]);
    *(double2 *)(p + i + 2) = make_double2(v[2], v[3]);
  }
};
template <> struct V4<float> {
  static __device__ void ld(const float *p, int64_t i, double v[4]) {
    const float4 a = *(const float4 *)(p + i);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  static __device__ void st(float *p, int64_t i, const double v[4]) {
    *(float4 *)(p + i) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
};

// The same update with four lanes per thread (lanes % 4 == 0): a block takes
// 256 / (lanes / 4) rows at a time when a row has at most 256 groups, else
// one row with its groups strided over the threads.
template <typename TS>
__global__ void k_filter_combine4(const TS *__restrict__ T, const TS *__restrict__ RY, const TS *__restrict__ Ylp,
                                  TS *__restrict__ RX, int64_t m, int lanes, int cplx,
                                  const double *__restrict__ lamk, double a, double ac, double s2) {
  const int G = lanes >> 2;
  const int R = G < (int)blockDim.x ? (int)blockDim.x / G : 1;
  const int rr = G < (int)blockDim.x ? (int)threadIdx.x / G : 0;
  const int q0 = G < (int)blockDim.x ? (int)threadIdx.x % G : (int)threadIdx.x;
  const int qs = G < (int)blockDim.x ? G : (int)blockDim.x;
  if (rr >= R) return;
  for (int64_t g = (int64_t)blockIdx.x * R + rr; g < m; g += (int64_t)gridDim.x * R) {
    for (int qg = q0; qg < G; qg += qs) {
      const int v = qg * 4;
      const int64_t t = g * lanes + v;
      double x[4], ry[4], yl[4], rx[4] = {0, 0, 0, 0};
      V4<TS>::ld(T, t, x);
      V4<TS>::ld(RY, t, ry);
      V4<TS>::ld(Ylp, t, yl);
      if (s2 != 0.0) V4<TS>::ld(RX, t, rx);
      double r[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double ly = lamk[cplx ? ((v + j) >> 1) : (v + j)];
        r[j] = a * x[j] - ac * ry[j] + a * ly * yl[j];
        if (s2 != 0.0) r[j] -= s2 * rx[j];
      }
      V4<TS>::st(RX, t, r);
    }
  }
}

// X = D^-1 R_Y + X Lambda_Y   (X FP64 [m][ldx], R_Y TS [m][lanes])
template <typename TS>
__global__ void k_filter_final(double *__restrict__ X, int64_t ldx, const TS *__restrict__ RY, int64_t m,
                               int lanes, int cplx, const double *__restrict__ dinv,
                               const double *__restrict__ LY) {
  const int64_t n = m * lanes;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = t / lanes;
    const int v = (int)(t - g * lanes);
    const double ly = LY[cplx ? (v >> 1) : v];
    X[g * ldx + v] = dinv[g] * VCvt<TS>::ld(RY, t) + X[g * ldx + v] * ly;
  }
}

// out[i] = sum_k part[k stride + i], k = 0..nparts-1 in order
__global__ void k_sum_parts(const double *__restrict__ part, int64_t stride, int nparts, int64_t len,
                            double *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += part[k * stride + i];
    out[i] = s;
  }
}

// out[g][v] = d[g]^pw * in[g][v] over [m][lanes] with leading dims
__global__ void k_scale_rows(const double *__restrict__ in, int64_t ldi, double *__restrict__ out, int64_t ldo,
                             int64_t m, int lanes, const double *__restrict__ d, int sqrt_pw) {
  const int64_t n = m * lanes;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = t / lanes;
    const int v = (int)(t - g * lanes);
    const double f = sqrt_pw ? sqrt(d[g]) : d[g];
    out[g * ldo + v] = f * in[g * ldi + v];
  }
}

// Lambda_Y of every recurrence step, table[(k - 2) nvec + i] for k = 2..p and
// the final value at table[p nvec + i] (Alg. 4's scalar recurrences)
__global__ void k_filter_tables(const double *__restrict__ lam, int64_t nvec, int degree, double e, double c,
                                double sigma1, double *__restrict__ table) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nvec) return;
  const double l = lam[i];
  const double gamma = 2.0 / sigma1;
  double sigma = sigma1, LX = 1.0, LY = sigma1 / e * (l - c);
  for (int k = 2; k <= degree; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    table[(int64_t)(k - 2) * nvec + i] = LY;
    const double lxn = 2.0 * sigma2 / e * LY * (l - c) - sigma * sigma2 * LX;
    LX = LY;
    LY = lxn;
    sigma = sigma2;
  }
  table[(int64_t)degree * nvec + i] = LY;
}

namespace {

inline dim3 rows_grid(int64_t m) { return dim3((unsigned)(m < 65536 ? m : 65536)); }

inline dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

// tiny symmetric tridiagonal eigenvalues by cyclic Jacobi on a dense copy
std::vector<double> tridiag_eigs(const std::vector<double> &al, const std::vector<double> &be) {
  const int n = (int)al.size();
  std::vector<double> A((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    A[i * n + i] = al[i];
    if (i + 1 < n) A[i * n + i + 1] = A[(i + 1) * n + i] = be[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
  std::sort(ev.begin(), ev.end());
  return ev;
}

struct Blas {
  rocblas_handle h = nullptr;
  ~Blas() { if (h) rocblas_destroy_handle(h); }
};

fe_status rb(rocblas_status st, const char *what) {
  if (st != rocblas_status_success) return set_error(FE_EDEVICE, std::string(what) + " failed: " + rocblas_status_to_string(st));
  return FE_OK;
}

}  // namespace


static size_t prec_bytes(int prec) { return prec == FE_F64 ? 8 : (prec == FE_F32 ? 4 : 2); }

fe_status filter_setup(FilterPlan &P, Mesh *m, double *X, int64_t ldx_l, const double *lam, int64_t nvec,
                       int degree, double lmin, double lT, double lmax, int prec) {
  P = FilterPlan();
  P.m = m; P.X = X; P.ldx = ldx_l; P.lam = lam; P.nvec = nvec; P.degree = degree; P.prec = prec;
  // BF16 steps keep the recurrence state in FP32; only the operator's
  // contractions take BF16 (hi/lo) operands on the matrix cores
  P.sprec = prec == FE_F64 ? FE_F64 : FE_F32;
  const int C = m->cplx ? 2 : 1;
  P.lanes = (int)(nvec * C);
  P.e = (lmax - lT) / 2.0;
  P.c = (lmax + lT) / 2.0;
  P.sigma1 = P.e / (lmin - P.c);
  double sigma = P.sigma1;
  const double gamma = 2.0 / P.sigma1;
  for (int k = 2; k <= degree; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    P.alpha.push_back(2.0 * sigma2 / P.e);
    P.s2.push_back(sigma * sigma2);
    sigma = sigma2;
  }
  const int64_t n = m->m * P.lanes;
  const size_t ts = prec_bytes(P.sprec);
  fe_status st;
  // FP32 / BF16: the FP64 Y lives in the R_X + H D^-1 R_Y block (it is dead
  // after the prologue, and those two are first written after it)
  const bool share = prec != FE_F64;
  if (!share && (st = ensure_workspace(m, 0, n * (int64_t)sizeof(double)))) return st;   // Y (FP64)
  if ((st = ensure_workspace(m, 1, n * (int64_t)ts))) return st;               // R_Y
  if ((st = ensure_workspace(m, 2, share ? filter_shared_bytes(n, (int64_t)ts) : n * (int64_t)ts))) return st;   // R_X
  const bool sep = prec != FE_F64;
  if (sep && (st = ensure_workspace(m, 3, n * (int64_t)ts))) return st;        // Y in the inner precision
  if ((st = ensure_workspace(m, 4, (int64_t)(degree + 1) * nvec * (int64_t)sizeof(double)))) return st;
  if (!share && (st = ensure_workspace(m, 8, n * (int64_t)ts))) return st;     // H D^-1 R_Y
  if (m->mass_kind == FE_MASS_CONSISTENT && (st = ensure_workspace(m, 9, n * (int64_t)sizeof(double))))
    return st;                                                                  // M X (FP64)
  if ((st = ensure_nl_workspace(m, P.lanes))) return st;
  P.Y = (double *)m->ws[share ? 2 : 0];
  P.RY = m->ws[1];
  P.RX = m->ws[2];
  P.Ylp = sep ? m->ws[3] : m->ws[0];
  P.tab = (double *)m->ws[4];
  P.T = share ? (void *)((char *)m->ws[2] + filter_t_offset(n, (int64_t)ts)) : m->ws[8];
  P.k = 2;
  return FE_OK;
}

fe_status filter_prologue(FilterPlan &P, hipStream_t s) {
  Mesh *m = P.m;
  hipLaunchKernelGGL(k_filter_tables, dim3((unsigned)((P.nvec + 255) / 256)), dim3(256), 0, s, P.lam, P.nvec,
                     P.degree, P.e, P.c, P.sigma1, P.tab);
  FE_HIP_TRY(hipGetLastError());
  // Y = H X (FP64), then Y - D X Lambda and the recurrence blocks in one pass
  LocalLaunch L0;
  L0.X = P.X; L0.Y = P.Y; L0.ldx = P.ldx; L0.ldy = P.lanes; L0.nlanes = P.lanes; L0.prec = FE_F64;
  L0.vt = m->vt_pref[FE_F64][0];
  fe_status st;
  if ((st = apply_with_nonlocal(m, L0, FE_F64, nullptr, 1.0, s))) return st;
  const double *MX = nullptr;
  if (m->mass_kind == FE_MASS_CONSISTENT) {
    LocalLaunch LM = L0;
    LM.Y = m->ws[9];
    LM.mass = true;
    if ((st = launch_local(m, LM, s))) return st;
    MX = (const double *)m->ws[9];
  }
  const double sc = P.sigma1 / P.e;
  const int cpl = m->cplx ? 1 : 0;
  switch (P.sprec) {
    case FE_F64:
      hipLaunchKernelGGL(k_filter_init<double>, rows_grid(m->m), dim3(256), 0, s, P.Y, P.X, P.ldx, MX, m->m,
                         P.lanes, cpl, m->dmass, P.lam, sc, (double *)P.RY, (double *)nullptr, (double *)P.RX);
      break;
    default:       // FP32 blocks; R_X overlaps Y here: cleared after Y is consumed
      hipLaunchKernelGGL(k_filter_init<float>, rows_grid(m->m), dim3(256), 0, s, P.Y, P.X, P.ldx, MX, m->m,
                         P.lanes, cpl, m->dmass, P.lam, sc, (float *)P.RY, (float *)P.Ylp, (float *)nullptr);
      FE_HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(k_zero<float>, grid_for(m->m * P.lanes), dim3(256), 0, s, (float *)P.RX, m->m * P.lanes);
  }
  FE_HIP_TRY(hipGetLastError());
  P.k = 2;
  return FE_OK;
}

// step k, operator part: T = H D^-1 R_Y (the local launch; the projector
// part follows in filter_step_rest)
LocalLaunch filter_step_local(const FilterPlan &P) {
  LocalLaunch L;
  L.X = P.RY; L.Y = P.T; L.ldx = P.lanes; L.ldy = P.lanes; L.nlanes = P.lanes; L.prec = P.prec;
  L.store32 = P.prec == FE_BF16;
  L.dinv_gather = P.m->dinv;
  L.vt = P.m->vt_pref[P.prec][1];
  return L;
}

fe_status filter_step_reduce(FilterPlan &P, hipStream_t s) {
  return nonlocal_reduce(P.m, P.RY, P.lanes, P.lanes, P.sprec, P.m->dinv, s);
}

// step k, rest: T += F W, then R_X <- a [T - c R_Y + Ylp Lambda_Y] - sigma sigma2 R_X
fe_status filter_step_rest(FilterPlan &P, hipStream_t s) {
  const int k = P.k;
  const double a = P.alpha[k - 2], s2 = k > 2 ? P.s2[k - 2] : 0.0;
  Mesh *m = P.m;
  fe_status st = nonlocal_update(m, P.T, P.lanes, P.lanes, P.sprec, 1.0, s);
  if (st) return st;
  const double *lamk = P.tab + (size_t)(k - 2) * P.nvec;
  const int cpl = m->cplx ? 1 : 0;
  if (P.lanes % 4 == 0) {
    const int G = P.lanes / 4;
    const int R = G < 256 ? 256 / G : 1;
    int64_t blocks = (m->m + R - 1) / R;
    if (blocks > 65536) blocks = 65536;
    const dim3 grid((unsigned)blocks);
    if (P.sprec == FE_F64)
      hipLaunchKernelGGL(k_filter_combine4<double>, grid, dim3(256), 0, s, (const double *)P.T,
                         (const double *)P.RY, (const double *)P.Ylp, (double *)P.RX, m->m, P.lanes, cpl, lamk, a,
                         a * P.c, s2);
    else
      hipLaunchKernelGGL(k_filter_combine4<float>, grid, dim3(256), 0, s, (const float *)P.T,
                         (const float *)P.RY, (const float *)P.Ylp, (float *)P.RX, m->m, P.lanes, cpl, lamk, a,
                         a * P.c, s2);
  } else {
    if (P.sprec == FE_F64)
      hipLaunchKernelGGL(k_filter_combine<double>, rows_grid(m->m), dim3(256), 0, s, (const double *)P.T,
                         (const double *)P.RY, (const double *)P.Ylp, (double *)P.RX, m->m, P.lanes, cpl, lamk, a,
                         a * P.c, s2);
    else
      hipLaunchKernelGGL(k_filter_combine<float>, rows_grid(m->m), dim3(256), 0, s, (const float *)P.T,
                         (const float *)P.RY, (const float *)P.Ylp, (float *)P.RX, m->m, P.lanes, cpl, lamk, a,
                         a * P.c, s2);
  }
  FE_HIP_TRY(hipGetLastError());
  std::swap(P.RX, P.RY);
  ++P.k;
  return FE_OK;
}

fe_status filter_final(FilterPlan &P, hipStream_t s) {
  Mesh *m = P.m;
  const int64_t n = m->m * P.lanes;
  const int cpl = m->cplx ? 1 : 0;
  const double *LY = P.tab + (size_t)P.degree * P.nvec;
  if (P.sprec == FE_F64)
    hipLaunchKernelGGL(k_filter_final<double>, grid_for(n), dim3(256), 0, s, P.X, P.ldx, (const double *)P.RY,
                       m->m, P.lanes, cpl, m->dinv, LY);
  else
    hipLaunchKernelGGL(k_filter_final<float>, grid_for(n), dim3(256), 0, s, P.X, P.ldx, (const float *)P.RY,
                       m->m, P.lanes, cpl, m->dinv, LY);
  FE_HIP_TRY(hipGetLastError());
  return FE_OK;
}

// the whole pass, enqueued (no host synchronisation)
static fe_status filter_enqueue(FilterPlan &P, hipStream_t s) {
  fe_status st;
  if ((st = filter_prologue(P, s))) return st;
  while (P.k <= P.degree) {
    LocalLaunch L = filter_step_local(P);
    if ((st = filter_step_reduce(P, s))) return st;
    if ((st = launch_local(P.m, L, s))) return st;
    if ((st = filter_step_rest(P, s))) return st;
  }
  return filter_final(P, s);
}

}  // namespace fehx

using namespace fehx;

extern "C" {

fe_status fe_cheb_filter(fe_mesh_t m, void *X, int64_t ldx, const double *lam, int64_t nvec, int32_t degree,
                         double lam_min, double lam_T, double lam_max, int32_t inner_prec, void *stream) {
  if (!m || !X || !lam) return set_error(FE_EINVAL, "NULL argument");
  if (nvec <= 0 || ldx < nvec) return set_error(FE_EINVAL, "bad nvec / ldx");
  if (degree < 1) return set_error(FE_EINVAL, "degree must be >= 1");
  if (!(lam_max > lam_T) || !(lam_min < lam_T)) return set_error(FE_EINVAL, "need lam_min < lam_T < lam_max");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  if (inner_prec < FE_F64 || inner_prec > FE_BF16) return set_error(FE_EINVAL, "unknown inner precision");
  const int C = m->cplx ? 2 : 1;
  FilterPlan P;
  fe_status st = filter_setup(P, m, (double *)X, ldx * C, lam, nvec, degree, lam_min, lam_T, lam_max, inner_prec);
  if (st) return st;
  return filter_enqueue(P, (hipStream_t)stream);
}

fe_status fe_lanczos(fe_mesh_t m, const void *v0, int32_t steps, double *theta, double *beta_last) {
  if (!m || !v0 || !theta || !beta_last) return set_error(FE_EINVAL, "NULL argument");
  if (steps < 1) return set_error(FE_EINVAL, "steps must be >= 1");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  const int C = m->cplx ? 2 : 1;
  const int64_t len = m->m * C;   // doubles per vector
  fe_status st;
  if ((st = ensure_workspace(m, 5, (int64_t)(steps + 1) * len * (int64_t)sizeof(double)))) return st;
  if ((st = ensure_workspace(m, 6, 3 * len * (int64_t)sizeof(double)))) return st;
  double *Q = (double *)m->ws[5];
  double *t = (double *)m->ws[6], *y = t + len, *hbuf = t + 2 * len;
  Blas B;
  if ((st = rb(rocblas_create_handle(&B.h), "rocblas_create_handle"))) return st;
  rocblas_set_pointer_mode(B.h, rocblas_pointer_mode_host);
  // q_0 = v0 / |v0|
  FE_HIP_TRY(hipMemcpy(Q, v0, len * sizeof(double), hipMemcpyDeviceToDevice));
  double nrm = 0;
  if ((st = rb(rocblas_dnrm2(B.h, (rocblas_int)len, Q, 1, &nrm), "nrm2"))) return st;
  double inv = 1.0 / nrm;
  if ((st = rb(rocblas_dscal(B.h, (rocblas_int)len, &inv, Q, 1), "scal"))) return st;
  std::vector<double> al, be;
  double beta_prev = 0;
  for (int j = 0; j < steps; ++j) {
    double *qj = Q + (int64_t)j * len;
    // w = D^-1/2 H D^-1/2 q_j
    hipLaunchKernelGGL(k_scale_rows, grid_for(len), dim3(256), 0, 0, qj, (int64_t)C, t, (int64_t)C, m->m, C, m->dinv, 1);
    LocalLaunch L;
    L.X = t; L.Y = y; L.ldx = C; L.ldy = C; L.nlanes = C; L.prec = FE_F64;
    if ((st = launch_local(m, L, 0))) return st;
    if ((st = launch_nonlocal(m, t, C, y, C, C, FE_F64, nullptr, 1.0, 0))) return st;
    double *w = Q + (int64_t)(j + 1) * len;
    hipLaunchKernelGGL(k_scale_rows, grid_for(len), dim3(256), 0, 0, y, (int64_t)C, w, (int64_t)C, m->m, C, m->dinv, 1);
    FE_HIP_TRY(hipGetLastError());
    if (j > 0) {
      double mb = -beta_prev;
      if ((st = rb(rocblas_daxpy(B.h, (rocblas_int)len, &mb, Q + (int64_t)(j - 1) * len, 1, w, 1), "axpy"))) return st;
    }
    double alpha = 0;   // Re(q^H w) = real dot product of the interleaved arrays
    if ((st = rb(rocblas_ddot(B.h, (rocblas_int)len, qj, 1, w, 1, &alpha), "dot"))) return st;
    double ma = -alpha;
    if ((st = rb(rocblas_daxpy(B.h, (rocblas_int)len, &ma, qj, 1, w, 1), "axpy"))) return st;
    // full reorthogonalisation against q_0..q_j:  w -= Q (Q^H w)
    const rocblas_int k = j + 1;
    if (C == 1) {
      const double one = 1.0, zero = 0.0, mone = -1.0;
      if ((st = rb(rocblas_dgemv(B.h, rocblas_operation_transpose, (rocblas_int)len, k, &one, Q, (rocblas_int)len, w, 1, &zero, hbuf, 1), "gemv"))) return st;
      if ((st = rb(rocblas_dgemv(B.h, rocblas_operation_none, (rocblas_int)len, k, &mone, Q, (rocblas_int)len, hbuf, 1, &one, w, 1), "gemv"))) return st;
    } else {
      const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0), mone(-1.0, 0.0);
      auto *Qz = (rocblas_double_complex *)Q;
      auto *wz = (rocblas_double_complex *)w;
      auto *hz = (rocblas_double_complex *)hbuf;
      if ((st = rb(rocblas_zgemv(B.h, rocblas_operation_conjugate_transpose, (rocblas_int)m->m, k, &one, Qz, (rocblas_int)m->m, wz, 1, &zero, hz, 1), "gemv"))) return st;
      if ((st = rb(rocblas_zgemv(B.h, rocblas_operation_none, (rocblas_int)m->m, k, &mone, Qz, (rocblas_int)m->m, hz, 1, &one, wz, 1), "gemv"))) return st;
    }
    double beta = 0;
    if ((st = rb(rocblas_dnrm2(B.h, (rocblas_int)len, w, 1, &beta), "nrm2"))) return st;
    al.push_back(alpha);
    be.push_back(beta);
    double ib = 1.0 / beta;
    if ((st = rb(rocblas_dscal(B.h, (rocblas_int)len, &ib, w, 1), "scal"))) return st;
    beta_prev = beta;
  }
  FE_HIP_TRY(hipDeviceSynchronize());
  std::vector<double> ev = tridiag_eigs(al, std::vector<double>(be.begin(), be.end() - 1));
  for (int i = 0; i < steps; ++i) theta[i] = ev[i];
  *beta_last = be.back();
  return FE_OK;
}

fe_status fe_rayleigh_ritz(fe_mesh_t m, void *Xv, int64_t ldx, int64_t nvec, double *ritz, void *stream) {
  if (!m || !Xv || !ritz) return set_error(FE_EINVAL, "NULL argument");
  if (nvec <= 0 || ldx < nvec) return set_error(FE_EINVAL, "bad nvec / ldx");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  const int C = m->cplx ? 2 : 1;
  hipStream_t s = (hipStream_t)stream;
  double *X = (double *)Xv;
  const int64_t lanes = nvec * C, ldl = ldx * C;
  fe_status st;
  if ((st = ensure_workspace(m, 5, m->m * lanes * (int64_t)sizeof(double)))) return st;
  if ((st = ensure_workspace(m, 6, (2 * nvec * nvec * C + 2 * nvec + 8) * (int64_t)sizeof(double)))) return st;
  double *W = (double *)m->ws[5];
  double *Hp = (double *)m->ws[6], *Sp = Hp + nvec * nvec * C, *E = Sp + nvec * nvec * C;
  rocblas_int *info = (rocblas_int *)(E + nvec);
  Blas B;
  if ((st = rb(rocblas_create_handle(&B.h), "rocblas_create_handle"))) return st;
  rocblas_set_stream(B.h, s);
  rocblas_set_pointer_mode(B.h, rocblas_pointer_mode_host);
  const rocblas_int n = (rocblas_int)nvec, mm = (rocblas_int)m->m;
  // W = H X
  LocalLaunch L;
  L.X = X; L.Y = W; L.ldx = ldl; L.ldy = lanes; L.nlanes = (int)lanes; L.prec = FE_F64;
  L.vt = m->vt_pref[FE_F64][0];
  if ((st = apply_with_nonlocal(m, L, FE_F64, nullptr, 1.0, s))) return st;
  // W = M X: the lumped D row scaling, or the consistent M (matrix-free)
  auto mass_into_W = [&]() -> fe_status {
    if (m->mass_kind == FE_MASS_CONSISTENT) {
      LocalLaunch LM;
      LM.X = X; LM.Y = W; LM.ldx = ldl; LM.ldy = lanes; LM.nlanes = (int)lanes; LM.prec = FE_F64;
      LM.vt = m->vt_pref[FE_F64][0];
      LM.mass = true;
      return launch_local(m, LM, s);
    }
    hipLaunchKernelGGL(k_scale_rows, grid_for(m->m * lanes), dim3(256), 0, s, X, ldl, W, lanes, m->m, (int)lanes,
                       m->dmass, 0);
    FE_HIP_TRY(hipGetLastError());
    return FE_OK;
  };
  // Gram matrices over the DoF axis (k = m, far longer than n): split into
  // NS chunks so that the product has enough tiles for the device, the
  // chunks' products into partial blocks (one strided-batched call, the
  // remainder one more), then summed in chunk order.
  const int64_t NS = std::min<int64_t>(64, m->m);
  const int64_t kc = m->m / NS, krem = m->m - NS * kc;
  const int64_t plen = (int64_t)nvec * nvec * C;       // doubles per partial
  if ((st = ensure_workspace(m, 10, (NS + 1) * plen * (int64_t)sizeof(double)))) return st;
  double *part = (double *)m->ws[10];
  auto sum_parts = [&](double *out) -> fe_status {
    hipLaunchKernelGGL(k_sum_parts, grid_for(plen), dim3(256), 0, s, part, plen, (int)(NS + (krem ? 1 : 0)), plen, out);
    FE_HIP_TRY(hipGetLastError());
    return FE_OK;
  };
  auto gram_d = [&](double *out) -> fe_status {   // out = W X^T (column-major views), real
    const double one = 1.0, zero = 0.0;
    fe_status e;
    if ((e = rb(rocblas_dgemm_strided_batched(B.h, rocblas_operation_none, rocblas_operation_transpose, n, n,
                                               (rocblas_int)kc, &one, W, (rocblas_int)lanes, kc * lanes, X,
                                               (rocblas_int)ldl, kc * ldl, &zero, part, n, plen, (rocblas_int)NS),
                "gemm_strided_batched"))) return e;
    if (krem)
      if ((e = rb(rocblas_dgemm(B.h, rocblas_operation_none, rocblas_operation_transpose, n, n, (rocblas_int)krem,
                                &one, W + NS * kc * lanes, (rocblas_int)lanes, X + NS * kc * ldl, (rocblas_int)ldl,
                                &zero, part + NS * plen, n), "gemm"))) return e;
    return sum_parts(out);
  };
  auto gram_z = [&](double *out) -> fe_status {   // out = W X^H (column-major views), complex
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    auto *Wz = (rocblas_double_complex *)W, *Xz = (rocblas_double_complex *)X;
    auto *Pz = (rocblas_double_complex *)part;
    const int64_t pz = (int64_t)nvec * nvec;
    fe_status e;
    if ((e = rb(rocblas_zgemm_strided_batched(B.h, rocblas_operation_none, rocblas_operation_conjugate_transpose, n,
                                               n, (rocblas_int)kc, &one, Wz, n, kc * nvec, Xz, (rocblas_int)ldx,
                                               kc * ldx, &zero, Pz, n, pz, (rocblas_int)NS), "gemm_strided_batched")))
      return e;
    if (krem)
      if ((e = rb(rocblas_zgemm(B.h, rocblas_operation_none, rocblas_operation_conjugate_transpose, n, n,
                                (rocblas_int)krem, &one, Wz + NS * kc * nvec, n, Xz + NS * kc * ldx, (rocblas_int)ldx,
                                &zero, Pz + NS * pz, n), "gemm"))) return e;
    return sum_parts(out);
  };
  // column-major views: X^T is (nvec x m) with ld = ldx elements
  if (C == 1) {
    const double one = 1.0, zero = 0.0;
    if ((st = gram_d(Hp))) return st;
    if ((st = mass_into_W())) return st;
    if ((st = gram_d(Sp))) return st;
    // H V = S V E: S = U^T U (Cholesky), A = U^-T H U^-1 with two blocked
    // triangular solves, A Q = Q E, V = U^-1 Q
    const rocblas_side L_ = rocblas_side_left, R_ = rocblas_side_right;
    const rocblas_fill up = rocblas_fill_upper;
    const rocblas_diagonal nu = rocblas_diagonal_non_unit;
    const rocblas_operation on = rocblas_operation_none, ot = rocblas_operation_transpose;
    if ((st = rb(rocsolver_dpotrf(B.h, up, n, Sp, n, info), "potrf"))) return st;
    if ((st = rb(rocblas_dtrsm(B.h, L_, up, ot, nu, n, n, &one, Sp, n, Hp, n), "trsm"))) return st;
    if ((st = rb(rocblas_dtrsm(B.h, R_, up, on, nu, n, n, &one, Sp, n, Hp, n), "trsm"))) return st;
    if ((st = rb(rocsolver_dsyevd(B.h, rocblas_evect_original, up, n, Hp, n, E, W, info + 1), "syevd"))) return st;
    if ((st = rb(rocblas_dtrsm(B.h, L_, up, on, nu, n, n, &one, Sp, n, Hp, n), "trsm"))) return st;
    // X <- X V : (X V)^T = V^T X^T
    if ((st = rb(rocblas_dgemm(B.h, rocblas_operation_transpose, rocblas_operation_none, n, mm, n, &one, Hp, n, X, (rocblas_int)ldl, &zero, W, (rocblas_int)lanes), "gemm"))) return st;
  } else {
    const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
    auto *Wz = (rocblas_double_complex *)W, *Xz = (rocblas_double_complex *)X;
    auto *Hz = (rocblas_double_complex *)Hp, *Sz = (rocblas_double_complex *)Sp;
    // G = (H X)^T conj(X): column-major G = conj(X^H H X)
    if ((st = gram_z(Hp))) return st;
    if ((st = mass_into_W())) return st;
    if ((st = gram_z(Sp))) return st;
    // eigenvectors of the conjugated pencil are conj(E); X E = (E^T X^T)^T = (V^H X^T)^T
    // the same reduction as the real case with U^H in place of U^T
    const rocblas_side L_ = rocblas_side_left, R_ = rocblas_side_right;
    const rocblas_fill up = rocblas_fill_upper;
    const rocblas_diagonal nu = rocblas_diagonal_non_unit;
    const rocblas_operation on = rocblas_operation_none, oc = rocblas_operation_conjugate_transpose;
    if ((st = rb(rocsolver_zpotrf(B.h, up, n, Sz, n, info), "potrf"))) return st;
    if ((st = rb(rocblas_ztrsm(B.h, L_, up, oc, nu, n, n, &one, Sz, n, Hz, n), "trsm"))) return st;
    if ((st = rb(rocblas_ztrsm(B.h, R_, up, on, nu, n, n, &one, Sz, n, Hz, n), "trsm"))) return st;
    if ((st = rb(rocsolver_zheevd(B.h, rocblas_evect_original, up, n, Hz, n, E, W, info + 1), "heevd"))) return st;
    if ((st = rb(rocblas_ztrsm(B.h, L_, up, on, nu, n, n, &one, Sz, n, Hz, n), "trsm"))) return st;
    if ((st = rb(rocblas_zgemm(B.h, rocblas_operation_conjugate_transpose, rocblas_operation_none, n, mm, n, &one, Hz, n, Xz, (rocblas_int)ldx, &zero, Wz, n), "gemm"))) return st;
  }
  FE_HIP_TRY(hipMemcpy2DAsync(X, ldl * sizeof(double), W, lanes * sizeof(double), lanes * sizeof(double), m->m,
                              hipMemcpyDeviceToDevice, s));
  FE_HIP_TRY(hipMemcpyAsync(ritz, E, nvec * sizeof(double), hipMemcpyDeviceToDevice, s));
  rocblas_int hinfo[2] = {0, 0};   // Cholesky of S, eigensolver
  FE_HIP_TRY(hipMemcpyAsync(hinfo, info, 2 * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
  FE_HIP_TRY(hipStreamSynchronize(s));
  if (hinfo[0] != 0)
    return set_error(FE_EDEVICE, "Gram matrix not positive definite (Cholesky info = " + std::to_string(hinfo[0]) + ")");
  if (hinfo[1] != 0) return set_error(FE_EDEVICE, "eigensolver reported info = " + std::to_string(hinfo[1]));
  return FE_OK;
}

fe_status fe_chfsi(fe_mesh_t m, void *X, int64_t ldx, int64_t nvec, const void *v0, int32_t outer,
                   int32_t degree, int32_t lanczos_steps, int32_t inner_prec, double *ritz, double *bounds,
                   void *stream) {
  if (!m || !X || !v0 || !ritz) return set_error(FE_EINVAL, "NULL argument");
  if (nvec <= 0 || ldx < nvec || outer < 0 || degree < 1 || lanczos_steps < 2)
    return set_error(FE_EINVAL, "bad nvec / ldx / outer / degree / lanczos_steps");
  if (nvec > m->m) return set_error(FE_EINVAL, "more vectors than DoFs");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  fe_status st;
  // spectral upper bound: largest Lanczos Ritz value plus the last residual norm
  std::vector<double> theta(lanczos_steps);
  double beta = 0;
  if ((st = fe_lanczos(m, v0, lanczos_steps, theta.data(), &beta))) return st;
  const double lmax = theta.back() + std::fabs(beta);
  if ((st = ensure_workspace(m, 7, nvec * (int64_t)sizeof(double)))) return st;
  double *lam = (double *)m->ws[7];
  hipStream_t s = (hipStream_t)stream;
  if ((st = fe_rayleigh_ritz(m, X, ldx, nvec, lam, stream))) return st;
  // first pass: lower end from Lanczos, cut from the free-electron count of nvec
  // states in the cell volume; later passes: the previous Ritz interval
  const fe_mesh_desc &d = m->desc;
  const double vol = std::fabs(d.lattice[0][0] * (d.lattice[1][1] * d.lattice[2][2] - d.lattice[1][2] * d.lattice[2][1]) -
                               d.lattice[0][1] * (d.lattice[1][0] * d.lattice[2][2] - d.lattice[1][2] * d.lattice[2][0]) +
                               d.lattice[0][2] * (d.lattice[1][0] * d.lattice[2][1] - d.lattice[1][1] * d.lattice[2][0]));
  double lmin = theta.front();
  double lT = lmin + 0.5 * std::pow(6.0 * M_PI * M_PI * (double)nvec / vol, 2.0 / 3.0);
  std::vector<double> hl(nvec);
  for (int it = 0; it < outer; ++it) {
    if (it > 0) {
      FE_HIP_TRY(hipMemcpy(hl.data(), lam, nvec * sizeof(double), hipMemcpyDeviceToHost));
      lmin = hl.front();
      lT = hl.back();
    }
    if (!(lT < lmax)) return set_error(FE_EINVAL, "Ritz interval reaches the spectral upper bound");
    if (bounds) { bounds[3 * it] = lmin; bounds[3 * it + 1] = lT; bounds[3 * it + 2] = lmax; }
    if ((st = fe_cheb_filter(m, X, ldx, lam, nvec, degree, lmin, lT, lmax, inner_prec, stream))) return st;
    if ((st = fe_rayleigh_ritz(m, X, ldx, nvec, lam, stream))) return st;
  }
  FE_HIP_TRY(hipMemcpyAsync(ritz, lam, nvec * sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_TRY(hipStreamSynchronize(s));
  return FE_OK;
}

struct fe_filter_graph_s {
  fehx::FilterPlan P;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
};

fe_status fe_filter_graph_create(fe_mesh_t m, void *X, int64_t ldx, const double *lam, int64_t nvec, int32_t degree,
                                 double lam_min, double lam_T, double lam_max, int32_t inner_prec,
                                 fe_filter_graph_t *out) {
  if (!out) return set_error(FE_EINVAL, "NULL output handle");
  *out = nullptr;
  if (!m || !X || !lam) return set_error(FE_EINVAL, "NULL argument");
  if (nvec <= 0 || ldx < nvec) return set_error(FE_EINVAL, "bad nvec / ldx");
  if (degree < 1) return set_error(FE_EINVAL, "degree must be >= 1");
  if (!(lam_max > lam_T) || !(lam_min < lam_T)) return set_error(FE_EINVAL, "need lam_min < lam_T < lam_max");
  if (inner_prec < FE_F64 || inner_prec > FE_BF16) return set_error(FE_EINVAL, "unknown inner precision");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  const int C = m->cplx ? 2 : 1;
  fe_filter_graph_s *G = new fe_filter_graph_s();
  fe_status st = filter_setup(G->P, m, (double *)X, ldx * C, lam, nvec, degree, lam_min, lam_T, lam_max, inner_prec);
  if (st) { delete G; return st; }
  hipStream_t cs = nullptr;
  if (hipStreamCreate(&cs) != hipSuccess) { delete G; return set_error(FE_EDEVICE, "hipStreamCreate failed"); }
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(cs);
    delete G;
    return set_error(FE_EDEVICE, "hipStreamBeginCapture failed");
  }
  FilterPlan P = G->P;   // enqueueing advances the step and swaps the blocks
  st = filter_enqueue(P, cs);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  hipStreamDestroy(cs);
  if (st == FE_OK && ec != hipSuccess) st = set_error(FE_EDEVICE, "hipStreamEndCapture failed");
  if (st == FE_OK && hipGraphInstantiate(&G->ex, g, nullptr, nullptr, 0) != hipSuccess)
    st = set_error(FE_EDEVICE, "hipGraphInstantiate failed");
  G->g = g;
  if (st) {
    if (G->ex) hipGraphExecDestroy(G->ex);
    if (G->g) hipGraphDestroy(G->g);
    delete G;
    return st;
  }
  ++m->graphs;
  *out = G;
  return FE_OK;
}

fe_status fe_filter_graph_launch(fe_filter_graph_t G, void *stream) {
  if (!G || !G->ex) return set_error(FE_EINVAL, "NULL graph");
  if (hipSetDevice(G->P.m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  FE_HIP_TRY(hipGraphLaunch(G->ex, (hipStream_t)stream));
  return FE_OK;
}

fe_status fe_filter_graph_destroy(fe_filter_graph_t G) {
  if (!G) return FE_OK;
  --G->P.m->graphs;
  if (G->ex) hipGraphExecDestroy(G->ex);
  if (G->g) hipGraphDestroy(G->g);
  delete G;
  return FE_OK;
}

}  // extern "C"
