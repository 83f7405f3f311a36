// Matrix-free local operator H_loc X on gfx950 (Sec. 3.2, eqns ggaReal /
// ggaCmplx, Alg. 2), one subdomain on one GPU.
//
// Work decomposition (the GPU analogue of the paper's multilevel batches,
// Sec. 4.1): a workgroup owns one column of cells along a_2 and one tile of
// VT real vector lanes (for complex meshes the real and imaginary parts of a
// vector sit in adjacent lanes, the paper's level-2 re/im batches).  It walks
// the column cell by cell: gather of the cell block X^(e) = Q^(e) X into LDS
// ([point][lane], lanes fastest), the eight 1D contraction sweeps of Alg. 2
// with the even-odd decomposition (each thread applies one 1D matrix to one
// line of points for one lane, coefficients read as wave-uniform scalars),
// the quadrature-point stage of eqn refact, and the transposed sweeps.
//
// Scatter Y += Q^(e)T Y^(e) without atomics and deterministically:
//  * along a_2 the shared node plane of consecutive cells is summed in LDS
//    (and the periodic first/last plane of the column at the end);
//  * across columns the columns are coloured 2 (or 3 for an odd count) per
//    axis and launched colour by colour; a node shared by several columns is
//    stored by the column of the lowest colour phase and read-modify-written
//    by the later ones, so no two concurrently running workgroups touch the
//    same node and the summation order is fixed.
// The first store of a node can fold in a linear epilogue (Chebyshev filter
// recurrence, residual), which is what lets a filter step run as one
// operator application.
#include "fe_internal.h"

namespace fehx {

// ---- storage conversions -----------------------------------------------------
struct bf16s { uint16_t b; };

__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}

template <typename TS, typename TC> struct Cvt;
template <> struct Cvt<double, double> {
  static __device__ __forceinline__ double ld(const double *p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(double *p, int64_t i, double v) { p[i] = v; }
};
template <> struct Cvt<float, float> {
  static __device__ __forceinline__ float ld(const float *p, int64_t i) { return p[i]; }
  static __device__ __forceinline__ void st(float *p, int64_t i, float v) { p[i] = v; }
};
template <> struct Cvt<bf16s, float> {
  static __device__ __forceinline__ float ld(const bf16s *p, int64_t i) { return bf16_to_f(p[i].b); }
  static __device__ __forceinline__ void st(bf16s *p, int64_t i, float v) { p[i].b = f_to_bf16(v); }
};

// ---- kernel arguments ----------------------------------------------------------
template <typename TC> struct KArgs {
  const void *X;
  void *Y;
  int64_t ldx, ldy;
  int nlanes;
  int N0, N1, N2, M0, M1, M2, p;
  const int *cols;
  int ncols, ntiles;
  const TC *tab;
  const TC *wq;
  const TC *coef;
  int gga;
  TC g0, g1, g2, k0, k1, k2;
  const double *dinv;
  int epi;
  TC alpha;
  const void *ein0, *ein1, *ein2;
  int64_t eld0, eld1, eld2;
  TC es0, es1, es2;
  int ed0, ed1, ed2;
  const double *elam0, *elam1, *elam2;
  const double *dmass;
};

// ---- even-odd application of a packed centro-(anti)symmetric 1D matrix ----------
// tab rows q < ceil(NOUT/2): E[q][0..ceil(NIN/2)) then O[q][0..floor(NIN/2)).
template <int NIN, int NOUT, int SYM, typename TC>
__device__ __forceinline__ void eo_apply(const TC *__restrict__ t, const TC (&x)[NIN], TC (&y)[NOUT]) {
  constexpr int CI = (NIN + 1) / 2, HI = NIN / 2, CO = (NOUT + 1) / 2, HO = NOUT / 2;
  TC xp[CI], xm[HI > 0 ? HI : 1];
#pragma unroll
  for (int i = 0; i < HI; ++i) {
    xp[i] = x[i] + x[NIN - 1 - i];
    xm[i] = x[i] - x[NIN - 1 - i];
  }
  if constexpr (NIN & 1) xp[HI] = x[HI];
#pragma unroll
  for (int q = 0; q < CO; ++q) {
    const TC *E = t + q * NIN;
    const TC *O = E + CI;
    TC e = 0, o = 0;
#pragma unroll
    for (int i = 0; i < CI; ++i) e = fma(E[i], xp[i], e);
#pragma unroll
    for (int i = 0; i < HI; ++i) o = fma(O[i], xm[i], o);
    if ((NOUT & 1) && q == HO) {
      y[q] = (SYM > 0) ? e : o;
    } else {
      y[q] = e + o;
      y[NOUT - 1 - q] = (SYM > 0) ? (e - o) : (o - e);
    }
  }
}

// One 1D contraction over every line of a block: each work item is one
// (line, lane); 'dec' maps a line to (source base, stride, destination base,
// stride) in points.
template <int NIN, int NOUT, int SYM, int VT, typename TC, typename Dec>
__device__ __forceinline__ void line_pass(const TC *__restrict__ src, TC *__restrict__ dst,
                                          const TC *__restrict__ tab, int nlines, Dec dec) {
  const int total = nlines * VT;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int v = t % VT, l = t / VT;
    int sb, ss, db, ds;
    dec(l, sb, ss, db, ds);
    TC x[NIN], y[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) x[i] = src[(sb + i * ss) * VT + v];
    const TC *tb = tab;
    asm volatile("" : "+s"(tb));   // keep the 1D table in scalar loads, not hoisted VGPRs
    eo_apply<NIN, NOUT, SYM>(tb, x, y);
#pragma unroll
    for (int i = 0; i < NOUT; ++i) dst[(db + i * ds) * VT + v] = y[i];
  }
}

// Quadrature-point stage for reference direction D (eqn refact / Alg. 2):
// for each line along D of the interpolated field Y0 (src):
//   T   = Dtilde u                                  (gradient along D)
//   F   = G_DD w T + Vtilde^G_D u                   (flux for Dtilde^T)
//   z   = Vtilde^G_D T  [+ (V + |k|^2/2) w u  for D = 0]  [- i kappa_D w T]
//   out = Dtilde^T F + z,   accumulated into dst (initialised by D = 0).
template <int D, int NQ, int VT, bool CPLX, typename TC>
__device__ __forceinline__ void dir_pass(const TC *__restrict__ src, TC *__restrict__ dst,
                                         const TC *__restrict__ tD, const TC *__restrict__ tDT,
                                         const KArgs<TC> &a, int64_t cell, int lane0) {
  constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
  const int total = NQ2 * VT;
  const TC gD = D == 0 ? a.g0 : (D == 1 ? a.g1 : a.g2);
  const TC kD = D == 0 ? a.k0 : (D == 1 ? a.k1 : a.k2);
  const TC *cL = a.coef + (cell * 4) * NQ3;
  const TC *cG = a.coef + (cell * 4 + 1 + D) * NQ3;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int v = t % VT, l = t / VT;
    int base, stride;
    if (D == 0) { base = l * NQ; stride = 1; }
    else if (D == 1) { base = (l / NQ) * NQ2 + (l % NQ); stride = NQ; }
    else { base = l; stride = NQ2; }
    TC u[NQ], T[NQ], F[NQ], z[NQ], o[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) u[i] = src[(base + i * stride) * VT + v];
    const TC *td = tD, *tdt = tDT;
    asm volatile("" : "+s"(td), "+s"(tdt));
    eo_apply<NQ, NQ, -1>(td, u, T);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int Q = base + i * stride;
      const TC w = a.wq[Q];
      F[i] = gD * w * T[i];
      z[i] = 0;
      if (a.gga) {
        const TC vg = cG[Q];
        F[i] = fma(vg, u[i], F[i]);
        z[i] = vg * T[i];
      }
      if (D == 0) z[i] = fma(cL[Q], u[i], z[i]);
      if constexpr (CPLX) {
        // -i kappa w T: real lane gets +kappa w T_im, imaginary lane -kappa w T_re
        const TC tp = __shfl_xor(T[i], 1);
        const TC kw = kD * w;
        z[i] = fma(((lane0 + v) & 1) ? -kw : kw, tp, z[i]);
      }
    }
    eo_apply<NQ, NQ, -1>(tdt, F, o);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int idx = (base + i * stride) * VT + v;
      if (D == 0) dst[idx] = o[i] + z[i];
      else dst[idx] += o[i] + z[i];
    }
  }
}

__device__ __forceinline__ int colour_of(int c, int n) { return ((n & 1) && c == n - 1) ? 2 : (c & 1); }

template <typename TS, typename TC>
__device__ __forceinline__ TC epi_term(const void *in, int64_t ld, TC s, int dpow, const double *lam,
                                       const double *dmass, int64_t g, int lane, bool cplx) {
  if (!in) return 0;
  TC c = s;
  if (dpow) c *= (TC)dmass[g];
  if (lam) c *= (TC)lam[cplx ? (lane >> 1) : lane];
  return c * Cvt<TS, TC>::ld((const TS *)in, g * ld + lane);
}

// FP64 blocks are capped at 512 threads so each lane may use 256 VGPRs.
template <typename TC> struct MaxThreads { static constexpr int value = sizeof(TC) == 8 ? 512 : 1024; };

template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC>
__global__ void __launch_bounds__(MaxThreads<TC>::value) k_local(KArgs<TC> a) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP, NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
  constexpr int OFF_N = 0;
  constexpr int OFF_NT = OFF_N + ((NQ + 1) / 2) * NP;
  constexpr int OFF_D = OFF_NT + ((NP + 1) / 2) * NQ;
  constexpr int OFF_DT = OFF_D + ((NQ + 1) / 2) * NQ;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC *A = reinterpret_cast<TC *>(smem_raw);
  TC *B = A + NQ3 * VT;
  TC *Ycar = B + NQ3 * VT;
  TC *Yfst = Ycar + NP2 * VT;

  // XCD-aware placement: block b runs on XCD b % 8; give each XCD a
  // contiguous range of work items so the tiles of one column share an L2.
  const int W = a.ncols * a.ntiles;
  const int per = gridDim.x >> 3;
  const int w = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w >= W) return;
  const int col = w / a.ntiles, tile = w - col * a.ntiles;
  const int cx = a.cols[2 * col], cy = a.cols[2 * col + 1];
  const int lane0 = tile * VT;
  const TS *__restrict__ X = (const TS *)a.X;
  TS *__restrict__ Y = (TS *)a.Y;
  const TC *tN = a.tab + OFF_N, *tNT = a.tab + OFF_NT, *tD = a.tab + OFF_D, *tDT = a.tab + OFF_DT;
  const int p = a.p;

  const int ax = colour_of(cx, a.N0), by = colour_of(cy, a.N1);
  const int axl = colour_of(cx == 0 ? a.N0 - 1 : cx - 1, a.N0);
  const int axr = colour_of(cx == a.N0 - 1 ? 0 : cx + 1, a.N0);
  const int byl = colour_of(cy == 0 ? a.N1 - 1 : cy - 1, a.N1);
  const int byr = colour_of(cy == a.N1 - 1 ? 0 : cy + 1, a.N1);

  auto gnode = [&](int i, int j, int k, int cz) -> int64_t {
    int gx = cx * p + i; if (gx >= a.M0) gx -= a.M0;
    int gy = cy * p + j; if (gy >= a.M1) gy -= a.M1;
    int gz = cz * p + k; if (gz >= a.M2) gz -= a.M2;
    return (int64_t)gx + (int64_t)a.M0 * ((int64_t)gy + (int64_t)a.M1 * gz);
  };

  for (int cz = 0; cz < a.N2; ++cz) {
    const int64_t cell = cx + (int64_t)a.N0 * (cy + (int64_t)a.N1 * cz);
    // gather X^(e) = Q^(e) X  ->  A[k][j][i][lane]
    for (int t = threadIdx.x; t < NP3 * VT; t += blockDim.x) {
      const int v = t % VT, n = t / VT;
      const int i = n % NP, j = (n / NP) % NP, k = n / NP2;
      const int64_t g = gnode(i, j, k, cz);
      const int lane = lane0 + v;
      TC val = 0;
      if (lane < a.nlanes) {
        val = Cvt<TS, TC>::ld(X, g * a.ldx + lane);
        if (a.dinv) val *= (TC)a.dinv[g];
      }
      A[n * VT + v] = val;
    }
    __syncthreads();
    // Y0 = (N x N x N) X^(e)
    line_pass<NP, NQ, 1, VT>(A, B, tN, NP2, [](int l, int &sb, int &ss, int &db, int &ds) {
      sb = l * NP; ss = 1; db = l * NQ; ds = 1; });
    __syncthreads();
    line_pass<NP, NQ, 1, VT>(B, A, tN, NP * NQ, [](int l, int &sb, int &ss, int &db, int &ds) {
      const int k = l / NQ, q1 = l % NQ;
      sb = k * NP * NQ + q1; ss = NQ; db = k * NQ2 + q1; ds = NQ; });
    __syncthreads();
    line_pass<NP, NQ, 1, VT>(A, B, tN, NQ2, [](int l, int &sb, int &ss, int &db, int &ds) {
      sb = l; ss = NQ2; db = l; ds = NQ2; });
    __syncthreads();
    // quadrature stage, direction by direction (diagonal metric)
    dir_pass<0, NQ, VT, CPLX>(B, A, tD, tDT, a, cell, lane0);
    __syncthreads();
    dir_pass<1, NQ, VT, CPLX>(B, A, tD, tDT, a, cell, lane0);
    __syncthreads();
    dir_pass<2, NQ, VT, CPLX>(B, A, tD, tDT, a, cell, lane0);
    __syncthreads();
    // Y^(e) = (N x N x N)^T Z
    line_pass<NQ, NP, 1, VT>(A, B, tNT, NQ2, [](int l, int &sb, int &ss, int &db, int &ds) {
      sb = l; ss = NQ2; db = l; ds = NQ2; });
    __syncthreads();
    line_pass<NQ, NP, 1, VT>(B, A, tNT, NP * NQ, [](int l, int &sb, int &ss, int &db, int &ds) {
      const int k = l / NQ, q1 = l % NQ;
      sb = k * NQ2 + q1; ss = NQ; db = k * NP * NQ + q1; ds = NQ; });
    __syncthreads();
    line_pass<NQ, NP, 1, VT>(A, B, tNT, NP2, [](int l, int &sb, int &ss, int &db, int &ds) {
      sb = l * NQ; ss = 1; db = l * NP; ds = 1; });
    __syncthreads();
    // node planes shared along a_2
    for (int t = threadIdx.x; t < NP2 * VT; t += blockDim.x) {
      if (cz == 0) Yfst[t] = B[t];
      else B[t] += Ycar[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NP2 * VT; t += blockDim.x) {
      TC *top = B + (NP - 1) * NP2 * VT;
      if (cz < a.N2 - 1) Ycar[t] = top[t];
      else top[t] += Yfst[t];
    }
    __syncthreads();
    // write the completed planes: store (first phase) or read-modify-write
    const int k0 = (cz == 0) ? 1 : 0;
    const int k1 = (cz == a.N2 - 1) ? NP : NP - 1;
    const int nw = (k1 - k0) * NP2 * VT;
    for (int t = threadIdx.x; t < nw; t += blockDim.x) {
      const int v = t % VT, n = t / VT + k0 * NP2;
      const int lane = lane0 + v;
      if (lane >= a.nlanes) continue;
      const int i = n % NP, j = (n / NP) % NP, k = n / NP2;
      const int64_t g = gnode(i, j, k, cz);
      const TC val = B[n * VT + v];
      const bool xs = (i == 0) || (i == NP - 1), ys = (j == 0) || (j == NP - 1);
      const int axo = (i == 0) ? axl : axr, byo = (j == 0) ? byl : byr;
      const bool store = (!xs || ax < axo) && (!ys || by < byo);
      const int64_t oi = g * a.ldy + lane;
      if (store) {
        TC out = val;
        if (a.epi) {
          out = a.alpha * val;
          out += epi_term<TS, TC>(a.ein0, a.eld0, a.es0, a.ed0, a.elam0, a.dmass, g, lane, CPLX);
          out += epi_term<TS, TC>(a.ein1, a.eld1, a.es1, a.ed1, a.elam1, a.dmass, g, lane, CPLX);
          out += epi_term<TS, TC>(a.ein2, a.eld2, a.es2, a.ed2, a.elam2, a.dmass, g, lane, CPLX);
        }
        Cvt<TS, TC>::st(Y, oi, out);
      } else {
        const TC add = a.epi ? a.alpha * val : val;
        Cvt<TS, TC>::st(Y, oi, Cvt<TS, TC>::ld(Y, oi) + add);
      }
    }
    __syncthreads();
  }
}

// ---- host-side dispatch ---------------------------------------------------------
namespace {

template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC>
fe_status run_local(Mesh *m, const LocalLaunch &L, hipStream_t s, int nt) {
  KArgs<TC> a{};
  a.X = L.X; a.Y = L.Y; a.ldx = L.ldx; a.ldy = L.ldy; a.nlanes = L.nlanes;
  a.N0 = m->N[0]; a.N1 = m->N[1]; a.N2 = m->N[2];
  a.M0 = m->Mn[0]; a.M1 = m->Mn[1]; a.M2 = m->Mn[2]; a.p = m->p;
  const bool f64 = std::is_same<TC, double>::value;
  a.tab = f64 ? (const TC *)m->tab64 : (const TC *)m->tab32;
  a.wq = f64 ? (const TC *)m->wq64 : (const TC *)m->wq32;
  a.coef = f64 ? (const TC *)m->coef64 : (const TC *)m->coef32;
  a.gga = m->has_gga ? 1 : 0;
  a.g0 = (TC)m->gdiag[0]; a.g1 = (TC)m->gdiag[1]; a.g2 = (TC)m->gdiag[2];
  a.k0 = (TC)m->kap[0]; a.k1 = (TC)m->kap[1]; a.k2 = (TC)m->kap[2];
  a.dinv = L.dinv_gather;
  a.epi = L.use_epi ? 1 : 0;
  a.alpha = (TC)L.epi.alpha;
  a.ein0 = L.epi.in[0]; a.ein1 = L.epi.in[1]; a.ein2 = L.epi.in[2];
  a.eld0 = L.epi.ld[0]; a.eld1 = L.epi.ld[1]; a.eld2 = L.epi.ld[2];
  a.es0 = (TC)L.epi.s[0]; a.es1 = (TC)L.epi.s[1]; a.es2 = (TC)L.epi.s[2];
  a.ed0 = L.epi.dpow[0]; a.ed1 = L.epi.dpow[1]; a.ed2 = L.epi.dpow[2];
  a.elam0 = L.epi.lam[0]; a.elam1 = L.epi.lam[1]; a.elam2 = L.epi.lam[2];
  a.dmass = m->dmass;
  a.ntiles = (L.nlanes + VT - 1) / VT;
  const size_t shm = (size_t)(2 * NQ * NQ * NQ + 2 * NP * NP) * VT * sizeof(TC);
  auto kern = k_local<NP, NQ, VT, CPLX, TS, TC>;
  static bool attr_done = false;
  if (!attr_done && shm > 65536) {
    FE_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    attr_done = true;
  }
  if (nt > MaxThreads<TC>::value) return set_error(FE_EINVAL, "thread count above the kernel's launch bound");
  if (nt <= 0) {
    int items = NQ * NQ * VT;
    nt = ((items + 63) / 64) * 64;
    if (nt > MaxThreads<TC>::value) nt = MaxThreads<TC>::value;
    if (nt < 128) nt = 128;
  }
  for (int ph = 0; ph < m->nphase; ++ph) {
    a.cols = m->cols + 2 * m->phase_off[ph];
    a.ncols = m->phase_off[ph + 1] - m->phase_off[ph];
    if (a.ncols == 0) continue;
    const int W = a.ncols * a.ntiles;
    const int nb = ((W + 7) / 8) * 8;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(nt), shm, s, a);
    FE_HIP_TRY(hipGetLastError());
  }
  return FE_OK;
}

template <int NP, int NQ, bool CPLX>
fe_status pick_vt(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  int vt = L.vt;
  int maxshm = 65536;
  hipDeviceGetAttribute(&maxshm, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
  auto need = [&](int v, int bytes) { return (size_t)(2 * NQ * NQ * NQ + 2 * NP * NP) * v * bytes; };
  if (L.prec == FE_F64) {
    if (vt == 0) vt = need(8, 8) <= (size_t)maxshm ? 8 : 4;
    if (vt == 16 && need(16, 8) <= (size_t)maxshm) return run_local<NP, NQ, 16, CPLX, double, double>(m, L, s, L.nt);
    if (vt == 8 && need(8, 8) <= (size_t)maxshm) return run_local<NP, NQ, 8, CPLX, double, double>(m, L, s, L.nt);
    if (vt == 4 && need(4, 8) <= (size_t)maxshm) return run_local<NP, NQ, 4, CPLX, double, double>(m, L, s, L.nt);
  } else if (L.prec == FE_F32) {
    if (vt == 0) vt = need(16, 4) <= (size_t)maxshm ? 16 : 8;
    if (vt == 32 && need(32, 4) <= (size_t)maxshm) return run_local<NP, NQ, 32, CPLX, float, float>(m, L, s, L.nt);
    if (vt == 16 && need(16, 4) <= (size_t)maxshm) return run_local<NP, NQ, 16, CPLX, float, float>(m, L, s, L.nt);
    if (vt == 8 && need(8, 4) <= (size_t)maxshm) return run_local<NP, NQ, 8, CPLX, float, float>(m, L, s, L.nt);
  } else if (L.prec == FE_BF16) {
    if (vt == 0) vt = need(32, 4) <= (size_t)maxshm ? 32 : (need(16, 4) <= (size_t)maxshm ? 16 : 8);
    if (vt == 32 && need(32, 4) <= (size_t)maxshm) return run_local<NP, NQ, 32, CPLX, bf16s, float>(m, L, s, L.nt);
    if (vt == 16 && need(16, 4) <= (size_t)maxshm) return run_local<NP, NQ, 16, CPLX, bf16s, float>(m, L, s, L.nt);
    if (vt == 8 && need(8, 4) <= (size_t)maxshm) return run_local<NP, NQ, 8, CPLX, bf16s, float>(m, L, s, L.nt);
  }
  return set_error(FE_EUNSUPPORTED, "no local-operator variant for this precision / vector tile / LDS size");
}

template <int NP, int NQ>
fe_status pick_cplx(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  return m->cplx ? pick_vt<NP, NQ, true>(m, L, s) : pick_vt<NP, NQ, false>(m, L, s);
}

}  // namespace

fe_status launch_local(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  if (m->nq != m->np) return set_error(FE_EUNSUPPORTED, "this build has kernels for n_q = n_p only");
  switch (m->np) {
    case 3: return pick_cplx<3, 3>(m, L, s);
    case 4: return pick_cplx<4, 4>(m, L, s);
    case 5: return pick_cplx<5, 5>(m, L, s);
    case 6: return pick_cplx<6, 6>(m, L, s);
    case 7: return pick_cplx<7, 7>(m, L, s);
    case 8: return pick_cplx<8, 8>(m, L, s);
    case 9: return pick_cplx<9, 9>(m, L, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
