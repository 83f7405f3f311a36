// Nonlocal pseudopotential term of eqn Vnonloc / eqn AXmatrixfreenonloc:
//   W = h (.) (F^H X)          one workgroup per (atom, vector tile); the sum
//                              over the atom's support nodes is split across
//                              threads and reduced in LDS in a fixed order
//   Y += alpha F W              one thread per (support node, vector): the
//                              node's row of F (its atoms' projectors) times W
// F here is the assembled node-level projector matrix of the paper's F^(a,e)
// cell blocks.  Both products stream the vectors of a node contiguously and
// keep the node's projector values wave-uniform.  The vector width of a
// workgroup is the whole block row (the paper's level-0 batch for the
// nonlocal rest of Alg. 1).
#include "fe_internal.h"

namespace fehx {

struct bf16n { uint16_t b; };
__device__ __forceinline__ float nl_bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t nl_f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename TS, typename TC> struct NCvt;
template <> struct NCvt<double, double> {
  static __device__ double ld(const double *p, int64_t i) { return p[i]; }
  static __device__ void st(double *p, int64_t i, double v) { p[i] = v; }
};
template <> struct NCvt<float, float> {
  static __device__ float ld(const float *p, int64_t i) { return p[i]; }
  static __device__ void st(float *p, int64_t i, float v) { p[i] = v; }
};
template <> struct NCvt<bf16n, float> {
  static __device__ float ld(const bf16n *p, int64_t i) { return nl_bf2f(p[i].b); }
  static __device__ void st(bf16n *p, int64_t i, float v) { p[i].b = nl_f2bf(v); }
};

constexpr int NL_MAXP = 10;     // projectors per atom (s, p, d = 9)
constexpr int NL_THREADS = 256;

// C = 1 real, C = 2 complex (lanes 2c, 2c+1 hold re, im of vector c).
template <int C, int VW, typename TS, typename TC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_w(const TS *__restrict__ X, int64_t ldx, int nlanes, const double *__restrict__ dinv,
       const int *__restrict__ atom_off, const int *__restrict__ nodes, const int *__restrict__ proj_off,
       const TC *__restrict__ F, int fstride, const double *__restrict__ h, TC *__restrict__ W, int64_t ldw) {
  constexpr int G = NL_THREADS / VW;          // node groups
  __shared__ TC red[G][NL_MAXP][C][VW];
  const int a = blockIdx.x;
  const int c = threadIdx.x % VW, gr = threadIdx.x / VW;
  const int vec = blockIdx.y * VW + c;        // vector index (complex vectors for C = 2)
  const int s0 = proj_off[a], ns = proj_off[a + 1] - s0;
  TC acc[NL_MAXP][C];
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s)
#pragma unroll
    for (int q = 0; q < C; ++q) acc[s][q] = 0;
  const bool on = vec * C < nlanes;
  for (int n = atom_off[a] + gr; n < atom_off[a + 1]; n += G) {
    const int64_t g = nodes[n];
    TC xr = 0, xi = 0;
    if (on) {
      xr = NCvt<TS, TC>::ld(X, g * ldx + (int64_t)vec * C);
      if (C == 2) xi = NCvt<TS, TC>::ld(X, g * ldx + (int64_t)vec * C + 1);
      if (dinv) { const TC d = (TC)dinv[g]; xr *= d; xi *= d; }
    }
    const TC *f = F + (int64_t)n * fstride * C;
#pragma unroll
    for (int s = 0; s < NL_MAXP; ++s) {
      if (s < ns) {
        const TC fr = f[s * C];
        if (C == 1) {
          acc[s][0] = fma(fr, xr, acc[s][0]);
        } else {
          const TC fi = f[s * C + 1];       // conj(F) x
          acc[s][0] = fma(fr, xr, fma(fi, xi, acc[s][0]));
          acc[s][C - 1] = fma(fr, xi, fma(-fi, xr, acc[s][C - 1]));
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s)
#pragma unroll
    for (int q = 0; q < C; ++q) red[gr][s][q][c] = acc[s][q];
  __syncthreads();
  // fixed-order reduction over node groups
  for (int t = threadIdx.x; t < ns * C * VW; t += NL_THREADS) {
    const int cc = t % VW, q = (t / VW) % C, s = t / (VW * C);
    TC sum = 0;
    for (int r = 0; r < G; ++r) sum += red[r][s][q][cc];
    const int v = blockIdx.y * VW + cc;
    if (v * C < nlanes) W[(int64_t)(s0 + s) * ldw + (int64_t)v * C + q] = (TC)h[s0 + s] * sum;
  }
}

template <int C, int VW, typename TS, typename TC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_y(TS *__restrict__ Y, int64_t ldy, int nlanes, const int *__restrict__ rows,
       const int *__restrict__ rowptr, const int *__restrict__ colidx, const TC *__restrict__ val,
       int64_t nrows, const TC *__restrict__ W, int64_t ldw, TC alpha) {
  constexpr int R = NL_THREADS / VW;
  const int c = threadIdx.x % VW;
  const int64_t r = (int64_t)blockIdx.x * R + threadIdx.x / VW;
  const int vec = blockIdx.y * VW + c;
  if (r >= nrows || vec * C >= nlanes) return;
  TC ar = 0, ai = 0;
  for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int s = colidx[e];
    const TC vr = val[(int64_t)e * C];
    const TC wr = W[(int64_t)s * ldw + (int64_t)vec * C];
    if (C == 1) {
      ar = fma(vr, wr, ar);
    } else {
      const TC vi = val[(int64_t)e * C + 1];
      const TC wi = W[(int64_t)s * ldw + (int64_t)vec * C + 1];
      ar = fma(vr, wr, fma(-vi, wi, ar));
      ai = fma(vr, wi, fma(vi, wr, ai));
    }
  }
  const int64_t g = rows[r];
  const int64_t o = g * ldy + (int64_t)vec * C;
  NCvt<TS, TC>::st(Y, o, NCvt<TS, TC>::ld(Y, o) + alpha * ar);
  if (C == 2) NCvt<TS, TC>::st(Y, o + 1, NCvt<TS, TC>::ld(Y, o + 1) + alpha * ai);
}

namespace {
template <int C, typename TS, typename TC>
fe_status run_nl(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes,
                 const double *dinv, double alpha, hipStream_t s) {
  constexpr int VW = 32;
  const bool f64 = std::is_same<TC, double>::value;
  const TC *F = f64 ? (const TC *)m->nl_F64 : (const TC *)m->nl_F32;
  const TC *val = f64 ? (const TC *)m->nl_val64 : (const TC *)m->nl_val32;
  const int64_t need = (int64_t)m->ns * nlanes * (int64_t)sizeof(double);
  if (m->nl_W == nullptr || m->nl_W_lanes < (int64_t)m->ns * nlanes) {
    if (m->nl_W) { hipFree(m->nl_W); m->footprint -= m->nl_W_lanes * (int64_t)sizeof(double); m->nl_W = nullptr; }
    FE_HIP_TRY(hipMalloc(&m->nl_W, need));
    m->nl_W_lanes = (int64_t)m->ns * nlanes;
    m->footprint += need;
  }
  TC *W = (TC *)m->nl_W;
  const int nvec = (nlanes + C - 1) / C;
  dim3 gw(m->natoms, (nvec + VW - 1) / VW);
  hipLaunchKernelGGL((k_nl_w<C, VW, TS, TC>), gw, dim3(NL_THREADS), 0, s, (const TS *)X, ldx, nlanes, dinv,
                     m->nl_atom_off, m->nl_atom_nodes, m->nl_atom_proj, F, m->nl_maxproj, m->nl_h, W,
                     (int64_t)nlanes);
  FE_HIP_TRY(hipGetLastError());
  constexpr int R = NL_THREADS / VW;
  dim3 gy((unsigned)((m->nl_nrows + R - 1) / R), (nvec + VW - 1) / VW);
  hipLaunchKernelGGL((k_nl_y<C, VW, TS, TC>), gy, dim3(NL_THREADS), 0, s, (TS *)Y, ldy, nlanes, m->nl_rows,
                     m->nl_rowptr, m->nl_colidx, val, m->nl_nrows, W, (int64_t)nlanes, (TC)alpha);
  FE_HIP_TRY(hipGetLastError());
  return FE_OK;
}
}  // namespace

fe_status launch_nonlocal(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, int prec,
                          const double *dinv, double alpha, hipStream_t s) {
  if (m->ns == 0) return FE_OK;
  if (m->nl_maxproj > NL_MAXP) return set_error(FE_EUNSUPPORTED, "more than 10 projectors on one atom");
  if (m->cplx) {
    if (prec == FE_F64) return run_nl<2, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
    if (prec == FE_F32) return run_nl<2, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
    return run_nl<2, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  }
  if (prec == FE_F64) return run_nl<1, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  if (prec == FE_F32) return run_nl<1, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  return run_nl<1, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
}

}  // namespace fehx
