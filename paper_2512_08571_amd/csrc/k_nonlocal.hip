// Nonlocal pseudopotential term of eqn Vnonloc / eqn AXmatrixfreenonloc,
// Y += alpha F diag(h) F^H X, with F the assembled node-level projector matrix
// (the paper's cell blocks F^(a,e) summed over cells).
//
//   k_nl_w    W_partial[chunk][s][lane] = sum over the chunk's support nodes of
//             conj(F[n][s]) X[node][lane]; one workgroup per (node chunk of one
//             atom, 64-lane vector tile); the four waves split the nodes and
//             are summed in LDS in a fixed order
//   k_nl_wsum W[s][lane] = h_s sum over the atom's chunks, in chunk order
//   k_nl_y    one wave per support node row: the row's (projector, value)
//             entries are wave-uniform scalar loads, W and Y are read and
//             written as coalesced 64-lane segments
// The vector width of these passes is the whole block row (the paper's
// level-0 batch for the nonlocal part of Alg. 1); complex lanes hold (re, im)
// pairs and exchange partners with a lane shuffle.
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

template <bool CPLX, typename TS, typename TC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_w(const TS *__restrict__ X, int64_t ldx, int nlanes, const double *__restrict__ dinv,
       const int *__restrict__ chunk_atom, const int *__restrict__ chunk_n0, const int *__restrict__ nodes,
       const int *__restrict__ atom_off, const int *__restrict__ proj_off, const TC *__restrict__ F, int fstride,
       TC *__restrict__ part, int64_t ldp) {
  __shared__ TC red[4][NL_MAXP][64];
  const int ch = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gl = blockIdx.y * 64 + lane;
  const int a = chunk_atom[ch];
  const int n0 = chunk_n0[ch];
  const int n1 = min(n0 + NL_CHUNK, atom_off[a + 1]);
  const int ns = proj_off[a + 1] - proj_off[a];
  const bool on = gl < nlanes;
  const bool odd = (gl & 1) != 0;
  TC acc[NL_MAXP];
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s) acc[s] = 0;
  constexpr int C = CPLX ? 2 : 1;
  for (int n = n0 + wv; n < n1; n += 4) {
    const int64_t g = nodes[n];
    TC x = on ? NCvt<TS, TC>::ld(X, g * ldx + gl) : (TC)0;
    if (dinv) x *= (TC)dinv[g];
    const TC xp = CPLX ? __shfl_xor(x, 1) : (TC)0;   // partner lane (im of re, re of im)
    const TC *f = F + (int64_t)n * fstride * C;
#pragma unroll
    for (int s = 0; s < NL_MAXP; ++s) {
      if (s < ns) {
        const TC fr = f[s * C];
        if (!CPLX) {
          acc[s] = fma(fr, x, acc[s]);
        } else {
          // conj(f) x:  re += fr xr + fi xi,  im += fr xi - fi xr
          const TC fi = f[s * C + 1];
          acc[s] = fma(fr, x, fma(odd ? -fi : fi, xp, acc[s]));
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s) red[wv][s][lane] = acc[s];
  __syncthreads();
  for (int t = threadIdx.x; t < ns * 64; t += NL_THREADS) {
    const int s = t / 64, l = t % 64;
    const TC sum = ((red[0][s][l] + red[1][s][l]) + red[2][s][l]) + red[3][s][l];
    const int glo = blockIdx.y * 64 + l;
    if (glo < nlanes) part[((int64_t)ch * NL_MAXP + s) * ldp + glo] = sum;
  }
}

template <typename TC>
__global__ void k_nl_wsum(const TC *__restrict__ part, int64_t ldp, const int *__restrict__ atom_chunk0,
                          const int *__restrict__ proj_off, const int *__restrict__ proj_atom,
                          const double *__restrict__ h, int ns, int nlanes, TC *__restrict__ W) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ns * nlanes) return;
  const int s = (int)(t / nlanes), l = (int)(t % nlanes);
  const int a = proj_atom[s];
  const int sl = s - proj_off[a];
  TC sum = 0;
  for (int ch = atom_chunk0[a]; ch < atom_chunk0[a + 1]; ++ch) sum += part[((int64_t)ch * NL_MAXP + sl) * ldp + l];
  W[(int64_t)s * nlanes + l] = (TC)h[s] * sum;
}

template <bool CPLX, typename TS, typename TC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_y(TS *__restrict__ Y, int64_t ldy, int nlanes, const int *__restrict__ rows, const int *__restrict__ rowptr,
       const int *__restrict__ colidx, const TC *__restrict__ val, int64_t nrows, const TC *__restrict__ W,
       TC alpha) {
  const int lane = threadIdx.x & 63;
  const int gl = blockIdx.y * 64 + lane;
  const bool on = gl < nlanes;
  const bool odd = (gl & 1) != 0;
  constexpr int C = CPLX ? 2 : 1;
  const int64_t wstride = (int64_t)gridDim.x * (NL_THREADS / 64);
  for (int64_t r = (int64_t)blockIdx.x * (NL_THREADS / 64) + (threadIdx.x >> 6); r < nrows; r += wstride) {
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    TC acc = 0;
    for (int e = e0; e < e1; ++e) {
      const int s = colidx[e];
      const TC w = on ? W[(int64_t)s * nlanes + gl] : (TC)0;
      const TC vr = val[(int64_t)e * C];
      if (!CPLX) {
        acc = fma(vr, w, acc);
      } else {
        // (vr + i vi)(wr + i wi): re += vr wr - vi wi, im += vr wi + vi wr
        const TC vi = val[(int64_t)e * C + 1];
        const TC wp = __shfl_xor(w, 1);
        acc = fma(vr, w, fma(odd ? vi : -vi, wp, acc));
      }
    }
    if (on) {
      const int64_t o = (int64_t)rows[r] * ldy + gl;
      NCvt<TS, TC>::st(Y, o, NCvt<TS, TC>::ld(Y, o) + alpha * acc);
    }
  }
}

namespace {
template <bool CPLX, typename TS, typename TC>
fe_status run_nl(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, const double *dinv,
                 double alpha, hipStream_t s) {
  const bool f64 = std::is_same<TC, double>::value;
  const TC *F = f64 ? (const TC *)m->nl_F64 : (const TC *)m->nl_F32;
  const TC *val = f64 ? (const TC *)m->nl_val64 : (const TC *)m->nl_val32;
  const int tiles = (nlanes + 63) / 64;
  // workspace: partials [nchunks][NL_MAXP][lanes] then W [ns][lanes]
  const int64_t ldp = nlanes;
  const int64_t need = ((int64_t)m->nl_nchunks * NL_MAXP + m->ns) * ldp * (int64_t)sizeof(double);
  if (m->nl_W == nullptr || m->nl_W_lanes < need) {
    if (m->nl_W) { hipFree(m->nl_W); m->footprint -= m->nl_W_lanes; m->nl_W = nullptr; }
    FE_HIP_TRY(hipMalloc(&m->nl_W, need));
    m->nl_W_lanes = need;
    m->footprint += need;
  }
  TC *part = (TC *)m->nl_W;
  TC *W = part + (int64_t)m->nl_nchunks * NL_MAXP * ldp;
  hipLaunchKernelGGL((k_nl_w<CPLX, TS, TC>), dim3(m->nl_nchunks, tiles), dim3(NL_THREADS), 0, s, (const TS *)X, ldx,
                     nlanes, dinv, m->nl_chunk_atom, m->nl_chunk_n0, m->nl_atom_nodes, m->nl_atom_off,
                     m->nl_atom_proj, F, m->nl_maxproj, part, ldp);
  FE_HIP_TRY(hipGetLastError());
  const int64_t nw = (int64_t)m->ns * nlanes;
  hipLaunchKernelGGL((k_nl_wsum<TC>), dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, part, ldp,
                     m->nl_atom_chunk0, m->nl_atom_proj, m->nl_proj_atom, m->nl_h, m->ns, nlanes, W);
  FE_HIP_TRY(hipGetLastError());
  int64_t blocks = (m->nl_nrows + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_nl_y<CPLX, TS, TC>), dim3((unsigned)blocks, tiles), dim3(NL_THREADS), 0, s, (TS *)Y, ldy,
                     nlanes, m->nl_rows, m->nl_rowptr, m->nl_colidx, val, m->nl_nrows, W, (TC)alpha);
  FE_HIP_TRY(hipGetLastError());
  return FE_OK;
}
}  // namespace

fe_status launch_nonlocal(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, int prec,
                          const double *dinv, double alpha, hipStream_t s) {
  if (m->ns == 0) return FE_OK;
  if (m->nl_maxproj > NL_MAXP) return set_error(FE_EUNSUPPORTED, "more than 10 projectors on one atom");
  if (m->cplx) {
    if (prec == FE_F64) return run_nl<true, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
    if (prec == FE_F32) return run_nl<true, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
    return run_nl<true, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  }
  if (prec == FE_F64) return run_nl<false, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  if (prec == FE_F32) return run_nl<false, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
  return run_nl<false, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, s);
}

}  // namespace fehx
