// Matrix-free local operator H_loc X on gfx950 (Sec. 3.2, eqns ggaReal /
// ggaCmplx, Alg. 2), one subdomain on one GPU.
//
// Work decomposition (the GPU analogue of the paper's multilevel batches,
// Sec. 4.1): a workgroup owns one column of cells along a_2 and one tile of
// VT real vector lanes (for complex meshes the real and imaginary parts of a
// vector sit in adjacent lanes, the paper's level-2 re/im batches).  It walks
// the column cell by cell: the 1D contraction sweeps of Alg. 2 with the
// even-odd decomposition (each thread applies one 1D matrix to one line of
// points for one lane, table rows read as wave-uniform scalars) and the
// quadrature-point stage of eqn refact, on LDS blocks [point][lane] (lanes
// fastest).  With n_q = n_p and a diagonal metric (local_column_lines) the
// gather X^(e) = Q^(e) X lands in registers as x-lines and seven passes run
// per cell: N along x, N along y, [N along z + the z-direction stage] on
// z-lines, the x-direction stage on x-lines, [the y-direction stage + N^T
// along y] on y-lines, N^T along x, [N^T along z + scatter] on z-lines (the
// transposed sweeps may run in any axis order and a line's owner can chain
// two steps).  Otherwise (n_q > n_p, the general metric, or a per-cell core)
// the block is staged in LDS first and every sweep is its own pass.
//
// Scatter Y += Q^(e)T Y^(e) without atomics and deterministically:
//  * along a_2 the shared node plane of consecutive cells is summed in
//    registers (line-gather path) or LDS (and the periodic first/last plane
//    of the column at the end);
//  * across columns the columns are coloured 2 (or 3 for an odd count) per
//    axis and launched colour by colour; a node shared by several columns is
//    stored by the column of the lowest colour phase and read-modify-written
//    by the later ones, so no two concurrently running workgroups touch the
//    same node and the summation order is fixed.
#pragma once
#include <type_traits>

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

// L consecutive lanes of one node row: global (storage type, 16-byte vector
// access for the wide forms) and LDS (compute type)
template <typename TS, typename TC, int L> struct VecIO;
template <typename TS, typename TC> struct VecIO<TS, TC, 1> {
  static __device__ __forceinline__ void ld(const TS *p, TC (&v)[1]) { v[0] = Cvt<TS, TC>::ld(p, 0); }
  static __device__ __forceinline__ void st(TS *p, const TC (&v)[1]) { Cvt<TS, TC>::st(p, 0, v[0]); }
};
template <> struct VecIO<double, double, 2> {
  static __device__ __forceinline__ void ld(const double *p, double (&v)[2]) {
    const double2 a = *(const double2 *)p; v[0] = a.x; v[1] = a.y;
  }
  static __device__ __forceinline__ void st(double *p, const double (&v)[2]) { *(double2 *)p = make_double2(v[0], v[1]); }
};
template <> struct VecIO<float, float, 4> {
  static __device__ __forceinline__ void ld(const float *p, float (&v)[4]) {
    const float4 a = *(const float4 *)p; v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
  static __device__ __forceinline__ void st(float *p, const float (&v)[4]) { *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]); }
};
template <> struct VecIO<bf16s, float, 8> {
  static __device__ __forceinline__ void ld(const bf16s *p, float (&v)[8]) {
    const uint4 a = *(const uint4 *)p;
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = __uint_as_float(w[i] << 16);
      v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
  static __device__ __forceinline__ void st(bf16s *p, const float (&v)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f_to_bf16(v[2 * i]) | ((uint32_t)f_to_bf16(v[2 * i + 1]) << 16);
    *(uint4 *)p = make_uint4(w[0], w[1], w[2], w[3]);
  }
};
template <typename TC, int L> struct LdsVec {
  static __device__ __forceinline__ void st(TC *p, const TC (&v)[L]) {
#pragma unroll
    for (int j = 0; j < L; ++j) p[j] = v[j];
  }
  static __device__ __forceinline__ void ld(const TC *p, TC (&v)[L]) {
#pragma unroll
    for (int j = 0; j < L; ++j) v[j] = p[j];
  }
};
template <> struct LdsVec<double, 2> {
  static __device__ __forceinline__ void st(double *p, const double (&v)[2]) { *(double2 *)p = make_double2(v[0], v[1]); }
  static __device__ __forceinline__ void ld(const double *p, double (&v)[2]) {
    const double2 a = *(const double2 *)p; v[0] = a.x; v[1] = a.y;
  }
};
template <> struct LdsVec<float, 4> {
  static __device__ __forceinline__ void st(float *p, const float (&v)[4]) { *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]); }
  static __device__ __forceinline__ void ld(const float *p, float (&v)[4]) {
    const float4 a = *(const float4 *)p; v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
};
template <> struct LdsVec<float, 8> {
  static __device__ __forceinline__ void st(float *p, const float (&v)[8]) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4 *)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  }
  static __device__ __forceinline__ void ld(const float *p, float (&v)[8]) {
    const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
};
// lanes per element of the wide form: 16 bytes of storage
template <typename TS> struct WideLanes { static constexpr int value = 16 / sizeof(TS); };

// ---- kernel arguments ----------------------------------------------------------
template <typename TC> struct KArgs {
  const void *X;
  void *Y;
  int64_t ldx, ldy;
  int nlanes;
  int N0, N1, N2, M0, M1, M2, p;
  int dmask;           // bit d: axis d has Dirichlet faces (interior nodes g - 1)
  int offd;            // off-diagonal metric terms (sheared box): gradients staged in LDS
  const int *cols;
  int ncols, ntiles;
  const TC *tab;
  const TC *wq;
  const TC *coef;
  int64_t coef_cell;   // coefficient elements per cell (0: one block for all cells)
  int gga;
  const double *dinv;
  const float *mxtab;  // full 1D matrices [4][8][8] (N, N^T, Dtilde, Dtilde^T) for the MFMA path
  int ncoef;           // coefficient blocks per cell (4, or NCOEF_GEN with the per-point metric)
};

// ---- even-odd application of a packed centro-(anti)symmetric 1D matrix ----------
// tab rows q < ceil(NOUT/2): E[q][0..ceil(NIN/2)) then O[q][0..floor(NIN/2)).
template <typename TC> using cptr = const __attribute__((address_space(4))) TC *;

// A wave-uniform table pointer whose value the compiler cannot see through:
// the table is re-read with scalar loads at each use instead of being hoisted
// out of the loops into (spilled) registers.
template <typename TC> __device__ __forceinline__ cptr<TC> scalar_table(const TC *p) {
  uint64_t a = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(a));
  return reinterpret_cast<cptr<TC>>(a);
}

template <int NIN, int NOUT, int SYM, typename TC>
__device__ __forceinline__ void eo_apply(cptr<TC> __restrict__ t, const TC (&x)[NIN], TC (&y)[NOUT]) {
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
    cptr<TC> E = t + q * NIN;
    cptr<TC> O = E + CI;
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
template <int NIN, int NOUT, int SYM, int VT, int NT, typename TC, typename Dec>
__device__ __forceinline__ void line_pass(const TC *__restrict__ src, TC *__restrict__ dst,
                                          const TC *__restrict__ tab, int nlines, Dec dec) {
  const int total = nlines * VT;
  for (int t = threadIdx.x; t < total; t += NT) {
    const int v = t % VT, l = t / VT;
    int sb, ss, db, ds;
    dec(l, sb, ss, db, ds);
    TC x[NIN], y[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) x[i] = src[(sb + i * ss) * VT + v];
    eo_apply<NIN, NOUT, SYM>(scalar_table(tab), x, y);
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
// C holds the cell's weighted coefficients [4][NQ3] staged in LDS (threads of
// one line read the same addresses).  The weight w_Q det J of a point on a
// line along D through (a, b) is W2[line] (w_a w_b, from LDS once per line)
// times the wave-uniform factor w_i det J, pre-multiplied in the table by
// g_DD (kinetic flux) and kappa_D (Bloch term).
// Value of the partner lane (lane ^ 1: the real / imaginary part of the same
// vector) by a DPP quad permutation [1, 0, 3, 2]; both lanes of a pair are
// always active together (tiles hold whole vectors, VT even).
__device__ __forceinline__ double swap_pair(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swap_pair(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// The quadrature-point work of one line along reference direction D: given
// the interpolated field u on the line's points, o = Dtilde^T F + z with
//   T = Dtilde u,  F = G_DD w T + Vtilde^G_D u,
//   z = Vtilde^G_D T  [+ (V + |k|^2/2) w u for D = 0]  [- i kappa_D w T],
// line l through (a, b) = (l % NQ, l / NQ) of the other two directions.
template <int D, int NQ, int VT, bool CPLX, typename TC, bool OFFD = false>
__device__ __forceinline__ void dir_line(const TC (&u)[NQ], TC (&out)[NQ], int l, int base, int stride,
                                         const TC *__restrict__ tD, const TC *__restrict__ tDT,
                                         const TC *__restrict__ tgw, const TC *__restrict__ tkw, const KArgs<TC> &a,
                                         const TC *__restrict__ C, const TC *__restrict__ W2, int lane,
                                         const TC *__restrict__ T3 = nullptr,
                                         int v = 0) {
  constexpr int NQ3 = NQ * NQ * NQ;
  const TC *cL = C;
  const TC *cG = C + (1 + D) * NQ3;
  TC T[NQ], F[NQ], z[NQ], o[NQ];
  eo_apply<NQ, NQ, -1>(scalar_table(tD), u, T);
  const TC w2 = W2[l];
  cptr<TC> gw = scalar_table(tgw + D * NQ);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int Q = base + i * stride;
    if constexpr (OFFD) {
      // general metric (sheared or distorted cells): the weighted metric row
      // of direction D at this point from the coefficient blocks 4-9, the
      // other two reference gradients from LDS
      constexpr int OD[3][3] = {{4, 7, 8}, {7, 5, 9}, {8, 9, 6}};
      F[i] = C[OD[D][D] * NQ3 + Q] * T[i];
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t != D) F[i] = fma(C[OD[D][t] * NQ3 + Q], T3[(t * NQ3 + Q) * VT + v], F[i]);
    } else {
      F[i] = (w2 * gw[i]) * T[i];
    }
    z[i] = 0;
    if (a.gga) {
      const TC vg = cG[Q];
      F[i] = fma(vg, u[i], F[i]);
      z[i] = vg * T[i];
    }
    if (D == 0) z[i] = fma(cL[Q], u[i], z[i]);
    if constexpr (CPLX) {
      // -i kappa w T: real lane gets +kappa w T_im, imaginary lane -kappa w T_re
      const TC tp = swap_pair(T[i]);
      const TC kw = OFFD ? C[(10 + D) * NQ3 + Q] : w2 * scalar_table(tkw + D * NQ)[i];
      z[i] = fma((lane & 1) ? -kw : kw, tp, z[i]);
    }
  }
  eo_apply<NQ, NQ, -1>(scalar_table(tDT), F, o);
#pragma unroll
  for (int i = 0; i < NQ; ++i) out[i] = o[i] + z[i];
}

// Lines along D of the interpolated field src (pass-per-sweep path): the
// D = 0 contribution initialises dst, the others are added.  OFFD: the
// off-diagonal metric terms read the other gradients from T3.
template <int D, int NQ, int VT, bool CPLX, typename TC, bool OFFD, int NT>
__device__ __forceinline__ void dir_pass(const TC *__restrict__ src, TC *__restrict__ dst, const TC *tD,
                                         const TC *tDT, const TC *tgw, const TC *tkw, const KArgs<TC> &a,
                                         const TC *__restrict__ C, const TC *__restrict__ W2, int lane0,
                                         const TC *__restrict__ T3) {
  constexpr int NQ2 = NQ * NQ;
  for (int t = threadIdx.x; t < NQ2 * VT; t += NT) {
    const int v = t % VT, l = t / VT;
    int base, stride;
    if (D == 0) { base = l * NQ; stride = 1; }
    else if (D == 1) { base = (l / NQ) * NQ2 + (l % NQ); stride = NQ; }
    else { base = l; stride = NQ2; }
    TC u[NQ], o[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) u[i] = src[(base + i * stride) * VT + v];
    dir_line<D, NQ, VT, CPLX, TC, OFFD>(u, o, l, base, stride, tD, tDT, tgw, tkw, a, C, W2, lane0 + v, T3, v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int idx = (base + i * stride) * VT + v;
      if (D == 0) dst[idx] = o[i];
      else dst[idx] += o[i];
    }
  }
}

// The three reference gradients of src (D-tilde along x, y, z lines) into
// T3[D][point][lane], one pass over the lines of all three directions.
template <int NQ, int VT, int NT, typename TC>
__device__ __forceinline__ void grad_pass(const TC *__restrict__ src, TC *__restrict__ T3, const TC *tD) {
  constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
  for (int t = threadIdx.x; t < 3 * NQ2 * VT; t += NT) {
    const int D = t / (NQ2 * VT), rem = t % (NQ2 * VT);
    const int v = rem % VT, l = rem / VT;
    int base, stride;
    if (D == 0) { base = l * NQ; stride = 1; }
    else if (D == 1) { base = (l / NQ) * NQ2 + (l % NQ); stride = NQ; }
    else { base = l; stride = NQ2; }
    TC u[NQ], g[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) u[i] = src[(base + i * stride) * VT + v];
    eo_apply<NQ, NQ, -1>(scalar_table(tD), u, g);
#pragma unroll
    for (int i = 0; i < NQ; ++i) T3[(D * NQ3 + base + i * stride) * VT + v] = g[i];
  }
}

// x-lines of the interpolated field src: dst += the x-direction contribution
template <int NQ, int VT, bool CPLX, int NT, typename TC>
__device__ __forceinline__ void xdir_pass(const TC *__restrict__ src, TC *__restrict__ dst, const TC *tD,
                                          const TC *tDT, const TC *tgw, const TC *tkw, const KArgs<TC> &a,
                                          const TC *__restrict__ C, const TC *__restrict__ W2, int lane0) {
  constexpr int NQ2 = NQ * NQ;
  for (int t = threadIdx.x; t < NQ2 * VT; t += NT) {
    const int v = t % VT, l = t / VT;
    const int base = l * NQ;
    TC u[NQ], o[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) u[i] = src[(base + i) * VT + v];
    dir_line<0, NQ, VT, CPLX>(u, o, l, base, 1, tD, tDT, tgw, tkw, a, C, W2, lane0 + v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) dst[(base + i) * VT + v] += o[i];
  }
}

// z-lines (NP = NQ): interpolation along z of buf (N_x, N_y already applied)
// written to u, and the z-direction contribution written over buf's line
template <int NQ, int VT, bool CPLX, int NT, typename TC>
__device__ __forceinline__ void zpass(TC *__restrict__ buf, TC *__restrict__ uout, const TC *tN, const TC *tD,
                                      const TC *tDT, const TC *tgw, const TC *tkw, const KArgs<TC> &a,
                                      const TC *__restrict__ C, const TC *__restrict__ W2, int lane0) {
  constexpr int NQ2 = NQ * NQ;
  for (int t = threadIdx.x; t < NQ2 * VT; t += NT) {
    const int v = t % VT, l = t / VT;
    TC x[NQ], u[NQ], o[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) x[i] = buf[(l + i * NQ2) * VT + v];
    eo_apply<NQ, NQ, 1>(scalar_table(tN), x, u);
#pragma unroll
    for (int i = 0; i < NQ; ++i) uout[(l + i * NQ2) * VT + v] = u[i];
    dir_line<2, NQ, VT, CPLX>(u, o, l, l, NQ2, tD, tDT, tgw, tkw, a, C, W2, lane0 + v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) buf[(l + i * NQ2) * VT + v] = o[i];
  }
}

// y-lines (NP = NQ): the y-direction contribution of u completes the sum in
// acc; the transposed interpolation along y of the complete line is written
// over u's line
template <int NQ, int VT, bool CPLX, int NT, typename TC>
__device__ __forceinline__ void ypass(TC *__restrict__ u_io, const TC *__restrict__ acc, const TC *tNT, const TC *tD,
                                      const TC *tDT, const TC *tgw, const TC *tkw, const KArgs<TC> &a,
                                      const TC *__restrict__ C, const TC *__restrict__ W2, int lane0) {
  constexpr int NQ2 = NQ * NQ;
  for (int t = threadIdx.x; t < NQ2 * VT; t += NT) {
    const int v = t % VT, l = t / VT;
    const int base = (l / NQ) * NQ2 + (l % NQ);
    TC u[NQ], o[NQ], y[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) u[i] = u_io[(base + i * NQ) * VT + v];
    dir_line<1, NQ, VT, CPLX>(u, o, l, base, NQ, tD, tDT, tgw, tkw, a, C, W2, lane0 + v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) o[i] += acc[(base + i * NQ) * VT + v];
    eo_apply<NQ, NQ, 1>(scalar_table(tNT), o, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) u_io[(base + i * NQ) * VT + v] = y[i];
  }
}

__device__ __forceinline__ int colour_of(int c, int n) { return ((n & 1) && c == n - 1) ? 2 : (c & 1); }

// FP64 blocks are capped at 512 threads so each lane may use 256 VGPRs.
template <typename TC> struct MaxThreads { static constexpr int value = sizeof(TC) == 8 ? 512 : 1024; };

// Threads per block: one work item per (line, lane) of the widest pass.
template <int NQ, int VT, typename TC> struct BlockSize {
  static constexpr int raw = ((NQ * NQ * VT + 63) / 64) * 64;
  static constexpr int value = raw > MaxThreads<TC>::value ? MaxThreads<TC>::value : (raw < 128 ? 128 : raw);
};
// A per-cell core (the sweeps of one cell between the staged block and the
// completed Y^(e)) other than the line passes below sets its own block size
// and may ask for LDS elements after the line weights.
template <class Core> struct CoreLds { static constexpr int elems = Core::extra_lds_elems; };
template <> struct CoreLds<void> { static constexpr int elems = 0; };
template <int NQ, int VT, typename TC, class Core> struct Threads { static constexpr int value = Core::threads; };
template <int NQ, int VT, typename TC> struct Threads<NQ, VT, TC, void> {
  static constexpr int value = BlockSize<NQ, VT, TC>::value;
};

// The line-gather path below serves FP64 with n_q = n_p and no per-cell core,
// except complex blocks at n_p = 8.  FP32 / BF16 blocks keep the staged path:
// their 16-byte element loads and stores (four or eight lanes per access) beat
// single-lane lines (FP32 filter steps, Mid operator, 512 vectors: 259 vs
// 313 ms per pass).  At n_p = 8 the 64 lines of a pass fill whole waves on
// either path, and complex blocks run 3.7% faster staged (12^3 cells, p = 7,
// 128 complex vectors, best tile each: 0.619 vs 0.642 ms per colour phase);
// real blocks there, and every other n_p measured (4, 6, 7, 9), run as fast
// or faster on lines (n_p = 7: 0.65 vs 0.79 ms on the Mid operator).
template <int NP, int NQ, typename TC, class Core, bool CPLX> struct LinesPath {
  static constexpr bool value =
      std::is_void<Core>::value && NP == NQ && std::is_same<TC, double>::value && !(CPLX && NP == 8);
};

// One work item on the line-gather path (n_q = n_p, diagonal metric, no
// per-cell core): the cell's block is gathered from X straight into x-lines
// (registers) and the completed Y^(e) leaves from z-lines (registers), so
// there is no staging pass through LDS, the node plane shared by consecutive
// cells of the column stays in registers (its z-line belongs to the same
// thread in every cell), and a cell takes six barriers.  Every thread keeps
// the same (line, lane) items in all passes, so their line bases are computed
// once per work item.  Passes (LDS A, B = [point][lane]):
//   1  x-lines: N along x of the gathered lines          (regs -> B)
//   2  y-lines: N along y                                (B -> A)
//   3  z-lines: N along z + the z-direction stage        (A -> u in B, z part in A)
//   4  x-lines: the x-direction stage                    (B -> A, added)
//   5  y-lines: the y-direction stage + N^T along y      (B, A -> B)
//   6  x-lines: N^T along x                              (B -> A)
//   7  z-lines: N^T along z, the carried plane, scatter  (A -> regs -> Y)
// The next cell's lines, D^-1 entries, coefficients and the values this
// cell's scatter reads back are loaded after pass 5 and land during 6 and 7.
template <int NP, int VT, bool CPLX, typename TS, typename TC, int NT>
__device__ __forceinline__ void local_column_lines(const KArgs<TC> &a, const int col, const int tile) {
  constexpr int NQ = NP, NP2 = NP * NP, NQ2 = NP2, NQ3 = NP2 * NP;
  constexpr int NI = NQ2 * VT;                      // (line, lane) items of a pass
  constexpr int IT = (NI + NT - 1) / NT;            // items per thread
  constexpr int CPT = (4 * NQ3 + NT - 1) / NT;      // coefficients per thread
  constexpr int OFF_N = 0;
  constexpr int OFF_NT = OFF_N + ((NQ + 1) / 2) * NP;
  constexpr int OFF_D = OFF_NT + ((NP + 1) / 2) * NQ;
  constexpr int OFF_DT = OFF_D + ((NQ + 1) / 2) * NQ;
  constexpr int OFF_GW = OFF_DT + ((NQ + 1) / 2) * NQ;
  constexpr int OFF_KW = OFF_GW + 3 * NQ;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC *A = reinterpret_cast<TC *>(smem_raw);
  TC *B = A + NQ3 * VT;
  TC *Cf = B + NQ3 * VT;             // cell coefficients [4][NQ3]
  TC *W2 = Cf + 4 * NQ3;             // w_a w_b per line [NQ2]

  const int cx = a.cols[2 * col], cy = a.cols[2 * col + 1];
  const int lane0 = tile * VT;
  const int tid = threadIdx.x;
  const TS *__restrict__ X = (const TS *)a.X;
  TS *__restrict__ Y = (TS *)a.Y;
  const TC *tN = a.tab + OFF_N, *tNT = a.tab + OFF_NT, *tD = a.tab + OFF_D, *tDT = a.tab + OFF_DT;
  const TC *tGW = a.tab + OFF_GW, *tKW = a.tab + OFF_KW;
  const int p = a.p;
  const int xoff = a.dmask & 1, yoff = (a.dmask >> 1) & 1, zoff = (a.dmask >> 2) & 1;
  const int ax = colour_of(cx, a.N0), by = colour_of(cy, a.N1);
  const int axl = colour_of(cx == 0 ? a.N0 - 1 : cx - 1, a.N0);
  const int axr = colour_of(cx == a.N0 - 1 ? 0 : cx + 1, a.N0);
  const int byl = colour_of(cy == 0 ? a.N1 - 1 : cy - 1, a.N1);
  const int byr = colour_of(cy == a.N1 - 1 ? 0 : cy + 1, a.N1);
  // node coordinate along an axis: cell c, local index i; periodic axes wrap,
  // a Dirichlet axis numbers its interior nodes g - 1 and has no DoF on its faces
  auto coord = [&](int c, int i, int off, int M, bool &in) {
    int g = c * p + i - off;
    if (off) in = in && g >= 0 && g < M;
    else if (g >= M) g -= M;
    return g;
  };

  // per item: line l = t / VT, lane v = t % VT; the gather x-line is
  // (j, k) = (l % NP, l / NP), the scatter z-line (i, j) = (l % NP, l / NP)
  int gxs[IT], gys[IT];      // scatter: node x and y of the z-line
  int gyg[IT], kg[IT];       // gather: node y and plane k of the x-line
  int flags[IT];             // bit 0 lane in range, 1 gather y in range, 2 scatter x/y in range, 3 read-modify-write
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int t = tid + r * NT;
    const int l = t / VT, v = t % VT;
    const bool item = t < NI && lane0 + v < a.nlanes;
    bool ing = true, ins = true;
    gyg[r] = coord(cy, l % NP, yoff, a.M1, ing);
    kg[r] = l / NP;
    const int i = l % NP, j = l / NP;
    gxs[r] = coord(cx, i, xoff, a.M0, ins);
    gys[r] = coord(cy, j, yoff, a.M1, ins);
    const bool xs = (i == 0) || (i == NP - 1), ys = (j == 0) || (j == NP - 1);
    const int axo = (i == 0) ? axl : axr, byo = (j == 0) ? byl : byr;
    const bool rmw = !((!xs || ax < axo) && (!ys || by < byo));
    flags[r] = (item ? 1 : 0) | (ing ? 2 : 0) | (ins ? 4 : 0) | (rmw ? 8 : 0);
  }
  const int64_t MM = (int64_t)a.M0 * a.M1;
  int ll[IT], vv[IT], py[IT];   // line index, lane, first point of the y-line
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int t = tid + r * NT;
    ll[r] = t / VT;
    vv[r] = t % VT;
    py[r] = (ll[r] / NQ) * NQ2 + ll[r] % NQ;
  }

  for (int t = tid; t < NQ2; t += NT) W2[t] = a.wq[t];
  TC xl[IT][NP], dl[IT][NP], cpre[CPT], ypre[IT][NP];
  // the gathered x-lines of cell cz (and their D^-1 entries) and its coefficients
  auto prefetch = [&](int cz) {
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int v = vv[r];
      bool in = (flags[r] & 3) == 3;
      const int gz = coord(cz, kg[r], zoff, a.M2, in);
      const int64_t row = (int64_t)gyg[r] * a.M0 + MM * gz;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        bool ini = in;
        const int gx = coord(cx, i, xoff, a.M0, ini);
        xl[r][i] = 0;
        dl[r][i] = 1;
        if (ini) {
          xl[r][i] = Cvt<TS, TC>::ld(X, (row + gx) * a.ldx + lane0 + v);
          if (a.dinv) dl[r][i] = (TC)a.dinv[row + gx];
        }
      }
    }
    const TC *src = a.coef + (cx + (int64_t)a.N0 * (cy + (int64_t)a.N1 * cz)) * a.coef_cell;
    const int nst = (a.ncoef < 4 ? a.ncoef : 4) * NQ3;
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + r * NT;
      cpre[r] = e < nst ? src[e] : (TC)0;
    }
  };
  auto stage_coef = [&]() {
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + r * NT;
      if (e < 4 * NQ3) Cf[e] = cpre[r];
    }
  };
  prefetch(0);
  stage_coef();
  TC carry[IT], first[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) carry[r] = first[r] = 0;

  for (int cz = 0; cz < a.N2; ++cz) {
    const int kskip0 = (cz == 0) ? 0 : -1;             // plane held back for the wrap
    const int kskip1 = (cz < a.N2 - 1) ? NP - 1 : -1;  // plane carried to the next cell
    // 1: N along x of the gathered lines (D^-1 applied first in filter steps)
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int t = tid + r * NT;
      if (t < NI) {
        const int v = vv[r], l = ll[r];
        TC x[NP], y[NQ];
#pragma unroll
        for (int i = 0; i < NP; ++i) x[i] = xl[r][i] * dl[r][i];
        eo_apply<NP, NQ, 1>(scalar_table(tN), x, y);
#pragma unroll
        for (int q = 0; q < NQ; ++q) B[(l * NQ + q) * VT + v] = y[q];
      }
    }
    __syncthreads();
    // 2: N along y
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (tid + r * NT >= NI) break;
      const int ey = py[r] * VT + vv[r];
      TC x[NP], y[NQ];
#pragma unroll
      for (int i = 0; i < NP; ++i) x[i] = B[ey + i * NQ * VT];
      eo_apply<NP, NQ, 1>(scalar_table(tN), x, y);
#pragma unroll
      for (int q = 0; q < NQ; ++q) A[ey + q * NQ * VT] = y[q];
    }
    __syncthreads();
    // 3: z sweep fused with the z-direction stage: u -> B, z part -> A
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (tid + r * NT >= NI) break;
      const int ez = ll[r] * VT + vv[r];
      TC x[NQ], u[NQ], o[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) x[i] = A[ez + i * NQ2 * VT];
      eo_apply<NQ, NQ, 1>(scalar_table(tN), x, u);
#pragma unroll
      for (int i = 0; i < NQ; ++i) B[ez + i * NQ2 * VT] = u[i];
      dir_line<2, NQ, VT, CPLX>(u, o, ll[r], ll[r], NQ2, tD, tDT, tGW, tKW, a, Cf, W2, lane0 + vv[r]);
#pragma unroll
      for (int i = 0; i < NQ; ++i) A[ez + i * NQ2 * VT] = o[i];
    }
    __syncthreads();
    // 4: the x-direction stage added into A
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (tid + r * NT >= NI) break;
      const int ex = ll[r] * NQ * VT + vv[r];
      TC u[NQ], o[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) u[i] = B[ex + i * VT];
      dir_line<0, NQ, VT, CPLX>(u, o, ll[r], ll[r] * NQ, 1, tD, tDT, tGW, tKW, a, Cf, W2, lane0 + vv[r]);
#pragma unroll
      for (int i = 0; i < NQ; ++i) A[ex + i * VT] += o[i];
    }
    __syncthreads();
    // 5: the y-direction stage completes the sum; N^T along y (-> B)
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (tid + r * NT >= NI) break;
      const int ey = py[r] * VT + vv[r];
      TC u[NQ], o[NQ], y[NP];
#pragma unroll
      for (int i = 0; i < NQ; ++i) u[i] = B[ey + i * NQ * VT];
      dir_line<1, NQ, VT, CPLX>(u, o, ll[r], py[r], NQ, tD, tDT, tGW, tKW, a, Cf, W2, lane0 + vv[r]);
#pragma unroll
      for (int i = 0; i < NQ; ++i) o[i] += A[ey + i * NQ * VT];
      eo_apply<NQ, NP, 1>(scalar_table(tNT), o, y);
#pragma unroll
      for (int i = 0; i < NP; ++i) B[ey + i * NQ * VT] = y[i];
    }
    // the next cell's lines and coefficients, and this cell's read-back values
    if (cz + 1 < a.N2) prefetch(cz + 1);
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int v = vv[r];
      const bool rm = (flags[r] & 13) == 13;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        ypre[r][k] = 0;
        bool in = rm && k != kskip0 && k != kskip1;
        const int gz = coord(cz, k, zoff, a.M2, in);
        if (in) ypre[r][k] = Cvt<TS, TC>::ld(Y, (gxs[r] + (int64_t)gys[r] * a.M0 + MM * gz) * a.ldy + lane0 + v);
      }
    }
    __syncthreads();
    // 6: N^T along x (B -> A)
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      if (tid + r * NT >= NI) break;
      const int ex = ll[r] * NQ * VT + vv[r];
      TC x[NQ], y[NP];
#pragma unroll
      for (int i = 0; i < NQ; ++i) x[i] = B[ex + i * VT];
      eo_apply<NQ, NP, 1>(scalar_table(tNT), x, y);
#pragma unroll
      for (int i = 0; i < NP; ++i) A[ex + i * VT] = y[i];
    }
    __syncthreads();
    // 7: N^T along z of the z-lines, the shared planes, the scatter
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int t = tid + r * NT;
      if (t < NI) {
        const int v = vv[r], l = ll[r];
        TC z[NQ], y[NP];
#pragma unroll
        for (int q = 0; q < NQ; ++q) z[q] = A[(l + q * NP2) * VT + v];
        eo_apply<NQ, NP, 1>(scalar_table(tNT), z, y);
        // plane 0 takes the carry (or, in the column's first cell, is held
        // back); plane NP-1 is carried, or in the last cell takes the first plane
        if (cz == 0) first[r] = y[0];
        else y[0] += carry[r];
        if (cz == a.N2 - 1) y[NP - 1] += (cz == 0) ? y[0] : first[r];
        carry[r] = y[NP - 1];
        if (flags[r] & 1 && flags[r] & 4) {
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            bool in = k != kskip0 && k != kskip1;
            const int gz = coord(cz, k, zoff, a.M2, in);
            if (in)
              Cvt<TS, TC>::st(Y, (gxs[r] + (int64_t)gys[r] * a.M0 + MM * gz) * a.ldy + lane0 + v,
                              (flags[r] & 8) ? ypre[r][k] + y[k] : y[k]);
          }
        }
      }
    }
    if (cz + 1 < a.N2) stage_coef();
  }
  __syncthreads();
}

// One work item: the column (cx, cy) = a.cols[col] of cells along a_2 for
// vector lanes [tile VT, tile VT + VT).  Ends with a barrier, so the block may
// start another item right away.
//
// Block elements: LPE consecutive lanes of one node (LPE = 1, or the 16-byte
// wide form when every block, leading dimension and lane count is aligned to
// it), so a node's VT lanes are VT / LPE elements and one element is one
// global and one LDS vector access.
template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC, int LPE, bool SH, class Core = void>
__device__ __forceinline__ void local_column(const KArgs<TC> &a, const int col, const int tile) {
  constexpr int NP2 = NP * NP, NP3 = NP2 * NP, NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
  constexpr int NT = Threads<NQ, VT, TC, Core>::value;
  if constexpr (LinesPath<NP, NQ, TC, Core, CPLX>::value) {
    if (!SH || !a.offd) {
      local_column_lines<NP, VT, CPLX, TS, TC, NT>(a, col, tile);
      return;
    }
  }
  static_assert(VT <= 255 && NP <= 15, "packed element metadata holds lane offsets < 256 and planes < 16");
  static_assert(VT % LPE == 0, "the vector tile must hold whole elements");
  static_assert(NQ >= NP, "n_q >= n_p");
  constexpr int NV = VT / LPE;                     // elements per node
  constexpr int XPT = (NP3 * NV + NT - 1) / NT;   // block elements per thread
  constexpr int NCF = SH ? NCOEF_GEN : 4;          // coefficient blocks staged per cell
  constexpr int CPT = (NCF * NQ3 + NT - 1) / NT;  // coefficients per thread
  constexpr int OFF_N = 0;
  constexpr int OFF_NT = OFF_N + ((NQ + 1) / 2) * NP;
  constexpr int OFF_D = OFF_NT + ((NP + 1) / 2) * NQ;
  constexpr int OFF_DT = OFF_D + ((NQ + 1) / 2) * NQ;
  constexpr int OFF_GW = OFF_DT + ((NQ + 1) / 2) * NQ;
  constexpr int OFF_KW = OFF_GW + 3 * NQ;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC *A = reinterpret_cast<TC *>(smem_raw);
  TC *B = A + NQ3 * VT;
  TC *Ycar = B + NQ3 * VT;
  TC *Yfst = Ycar + NP2 * VT;
  TC *Cf = Yfst + NP2 * VT;          // cell coefficients [NCF][NQ3]
  TC *W2 = Cf + NCF * NQ3;           // w_a w_b per line [NQ2]
  TC *T3 = W2 + NQ2;                 // [3][NQ3][VT] gradients (sheared boxes only)

  const int cx = a.cols[2 * col], cy = a.cols[2 * col + 1];
  const int lane0 = tile * VT;
  const int tid = threadIdx.x;
  const TS *__restrict__ X = (const TS *)a.X;
  TS *__restrict__ Y = (TS *)a.Y;
  const TC *tN = a.tab + OFF_N, *tNT = a.tab + OFF_NT, *tD = a.tab + OFF_D, *tDT = a.tab + OFF_DT;
  const TC *tGW = a.tab + OFF_GW, *tKW = a.tab + OFF_KW;
  const int p = a.p;
  const int ax = colour_of(cx, a.N0), by = colour_of(cy, a.N1);
  const int axl = colour_of(cx == 0 ? a.N0 - 1 : cx - 1, a.N0);
  const int axr = colour_of(cx == a.N0 - 1 ? 0 : cx + 1, a.N0);
  const int byl = colour_of(cy == 0 ? a.N1 - 1 : cy - 1, a.N1);
  const int byr = colour_of(cy == a.N1 - 1 ? 0 : cy + 1, a.N1);

  // this thread's block elements e = tid + r NT: the x/y part of the node
  // index, and packed {plane k, lane offset v, in range, read-modify-write}
  int exy[XPT], emeta[XPT];
#pragma unroll
  for (int r = 0; r < XPT; ++r) {
    const int e = tid + r * NT;
    const int v = (e % NV) * LPE, n = e / NV;
    const int i = n % NP, j = (n / NP) % NP;
    // periodic axes wrap; a Dirichlet axis numbers its interior nodes g - 1
    // and has no DoF on its faces (such nodes are gathered as zero and not
    // stored)
    int gx = cx * p + i, gy = cy * p + j;
    bool inb = true;
    if (a.dmask & 1) { gx -= 1; inb = inb && gx >= 0 && gx < a.M0; } else if (gx >= a.M0) gx -= a.M0;
    if (a.dmask & 2) { gy -= 1; inb = inb && gy >= 0 && gy < a.M1; } else if (gy >= a.M1) gy -= a.M1;
    exy[r] = gx + a.M0 * gy;
    const bool xs = (i == 0) || (i == NP - 1), ys = (j == 0) || (j == NP - 1);
    const int axo = (i == 0) ? axl : axr, byo = (j == 0) ? byl : byr;
    const bool rmw = !((!xs || ax < axo) && (!ys || by < byo));
    const bool ok = e < NP3 * NV && lane0 + v < a.nlanes && inb;
    emeta[r] = (n / NP2) | (v << 4) | (ok ? 1 << 12 : 0) | (rmw ? 1 << 13 : 0);
  }
  auto ek = [&](int r) { return emeta[r] & 15; };
  auto elane = [&](int r) { return lane0 + ((emeta[r] >> 4) & 255); };
  auto eok = [&](int r) { return (emeta[r] >> 12) & 1; };
  auto ermw = [&](int r) { return (emeta[r] >> 13) & 1; };
  const int64_t MM = (int64_t)a.M0 * a.M1;
  const int zoff = (a.dmask & 4) ? 1 : 0;
  auto node_of = [&](int r, int cz) -> int64_t {
    int gz = cz * p + ek(r) - zoff;
    if (!zoff && gz >= a.M2) gz -= a.M2;
    return (int64_t)exy[r] + MM * gz;
  };
  // plane k of cell cz holds DoFs (always on a periodic a_2)
  auto zin = [&](int k, int cz) { const int gz = cz * p + k - zoff; return !zoff || (gz >= 0 && gz < a.M2); };

  for (int t = tid; t < NQ2; t += NT) W2[t] = a.wq[t];
  if constexpr (!std::is_void<Core>::value) Core::begin(W2 + NQ2, a);   // read after the first barrier
  // dpre: the node's D^-1 entry (filter steps), applied when the block is
  // staged so that its load stays in flight with the others
  TC xpre[XPT][LPE], dpre[XPT], cpre[CPT], ypre[XPT][LPE];
  auto prefetch = [&](int cz) {
#pragma unroll
    for (int r = 0; r < XPT; ++r) {
#pragma unroll
      for (int jj = 0; jj < LPE; ++jj) xpre[r][jj] = 0;
      dpre[r] = 0;
      if (eok(r) && zin(ek(r), cz)) {
        const int64_t g = node_of(r, cz);
        VecIO<TS, TC, LPE>::ld(X + g * a.ldx + elane(r), xpre[r]);
        if (a.dinv) dpre[r] = (TC)a.dinv[g];
      }
    }
    const TC *src = a.coef + (cx + (int64_t)a.N0 * (cy + (int64_t)a.N1 * cz)) * a.coef_cell;
    const int nst = (a.ncoef < NCF ? a.ncoef : NCF) * NQ3;   // the blocks this instance reads
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + r * NT;
      cpre[r] = e < nst ? src[e] : (TC)0;
    }
  };
  prefetch(0);

  for (int cz = 0; cz < a.N2; ++cz) {
    // stage X^(e) = Q^(e) X -> A[k][j][i][lane] and the coefficients -> Cf
#pragma unroll
    for (int r = 0; r < XPT; ++r) {
      const int e = tid + r * NT;
      if (a.dinv) {
#pragma unroll
        for (int jj = 0; jj < LPE; ++jj) xpre[r][jj] *= dpre[r];
      }
      if (e < NP3 * NV) LdsVec<TC, LPE>::st(A + e * LPE, xpre[r]);
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + r * NT;
      if (e < NCF * NQ3) Cf[e] = cpre[r];
    }
    const int kskip0 = (cz == 0) ? 0 : -1;             // plane held back for the wrap
    const int kskip1 = (cz < a.N2 - 1) ? NP - 1 : -1;  // plane carried to the next cell
    __syncthreads();
    // Y0 = (N x N x N) X^(e): along x and y here (a core does all its sweeps)
    if constexpr (std::is_void<Core>::value) {
      line_pass<NP, NQ, 1, VT, NT>(A, B, tN, NP2, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l * NP; ss = 1; db = l * NQ; ds = 1; });
      __syncthreads();
      line_pass<NP, NQ, 1, VT, NT>(B, A, tN, NP * NQ, [](int l, int &sb, int &ss, int &db, int &ds) {
        const int k = l / NQ, q1 = l % NQ;
        sb = k * NP * NQ + q1; ss = NQ; db = k * NQ2 + q1; ds = NQ; });
      __syncthreads();
    }
    // next cell's block and coefficients, and the values this cell will
    // read-modify-write (stored by earlier phases), in flight from here on
    auto prefetch_next = [&]() {
      if (cz + 1 < a.N2) prefetch(cz + 1);
#pragma unroll
      for (int r = 0; r < XPT; ++r) {
#pragma unroll
        for (int jj = 0; jj < LPE; ++jj) ypre[r][jj] = 0;
        if (eok(r) && ermw(r) && ek(r) != kskip0 && ek(r) != kskip1 && zin(ek(r), cz))
          VecIO<TS, TC, LPE>::ld(Y + node_of(r, cz) * a.ldy + elane(r), ypre[r]);
      }
    };
    // every sweep its own pass: n_q > n_p (the line lengths change between
    // the sweeps), or a sheared box (the off-diagonal metric needs all three
    // gradients at a point, staged in T3 first)
    auto separate_passes = [&](auto offd_tag) {
      constexpr bool OFFD = decltype(offd_tag)::value;
      line_pass<NP, NQ, 1, VT, NT>(A, B, tN, NQ2, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l; ss = NQ2; db = l; ds = NQ2; });
      __syncthreads();
      if constexpr (OFFD) {
        grad_pass<NQ, VT, NT>(B, T3, tD);
        __syncthreads();
      }
      dir_pass<0, NQ, VT, CPLX, TC, OFFD, NT>(B, A, tD, tDT, tGW, tKW, a, Cf, W2, lane0, T3);
      __syncthreads();
      dir_pass<1, NQ, VT, CPLX, TC, OFFD, NT>(B, A, tD, tDT, tGW, tKW, a, Cf, W2, lane0, T3);
      __syncthreads();
      dir_pass<2, NQ, VT, CPLX, TC, OFFD, NT>(B, A, tD, tDT, tGW, tKW, a, Cf, W2, lane0, T3);
      prefetch_next();
      __syncthreads();
      // Y^(e) = (N x N x N)^T Z: along z (A -> B), y (B -> A), x (A -> B)
      line_pass<NQ, NP, 1, VT, NT>(A, B, tNT, NQ2, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l; ss = NQ2; db = l; ds = NQ2; });
      __syncthreads();
      line_pass<NQ, NP, 1, VT, NT>(B, A, tNT, NP * NQ, [](int l, int &sb, int &ss, int &db, int &ds) {
        const int k = l / NQ, q1 = l % NQ;
        sb = k * NQ2 + q1; ss = NQ; db = k * NP * NQ + q1; ds = NQ; });
      __syncthreads();
      line_pass<NQ, NP, 1, VT, NT>(A, B, tNT, NP2, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l * NQ; ss = 1; db = l * NP; ds = 1; });
      __syncthreads();
    };
    if constexpr (!std::is_void<Core>::value) {
      // the seven sweeps of the cell by the core (n_q = n_p, diagonal metric)
      Core::template cell<NP, VT, CPLX>(A, B, Cf, W2, a, lane0, prefetch_next);
    } else if (SH && a.offd) {
      if constexpr (SH) separate_passes(std::true_type{});
    } else if constexpr (NP != NQ) {
      separate_passes(std::false_type{});
    } else {
      // z sweep fused with the z-direction quadrature work: u -> B, z part -> A
      zpass<NQ, VT, CPLX, NT>(A, B, tN, tD, tDT, tGW, tKW, a, Cf, W2, lane0);
      __syncthreads();
      // x-direction quadrature work added into A
      xdir_pass<NQ, VT, CPLX, NT>(B, A, tD, tDT, tGW, tKW, a, Cf, W2, lane0);
      prefetch_next();
      __syncthreads();
      // y-direction work completes the sum; its owner applies N^T along y (-> B)
      ypass<NQ, VT, CPLX, NT>(B, A, tNT, tD, tDT, tGW, tKW, a, Cf, W2, lane0);
      __syncthreads();
      // the rest of Y^(e) = (N x N x N)^T Z: along x (B -> A), then z (A -> B)
      line_pass<NQ, NP, 1, VT, NT>(B, A, tNT, NP * NQ, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l * NQ; ss = 1; db = l * NP; ds = 1; });
      __syncthreads();
      line_pass<NQ, NP, 1, VT, NT>(A, B, tNT, NP2, [](int l, int &sb, int &ss, int &db, int &ds) {
        sb = l; ss = NQ * NP; db = l; ds = NP2; });
      __syncthreads();
    }
    // node planes shared along a_2: plane 0 takes the carry, plane NP-1 is
    // carried (or, in the last cell, takes the column's first plane)
    for (int t = tid; t < NP2 * VT; t += NT) {
      TC *top = B + (NP - 1) * NP2 * VT;
      if (cz == 0) Yfst[t] = B[t];
      else B[t] += Ycar[t];
      if (cz == a.N2 - 1) top[t] += (cz == 0) ? B[t] : Yfst[t];
    }
    __syncthreads();
    if (cz < a.N2 - 1)
      for (int t = tid; t < NP2 * VT; t += NT) Ycar[t] = B[(NP - 1) * NP2 * VT + t];
    // write the completed planes: store (first phase) or read-modify-write
#pragma unroll
    for (int r = 0; r < XPT; ++r) {
      if (!eok(r) || ek(r) == kskip0 || ek(r) == kskip1 || !zin(ek(r), cz)) continue;
      const int e = tid + r * NT;
      const int64_t g = node_of(r, cz);
      TC val[LPE], out[LPE];
      LdsVec<TC, LPE>::ld(B + e * LPE, val);
#pragma unroll
      for (int jj = 0; jj < LPE; ++jj) out[jj] = ermw(r) ? ypre[r][jj] + val[jj] : val[jj];
      VecIO<TS, TC, LPE>::st(Y + g * a.ldy + elane(r), out);
    }
    __syncthreads();
  }
}

// XCD-aware placement: block b runs on XCD b % 8; each XCD gets a contiguous
// range of work items so the tiles of one column share an L2.  'grid' must be
// a multiple of 8.
__device__ __forceinline__ int xcd_item(int b, int grid) { return (b & 7) * (grid >> 3) + (b >> 3); }

// Register budget: at most 128 VGPRs (4 waves per SIMD), so that two FP64
// blocks of 7 waves, or one FP32/BF16 block of up to 16 waves, are resident
// per CU.  FP64 kernels of degree 7 and up (or with 8 and more quadrature
// points per direction) hold more live values in the line passes than 128
// registers: they get 256 (2 waves per SIMD) rather than spilling to scratch
// (measured per H X: complex p = 7, 24^3 cells, 512 vectors 90 -> 61 ms;
// real p = 8, 12^3 cells, 256 vectors 7.5 -> 3.7 ms).
template <int NP, int NQ, typename TC> struct LocalWaves {
  static constexpr int value = std::is_same<TC, double>::value && (NP >= 7 || NQ >= 8) ? 2 : 4;
};
#define FEHX_LOCAL_BOUNDS __launch_bounds__((Threads<NQ, VT, TC, Core>::value)) __attribute__((amdgpu_waves_per_eu(LocalWaves<NP, NQ, TC>::value)))

// One system, one colour phase: one block per (column, tile).
template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC, int LPE, bool SH, class Core = void>
__global__ void FEHX_LOCAL_BOUNDS k_local(KArgs<TC> a) {
  const int w = xcd_item(blockIdx.x, gridDim.x);
  if (w >= a.ncols * a.ntiles) return;
  const int col = w / a.ntiles;
  local_column<NP, NQ, VT, CPLX, TS, TC, LPE, SH, Core>(a, col, w - col * a.ntiles);
}

// Several systems of one class (n_p, n_q, precision, real/complex), one colour
// phase each, in one persistent launch: the blocks stride over the
// concatenated work lists (system s owns items [off[s], off[s+1])).
constexpr int LOCAL_MAXB = 8;
template <typename TC> struct BatchArgs {
  int nsys, total;
  int off[LOCAL_MAXB + 1];
  KArgs<TC> sys[LOCAL_MAXB];
};

template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC, int LPE, bool SH, class Core = void>
__global__ void FEHX_LOCAL_BOUNDS k_local_batch(BatchArgs<TC> B) {
  for (int base = 0; base < B.total; base += gridDim.x) {
    const int w = base + xcd_item(blockIdx.x, gridDim.x);
    if (w >= B.total) return;
    int sidx = 0;
    while (sidx + 1 < B.nsys && w >= B.off[sidx + 1]) ++sidx;
    const KArgs<TC> &a = B.sys[sidx];
    const int lw = w - B.off[sidx];
    const int col = lw / a.ntiles;
    local_column<NP, NQ, VT, CPLX, TS, TC, LPE, SH, Core>(a, col, lw - col * a.ntiles);
  }
}

// ---- host-side dispatch (templates; instantiated per precision) -------------

template <typename TC> KArgs<TC> make_args(Mesh *m, const LocalLaunch &L, int vt) {
  KArgs<TC> a{};
  a.X = L.X; a.Y = L.Y; a.ldx = L.ldx; a.ldy = L.ldy; a.nlanes = L.nlanes;
  a.N0 = m->N[0]; a.N1 = m->N[1]; a.N2 = m->N[2];
  a.M0 = m->Mn[0]; a.M1 = m->Mn[1]; a.M2 = m->Mn[2]; a.p = m->p;
  a.dmask = (m->desc.periodic[0] ? 0 : 1) | (m->desc.periodic[1] ? 0 : 2) | (m->desc.periodic[2] ? 0 : 4);
  a.offd = (m->offd && !L.mass) ? 1 : 0;
  const bool f64 = std::is_same<TC, double>::value;
  a.tab = f64 ? (const TC *)m->tab64 : (const TC *)m->tab32;
  a.wq = f64 ? (const TC *)m->wq64 : (const TC *)m->wq32;
  a.coef = f64 ? (const TC *)m->coef64 : (const TC *)m->coef32;
  a.coef_cell = (int64_t)m->ncoef * m->nq * m->nq * m->nq;
  a.ncoef = m->ncoef;
  a.gga = m->has_gga ? 1 : 0;
  if (L.mass) {
    a.tab = f64 ? (const TC *)m->tabM64 : (const TC *)m->tabM32;
    a.coef = f64 ? (const TC *)m->coefM64 : (const TC *)m->coefM32;
    a.coef_cell = m->coefM_cell;
    a.gga = 0;
  }
  a.dinv = L.dinv_gather;
  a.mxtab = m->tabmx;
  a.ntiles = (L.nlanes + vt - 1) / vt;
  return a;
}

// LDS per workgroup on gfx950; tiles whose block cannot fit are not instantiated
constexpr size_t LDS_MAX = 160 * 1024;
template <int NP, int NQ> constexpr size_t lds_need(int vt, int bytes, bool offd = false) {
  return ((size_t)(2 * NQ * NQ * NQ + 2 * NP * NP) * vt + (offd ? NCOEF_GEN : 4) * NQ * NQ * NQ + NQ * NQ +
          (offd ? (size_t)3 * NQ * NQ * NQ * vt : 0)) * bytes;
}

// LDS of one block as launched: the line-gather path holds no staged carry
// planes
template <int NP, int NQ, typename TC, class Core, bool CPLX>
constexpr size_t lds_local(int vt, int bytes, bool offd) {
  return (LinesPath<NP, NQ, TC, Core, CPLX>::value && !offd)
             ? ((size_t)2 * NQ * NQ * NQ * vt + 4 * NQ * NQ * NQ + NQ * NQ) * bytes
             : lds_need<NP, NQ>(vt, bytes, offd);
}

inline int device_cus(int dev) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  return n;
}

// Single system: one launch per colour phase, one block per (column, tile).
// Batch (several systems of one class, or persistent=true): one persistent
// launch per colour phase over the concatenated work lists of up to
// LOCAL_MAXB systems, grid = the resident block count (rounded to 8 XCDs).
inline int max_lds(Mesh *m) {
  int maxshm = 65536;
  (void)hipDeviceGetAttribute(&maxshm, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
  return maxshm;
}

template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC, int LPE, bool SH, class Core = void>
inline fe_status run_local_lpe(const LocalBatch &Bt, hipStream_t s) {
  // sheared boxes add the three staged gradients to the LDS block; a launch
  // above 64 KiB raises the kernel's dynamic-LDS attribute to its size first
  bool offd = false;
  for (int i = 0; i < Bt.n; ++i) offd = offd || (Bt.ms[i]->offd && !Bt.Ls[i].mass);
  const size_t shm = lds_local<NP, NQ, TC, Core, CPLX>(VT, sizeof(TC), offd) + CoreLds<Core>::elems * sizeof(TC);
  constexpr int NTB = Threads<NQ, VT, TC, Core>::value;
  if (Bt.n == 1 && !Bt.persistent) {
    Mesh *m = Bt.ms[0];
    const LocalLaunch &L = Bt.Ls[0];
    KArgs<TC> a = make_args<TC>(m, L, VT);
    auto kern = k_local<NP, NQ, VT, CPLX, TS, TC, LPE, SH, Core>;
    static size_t attr_set = 65536;
    if (shm > attr_set) {
      FE_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
      attr_set = shm;
    }
    for (int ph = 0; ph < m->nphase; ++ph) {
      a.cols = m->cols + 2 * m->phase_off[ph];
      a.ncols = m->phase_off[ph + 1] - m->phase_off[ph];
      if (a.ncols == 0) continue;
      const int W = a.ncols * a.ntiles;
      const int nb = ((W + 7) / 8) * 8;
      hipLaunchKernelGGL(kern, dim3(nb), dim3(NTB), shm, s, a);
      FE_HIP_TRY(hipGetLastError());
    }
    return FE_OK;
  }
  auto kern = k_local_batch<NP, NQ, VT, CPLX, TS, TC, LPE, SH, Core>;
  static size_t battr_set = 65536;
  static int resident[2] = {0, 0};   // resident blocks without / with the staged gradients
  if (shm > battr_set) {
    FE_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    battr_set = shm;
  }
  if (!resident[offd]) {
    int per_cu = 0;
    FE_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, NTB, shm));
    resident[offd] = (per_cu > 0 ? per_cu : 1) * device_cus(Bt.ms[0]->device);
  }
  const int cap = Bt.blocks_per_cu > 0 ? Bt.blocks_per_cu * device_cus(Bt.ms[0]->device) : resident[offd];
  int nphase = 0;
  for (int i = 0; i < Bt.n; ++i) nphase = nphase > Bt.ms[i]->nphase ? nphase : Bt.ms[i]->nphase;
  for (int ph = 0; ph < nphase; ++ph) {
    for (int i0 = 0; i0 < Bt.n;) {
      BatchArgs<TC> B{};
      B.nsys = 0;
      B.off[0] = 0;
      for (; i0 < Bt.n && B.nsys < LOCAL_MAXB; ++i0) {
        Mesh *m = Bt.ms[i0];
        if (ph >= m->nphase) continue;
        const int ncols = m->phase_off[ph + 1] - m->phase_off[ph];
        if (ncols == 0) continue;
        KArgs<TC> a = make_args<TC>(m, Bt.Ls[i0], VT);
        a.cols = m->cols + 2 * m->phase_off[ph];
        a.ncols = ncols;
        B.sys[B.nsys] = a;
        B.off[B.nsys + 1] = B.off[B.nsys] + ncols * a.ntiles;
        ++B.nsys;
      }
      if (B.nsys == 0) continue;
      B.total = B.off[B.nsys];
      int grid = B.total < cap ? B.total : cap;
      grid = ((grid + 7) / 8) * 8;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(NTB), shm, s, B);
      FE_HIP_TRY(hipGetLastError());
    }
  }
  return FE_OK;
}

// The wide (16-byte) element form when every block of every system allows it.
inline bool wide_ok(const LocalBatch &Bt, int lpe, size_t ts) {
  const uintptr_t al = (uintptr_t)lpe * ts;
  auto ok_block = [&](const void *p, int64_t ld) { return p == nullptr || ((uintptr_t)p % al == 0 && ld % lpe == 0); };
  for (int i = 0; i < Bt.n; ++i) {
    const LocalLaunch &L = Bt.Ls[i];
    if (L.nlanes % lpe != 0 || !ok_block(L.X, L.ldx) || !ok_block(L.Y, L.ldy)) return false;
  }
  return true;
}

template <int NP, int NQ, int VT, bool CPLX, typename TS, typename TC, bool SH = false, class Core = void>
inline fe_status run_local(const LocalBatch &Bt, hipStream_t s) {
  constexpr int W = WideLanes<TS>::value;
  // the line-gather path moves single lanes: one instance serves every block
  constexpr bool lines_only = LinesPath<NP, NQ, TC, Core, CPLX>::value && !SH;
  if constexpr (!lines_only)
    if (VT % W == 0 && wide_ok(Bt, W, sizeof(TS))) return run_local_lpe<NP, NQ, VT, CPLX, TS, TC, W, SH, Core>(Bt, s);
  return run_local_lpe<NP, NQ, VT, CPLX, TS, TC, 1, SH, Core>(Bt, s);
}


// Vector tile per precision: the caller's (the autotuner's) choice when it is
// set and fits, else the widest default whose LDS fits.
template <int NP, int NQ, bool CPLX>
fe_status pick_vt_f64(const LocalBatch &B, hipStream_t s) {
  const size_t mx = (size_t)max_lds(B.ms[0]);
  bool od = false;   // any system of a sheared box: the staged gradients must fit too
  for (int i = 0; i < B.n; ++i) od = od || (B.ms[i]->offd && !B.Ls[i].mass);
  int vt = B.Ls[0].vt ? B.Ls[0].vt
                      : (lds_need<NP, NQ>(8, 8, od) <= mx ? 8 : (lds_need<NP, NQ>(4, 8, od) <= mx ? 4 : 2));
  if constexpr (lds_need<NP, NQ>(16, 8) <= LDS_MAX)
    if (vt == 16 && lds_need<NP, NQ>(16, 8, od) <= mx)
      return od ? run_local<NP, NQ, 16, CPLX, double, double, true>(B, s) : run_local<NP, NQ, 16, CPLX, double, double>(B, s);
  // ten lanes: 7^2 lines x 10 lanes fill 490 of a 512-thread block at n_p = 7
  if constexpr (NP == NQ && lds_need<NP, NQ>(10, 8) <= LDS_MAX)
    if (vt == 10 && lds_need<NP, NQ>(10, 8, od) <= mx)
      return od ? run_local<NP, NQ, 10, CPLX, double, double, true>(B, s) : run_local<NP, NQ, 10, CPLX, double, double>(B, s);
  if constexpr (lds_need<NP, NQ>(8, 8) <= LDS_MAX)
    if (vt == 8 && lds_need<NP, NQ>(8, 8, od) <= mx)
      return od ? run_local<NP, NQ, 8, CPLX, double, double, true>(B, s) : run_local<NP, NQ, 8, CPLX, double, double>(B, s);
  if constexpr (lds_need<NP, NQ>(4, 8) <= LDS_MAX)
    if (vt == 4 && lds_need<NP, NQ>(4, 8, od) <= mx)
      return od ? run_local<NP, NQ, 4, CPLX, double, double, true>(B, s) : run_local<NP, NQ, 4, CPLX, double, double>(B, s);
  // two lanes (one complex vector): only where four do not fit (n_q = 12)
  if constexpr (lds_need<NP, NQ>(4, 8) > LDS_MAX && lds_need<NP, NQ>(2, 8) <= LDS_MAX)
    if (vt == 2 && lds_need<NP, NQ>(2, 8, od) <= mx)
      return od ? run_local<NP, NQ, 2, CPLX, double, double, true>(B, s) : run_local<NP, NQ, 2, CPLX, double, double>(B, s);
  return set_error(FE_EUNSUPPORTED, "no FP64 local-operator variant for this vector tile / LDS size");
}
template <int NP, int NQ, bool CPLX>
fe_status pick_vt_f32(const LocalBatch &B, hipStream_t s) {
  const size_t mx = (size_t)max_lds(B.ms[0]);
  bool od = false;   // any system of a sheared box: the staged gradients must fit too
  for (int i = 0; i < B.n; ++i) od = od || (B.ms[i]->offd && !B.Ls[i].mass);
  int vt = B.Ls[0].vt ? B.Ls[0].vt : (lds_need<NP, NQ>(16, 4, od) <= mx ? 16 : 8);
  if constexpr (lds_need<NP, NQ>(32, 4) <= LDS_MAX)
    if (vt == 32 && lds_need<NP, NQ>(32, 4, od) <= mx)
      return od ? run_local<NP, NQ, 32, CPLX, float, float, true>(B, s) : run_local<NP, NQ, 32, CPLX, float, float>(B, s);
  if constexpr (lds_need<NP, NQ>(16, 4) <= LDS_MAX)
    if (vt == 16 && lds_need<NP, NQ>(16, 4, od) <= mx)
      return od ? run_local<NP, NQ, 16, CPLX, float, float, true>(B, s) : run_local<NP, NQ, 16, CPLX, float, float>(B, s);
  if constexpr (lds_need<NP, NQ>(8, 4) <= LDS_MAX)
    if (vt == 8 && lds_need<NP, NQ>(8, 4, od) <= mx)
      return od ? run_local<NP, NQ, 8, CPLX, float, float, true>(B, s) : run_local<NP, NQ, 8, CPLX, float, float>(B, s);
  return set_error(FE_EUNSUPPORTED, "no FP32 local-operator variant for this vector tile / LDS size");
}
template <int NP, int NQ, bool CPLX>
fe_status pick_vt_bf16(const LocalBatch &B, hipStream_t s) {
  const size_t mx = (size_t)max_lds(B.ms[0]);
  bool od = false;   // any system of a sheared box: the staged gradients must fit too
  for (int i = 0; i < B.n; ++i) od = od || (B.ms[i]->offd && !B.Ls[i].mass);
  int vt = B.Ls[0].vt ? B.Ls[0].vt : (lds_need<NP, NQ>(32, 4, od) <= mx ? 32 : (lds_need<NP, NQ>(16, 4, od) <= mx ? 16 : 8));
  if constexpr (lds_need<NP, NQ>(32, 4) <= LDS_MAX)
    if (vt == 32 && lds_need<NP, NQ>(32, 4, od) <= mx)
      return od ? run_local<NP, NQ, 32, CPLX, bf16s, float, true>(B, s) : run_local<NP, NQ, 32, CPLX, bf16s, float>(B, s);
  if constexpr (lds_need<NP, NQ>(16, 4) <= LDS_MAX)
    if (vt == 16 && lds_need<NP, NQ>(16, 4, od) <= mx)
      return od ? run_local<NP, NQ, 16, CPLX, bf16s, float, true>(B, s) : run_local<NP, NQ, 16, CPLX, bf16s, float>(B, s);
  if constexpr (lds_need<NP, NQ>(8, 4) <= LDS_MAX)
    if (vt == 8 && lds_need<NP, NQ>(8, 4, od) <= mx)
      return od ? run_local<NP, NQ, 8, CPLX, bf16s, float, true>(B, s) : run_local<NP, NQ, 8, CPLX, bf16s, float>(B, s);
  return set_error(FE_EUNSUPPORTED, "no BF16 local-operator variant for this vector tile / LDS size");
}
template <int NP, int NQ> fe_status pick_cplx_f64(const LocalBatch &B, hipStream_t s) {
  return B.ms[0]->cplx ? pick_vt_f64<NP, NQ, true>(B, s) : pick_vt_f64<NP, NQ, false>(B, s);
}
template <int NP, int NQ> fe_status pick_cplx_f32(const LocalBatch &B, hipStream_t s) {
  return B.ms[0]->cplx ? pick_vt_f32<NP, NQ, true>(B, s) : pick_vt_f32<NP, NQ, false>(B, s);
}
template <int NP, int NQ> fe_status pick_cplx_bf16(const LocalBatch &B, hipStream_t s) {
  return B.ms[0]->cplx ? pick_vt_bf16<NP, NQ, true>(B, s) : pick_vt_bf16<NP, NQ, false>(B, s);
}

}  // namespace fehx
static_assert(sizeof(fehx::BatchArgs<double>) <= 4096, "batched kernel arguments exceed the 4 KB kernarg limit");
