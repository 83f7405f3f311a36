// The sweeps of one cell on the matrix cores (MFMA), for FE_BF16 requests:
// BF16 operands with FP32 accumulation, each FP32 value and each 1D matrix
// entry carried as a pair of BF16 numbers (hi + lo), so a contraction keeps
// about 17 significant bits instead of BF16's 8.
//
// Each 1D contraction of Alg. 2 (N, Dtilde and their transposes along one
// reference direction, n_q = n_p <= 8) is a 16 x 16 x 16 MFMA
// (v_mfma_f32_16x16x16_bf16) over 16 vector lanes of two lines at once: the
// 16 x 16 operand A holds the 1D matrix twice on its block diagonal (rows and
// columns 0..7 for the first line, 8..15 for the second), B holds the two
// lines' points (k = point along the line, column = vector lane).  With
// x = x_hi + x_lo and M = M_hi + M_lo the product is
//   M x ~ M_hi x_hi + M_hi x_lo + M_lo x_hi        (three MFMAs, FP32 sums),
// the dropped M_lo x_lo and the split residue being ~2^-17 relative.
//
// Register layout of v_mfma_f32_16x16x16_bf16 (lane l, g = l / 16, n = l % 16):
//   A: row n, columns 4g .. 4g + 3;   B: rows 4g .. 4g + 3, column n;
//   C: rows 4g .. 4g + 3, column n.
// B and C share their mapping, so a contraction's output is the next
// contraction's input along the same line without leaving the registers:
// the quadrature-point stage of a direction (gradient Dtilde u, fluxes,
// transposed gradient) runs in registers on one pair of lines.  Lane l holds
// points 4 (g % 2) .. + 3 of line g / 2 of the pair for vector lane n.
//
// The cell is swept in the same seven LDS passes as the vector-ALU kernel
// (N along x, N along y, [N along z + the z-direction stage], the
// x-direction stage, [the y-direction stage + N^T along y], N^T along x,
// N^T along z), on the same [point][lane] LDS blocks in FP32.
#pragma once
#include "k_local_impl.h"

namespace fehx {

typedef short mx_s4 __attribute__((ext_vector_type(4)));
typedef float mx_f4 __attribute__((ext_vector_type(4)));

// bfloat16 bits of x, round to nearest even (finite x)
__device__ __forceinline__ uint32_t mx_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// x ~ hi + lo (both BF16, round to nearest even)
__device__ __forceinline__ void mx_split(const float (&x)[4], mx_s4 &hi, mx_s4 &lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t h = mx_bf16(x[j]);
    hi[j] = (short)h;
    lo[j] = (short)mx_bf16(x[j] - __uint_as_float(h << 16));
  }
}

struct MxMat {
  mx_s4 hi, lo;
};

// This lane's part of the block-diagonal operand A of a matrix M[8][8]
// (row = output point, column = input point, zero padded):
// A[r][c] = M[r % 8][c % 8] when r / 8 == c / 8, else 0.
__device__ __forceinline__ MxMat mx_operand(const float *__restrict__ M) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  MxMat a;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * g + j;
    const float v = ((r >> 3) == (c >> 3)) ? M[(r & 7) * 8 + (c & 7)] : 0.0f;
    const uint32_t h = mx_bf16(v);
    a.hi[j] = (short)h;
    a.lo[j] = (short)mx_bf16(v - __uint_as_float(h << 16));
  }
  return a;
}

// y = M x for this pair of lines (x in B layout, y in C layout)
__device__ __forceinline__ void mx_apply(const MxMat &M, const float (&x)[4], float (&y)[4]) {
  mx_s4 hi, lo;
  mx_split(x, hi, lo);
  mx_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(M.hi, hi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(M.hi, lo, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(M.lo, hi, acc, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = acc[j];
}

// Line geometry of the passes: line l of direction D through the other two
// coordinates; point i of the line sits at base + i * stride.
template <int D, int NQ> __device__ __forceinline__ void mx_line(int l, int &base, int &stride) {
  constexpr int NQ2 = NQ * NQ;
  if (D == 0) { base = l * NQ; stride = 1; }
  else if (D == 1) { base = (l / NQ) * NQ2 + (l % NQ); stride = NQ; }
  else { base = l; stride = NQ2; }
}

// offsets of the per-direction point factors g_DD w_i det J and
// kappa_D w_i det J in the packed table (see tab_layout), n_p = n_q
template <int NQ> constexpr int mx_gw_off() { return 4 * ((NQ + 1) / 2) * NQ; }
template <int NQ> constexpr int mx_kw_off() { return mx_gw_off<NQ>() + 3 * NQ; }

// a wave-uniform table pointer, made scalar (the batched kernel may hold the
// kernel arguments in vector registers)
__device__ __forceinline__ cptr<float> mx_uniform(const float *p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return reinterpret_cast<cptr<float>>(((uint64_t)hi << 32) | lo);
}

// g[k0 + j] for a lane whose first point is k0 (0 or 4), g a wave-uniform
// table of NQ entries read with scalar loads
template <int NQ> __device__ __forceinline__ float mx_pick(cptr<float> g, int k0, int j) {
  const float lo = g[j];
  const float hi = (j + 4 < NQ) ? g[j + 4 < NQ ? j + 4 : 0] : 0.0f;
  return k0 ? hi : lo;
}

template <int NQ, int VT, int NT, bool CPLX> struct MxCell {
  static constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ, TV = VT / 16, NW = NT / 64;
  static constexpr int NPAIR = (NQ2 + 1) / 2;

  // the lane's slot: pair p, column tile ct -> line, first point, vector lane
  struct Slot {
    int line, k0, v;
    bool ok;
  };
  static __device__ __forceinline__ Slot slot(int item) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const int pr = item / TV, ct = item - pr * TV;
    Slot s;
    s.line = 2 * pr + (g >> 1);
    s.k0 = (g & 1) * 4;
    s.v = ct * 16 + (lane & 15);
    s.ok = s.line < NQ2;
    if (!s.ok) s.line = 0;
    return s;
  }

  template <int D>
  static __device__ __forceinline__ void load(const float *__restrict__ src, const Slot &s, float (&x)[4]) {
    int base, stride;
    mx_line<D, NQ>(s.line, base, stride);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = s.k0 + j;
      x[j] = (s.ok && k < NQ) ? src[(base + k * stride) * VT + s.v] : 0.0f;
    }
  }
  template <int D>
  static __device__ __forceinline__ void store(float *__restrict__ dst, const Slot &s, const float (&y)[4]) {
    int base, stride;
    mx_line<D, NQ>(s.line, base, stride);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = s.k0 + j;
      if (s.ok && k < NQ) dst[(base + k * stride) * VT + s.v] = y[j];
    }
  }
  template <int D>
  static __device__ __forceinline__ void add(const float *__restrict__ src, const Slot &s, float (&y)[4]) {
    int base, stride;
    mx_line<D, NQ>(s.line, base, stride);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = s.k0 + j;
      if (s.ok && k < NQ) y[j] += src[(base + k * stride) * VT + s.v];
    }
  }

  // the quadrature-point work of direction D on the pair's lines (eqn refact):
  //   T = Dtilde u,  F = G_DD w T + Vtilde^G_D u,
  //   o = Dtilde^T F + Vtilde^G_D T [+ (V + |k|^2/2) w u for D = 0] [- i kappa_D w T]
  template <int D>
  static __device__ __forceinline__ void stage(const float (&u)[4], float (&o)[4], const Slot &s, const MxMat &Dm,
                                               const MxMat &DTm, const KArgs<float> &a, const float *__restrict__ C,
                                               const float *__restrict__ W2, int lane0) {
    int base, stride;
    mx_line<D, NQ>(s.line, base, stride);
    float T[4], F[4], z[4];
    mx_apply(Dm, u, T);
    const float w2 = W2[s.line];
    cptr<float> gw = mx_uniform(a.tab + mx_gw_off<NQ>() + D * NQ);
    cptr<float> kw = mx_uniform(a.tab + mx_kw_off<NQ>() + D * NQ);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = s.k0 + j;
      const bool in = s.ok && k < NQ;
      const int kk = in ? k : 0;
      const int Q = base + kk * stride;
      F[j] = (w2 * mx_pick<NQ>(gw, s.k0, j)) * T[j];
      z[j] = 0.0f;
      if (a.gga) {
        const float vg = C[(1 + D) * NQ3 + Q];
        F[j] = fmaf(vg, u[j], F[j]);
        z[j] = vg * T[j];
      }
      if (D == 0) z[j] = fmaf(C[Q], u[j], z[j]);
      if constexpr (CPLX) {
        // -i kappa w T: the real lane gets +kappa w T_im, the imaginary lane -kappa w T_re
        const float tp = swap_pair(T[j]);
        const float kwv = w2 * mx_pick<NQ>(kw, s.k0, j);
        z[j] = fmaf((lane & 1) ? -kwv : kwv, tp, z[j]);
      }
      if (!in) F[j] = 0.0f;
    }
    mx_apply(DTm, F, o);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] += z[j];
  }

  // the seven sweeps of one cell: X^(e) in A on entry, Y^(e) in B on exit
  template <int NP, typename Pre>
  static __device__ __forceinline__ void run(float *__restrict__ A, float *__restrict__ B, const float *__restrict__ C,
                                             const float *__restrict__ W2, const KArgs<float> &a, int lane0,
                                             Pre &&prefetch_next) {
    static_assert(NP == NQ && NQ <= 8, "the MFMA cell core needs n_q = n_p <= 8");
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform item loops
    const MxMat Nm = mx_operand(a.mxtab), NTm = mx_operand(a.mxtab + 64);
    const MxMat Dm = mx_operand(a.mxtab + 128), DTm = mx_operand(a.mxtab + 192);
    constexpr int ITEMS = NPAIR * TV;
    // N along x (A -> B), N along y (B -> A)
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float x[4], y[4];
      load<0>(A, s, x);
      mx_apply(Nm, x, y);
      store<0>(B, s, y);
    }
    __syncthreads();
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float x[4], y[4];
      load<1>(B, s, x);
      mx_apply(Nm, x, y);
      store<1>(A, s, y);
    }
    __syncthreads();
    // z-lines: u = N_z (A) -> B; the z-direction stage -> A
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float x[4], u[4], o[4];
      load<2>(A, s, x);
      mx_apply(Nm, x, u);
      store<2>(B, s, u);
      stage<2>(u, o, s, Dm, DTm, a, C, W2, lane0);
      store<2>(A, s, o);
    }
    __syncthreads();
    // x-lines of u: the x-direction stage added into A
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float u[4], o[4];
      load<0>(B, s, u);
      stage<0>(u, o, s, Dm, DTm, a, C, W2, lane0);
      add<0>(A, s, o);
      store<0>(A, s, o);
    }
    prefetch_next();
    __syncthreads();
    // y-lines: the y-direction stage completes the sum; N^T along y -> B
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float u[4], o[4], y[4];
      load<1>(B, s, u);
      stage<1>(u, o, s, Dm, DTm, a, C, W2, lane0);
      add<1>(A, s, o);
      mx_apply(NTm, o, y);
      store<1>(B, s, y);
    }
    __syncthreads();
    // N^T along x (B -> A), then along z (A -> B)
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float x[4], y[4];
      load<0>(B, s, x);
      mx_apply(NTm, x, y);
      store<0>(A, s, y);
    }
    __syncthreads();
    for (int it = wave; it < ITEMS; it += NW) {
      const Slot s = slot(it);
      float x[4], y[4];
      load<2>(A, s, x);
      mx_apply(NTm, x, y);
      store<2>(B, s, y);
    }
    __syncthreads();
  }
};

// The core hook of local_column: NT threads per block.
template <int NT> struct MxCore {
  static constexpr int threads = NT;
  template <int NP, int VT, bool CPLX, typename TC, typename Pre>
  static __device__ __forceinline__ void cell(TC *A, TC *B, const TC *C, const TC *W2, const KArgs<TC> &a, int lane0,
                                              Pre &&prefetch_next) {
    static_assert(std::is_same<TC, float>::value, "the MFMA core computes in float");
    MxCell<NP, VT, NT, CPLX>::template run<NP>(A, B, C, W2, a, lane0, prefetch_next);
  }
};

}  // namespace fehx
