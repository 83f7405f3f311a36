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

// x ~ hi + lo, both BF16 rounded to nearest even (gfx950 converts a pair of
// floats to packed BF16 in one instruction)
__device__ __forceinline__ void mx_split1(float x, short &hi, short &lo) {
  const __bf16 h = (__bf16)x;
  hi = __builtin_bit_cast(short, h);
  lo = __builtin_bit_cast(short, (__bf16)(x - (float)h));
}
__device__ __forceinline__ void mx_split(const float (&x)[4], mx_s4 &hi, mx_s4 &lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    short h, l;
    mx_split1(x[j], h, l);
    hi[j] = h;
    lo[j] = l;
  }
}

struct MxMat {
  mx_s4 hi, lo;
};

// Lane 'lane''s part of the block-diagonal operand A of a matrix M[8][8]
// (row = output point, column = input point, zero padded):
// A[r][c] = M[r % 8][c % 8] when r / 8 == c / 8, else 0.
__device__ __forceinline__ MxMat mx_operand(const float *__restrict__ M, int lane) {
  const int r = lane & 15, g = lane >> 4;
  MxMat a;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * g + j;
    const float v = ((r >> 3) == (c >> 3)) ? M[(r & 7) * 8 + (c & 7)] : 0.0f;
    short h, l;
    mx_split1(v, h, l);
    a.hi[j] = h;
    a.lo[j] = l;
  }
  return a;
}

// The operands of the four 1D matrices (N, N^T, Dtilde, Dtilde^T), formed
// once per work item into LDS (frag[matrix][lane] = hi.xy, lo.xy) and read
// back by each pass: short live ranges without a global round trip per pass.
constexpr int MX_FRAG_ELEMS = 4 * 64 * 4;
__device__ __forceinline__ uint32_t mx_pack(short a, short b) {
  return (uint32_t)(uint16_t)a | ((uint32_t)(uint16_t)b << 16);
}
// the fragments' place after the masked-store slot, aligned for 16-byte reads
__device__ __forceinline__ uint32_t *mx_frag_at(float *tail) {
  return reinterpret_cast<uint32_t *>((reinterpret_cast<uintptr_t>(tail + 16) + 15) & ~(uintptr_t)15);
}
__device__ __forceinline__ void mx_frag_store(uint32_t *__restrict__ frag, const float *__restrict__ tab) {
  for (int t = threadIdx.x; t < 4 * 64; t += blockDim.x) {
    const MxMat a = mx_operand(tab + (t >> 6) * 64, t & 63);
    uint32_t *p = frag + 4 * t;
    p[0] = mx_pack(a.hi[0], a.hi[1]);
    p[1] = mx_pack(a.hi[2], a.hi[3]);
    p[2] = mx_pack(a.lo[0], a.lo[1]);
    p[3] = mx_pack(a.lo[2], a.lo[3]);
  }
}
__device__ __forceinline__ MxMat mx_frag(const uint32_t *__restrict__ frag, int mat) {
  const uint4 v = *(const uint4 *)(frag + 4 * (mat * 64 + (threadIdx.x & 63)));
  MxMat a;
  a.hi[0] = (short)(v.x & 0xffffu); a.hi[1] = (short)(v.x >> 16);
  a.hi[2] = (short)(v.y & 0xffffu); a.hi[3] = (short)(v.y >> 16);
  a.lo[0] = (short)(v.z & 0xffffu); a.lo[1] = (short)(v.z >> 16);
  a.lo[2] = (short)(v.w & 0xffffu); a.lo[3] = (short)(v.w >> 16);
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
  static constexpr int NPAIR = (NQ2 + 1) / 2, ITEMS = NPAIR * TV;
  static constexpr int U = 2;                  // items in flight per wave

  // An item is (pair of lines, column tile); the lane's part of it: its
  // line, first point k0 (0 or 4), vector lane v, and per point j whether
  // it exists (bit j of 'valid').  Invalid points read a clamped address and
  // use zero, and store into the trash slot, so no access is predicated.
  struct Slot {
    int line, k0, v, valid;
  };
  static __device__ __forceinline__ Slot slot(int item) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const int pr = item / TV, ct = item - pr * TV;
    Slot s;
    s.line = 2 * pr + (g >> 1);
    s.k0 = (g & 1) * 4;
    s.v = ct * 16 + (lane & 15);
    const bool ok = item < ITEMS && s.line < NQ2;
    s.valid = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s.valid |= (ok && s.k0 + j < NQ) ? 1 << j : 0;
    if (!ok) s.line = 0;
    return s;
  }
  // element offsets of the lane's four points (invalid: point 0 for loads)
  template <int D>
  static __device__ __forceinline__ void offsets(const Slot &s, int (&o)[4]) {
    int base, stride;
    mx_line<D, NQ>(s.line, base, stride);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = s.k0 + j < NQ ? s.k0 + j : NQ - 1;
      o[j] = (base + k * stride) * VT + s.v;
    }
  }
  static __device__ __forceinline__ void load(const float *__restrict__ src, const Slot &s, const int (&o)[4],
                                              float (&x)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = src[o[j]];
      x[j] = (s.valid >> j & 1) ? v : 0.0f;
    }
  }
  // dst[o] = y for the valid points; the others go to the trash slot of A
  static __device__ __forceinline__ void store(float *__restrict__ dst, float *__restrict__ trash, const Slot &s,
                                               const int (&o)[4], const float (&y)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float *p = (s.valid >> j & 1) ? dst + o[j] : trash + (threadIdx.x & 15);
      *p = y[j];
    }
  }

  // the quadrature-point work of direction D on the pair's lines (eqn refact):
  //   T = Dtilde u,  F = G_DD w T + Vtilde^G_D u,
  //   o = Dtilde^T F + Vtilde^G_D T [+ (V + |k|^2/2) w u for D = 0] [- i kappa_D w T]
  template <int D>
  static __device__ __forceinline__ void stage(const float (&u)[4], float (&o)[4], const Slot &s, const MxMat &Dm,
                                               const MxMat &DTm, const KArgs<float> &a, const float *__restrict__ C,
                                               const float *__restrict__ W2) {
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
      const int k = s.k0 + j < NQ ? s.k0 + j : NQ - 1;
      const int Q = base + k * stride;
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
      if (!(s.valid >> j & 1)) F[j] = 0.0f;
    }
    mx_apply(DTm, F, o);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] += z[j];
  }

  // one pass over the items, U per wave at a time: body(slot, u) for each
  template <typename Body>
  static __device__ __forceinline__ void items(int wave, Body &&body) {
    for (int it0 = wave; it0 < ITEMS; it0 += NW * U) {
      Slot s[U];
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] = slot(it0 + u * NW);
      body(s);
    }
  }

  // the seven sweeps of one cell: X^(e) in A on entry, Y^(e) in B on exit
  template <int NP, typename Pre>
  static __device__ __forceinline__ void run(float *__restrict__ A, float *__restrict__ B, const float *__restrict__ C,
                                             const float *__restrict__ W2, const KArgs<float> &a, int lane0,
                                             Pre &&prefetch_next) {
    static_assert(NP == NQ && NQ <= 8, "the MFMA cell core needs n_q = n_p <= 8");
    (void)lane0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform item loops
    // masked stores land in the slot after the line weights (the LDS tail),
    // the operand fragments follow it
    float *trash = const_cast<float *>(W2) + NQ2;
    const uint32_t *frag = mx_frag_at(trash);
    constexpr int tN = 0, tNT = 1, tD = 2, tDT = 3;
    // a plain contraction along direction D: src -> dst
    auto sweep = [&](auto dtag, int tM, const float *src, float *dst) {
      constexpr int D = decltype(dtag)::value;
      const MxMat M = mx_frag(frag, tM);
      items(wave, [&](const Slot (&s)[U]) {
        int o[U][4];
        float x[U][4], y[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) { offsets<D>(s[u], o[u]); load(src, s[u], o[u], x[u]); }
#pragma unroll
        for (int u = 0; u < U; ++u) mx_apply(M, x[u], y[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) store(dst, trash, s[u], o[u], y[u]);
      });
    };
    using X0 = std::integral_constant<int, 0>;
    using X1 = std::integral_constant<int, 1>;
    using X2 = std::integral_constant<int, 2>;
    // N along x (A -> B), N along y (B -> A)
    sweep(X0{}, tN, A, B);
    __syncthreads();
    sweep(X1{}, tN, B, A);
    __syncthreads();
    // z-lines: u = N_z (A) -> B; the z-direction stage -> A
    {
    const MxMat Nm = mx_frag(frag, tN), Dm = mx_frag(frag, tD), DTm = mx_frag(frag, tDT);
    items(wave, [&](const Slot (&s)[U]) {
      int o[U][4];
      float x[U][4], uu[U][4], r[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) { offsets<2>(s[u], o[u]); load(A, s[u], o[u], x[u]); }
#pragma unroll
      for (int u = 0; u < U; ++u) mx_apply(Nm, x[u], uu[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) store(B, trash, s[u], o[u], uu[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) stage<2>(uu[u], r[u], s[u], Dm, DTm, a, C, W2);
#pragma unroll
      for (int u = 0; u < U; ++u) store(A, trash, s[u], o[u], r[u]);
    });
    }
    __syncthreads();
    // x-lines of u: the x-direction stage added into A
    {
    const MxMat Dm = mx_frag(frag, tD), DTm = mx_frag(frag, tDT);
    items(wave, [&](const Slot (&s)[U]) {
      int o[U][4];
      float uu[U][4], r[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        offsets<0>(s[u], o[u]);
        load(B, s[u], o[u], uu[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) stage<0>(uu[u], r[u], s[u], Dm, DTm, a, C, W2);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float acc[4];
        load(A, s[u], o[u], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) r[u][j] += acc[j];
        store(A, trash, s[u], o[u], r[u]);
      }
    });
    }
    prefetch_next();
    __syncthreads();
    // y-lines: the y-direction stage completes the sum; N^T along y -> B
    {
    const MxMat Dm = mx_frag(frag, tD), DTm = mx_frag(frag, tDT), NTm = mx_frag(frag, tNT);
    items(wave, [&](const Slot (&s)[U]) {
      int o[U][4];
      float uu[U][4], r[U][4], y[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        offsets<1>(s[u], o[u]);
        load(B, s[u], o[u], uu[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) stage<1>(uu[u], r[u], s[u], Dm, DTm, a, C, W2);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float acc[4];
        load(A, s[u], o[u], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) r[u][j] = (s[u].valid >> j & 1) ? r[u][j] + acc[j] : 0.0f;
        mx_apply(NTm, r[u], y[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) store(B, trash, s[u], o[u], y[u]);
    });
    }
    __syncthreads();
    // N^T along x (B -> A), then along z (A -> B)
    sweep(X0{}, tNT, B, A);
    __syncthreads();
    sweep(X2{}, tNT, A, B);
    __syncthreads();
  }
};

// The core hook of local_column: NT threads per block.
template <int NT> struct MxCore {
  static constexpr int threads = NT;
  // LDS after the line weights: the masked-store slot, then the operand fragments
  static constexpr int extra_lds_elems = 16 + 4 + MX_FRAG_ELEMS;
  template <typename TC> static __device__ __forceinline__ void begin(TC *tail, const KArgs<TC> &a) {
    mx_frag_store(mx_frag_at(tail), a.mxtab);
  }
  template <int NP, int VT, bool CPLX, typename TC, typename Pre>
  static __device__ __forceinline__ void cell(TC *A, TC *B, const TC *C, const TC *W2, const KArgs<TC> &a, int lane0,
                                              Pre &&prefetch_next) {
    static_assert(std::is_same<TC, float>::value, "the MFMA core computes in float");
    MxCell<NP, VT, NT, CPLX>::template run<NP>(A, B, C, W2, a, lane0, prefetch_next);
  }
};

}  // namespace fehx
