// Nonlocal pseudopotential term of eqn Vnonloc / eqn AXmatrixfreenonloc,
// Y += alpha F diag(h) F^H X, with F the assembled node-level projector matrix
// (the paper's cell blocks F^(a,e) summed over cells).
//
//   k_nl_w    W_partial[chunk][s][lane] = sum over the chunk's support nodes of
//             conj(F[n][s]) X[node][lane]; one workgroup per (node chunk of one
//             atom, 256-lane tile), the chunks run in order of position, each
//             XCD taking a contiguous run of them, so that overlapping atoms'
//             chunks share cached X rows in one L2; the four waves
//             split the nodes and are summed in LDS in a fixed order
//   k_nl_wsum W[s][lane] = h_s sum over the atom's chunks, in chunk order
//   k_nl_yb   the rows grouped by node bricks: one workgroup per (brick, lane
//             tile) stages the W rows of the brick's projectors in LDS once,
//             then each wave updates one Y row at a time reading W from LDS
//             (W crosses the L2 once per brick instead of once per entry)
//   k_nl_ybm  the FP64 form of the brick update on the matrix cores: the
//             brick's projector values as a dense block times the brick's W
//             rows, v_mfma_f64_16x16x4 over 16-row tiles
//   k_nl_y    the rows no brick of at most NL_BPMAX projectors holds: one wave
//             per row at a time, the row's (projector, value) entries are
//             wave-uniform scalar loads taken eight at a time, W and Y are
//             read and written as 256-lane rows
// Every thread owns four adjacent lanes (one 16/32-byte vector access per
// row when the block is aligned), so a wave moves a whole 256-lane row per
// access and complex (re, im) pairs stay inside one thread.  The vector
// width of these passes is the whole block row (the paper's level-0 batch
// for the nonlocal part of Alg. 1).
#include <mutex>
#include <string>

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
constexpr int NL_THREADS = 256;
constexpr int NL_TILE = 256;    // lanes per wave (4 per thread)

// Four adjacent lanes starting at element offset o of a row; VEC: the four
// are in range and 4-element aligned, so one vector access moves them.
// (Pair: the same for two FP64 lanes.)
template <typename TS, typename TC, bool VEC> struct Quad;
template <bool VEC> struct Quad<double, double, VEC> {
  static __device__ __forceinline__ void ld(const double *p, int64_t o, int nv, double v[4]) {
    if (VEC) {
      const double2 a = *(const double2 *)(p + o), b = *(const double2 *)(p + o + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = j < nv ? p[o + j] : 0.0;
    }
  }
  static __device__ __forceinline__ void st(double *p, int64_t o, int nv, const double v[4]) {
    if (VEC) {
      *(double2 *)(p + o) = make_double2(v[0], v[1]);
      *(double2 *)(p + o + 2) = make_double2(v[2], v[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) if (j < nv) p[o + j] = v[j];
    }
  }
};
template <bool VEC> struct Quad<float, float, VEC> {
  static __device__ __forceinline__ void ld(const float *p, int64_t o, int nv, float v[4]) {
    if (VEC) {
      const float4 a = *(const float4 *)(p + o);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = j < nv ? p[o + j] : 0.0f;
    }
  }
  static __device__ __forceinline__ void st(float *p, int64_t o, int nv, const float v[4]) {
    if (VEC) {
      *(float4 *)(p + o) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) if (j < nv) p[o + j] = v[j];
    }
  }
};
template <bool VEC> struct Quad<bf16n, float, VEC> {
  static __device__ __forceinline__ void ld(const bf16n *p, int64_t o, int nv, float v[4]) {
    if (VEC) {
      const uint2 a = *(const uint2 *)(p + o);
      v[0] = __uint_as_float(a.x << 16); v[1] = __uint_as_float(a.x & 0xffff0000u);
      v[2] = __uint_as_float(a.y << 16); v[3] = __uint_as_float(a.y & 0xffff0000u);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = j < nv ? nl_bf2f(p[o + j].b) : 0.0f;
    }
  }
  static __device__ __forceinline__ void st(bf16n *p, int64_t o, int nv, const float v[4]) {
    if (VEC) {
      uint2 a;
      a.x = (uint32_t)nl_f2bf(v[0]) | ((uint32_t)nl_f2bf(v[1]) << 16);
      a.y = (uint32_t)nl_f2bf(v[2]) | ((uint32_t)nl_f2bf(v[3]) << 16);
      *(uint2 *)(p + o) = a;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) if (j < nv) p[o + j].b = nl_f2bf(v[j]);
    }
  }
};

template <bool VEC> struct Pair {
  static __device__ __forceinline__ void ld(const double *p, int64_t o, int nv, double v[2]) {
    if (VEC) {
      const double2 a = *(const double2 *)(p + o);
      v[0] = a.x; v[1] = a.y;
    } else {
      v[0] = nv > 0 ? p[o] : 0.0;
      v[1] = nv > 1 ? p[o + 1] : 0.0;
    }
  }
  static __device__ __forceinline__ void st(double *p, int64_t o, int nv, const double v[2]) {
    if (VEC) {
      *(double2 *)(p + o) = make_double2(v[0], v[1]);
    } else {
      if (nv > 0) p[o] = v[0];
      if (nv > 1) p[o + 1] = v[1];
    }
  }
};

// 16 bytes of compute-type lanes per thread in the brick update
template <typename TS, typename TC, bool VEC> struct BrickIO { using T = Quad<TS, TC, VEC>; };
template <bool VEC> struct BrickIO<double, double, VEC> { using T = Pair<VEC>; };

// acc += conj(f) x (complex: lanes (re, im, re, im)) or f x (real)
template <bool CPLX, typename TC>
__device__ __forceinline__ void nl_conj_fma(TC fr, TC fi, const TC x[4], TC acc[4]) {
  if (!CPLX) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = fma(fr, x[j], acc[j]);
  } else {
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
      acc[j] = fma(fr, x[j], fma(fi, x[j + 1], acc[j]));
      acc[j + 1] = fma(fr, x[j + 1], fma(-fi, x[j], acc[j + 1]));
    }
  }
}

template <bool CPLX, typename TS, typename TC, bool VEC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_w(const TS *__restrict__ X, int64_t ldx, int nlanes, const double *__restrict__ dinv,
       const int *__restrict__ chunk_order, int nchunks, const int *__restrict__ chunk_atom, const int *__restrict__ chunk_n0,
       const int *__restrict__ nodes,
       const int *__restrict__ atom_off, const int *__restrict__ proj_off, const TC *__restrict__ F, int fstride,
       TC *__restrict__ part, int64_t ldp) {
  __shared__ TC red[4][NL_TILE];
  // XCD-aware: block x runs on XCD x % 8, and each XCD takes a contiguous run
  // of the position-ordered chunks, so overlapping atoms' chunks share an L2
  const int item = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (item >= nchunks) return;                   // whole block: before any barrier
  const int ch = chunk_order[item];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l0 = blockIdx.y * NL_TILE + (threadIdx.x & 63) * 4;
  const int nv = min(4, nlanes - l0);            // lanes of this thread in range
  const int a = chunk_atom[ch];
  const int n0 = chunk_n0[ch];
  const int n1 = min(n0 + NL_CHUNK, atom_off[a + 1]);
  const int ns = proj_off[a + 1] - proj_off[a];
  TC acc[NL_MAXP][4];
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[s][j] = 0;
  constexpr int C = CPLX ? 2 : 1;
#pragma unroll 2
  for (int n = n0 + wv; n < n1; n += 4) {
    const int64_t g = nodes[n];
    TC x[4];
    if (nv > 0) Quad<TS, TC, VEC>::ld(X, g * ldx + l0, nv, x);
    else x[0] = x[1] = x[2] = x[3] = 0;
    if (dinv) {
      const TC d = (TC)dinv[g];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] *= d;
    }
    const TC *f = F + (int64_t)n * fstride * C;
#pragma unroll
    for (int s = 0; s < NL_MAXP; ++s)
      if (s < ns) nl_conj_fma<CPLX>(f[s * C], CPLX ? f[s * C + 1] : (TC)0, x, acc[s]);
  }
  // fixed-order sum of the four waves, one projector at a time
#pragma unroll
  for (int s = 0; s < NL_MAXP; ++s) {
    if (s < ns) {
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wv][(threadIdx.x & 63) * 4 + j] = acc[s][j];
      __syncthreads();
      const int l = threadIdx.x;                 // one lane of the tile per thread
      const TC sum = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
      const int glo = blockIdx.y * NL_TILE + l;
      if (glo < nlanes) part[((int64_t)ch * NL_MAXP + s) * ldp + glo] = sum;
      __syncthreads();
    }
  }
}

template <typename TC>
__global__ void k_nl_wsum(const TC *__restrict__ part, int64_t ldp, const int *__restrict__ atom_chunk0,
                          const int *__restrict__ proj_off, const int *__restrict__ proj_atom,
                          const double *__restrict__ h, int ns, int nlanes, TC *__restrict__ W, int64_t ldw) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ns * nlanes) return;
  const int s = (int)(t / nlanes), l = (int)(t % nlanes);
  const int a = proj_atom[s];
  const int sl = s - proj_off[a];
  TC sum = 0;
  for (int ch = atom_chunk0[a]; ch < atom_chunk0[a + 1]; ++ch) sum += part[((int64_t)ch * NL_MAXP + sl) * ldp + l];
  W[(int64_t)s * ldw + l] = (TC)h[s] * sum;
}

template <bool CPLX, typename TS, typename TC, bool VEC>
__global__ void __launch_bounds__(NL_THREADS)
k_nl_y(TS *__restrict__ Y, int64_t ldy, int nlanes, const int *__restrict__ rows, const int *__restrict__ rowptr,
       const int *__restrict__ colidx, const TC *__restrict__ val, int64_t nrows, const TC *__restrict__ W,
       int64_t ldw, TC alpha) {
  const int l0 = blockIdx.y * NL_TILE + (threadIdx.x & 63) * 4;
  const int nv = min(4, nlanes - l0);
  const bool on = nv > 0;
  constexpr int C = CPLX ? 2 : 1;
  const int64_t wstride = (int64_t)gridDim.x * (NL_THREADS / 64);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t r = (int64_t)blockIdx.x * (NL_THREADS / 64) + wv; r < nrows; r += wstride) {
    const int e0 = rowptr[r], e1 = rowptr[r + 1];
    const int64_t o = (int64_t)rows[r] * ldy + l0;
    TC y[4] = {0, 0, 0, 0};
    if (on) Quad<TS, TC, VEC>::ld(Y, o, nv, y);        // in flight with the W reads
    TC acc[4] = {0, 0, 0, 0};
    for (int eb = e0; eb < e1; eb += 8) {
      // eight entries at a time: independent W rows keep several loads in flight
      int sidx[8];
      TC vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = eb + u < e1;
        const int e = in ? eb + u : e1 - 1;
        sidx[u] = colidx[e];
        vr[u] = in ? val[(int64_t)e * C] : (TC)0;
        vi[u] = (CPLX && in) ? val[(int64_t)e * C + 1] : (TC)0;
      }
      TC w[8][4];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (on) Quad<TC, TC, VEC>::ld(W, (int64_t)sidx[u] * ldw + l0, nv, w[u]);
        else w[u][0] = w[u][1] = w[u][2] = w[u][3] = 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (!CPLX) {
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] = fma(vr[u], w[u][j], acc[j]);
        } else {
          // (vr + i vi)(wr + i wi): re += vr wr - vi wi, im += vr wi + vi wr
#pragma unroll
          for (int j = 0; j < 4; j += 2) {
            acc[j] = fma(vr[u], w[u][j], fma(-vi[u], w[u][j + 1], acc[j]));
            acc[j + 1] = fma(vr[u], w[u][j + 1], fma(vi[u], w[u][j], acc[j + 1]));
          }
        }
      }
    }
    if (on) {
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] += alpha * acc[j];
      Quad<TS, TC, VEC>::st(Y, o, nv, y);
    }
  }
}

constexpr int NL_BTHREADS = 1024;
constexpr int NL_YPF = 4;      // Y rows in flight per wave in the brick update

// Y[row] += alpha sum_e val_e W[proj_e] over the rows of one brick.  Each
// thread owns LPT = 16 / sizeof(TC) adjacent lanes (FP64: 2, FP32: 4), so a
// complex (re, im) pair stays in one thread and a wave covers a 64 LPT-lane
// tile; the staged block is np x tile (at most NL_BPMAX x 1 KiB).  A row's
// entries come in groups of four, two groups per step as wave-uniform scalar
// loads.  Blocks are numbered so that the lane tiles of one brick run on one
// XCD (dispatch deals consecutive blocks to the eight XCDs in turn): the
// brick's entry list is fetched from HBM once and then hit in that L2.
template <bool CPLX, typename TS, typename TC, bool VEC>
__global__ void __launch_bounds__(NL_BTHREADS)
k_nl_yb(TS *__restrict__ Y, int64_t ldy, int nlanes, int nbrick, const int *__restrict__ b_row0, const int *__restrict__ b_p0,
        const int *__restrict__ b_proj, const int *__restrict__ b_rows, const int *__restrict__ b_rowptr,
        const int4 *__restrict__ gcol, const TC *__restrict__ gval, const TC *__restrict__ W, int64_t ldw,
        TC alpha) {
  constexpr int LPT = 16 / sizeof(TC);
  constexpr int TILE = 64 * LPT;
  constexpr int C = CPLX ? 2 : 1;
  constexpr int GV = 4 * C;                          // values per group
  constexpr int NW = NL_BTHREADS / 64;
  using IO = typename BrickIO<TS, TC, VEC>::T;
  using IOW = typename BrickIO<TC, TC, VEC>::T;
  extern __shared__ __align__(16) unsigned char nl_smem[];
  TC *Wl = (TC *)nl_smem;
  const int tiles = (nlanes + TILE - 1) / TILE;
  const int xcd = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int b = (rest / tiles) * 8 + xcd, tile = rest % tiles;
  if (b >= nbrick) return;                           // whole block: before any barrier
  const int lt = (threadIdx.x & 63) * LPT;
  const int l0 = tile * TILE + lt;
  const int nv = min(LPT, nlanes - l0);
  const bool on = nv > 0;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p0 = b_p0[b], np = b_p0[b + 1] - p0;
  for (int i = wv; i < np; i += NW) {
    TC w[LPT];
    if (on) IOW::ld(W, (int64_t)b_proj[p0 + i] * ldw + l0, nv, w);
    else
#pragma unroll
      for (int j = 0; j < LPT; ++j) w[j] = 0;
#pragma unroll
    for (int j = 0; j < LPT; ++j) Wl[i * TILE + lt + j] = w[j];
  }
  __syncthreads();
  const TC *Wt = Wl + lt;
  const int r1 = b_row0[b + 1];
  // Each wave's Y rows are read NL_YPF rows ahead, one register slot per
  // row in flight (the row loop is unrolled over the slots, so a pending read
  // is never moved between registers): enough HBM reads in flight per CU to
  // cover their latency.
  // Reads are unconditional so that the waits stay counted: a lane past the
  // block reads the row's first lanes, a slot past the wave's last row reads
  // that row again; neither value is used.
  TC yq[NL_YPF][LPT];
  const int rw = b_row0[b] + wv;
  const int lc = on ? l0 : 0, nc = on ? nv : min(LPT, nlanes);
  if (rw < r1) {
#pragma unroll
    for (int k = 0; k < NL_YPF; ++k) {
      const int rk = min(rw + k * NW, r1 - 1);
      IO::ld(Y, (int64_t)b_rows[rk] * ldy + lc, nc, yq[k]);
    }
  }
  for (int r0 = rw; r0 < r1; r0 += NL_YPF * NW)
#pragma unroll
  for (int q = 0; q < NL_YPF; ++q) {
    const int r = r0 + q * NW;
    if (r >= r1) break;
    const int g0 = b_rowptr[r], g1 = b_rowptr[r + 1];
    TC acc[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) acc[j] = 0;
    for (int g = g0; g < g1; g += 2) {
      // two groups (eight entries) per step: one scalar-load round trip,
      // eight LDS reads in flight
      int cc[8];
      TC vc[2 * GV];
      const int4 ca = gcol[g], cb = gcol[g + 1];
      cc[0] = ca.x; cc[1] = ca.y; cc[2] = ca.z; cc[3] = ca.w;
      cc[4] = cb.x; cc[5] = cb.y; cc[6] = cb.z; cc[7] = cb.w;
#pragma unroll
      for (int k = 0; k < 2 * GV; ++k) vc[k] = gval[(int64_t)g * GV + k];
      TC w[8][LPT];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int j = 0; j < LPT; ++j) w[u][j] = Wt[cc[u] * TILE + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const TC vr = vc[u * C], vi = CPLX ? vc[u * C + 1] : (TC)0;
        if (!CPLX) {
#pragma unroll
          for (int j = 0; j < LPT; ++j) acc[j] = fma(vr, w[u][j], acc[j]);
        } else {
          // (vr + i vi)(wr + i wi): re += vr wr - vi wi, im += vr wi + vi wr
#pragma unroll
          for (int j = 0; j < LPT; j += 2) {
            acc[j] = fma(vr, w[u][j], fma(-vi, w[u][j + 1], acc[j]));
            acc[j + 1] = fma(vr, w[u][j + 1], fma(vi, w[u][j], acc[j + 1]));
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < LPT; ++j) yq[q][j] += alpha * acc[j];
    if (on) IO::st(Y, (int64_t)b_rows[r] * ldy + l0, nv, yq[q]);
    const int rn = r + NL_YPF * NW;
    IO::ld(Y, (int64_t)b_rows[rn < r1 ? rn : r] * ldy + lc, nc, yq[q]);
  }
}

// FP64 brick update on the matrix cores: Y[rows of brick b] += alpha A_b B_b.
// A_b is the brick's dense projector block (rows x K_b, columns (p, re) and
// (p, im) for complex, zero-padded to a multiple of 4); B_b (K_b x 64 lanes,
// staged in LDS) holds the W rows of the brick's projectors, the (p, im) row
// as i W_p, so that one real product yields both parts of F W:
//   re += Fr Wr + Fi (-Wi),  im += Fr Wi + Fi Wr.
// One workgroup per (brick, 64-lane tile); each wave takes 16-row tiles and
// accumulates four 16 x 16 column blocks over K with v_mfma_f64_16x16x4
// (operands: lane l holds A[l & 15][l >> 4] and B[l >> 4][l & 15]; item v of
// the result is row (l >> 4) + 4 v, column l & 15).  The K order is fixed, so
// the update is reproducible bit for bit.  The four A values of a step come
// eight steps at a time, so one load latency covers 32 columns of K.
constexpr int NL_MT = 512;   // threads of the matrix-core brick update
constexpr int NL_MN = 64;    // lanes per workgroup tile
typedef double nl_v4d __attribute__((ext_vector_type(4)));
// the staged block (at most 2 NL_BPMAX rows of 64 lanes) must stay within the
// 64 KiB of dynamic LDS a launch gets without a function attribute
static_assert(2 * NL_BPMAX * NL_MN * sizeof(double) <= 65536, "k_nl_ybm's LDS block exceeds 64 KiB");

template <bool CPLX>
__global__ void __launch_bounds__(NL_MT)
k_nl_ybm(double *__restrict__ Y, int64_t ldy, int nlanes, int nbrick, const int *__restrict__ b_row0,
         const int *__restrict__ b_p0, const int *__restrict__ b_proj, const int *__restrict__ b_rows,
         const int64_t *__restrict__ a_off, const int *__restrict__ kb, const double *__restrict__ A,
         const double *__restrict__ W, int64_t ldw, double alpha) {
  constexpr int NCB = NL_MN / 16;
  constexpr int NW = NL_MT / 64;
  extern __shared__ __align__(16) unsigned char nl_smem[];
  double *Bl = (double *)nl_smem;
  const int tiles = (nlanes + NL_MN - 1) / NL_MN;
  const int xcd = blockIdx.x & 7, rest = blockIdx.x >> 3;   // a brick's tiles on one XCD, as in k_nl_yb
  const int b = (rest / tiles) * 8 + xcd, tile = rest % tiles;
  if (b >= nbrick) return;                                   // whole block: before any barrier
  const int n0 = tile * NL_MN;
  const int p0 = b_p0[b], np = b_p0[b + 1] - p0, K = kb[b];
  for (int e = threadIdx.x; e < K * NL_MN; e += NL_MT) {
    const int k = e / NL_MN, j = e - k * NL_MN;
    const int p = CPLX ? k >> 1 : k;
    double v = 0.0;
    if (p < np && n0 + j < nlanes) {          // complex: nlanes even, so n0 + (j | 1) < nlanes too
      const double *w = W + (int64_t)b_proj[p0 + p] * ldw + n0;
      if (!CPLX || !(k & 1)) v = w[j];
      else v = (j & 1) ? w[j - 1] : -w[j + 1];
    }
    Bl[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int r0 = b_row0[b], R = b_row0[b + 1] - r0;
  const double *Ab = A + a_off[b];
  for (int mt = wv; mt * 16 < R; mt += NW) {
    // this tile's Y values (rows past the brick read its last row, columns
    // past the block its last column; neither is written back)
    double y[4][NCB];
    int64_t yo[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      yo[v] = (int64_t)b_rows[r0 + min(mt * 16 + kq + 4 * v, R - 1)] * ldy;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) y[v][cb] = Y[yo[v] + min(n0 + cb * 16 + i, nlanes - 1)];
    }
    nl_v4d acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = (nl_v4d){0.0, 0.0, 0.0, 0.0};
    const bool arow = mt * 16 + i < R;
    const double *ap = Ab + (int64_t)min(mt * 16 + i, R - 1) * K + kq;
    for (int k0 = 0; k0 < K; k0 += 32) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = (arow && k0 + 4 * u < K) ? ap[k0 + 4 * u] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k0 + 4 * u >= K) break;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], Bl[(k0 + 4 * u + kq) * NL_MN + cb * 16 + i],
                                                         acc[cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (mt * 16 + kq + 4 * v >= R) continue;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int col = n0 + cb * 16 + i;
        if (col < nlanes) Y[yo[v] + col] = y[v][cb] + alpha * acc[cb][v];
      }
    }
  }
}

namespace {
template <bool CPLX, typename TS, typename TC, bool VEC>
void launch_nl_w(Mesh *m, const TS *X, int64_t ldx, int nlanes, const double *dinv, const TC *F, TC *part,
                 int64_t ldp, TC *W, int64_t ldw, hipStream_t s) {
  const int tiles = (nlanes + NL_TILE - 1) / NL_TILE;
  const unsigned gx = (unsigned)(m->nl_nchunks + 7) / 8 * 8;   // a multiple of the 8 XCDs
  hipLaunchKernelGGL((k_nl_w<CPLX, TS, TC, VEC>), dim3(gx, tiles), dim3(NL_THREADS), 0, s, X, ldx,
                     nlanes, dinv, m->nl_chunk_order, m->nl_nchunks, m->nl_chunk_atom, m->nl_chunk_n0, m->nl_atom_nodes, m->nl_atom_off,
                     m->nl_atom_proj, F, m->nl_maxproj, part, ldp);
  const int64_t nw = (int64_t)m->ns * nlanes;
  hipLaunchKernelGGL((k_nl_wsum<TC>), dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, part, ldp,
                     m->nl_atom_chunk0, m->nl_atom_proj, m->nl_proj_atom, m->nl_h, m->ns, nlanes, W, ldw);
}

template <bool CPLX, typename TS, typename TC, bool VEC>
void launch_nl_y(Mesh *m, TS *Y, int64_t ldy, int nlanes, const TC *val, const TC *W, int64_t ldw, TC alpha,
                 hipStream_t s) {
  if constexpr (std::is_same<TC, double>::value) {
    if (m->nl_nbrick > 0) {
      const int64_t blocks = ((int64_t)m->nl_nbrick + 7) / 8 * 8 * ((nlanes + NL_MN - 1) / NL_MN);
      const size_t shm = (size_t)m->nl_b_kmax * NL_MN * sizeof(double);
      hipLaunchKernelGGL((k_nl_ybm<CPLX>), dim3((unsigned)blocks), dim3(NL_MT), shm, s, (double *)Y, ldy, nlanes,
                         m->nl_nbrick, m->nl_b_row0, m->nl_b_p0, m->nl_b_proj, m->nl_b_rows, m->nl_b_aoff,
                         m->nl_b_k, m->nl_b_A64, (const double *)W, ldw, (double)alpha);
    }
  } else if (m->nl_nbrick > 0) {
    const TC *bval = (const TC *)m->nl_b_val32;
    constexpr int BT = 64 * (16 / (int)sizeof(TC));
    const int64_t btiles = (nlanes + BT - 1) / BT;
    const size_t shm = (size_t)m->nl_bmaxp * BT * sizeof(TC);
    const int64_t blocks = ((int64_t)m->nl_nbrick + 7) / 8 * 8 * btiles;
    hipLaunchKernelGGL((k_nl_yb<CPLX, TS, TC, VEC>), dim3((unsigned)blocks), dim3(NL_BTHREADS), shm, s, Y,
                       ldy, nlanes, m->nl_nbrick, m->nl_b_row0, m->nl_b_p0, m->nl_b_proj, m->nl_b_rows, m->nl_b_rowptr,
                       (const int4 *)m->nl_b_lcol, bval, W, ldw, alpha);
  }
  if (m->nl_nrows > 0) {
    const int tiles = (nlanes + NL_TILE - 1) / NL_TILE;
    int64_t blocks = (m->nl_nrows + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_nl_y<CPLX, TS, TC, VEC>), dim3((unsigned)blocks, tiles), dim3(NL_THREADS), 0, s, Y, ldy,
                       nlanes, m->nl_rows, m->nl_rowptr, m->nl_colidx, val, m->nl_nrows, W, ldw, alpha);
  }
}

// part 1: W = diag(h) F^H (D^-1) X;  part 2: Y += alpha F W;  3: both.
// ws: the partials + W workspace (nl_workspace_bytes), or null for the mesh's own
template <bool CPLX, typename TS, typename TC>
fe_status run_nl(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, const double *dinv,
                 double alpha, int parts, void *ws, hipStream_t s) {
  const bool f64 = std::is_same<TC, double>::value;
  const TC *F = f64 ? (const TC *)m->nl_F64 : (const TC *)m->nl_F32;
  const TC *val = f64 ? (const TC *)m->nl_val64 : (const TC *)m->nl_val32;
  // workspace: partials [nchunks][NL_MAXP][ldp] then W [ns][ldw], rows padded to 4 lanes
  const int64_t ldp = (nlanes + 3) / 4 * 4, ldw = ldp;
  if (!ws) {
    fe_status st = ensure_nl_workspace(m, nlanes);
    if (st) return st;
    ws = m->nl_W;
  }
  TC *part = (TC *)ws;
  TC *W = part + (int64_t)m->nl_nchunks * NL_MAXP * ldp;
  // vector accesses need every thread's four lanes in range and 4-element aligned
  const uintptr_t al = 4 * sizeof(TS);
  if (parts & 1) {
    const bool vec = nlanes % 4 == 0 && ldx % 4 == 0 && (uintptr_t)X % al == 0;
    if (vec) launch_nl_w<CPLX, TS, TC, true>(m, (const TS *)X, ldx, nlanes, dinv, F, part, ldp, W, ldw, s);
    else launch_nl_w<CPLX, TS, TC, false>(m, (const TS *)X, ldx, nlanes, dinv, F, part, ldp, W, ldw, s);
  }
  if (parts & 2) {
    const bool vec = nlanes % 4 == 0 && ldy % 4 == 0 && (uintptr_t)Y % al == 0;
    if (vec) launch_nl_y<CPLX, TS, TC, true>(m, (TS *)Y, ldy, nlanes, val, W, ldw, (TC)alpha, s);
    else launch_nl_y<CPLX, TS, TC, false>(m, (TS *)Y, ldy, nlanes, val, W, ldw, (TC)alpha, s);
  }
  FE_HIP_TRY(hipGetLastError());
  return FE_OK;
}

fe_status dispatch_nl(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, int prec,
                      const double *dinv, double alpha, int parts, hipStream_t s, void *ws = nullptr) {
  if (m->ns == 0) return FE_OK;
  if (m->nl_maxproj > NL_MAXP) return set_error(FE_EUNSUPPORTED, "more than 10 projectors on one atom");
  if (m->cplx) {
    if (prec == FE_F64) return run_nl<true, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
    if (prec == FE_F32) return run_nl<true, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
    return run_nl<true, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
  }
  if (prec == FE_F64) return run_nl<false, double, double>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
  if (prec == FE_F32) return run_nl<false, float, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
  return run_nl<false, bf16n, float>(m, X, ldx, Y, ldy, nlanes, dinv, alpha, parts, ws, s);
}
}  // namespace

// bytes of the projector workspace for nlanes real lanes: the per-chunk
// partials [nchunks][NL_MAXP][ldp] and W [ns][ldp] (sized for FP64)
int64_t nl_workspace_bytes(const Mesh *m, int nlanes) {
  if (m->ns == 0) return 0;
  const int64_t ldp = (nlanes + 3) / 4 * 4;
  return ((int64_t)m->nl_nchunks * NL_MAXP * ldp + (int64_t)m->ns * ldp) * (int64_t)sizeof(double);
}

fe_status ensure_nl_workspace(Mesh *m, int nlanes) {
  if (m->ns == 0) return FE_OK;
  const int64_t need = nl_workspace_bytes(m, nlanes);
  if (m->nl_W != nullptr && m->nl_W_lanes >= need) return FE_OK;
  if (m->nl_W != nullptr && m->graphs > 0)
    return set_error(FE_ESTATE, "a captured filter graph holds this mesh's projector workspace; destroy it before a "
                                "call with more vectors");
  if (m->nl_W) { hipFree(m->nl_W); m->footprint -= m->nl_W_lanes; m->nl_W = nullptr; m->nl_W_lanes = 0; }
  if (hipMalloc(&m->nl_W, need) != hipSuccess) { m->nl_W = nullptr; return set_error(FE_ENOMEM, "nonlocal workspace allocation failed"); }
  m->nl_W_lanes = need;
  m->footprint += need;
  return FE_OK;
}

fe_status launch_nonlocal(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy, int nlanes, int prec,
                          const double *dinv, double alpha, hipStream_t s) {
  return dispatch_nl(m, X, ldx, Y, ldy, nlanes, prec, dinv, alpha, 3, s);
}

fe_status launch_nonlocal_w(Mesh *m, const void *X, int64_t ldx, int nlanes, int prec, const double *dinv,
                            hipStream_t s) {
  return dispatch_nl(m, X, ldx, nullptr, 0, nlanes, prec, dinv, 0.0, 1, s);
}

fe_status launch_nonlocal_y(Mesh *m, void *Y, int64_t ldy, int nlanes, int prec, double alpha, hipStream_t s) {
  return dispatch_nl(m, nullptr, 0, Y, ldy, nlanes, prec, nullptr, alpha, 2, s);
}

fe_status ensure_side_stream(Mesh *m) {
  if (m->side) return FE_OK;
  if (hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess) {
    m->side = nullptr;
    return set_error(FE_EDEVICE, "hipStreamCreate failed");
  }
  if (hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) != hipSuccess)
    return set_error(FE_EDEVICE, "hipEventCreate failed");
  return FE_OK;
}

// An application runs the projector reduction W before the local-operator
// launches and the projector update Y += alpha F W after them.  FP64: all on
// the caller's stream.  FP32 / BF16: the reduction is forked to the mesh's
// second stream, beside the local launches (both only read X), and joined
// back before the update.  The choice is measured: the FP64 line-gather
// local kernel fills the CUs' registers and loses more to a co-running
// reduction than the reduction takes on its own (Mid: step 3.57 ms forked,
// 3.53 ms in order), while the FP32 staged kernel loses less (filter pass at
// 512 vectors: 258 ms forked, 264 ms in order).
static bool nl_forked(int prec) { return prec != FE_F64; }

fe_status nonlocal_reduce(Mesh *m, const void *X, int64_t ldx, int nlanes, int prec, const double *dinv,
                          hipStream_t s) {
  if (m->ns == 0) return FE_OK;
  fe_status st;
  if ((st = ensure_nl_workspace(m, nlanes))) return st;
  if (!nl_forked(prec)) return launch_nonlocal_w(m, X, ldx, nlanes, prec, dinv, s);
  if ((st = ensure_side_stream(m))) return st;
  FE_HIP_TRY(hipEventRecord(m->ev_fork, s));
  FE_HIP_TRY(hipStreamWaitEvent(m->side, m->ev_fork, 0));
  if ((st = launch_nonlocal_w(m, X, ldx, nlanes, prec, dinv, m->side))) return st;
  FE_HIP_TRY(hipEventRecord(m->ev_join, m->side));
  return FE_OK;
}

fe_status nonlocal_update(Mesh *m, void *Y, int64_t ldy, int nlanes, int prec, double alpha, hipStream_t s) {
  if (m->ns == 0) return FE_OK;
  if (nl_forked(prec)) FE_HIP_TRY(hipStreamWaitEvent(s, m->ev_join, 0));
  return launch_nonlocal_y(m, Y, ldy, nlanes, prec, alpha, s);
}

fe_status apply_with_nonlocal(Mesh *m, const LocalLaunch &L, int prec, const double *dinv, double alpha,
                              hipStream_t s) {
  fe_status st;
  if ((st = nonlocal_reduce(m, L.X, L.ldx, L.nlanes, prec, dinv, s))) return st;
  if ((st = launch_local(m, L, s))) return st;
  return nonlocal_update(m, L.Y, L.ldy, L.nlanes, prec, alpha, s);
}

// ---- the application that allocates nothing ----------------------------------
// Scratch for fe_apply_H_noalloc: the projector partials and W of one
// application, in a file-scope device array (each device holds its own copy
// for the life of the process).  Host code never passes the array's name to a
// kernel: its device address comes from hipGetSymbolAddress, once per device
// with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[FE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAXDEV = 64;
std::mutex g_scratch_mu;
void *g_scratch[SCRATCH_MAXDEV] = {};

fe_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= SCRATCH_MAXDEV) return set_error(FE_EUNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(FE_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FE_OK;
}
}  // namespace

}  // namespace fehx

using namespace fehx;

extern "C" fe_status fe_apply_H_noalloc(fe_mesh_t m, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t nvec,
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
  const int nlanes = (int)(nvec * C);
  if (nl_workspace_bytes(m, nlanes) > FE_NOALLOC_SCRATCH_BYTES)
    return set_error(FE_EINVAL, "projector workspace of " + std::to_string(nl_workspace_bytes(m, nlanes)) +
                                    " bytes exceeds the static scratch of " + std::to_string((long long)FE_NOALLOC_SCRATCH_BYTES) +
                                    " bytes; use fe_apply_H");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  void *ws = nullptr;
  fe_status st;
  if (m->ns > 0 && (st = scratch_address(m->device, &ws))) return st;
  hipStream_t s = (hipStream_t)stream;
  LocalLaunch L;
  L.X = X; L.Y = Y; L.ldx = ldx * C; L.ldy = ldy * C; L.nlanes = nlanes; L.prec = prec;
  L.vt = m->vt_pref[prec][0];
  // projector reduction, local operator, projector update on the caller's
  // stream, as in fe_apply_H
  if ((st = dispatch_nl(m, X, L.ldx, nullptr, 0, nlanes, prec, nullptr, 0.0, 1, s, ws))) return st;
  if ((st = launch_local(m, L, s))) return st;
  return dispatch_nl(m, nullptr, 0, Y, L.ldy, nlanes, prec, nullptr, 1.0, 2, s, ws);
}
