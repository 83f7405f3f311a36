// Autotuner for the local-operator launch shape.
//
// The vector tile VT (real lanes per workgroup) sets the LDS footprint
// ((2 n_q^3 + 2 n_p^2) VT + 4 n_q^3 + n_q^2 elements), the threads per block
// and so the occupancy, and the width of each node's coalesced segment.  Which
// VT is fastest depends on the precision, on whether the launch scales the
// gathered block by D^-1 (filter steps), on real vs complex and on the vector
// count, so the library measures it on the mesh itself: every
// candidate VT is run on scratch blocks of the requested width and timed with
// HIP events, and the fastest is kept per (precision, launch kind).
#include <algorithm>
#include <cmath>
#include <vector>

#include "fe_internal.h"

namespace fehx {

struct bf16t { uint16_t b; };

template <typename TS> __device__ __forceinline__ TS fill_value(double v);
template <> __device__ __forceinline__ double fill_value<double>(double v) { return v; }
template <> __device__ __forceinline__ float fill_value<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16t fill_value<bf16t>(double v) {
  bf16t r;
  r.b = (uint16_t)(__float_as_uint((float)v) >> 16);
  return r;
}

// x[i] in [-1, 1) from a 64-bit mix of i (timing data only)
template <typename TS>
__global__ void k_fill(TS *__restrict__ x, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = (uint64_t)i + seed * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    x[i] = fill_value<TS>((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
  }
}

namespace {

struct Scratch {
  std::vector<void *> p;
  ~Scratch() {
    for (void *q : p) hipFree(q);
  }
  void *get(size_t bytes) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
    p.push_back(q);
    return q;
  }
};

template <typename TS>
void fill(void *x, int64_t n, uint64_t seed, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_fill<TS>, dim3((unsigned)b), dim3(256), 0, s, (TS *)x, n, seed);
}

// FP64 offers ten lanes on the line-gather path (n_q = n_p)
constexpr int MAX_CAND = FE_TILE_CANDIDATES;
int candidates(int prec, bool nq_eq_np, int *out) {
  if (prec == FE_F64) {
    int n = 0;
    out[n++] = 2; out[n++] = 4; out[n++] = 8;
    if (nq_eq_np) out[n++] = 10;
    out[n++] = 16;
    return n;
  }
  out[0] = 8; out[1] = 16; out[2] = 32;
  return 3;
}

// a tile the local-operator launchers run on this mesh: its staged block fits
// the LDS, and FP64 takes two lanes only where four do not fit (as the
// launchers choose)
bool tile_fits(const Mesh *m, int prec, int vt) {
  int mx = 65536;
  (void)hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
  const size_t lim = std::min((size_t)mx, LOCAL_LDS_MAX);
  const int bytes = prec == FE_F64 ? 8 : 4;
  const bool od = m->offd;
  auto fits = [&](int v) { return local_lds_bytes(m->np, m->nq, v, bytes, od) <= lim; };
  if (prec == FE_F64 && vt == 2) return !fits(4) && fits(2);
  return fits(vt);
}

bool valid_tile(int prec, bool nq_eq_np, int vt) {
  int c[MAX_CAND];
  const int n = candidates(prec, nq_eq_np, c);
  for (int i = 0; i < n; ++i)
    if (c[i] == vt) return true;
  return vt == 0;
}

}  // namespace
}  // namespace fehx

using namespace fehx;

extern "C" {

fe_status fe_set_tile(fe_mesh_t m, int32_t prec, int32_t kind, int32_t vt) {
  if (!m) return set_error(FE_EINVAL, "NULL mesh");
  if (prec < FE_F64 || prec > FE_BF16 || kind < 0 || kind > 1) return set_error(FE_EINVAL, "bad precision / kind");
  if (!valid_tile(prec, m->nq == m->np, vt)) return set_error(FE_EINVAL, "vector tile not offered for this precision");
  if (vt != 0 && !m->host_only && !tile_fits(m, prec, vt))
    return set_error(FE_EINVAL, "vector tile does not fit this mesh's local-operator block in LDS");
  m->vt_pref[prec][kind] = vt;
  return FE_OK;
}

fe_status fe_get_tile(fe_mesh_t m, int32_t prec, int32_t kind, int32_t *vt) {
  if (!m || !vt) return set_error(FE_EINVAL, "NULL argument");
  if (prec < FE_F64 || prec > FE_BF16 || kind < 0 || kind > 1) return set_error(FE_EINVAL, "bad precision / kind");
  *vt = m->vt_pref[prec][kind];
  return FE_OK;
}

fe_status fe_autotune(fe_mesh_t m, int32_t prec, int32_t kind, int64_t nvec, int32_t reps, int32_t *best_vt,
                      int32_t *cand_vt, double *cand_ms, int32_t *ncand) {
  if (!m || !best_vt) return set_error(FE_EINVAL, "NULL argument");
  if (prec < FE_F64 || prec > FE_BF16 || kind < 0 || kind > 1) return set_error(FE_EINVAL, "bad precision / kind");
  if (nvec <= 0 || reps <= 0) return set_error(FE_EINVAL, "nvec and reps must be positive");
  if (m->host_only) return set_error(FE_ESTATE, "host-only mesh (device < 0)");
  if (hipSetDevice(m->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  const int C = m->cplx ? 2 : 1;
  const int64_t lanes = nvec * C;
  // filter steps in BF16 run on FP32 blocks (the recurrence state)
  const bool store32 = prec == FE_BF16 && kind == 1;
  const size_t es = prec == FE_F64 ? 8 : ((prec == FE_F32 || store32) ? 4 : 2);
  const int64_t n = m->m * lanes;
  Scratch S;
  void *X = S.get((size_t)n * es), *Y = S.get((size_t)n * es);
  if (!X || !Y) return set_error(FE_ENOMEM, "autotune scratch allocation failed");
  hipStream_t s = nullptr;
  FE_HIP_TRY(hipStreamCreate(&s));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { hipStreamDestroy(s); }
  } sg{s};
  if (prec == FE_F64) { fill<double>(X, n, 1, s); fill<double>(Y, n, 2, s); }
  else if (prec == FE_F32 || store32) { fill<float>(X, n, 1, s); fill<float>(Y, n, 2, s); }
  else { fill<bf16t>(X, n, 1, s); fill<bf16t>(Y, n, 2, s); }
  FE_HIP_TRY(hipGetLastError());
  hipEvent_t e0, e1;
  FE_HIP_TRY(hipEventCreate(&e0));
  FE_HIP_TRY(hipEventCreate(&e1));
  struct EventGuard {
    hipEvent_t a, b;
    ~EventGuard() { hipEventDestroy(a); hipEventDestroy(b); }
  } eg{e0, e1};
  int cand[MAX_CAND];
  const int nc = candidates(prec, m->nq == m->np, cand);
  float best = INFINITY;
  int bestv = 0;
  for (int i = 0; i < nc; ++i) {
    LocalLaunch L;
    L.X = X; L.Y = Y; L.ldx = lanes; L.ldy = lanes; L.nlanes = (int)lanes; L.prec = prec; L.vt = cand[i];
    L.store32 = store32;
    if (kind == 1) L.dinv_gather = m->dinv;   // a filter step: D^-1 applied at the gather
    float ms = INFINITY;
    fe_status st = launch_local(m, L, s);   // warm-up; a tile whose LDS does not fit is skipped
    if (st == FE_OK) {
      FE_HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < reps && st == FE_OK; ++r) st = launch_local(m, L, s);
      FE_HIP_TRY(hipEventRecord(e1, s));
      FE_HIP_TRY(hipEventSynchronize(e1));
      if (st == FE_OK) {
        FE_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms /= (float)reps;
      }
    } else if (st != FE_EUNSUPPORTED) {
      return st;
    }
    if (cand_vt) cand_vt[i] = cand[i];
    if (cand_ms) cand_ms[i] = std::isfinite(ms) ? (double)ms : -1.0;
    if (ms < best) { best = ms; bestv = cand[i]; }
  }
  if (ncand) *ncand = nc;
  if (bestv == 0) return set_error(FE_EUNSUPPORTED, "no vector tile fits this mesh");
  m->vt_pref[prec][kind] = bestv;
  *best_vt = bestv;
  return FE_OK;
}

}  // extern "C"
