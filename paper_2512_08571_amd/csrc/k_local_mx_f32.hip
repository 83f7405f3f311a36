// Instantiations of the matrix-core local operator (k_local_mx.h) for FP32 blocks (the filter's recurrence state).
#include "k_local_mx.h"

namespace fehx {

namespace {

constexpr int MX_THREADS = 512;   // 8 waves: the gather's per-thread share fits 128 VGPRs
using Core = MxCore<MX_THREADS>;
using TS = float;

template <int NP, bool CPLX>
fe_status mx_pick_vt(const LocalBatch &B, hipStream_t s) {
  const size_t mx = (size_t)max_lds(B.ms[0]);
  const int want = B.Ls[0].vt >= 32 ? 32 : 16;
  if constexpr ((lds_need<NP, NP>(32, 4) + 80 + 4 * MX_FRAG_ELEMS) <= LDS_MAX)
    if (want == 32 && (lds_need<NP, NP>(32, 4) + 80 + 4 * MX_FRAG_ELEMS) <= mx) return run_local<NP, NP, 32, CPLX, TS, float, false, Core>(B, s);
  if ((lds_need<NP, NP>(16, 4) + 80 + 4 * MX_FRAG_ELEMS) <= mx) return run_local<NP, NP, 16, CPLX, TS, float, false, Core>(B, s);
  return set_error(FE_EUNSUPPORTED, "no MFMA local-operator tile fits the LDS");
}

template <int NP>
fe_status mx_cplx(const LocalBatch &B, hipStream_t s) {
  return B.ms[0]->cplx ? mx_pick_vt<NP, true>(B, s) : mx_pick_vt<NP, false>(B, s);
}

}  // namespace

fe_status local_mx_f32(const LocalBatch &B, hipStream_t s) {
  switch (B.ms[0]->np) {
    case 3: return mx_cplx<3>(B, s);
    case 4: return mx_cplx<4>(B, s);
    case 5: return mx_cplx<5>(B, s);
    case 6: return mx_cplx<6>(B, s);
    case 7: return mx_cplx<7>(B, s);
    case 8: return mx_cplx<8>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "the MFMA local operator covers n_p <= 8");
  }
}

}  // namespace fehx
