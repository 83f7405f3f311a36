// Local-operator launcher instantiations for f32 (see k_local_impl.h).
#include "k_local_impl.h"

namespace fehx {

fe_status local_f32_acc(const LocalBatch &B, hipStream_t s);
fe_status local_f32_acc3(const LocalBatch &B, hipStream_t s);

fe_status launch_local_f32(const LocalBatch &B, hipStream_t s) {
  if (B.ms[0]->nq == B.ms[0]->np + 2) return local_f32_acc(B, s);   // the accurate rule
  if (B.ms[0]->nq == B.ms[0]->np + 3) return local_f32_acc3(B, s);  // one point more
  if (B.ms[0]->nq != B.ms[0]->np) return set_error(FE_EUNSUPPORTED, "n_q must be n_p, n_p + 2 or n_p + 3");
  switch (B.ms[0]->np) {
    case 3: return pick_cplx_f32<3, 3>(B, s);
    case 4: return pick_cplx_f32<4, 4>(B, s);
    case 5: return pick_cplx_f32<5, 5>(B, s);
    case 6: return pick_cplx_f32<6, 6>(B, s);
    case 7: return pick_cplx_f32<7, 7>(B, s);
    case 8: return pick_cplx_f32<8, 8>(B, s);
    case 9: return pick_cplx_f32<9, 9>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
