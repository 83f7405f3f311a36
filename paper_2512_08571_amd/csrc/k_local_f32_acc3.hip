// Local-operator launcher instantiations for f32 (see k_local_impl.h), n_q = n_p + 3.
#include "k_local_impl.h"

namespace fehx {

fe_status local_f32_acc3(const LocalBatch &B, hipStream_t s) {
  switch (B.ms[0]->np) {
    case 3: return pick_cplx_f32<3, 6>(B, s);
    case 4: return pick_cplx_f32<4, 7>(B, s);
    case 5: return pick_cplx_f32<5, 8>(B, s);
    case 6: return pick_cplx_f32<6, 9>(B, s);
    case 7: return pick_cplx_f32<7, 10>(B, s);
    case 8: return pick_cplx_f32<8, 11>(B, s);
    case 9: return pick_cplx_f32<9, 12>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
