// Local-operator launcher instantiations for f64 (see k_local_impl.h), n_q = n_p + 3, n_p <= 6.
#include "k_local_impl.h"

namespace fehx {

fe_status local_f64_acc3_lo(const LocalBatch &B, hipStream_t s) {
  switch (B.ms[0]->np) {
    case 3: return pick_cplx_f64<3, 6>(B, s);
    case 4: return pick_cplx_f64<4, 7>(B, s);
    case 5: return pick_cplx_f64<5, 8>(B, s);
    case 6: return pick_cplx_f64<6, 9>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
