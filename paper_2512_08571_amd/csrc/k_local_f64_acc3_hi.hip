// Local-operator launcher instantiations for f64 (see k_local_impl.h), n_q = n_p + 3, n_p >= 7.
#include "k_local_impl.h"

namespace fehx {

fe_status local_f64_acc3_hi(const LocalBatch &B, hipStream_t s) {
  switch (B.ms[0]->np) {
    case 7: return pick_cplx_f64<7, 10>(B, s);
    case 8: return pick_cplx_f64<8, 11>(B, s);
    case 9: return pick_cplx_f64<9, 12>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
