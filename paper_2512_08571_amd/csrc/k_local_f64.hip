// Local-operator launcher instantiations for f64 (see k_local_impl.h).
#include "k_local_impl.h"

namespace fehx {

fe_status launch_local_f64(const LocalBatch &B, hipStream_t s) {
  if (B.ms[0]->nq == B.ms[0]->np + 2) {
    // the accurate rule n_q = n_p + 2 (FP64 only)
    switch (B.ms[0]->np) {
      case 3: return pick_cplx_f64<3, 5>(B, s);
      case 4: return pick_cplx_f64<4, 6>(B, s);
      case 5: return pick_cplx_f64<5, 7>(B, s);
      case 6: return pick_cplx_f64<6, 8>(B, s);
      case 7: return pick_cplx_f64<7, 9>(B, s);
      case 8: return pick_cplx_f64<8, 10>(B, s);
      case 9: return pick_cplx_f64<9, 11>(B, s);
      default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
    }
  }
  switch (B.ms[0]->np) {
    case 3: return pick_cplx_f64<3, 3>(B, s);
    case 4: return pick_cplx_f64<4, 4>(B, s);
    case 5: return pick_cplx_f64<5, 5>(B, s);
    case 6: return pick_cplx_f64<6, 6>(B, s);
    case 7: return pick_cplx_f64<7, 7>(B, s);
    case 8: return pick_cplx_f64<8, 8>(B, s);
    case 9: return pick_cplx_f64<9, 9>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
