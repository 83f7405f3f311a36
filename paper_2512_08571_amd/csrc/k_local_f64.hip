// Local-operator launcher instantiations for f64 (see k_local_impl.h).
#include "k_local_impl.h"

namespace fehx {

fe_status launch_local_f64(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  switch (m->np) {
    case 3: return pick_cplx_f64<3, 3>(m, L, s);
    case 4: return pick_cplx_f64<4, 4>(m, L, s);
    case 5: return pick_cplx_f64<5, 5>(m, L, s);
    case 6: return pick_cplx_f64<6, 6>(m, L, s);
    case 7: return pick_cplx_f64<7, 7>(m, L, s);
    case 8: return pick_cplx_f64<8, 8>(m, L, s);
    case 9: return pick_cplx_f64<9, 9>(m, L, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
