// Matrix-free local operator: dispatch by precision (kernels in k_local_impl.h,
// instantiated in k_local_f64.hip, k_local_f32.hip, k_local_bf16.hip).
#include "fe_internal.h"

namespace fehx {

fe_status launch_local_f64(Mesh *m, const LocalLaunch &L, hipStream_t s);
fe_status launch_local_f32(Mesh *m, const LocalLaunch &L, hipStream_t s);
fe_status launch_local_bf16(Mesh *m, const LocalLaunch &L, hipStream_t s);

fe_status launch_local(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  if (m->nq != m->np) return set_error(FE_EUNSUPPORTED, "this build has kernels for n_q = n_p only");
  if (L.prec == FE_F64) return launch_local_f64(m, L, s);
  if (L.prec == FE_F32) return launch_local_f32(m, L, s);
  if (L.prec == FE_BF16) return launch_local_bf16(m, L, s);
  return set_error(FE_EINVAL, "unknown precision");
}

}  // namespace fehx
