// Matrix-free local operator: dispatch by precision (kernels in k_local_impl.h,
// instantiated in k_local_f64.hip, k_local_f32.hip, k_local_bf16.hip).
#include "fe_internal.h"

namespace fehx {

fe_status launch_local_f64(const LocalBatch &B, hipStream_t s);
fe_status launch_local_f32(const LocalBatch &B, hipStream_t s);
fe_status launch_local_bf16(const LocalBatch &B, hipStream_t s);

fe_status launch_local_batch(const LocalBatch &B, hipStream_t s) {
  if (B.n < 1) return FE_OK;
  Mesh *m0 = B.ms[0];
  for (int i = 0; i < B.n; ++i) {
    Mesh *m = B.ms[i];
    if (m->nq != m->np && m->nq != m->np + 2 && m->nq != m->np + 3)
      return set_error(FE_EUNSUPPORTED, "this build has kernels for n_q = n_p, n_p + 2 and n_p + 3 only");
    if (m->np != m0->np || m->nq != m0->nq || m->cplx != m0->cplx || m->device != m0->device)
      return set_error(FE_EINVAL, "a batched launch needs one degree, quadrature, field type and device");
    if (B.Ls[i].prec != B.Ls[0].prec || B.Ls[i].vt != B.Ls[0].vt || B.Ls[i].store32 != B.Ls[0].store32)
      return set_error(FE_EINVAL, "a batched launch needs one precision, block type and vector tile");
  }
  if (B.Ls[0].prec == FE_F64) return launch_local_f64(B, s);
  if (B.Ls[0].prec == FE_F32) return launch_local_f32(B, s);
  if (B.Ls[0].prec == FE_BF16) return launch_local_bf16(B, s);
  return set_error(FE_EINVAL, "unknown precision");
}

fe_status launch_local(Mesh *m, const LocalLaunch &L, hipStream_t s) {
  Mesh *ms[1] = {m};
  LocalBatch B;
  B.ms = ms;
  B.Ls = &L;
  B.n = 1;
  return launch_local_batch(B, s);
}

}  // namespace fehx
