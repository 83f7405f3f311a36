// FE_BF16 local operator on the matrix cores (k_local_mx.h): dispatch.  The
// instantiations (n_q = n_p <= 8, orthorhombic boxes, vector tiles of 16 and
// 32 lanes) sit in k_local_mx_f32.hip (FP32 blocks: the filter's recurrence
// state) and k_local_mx_bf16.hip (BF16 blocks: fe_apply_H), compiled in
// parallel.
#include "fe_internal.h"

namespace fehx {

fe_status local_mx_f32(const LocalBatch &B, hipStream_t s);
fe_status local_mx_bf16(const LocalBatch &B, hipStream_t s);

// Whether every system of the batch is one the MFMA core covers: n_q = n_p
// <= 8 and a diagonal metric (the sheared-box flux terms are not in it).
bool local_mx_ok(const LocalBatch &B) {
  for (int i = 0; i < B.n; ++i) {
    const Mesh *m = B.ms[i];
    if (m->nq != m->np || m->np > 8 || (m->offd && !B.Ls[i].mass)) return false;
  }
  return true;
}

fe_status launch_local_mx(const LocalBatch &B, hipStream_t s) {
  if (!local_mx_ok(B)) return set_error(FE_EUNSUPPORTED, "the MFMA local operator needs n_q = n_p <= 8 and a diagonal metric");
  return B.Ls[0].store32 ? local_mx_f32(B, s) : local_mx_bf16(B, s);
}

}  // namespace fehx
