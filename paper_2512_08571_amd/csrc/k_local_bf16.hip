// Local-operator launcher instantiations for bf16 (see k_local_impl.h).
#include "k_local_impl.h"

namespace fehx {

fe_status local_bf16_acc(const LocalBatch &B, hipStream_t s);
bool local_mx_ok(const LocalBatch &B);
fe_status launch_local_mx(const LocalBatch &B, hipStream_t s);
fe_status launch_local_f32(const LocalBatch &B, hipStream_t s);

// FE_BF16: on the matrix cores (BF16 hi/lo operands, FP32 accumulation) where
// that core applies (n_q = n_p <= 8, diagonal metric).  Elsewhere BF16 blocks
// run the vector-ALU kernels below (float arithmetic), and FP32 blocks (the
// filter's recurrence state) the FP32 kernels.
fe_status launch_local_bf16(const LocalBatch &B, hipStream_t s) {
  if (local_mx_ok(B)) return launch_local_mx(B, s);
  if (B.Ls[0].store32) return launch_local_f32(B, s);
  if (B.ms[0]->nq == B.ms[0]->np + 2) return local_bf16_acc(B, s);   // the accurate rule
  if (B.ms[0]->nq == B.ms[0]->np + 3)
    return set_error(FE_EUNSUPPORTED, "BF16 blocks with n_q = n_p + 3 are not built (FP64 and FP32 are)");
  if (B.ms[0]->nq != B.ms[0]->np) return set_error(FE_EUNSUPPORTED, "n_q must be n_p or n_p + 2");
  switch (B.ms[0]->np) {
    case 3: return pick_cplx_bf16<3, 3>(B, s);
    case 4: return pick_cplx_bf16<4, 4>(B, s);
    case 5: return pick_cplx_bf16<5, 5>(B, s);
    case 6: return pick_cplx_bf16<6, 6>(B, s);
    case 7: return pick_cplx_bf16<7, 7>(B, s);
    case 8: return pick_cplx_bf16<8, 8>(B, s);
    case 9: return pick_cplx_bf16<9, 9>(B, s);
    default: return set_error(FE_EUNSUPPORTED, "FE degree outside 2..8");
  }
}

}  // namespace fehx
