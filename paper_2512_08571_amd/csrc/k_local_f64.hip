// FP64 local-operator launcher: dispatch on (n_p, n_q) to the instantiation
// files (split so that they compile in parallel; see k_local_impl.h).
#include "k_local_impl.h"

namespace fehx {

fe_status local_f64_eq_lo(const LocalBatch &B, hipStream_t s);
fe_status local_f64_eq_hi(const LocalBatch &B, hipStream_t s);
fe_status local_f64_acc_lo(const LocalBatch &B, hipStream_t s);
fe_status local_f64_acc_hi(const LocalBatch &B, hipStream_t s);
fe_status local_f64_acc3_lo(const LocalBatch &B, hipStream_t s);
fe_status local_f64_acc3_hi(const LocalBatch &B, hipStream_t s);

fe_status launch_local_f64(const LocalBatch &B, hipStream_t s) {
  const int np = B.ms[0]->np, nq = B.ms[0]->nq;
  if (nq == np) return np <= 6 ? local_f64_eq_lo(B, s) : local_f64_eq_hi(B, s);
  // the accurate rule n_q = n_p + 2
  if (nq == np + 2) return np <= 6 ? local_f64_acc_lo(B, s) : local_f64_acc_hi(B, s);
  if (nq == np + 3) return np <= 6 ? local_f64_acc3_lo(B, s) : local_f64_acc3_hi(B, s);
  return set_error(FE_EUNSUPPORTED, "n_q must be n_p, n_p + 2 or n_p + 3");
}

}  // namespace fehx

// the host-side tile check (fe_set_tile) sizes blocks with the same formula
static_assert(fehx::lds_need<7, 7>(10, 8) == fehx::local_lds_bytes(7, 7, 10, 8, false), "LDS size formulas differ");
static_assert(fehx::lds_need<9, 11>(4, 8, true) == fehx::local_lds_bytes(9, 11, 4, 8, true), "LDS size formulas differ");
static_assert(fehx::LDS_MAX == fehx::LOCAL_LDS_MAX, "LDS limits differ");
