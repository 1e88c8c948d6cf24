// Learned residual -> correction preconditioner (inference/training kernels).
#include "dense.h"

namespace qm {
void mlp_precondition(qm_hpsi_plan*, const DJobs&, const void*, hipStream_t) {
  throw Error(QM_E_STATE, "learned preconditioner not available in this build");
}
}  // namespace qm

extern "C" {
qm_status qm_mlp_forward(const float*, const float*, float*, int64_t, void*) { return QM_E_STATE; }
qm_status qm_mlp_loss_grad(const float*, const float*, const float*, const float*, int64_t, float*,
                           double*, void*) {
  return QM_E_STATE;
}
qm_status qm_mlp_adam(float*, const float*, float*, float*, int32_t, float, float, float, float,
                      void*) {
  return QM_E_STATE;
}
}
