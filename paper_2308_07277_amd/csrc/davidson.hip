// Block Davidson driver (placeholder until the GPU eigensolver lands).
#include "qm_internal.h"

namespace qm {
struct DavState {};
void davidson_free(qm_hpsi_plan* p) {
  delete p->dav;
  p->dav = nullptr;
}
}  // namespace qm

extern "C" {
qm_status qm_davidson_step(qm_hpsi_plan* plan, int32_t, void*, double*, double*, int32_t,
                           const qm_dav_opts*, int32_t*, void*) {
  if (plan) plan->err = "qm_davidson_step: not available in this build";
  return QM_E_STATE;
}
qm_status qm_davidson_solve(qm_hpsi_plan* plan, int32_t, void*, double*, double*, int32_t,
                            const qm_dav_opts*, qm_dav_stats*, void*) {
  if (plan) plan->err = "qm_davidson_solve: not available in this build";
  return QM_E_STATE;
}
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
