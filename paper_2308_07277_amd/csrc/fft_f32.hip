// float32 instantiation of the local-part kernels.
#include "fft_launch.h"
namespace qm {
void launch_local_f32(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi,
                      void* hpsi, hipStream_t s, StageEvents* ev, const HpsiWork* wk) {
  launch_local_t<float>(p, sl, psi, hpsi, s, ev, wk);
}
}  // namespace qm
