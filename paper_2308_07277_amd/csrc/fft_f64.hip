// float64 instantiation of the local-part kernels.
#include "fft_launch.h"
namespace qm {
void launch_local_f64(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi,
                      void* hpsi, hipStream_t s, StageEvents* ev, const HpsiWork* wk) {
  launch_local_t<double>(p, sl, psi, hpsi, s, ev, wk);
}
void launch_zinv_f64(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, hipStream_t s) {
  int64_t nblk_z = 0, npair = 0;
  const LocalArgs a = make_local_args<double>(p, sl, psi, nullptr, nullptr, nblk_z, npair);
  launch_zinv_t<double>(a, nblk_z, p->N3, s);
}
}  // namespace qm
