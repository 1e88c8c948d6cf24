// H|psi> for callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc): the same operation as qm_apply_h, with the
// working memory that the plan's buffers give qm_apply_h (stick buffer, projections P and
// D P, split-K partial sums) taken from one static device array of fixed size instead.
// k-points are processed one at a time, their bands in chunks sized so that one chunk's
// working memory fits in the array; the kernels are the ones qm_apply_h launches.
#include <mutex>

#include "qm_internal.h"

namespace qm {

constexpr size_t kScratchBytes = size_t(QM_NOALLOC_SCRATCH_MIB) << 20;

// The library's scratch array.  Each GPU the library runs on holds its own copy, at its
// own address, until the process ends.  In host code the name is only a host-side stand-in:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static char* scratch_ptr() {
  int dev = 0;
  QM_HIP(hipGetDevice(&dev));
  QM_REQUIRE(dev >= 0 && dev < kMaxDevices, QM_E_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    QM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    QM_REQUIRE(ptr != nullptr, QM_E_HIP, "no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

static void apply_noalloc(qm_hpsi_plan* p, int k, const void* psi, void* hpsi, int nbnd,
                          hipStream_t s) {
  QM_REQUIRE(psi && hpsi, QM_E_ARG, "psi and hpsi must be non-NULL");
  QM_REQUIRE(psi != hpsi, QM_E_ARG, "hpsi must not alias psi");
  QM_REQUIRE(nbnd >= 1 && nbnd <= p->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
  QM_REQUIRE(k >= -1 && k < p->nk, QM_E_ARG, "k out of range");
  const int lp = p->prec == QM_PREC_FP64 ? 0 : (p->prec == QM_PREC_FP32 ? 1 : 2);
  QM_REQUIRE(lp == 0 || p->nproj == 0 || p->beta_lp_kind == lp, QM_E_STATE,
             "the reduced-precision copy of beta is not built: call qm_hpsi_plan_set_precision "
             "before capturing");
  const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? p->nk : k + 1;
  const int64_t csz = lp == 0 ? 16 : 8;   // stick buffer element: c128 or c64
  const int64_t pq_band = int64_t(p->nproj) * 16;
  // one chunk: stick block, P, Q and at least one split of partial sums, each 256-aligned
  const int64_t avail = int64_t(kScratchBytes) - 4 * 256;
  // validate every k before any launch, so a size error leaves no partial result
  for (int kk = k0; kk < k1; ++kk) {
    const int64_t per_band = int64_t(p->kinfo[kk].nstick) * p->N3 * csz + 3 * pq_band;
    QM_REQUIRE(per_band <= avail, QM_E_ARG,
               "one band of this k-point needs more working memory than the "
               "allocation-free scratch array holds (QM_NOALLOC_SCRATCH_MIB)");
  }
  char* base = scratch_ptr();
  const int64_t g0 = p->kinfo[k0].g_off;
  for (int kk = k0; kk < k1; ++kk) {
    const KInfo& ki = p->kinfo[kk];
    const int64_t sb_band = int64_t(ki.nstick) * p->N3 * csz;
    const int nbc = int(std::min<int64_t>(nbnd, avail / (sb_band + 3 * pq_band)));
    for (int b0 = 0; b0 < nbnd; b0 += nbc) {
      const int nb = std::min(nbc, nbnd - b0);
      HpsiWork wk;
      int64_t off = 0;
      wk.sbuf = base + off;
      off += align256(nb * sb_band);
      wk.P = reinterpret_cast<double2*>(base + off);
      off += align256(nb * pq_band);
      wk.Q = reinterpret_cast<double2*>(base + off);
      off += align256(nb * pq_band);
      wk.part = base + off;
      wk.part_bytes = int64_t(kScratchBytes) - off;
      const int64_t o = int64_t(nbnd) * (ki.g_off - g0) + int64_t(b0) * ki.npw;
      apply_h_slices(p, std::vector<KSlice>{KSlice{kk, nb, o, o}}, psi, hpsi, s, p->prec, nullptr,
                     nullptr, &wk);
    }
  }
}

}  // namespace qm

using namespace qm;

extern "C" qm_status qm_apply_h_noalloc(qm_hpsi_plan* plan, int32_t k, const void* psi, void* hpsi,
                                        int32_t nbnd, void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    apply_noalloc(plan, k, psi, hpsi, nbnd, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  } catch (const Error& e) {
    plan->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    plan->err = e.what();
    return QM_E_STATE;
  }
}
