// Real-time propagation of the time-dependent Kohn-Sham equations (Sec. 2.4; Sec. 5,
// 'tddft' module): the Taylor-series exponential exp(-i dt H) psi ~ sum_{r<=k} (-i dt)^r/r!
// H^r psi applied with the plan's H|psi>, and the enforced-time-reversal-symmetry (ETRS)
// step with the Hamiltonian rebuilt from the instantaneous density (Hartree-only model:
// V = V_ext + V_H[n(psi)]).
#include <cmath>
#include <cstring>

#include "qm_internal.h"

namespace qm {

// term <- (-i c) hterm, out += term (c = dt / r), over n complex entries
__global__ void k_taylor_term(double2* __restrict__ out, double2* __restrict__ term,
                              const double2* __restrict__ hterm, double c, int64_t n) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const double2 h = hterm[t];
    const double2 v = make_double2(c * h.y, -c * h.x);
    term[t] = v;
    const double2 o = out[t];
    out[t] = make_double2(o.x + v.x, o.y + v.y);
  }
}

struct TdWork {
  double2* term = nullptr;
  double2* hterm = nullptr;
  double2* half = nullptr;
  double2* bar = nullptr;
  double* rho = nullptr;
  double* vh = nullptr;
  double* vtot = nullptr;
  int64_t nband_elems = 0;
};

static TdWork* td_work(qm_hpsi_plan* p) {
  if (!p->td) {
    TdWork* w = new TdWork();
    try {
      const int64_t n = int64_t(p->nbnd_max) * p->npw_total;
      const int64_t nr = int64_t(p->N1) * p->N2 * p->N3;
      QM_HIP(hipMalloc(&w->term, size_t(n) * sizeof(double2)));
      QM_HIP(hipMalloc(&w->hterm, size_t(n) * sizeof(double2)));
      QM_HIP(hipMalloc(&w->half, size_t(n) * sizeof(double2)));
      QM_HIP(hipMalloc(&w->bar, size_t(n) * sizeof(double2)));
      QM_HIP(hipMalloc(&w->rho, size_t(nr) * sizeof(double)));
      QM_HIP(hipMalloc(&w->vh, size_t(nr) * sizeof(double)));
      QM_HIP(hipMalloc(&w->vtot, size_t(nr) * sizeof(double)));
      w->nband_elems = n;
    } catch (...) {
      void* q[] = {w->term, w->hterm, w->half, w->bar, w->rho, w->vh, w->vtot};
      for (void* x : q)
        if (x) (void)hipFree(x);
      delete w;
      throw;
    }
    p->td = w;
  }
  return p->td;
}

void td_free(qm_hpsi_plan* p) {
  if (!p->td) return;
  TdWork* w = p->td;
  void* q[] = {w->term, w->hterm, w->half, w->bar, w->rho, w->vh, w->vtot};
  for (void* x : q)
    if (x) (void)hipFree(x);
  delete w;
  p->td = nullptr;
}

// out = sum_{r=0}^{order} (-i dt)^r / r! H^r in, for the bands of k (-1: all k); in may equal out
static void expm_taylor(qm_hpsi_plan* p, int k, const void* in, void* out, int nbnd, double dt, int order,
                        hipStream_t s) {
  QM_REQUIRE(in && out, QM_E_ARG, "psi_in and psi_out must be non-NULL");
  QM_REQUIRE(nbnd >= 1 && nbnd <= p->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
  QM_REQUIRE(k >= -1 && k < p->nk, QM_E_ARG, "k out of range");
  QM_REQUIRE(order >= 1 && order <= 64, QM_E_ARG, "need 1 <= order <= 64");
  QM_REQUIRE(std::isfinite(dt), QM_E_ARG, "dt must be finite");
  TdWork* w = td_work(p);
  const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? p->nk : k + 1;
  const int64_t n = int64_t(nbnd) * (p->kinfo[k1 - 1].g_off + p->kinfo[k1 - 1].npw - p->kinfo[k0].g_off);
  QM_REQUIRE(n <= w->nband_elems, QM_E_STATE, "band block larger than the work buffers");
  QM_HIP(hipMemcpyAsync(w->term, in, size_t(n) * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (out != in) QM_HIP(hipMemcpyAsync(out, in, size_t(n) * sizeof(double2), hipMemcpyDeviceToDevice, s));
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 16384));
  for (int r = 1; r <= order; ++r) {
    const qm_status st = qm_apply_h(p, k, w->term, w->hterm, nbnd, s);
    if (st != QM_OK) throw Error(st, p->err);
    hipLaunchKernelGGL(k_taylor_term, dim3(blocks), dim3(256), 0, s, reinterpret_cast<double2*>(out),
                       w->term, w->hterm, dt / double(r), n);
    QM_HIP(hipGetLastError());
  }
}

// the Hartree-only H of the density of psi: V = V_ext + V_H[n(psi)] into the plan
static void set_h_of(qm_hpsi_plan* p, const double* vext, const double* kw, const double* occ,
                     const void* psi, int nbnd, hipStream_t s) {
  TdWork* w = p->td;
  qm_status st = qm_density(p, -1, psi, nbnd, kw, occ, w->rho, s);
  if (st == QM_OK) st = qm_hartree(p, w->rho, w->vh, nullptr, s);
  if (st != QM_OK) throw Error(st, p->err);
  grid_add(p, vext, w->vh, w->vtot, s);
  launch_vplan(p, w->vtot, s);
}

static void etrs_step(qm_hpsi_plan* p, const double* vext, const double* kw, const double* occ, void* psi,
                      int nbnd, double dt, int order, hipStream_t s) {
  QM_REQUIRE(vext && kw && occ && psi, QM_E_ARG, "vext, kweights, occ and psi must be non-NULL");
  QM_REQUIRE(p->nk <= kMaxSlices, QM_E_ARG, "at most 32 k-points");
  TdWork* w = td_work(p);
  set_h_of(p, vext, kw, occ, psi, nbnd, s);                  // H[psi_n]
  expm_taylor(p, -1, psi, w->half, nbnd, 0.5 * dt, order, s);
  expm_taylor(p, -1, psi, w->bar, nbnd, dt, order, s);
  set_h_of(p, vext, kw, occ, w->bar, nbnd, s);               // H[psi_bar]
  expm_taylor(p, -1, w->half, psi, nbnd, 0.5 * dt, order, s);
}

}  // namespace qm

using namespace qm;

extern "C" {

qm_status qm_expm_taylor(qm_hpsi_plan* plan, int32_t k, const void* psi_in, void* psi_out, int32_t nbnd,
                         double dt, int32_t order, void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    expm_taylor(plan, k, psi_in, psi_out, nbnd, dt, order, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  } catch (const Error& e) {
    plan->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    plan->err = e.what();
    return QM_E_STATE;
  }
}

qm_status qm_td_etrs(qm_hpsi_plan* plan, const double* vext_r, const double* kweights, const double* occ,
                     void* psi, int32_t nbnd, double dt, int32_t order, int32_t nsteps, void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    QM_REQUIRE(nsteps >= 0, QM_E_ARG, "nsteps must be >= 0");
    for (int i = 0; i < nsteps; ++i)
      etrs_step(plan, vext_r, kweights, occ, psi, nbnd, dt, order, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  } catch (const Error& e) {
    plan->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    plan->err = e.what();
    return QM_E_STATE;
  }
}

}  // extern "C"
