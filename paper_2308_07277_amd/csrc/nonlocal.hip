// Kleinman-Bylander non-local term of H|psi> (Sec. 2.3, separable form
// sum_ij |beta_i> D_ij <beta_j|):  P = beta^dagger psi (CN GEMM),
// Q = D P (banded row ranges of D), H psi += beta Q (EX GEMM, accumulating).
#include "cplx.h"
#include "qm_internal.h"

namespace qm {

// Q[k](i, j) = sum_{l in range(i)} D(i, l) P[k](l, j); P, Q c128 [nproj][nbnd] per k
__global__ void k_apply_d(const double2* __restrict__ P, double2* __restrict__ Q,
                          const double* __restrict__ D, const int32_t* __restrict__ drange,
                          int nproj, int nbnd, int64_t total) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(t % nbnd);
    const int64_t r = t / nbnd;
    const int i = int(r % nproj);
    const int64_t kb = (r / nproj) * int64_t(nproj) * nbnd;
    const int lo = drange[2 * i], hi = drange[2 * i + 1];
    double sr = 0, si = 0;
    for (int l = lo; l < hi; ++l) {
      const double d = D[int64_t(i) * nproj + l];
      const double2 p = P[kb + int64_t(l) * nbnd + j];
      sr += d * p.x;
      si += d * p.y;
    }
    Q[t] = make_double2(sr, si);
  }
}

void launch_nonlocal_fp64(qm_hpsi_plan* p, int k0, int k1, int nbnd, const void* psi, void* hpsi,
                          hipStream_t s, StageEvents* ev) {
  if (p->nproj == 0) return;
  const int np = p->nproj;
  double2* P = reinterpret_cast<double2*>(p->proj_q);
  double2* Q = P + int64_t(p->nk) * np * p->nbnd_max;
  std::vector<GemmCN> cn;
  std::vector<GemmEX> ex;
  const int64_t g0 = p->kinfo[k0].g_off;
  for (int k = k0; k < k1; ++k) {
    const KInfo& ki = p->kinfo[k];
    const double2* bk = reinterpret_cast<const double2*>(p->beta64) + ki.beta_off;
    const double2* pk = reinterpret_cast<const double2*>(psi) + int64_t(nbnd) * (ki.g_off - g0);
    double2* hk = reinterpret_cast<double2*>(hpsi) + int64_t(nbnd) * (ki.g_off - g0);
    double2* Pk = P + int64_t(k - k0) * np * nbnd;
    double2* Qk = Q + int64_t(k - k0) * np * nbnd;
    cn.push_back(GemmCN{bk, pk, Pk, np, nbnd, ki.npw, ki.npw, ki.npw, nbnd});
    ex.push_back(GemmEX{Qk, bk, hk, nbnd, ki.npw, np, nbnd, ki.npw, ki.npw});
  }
  zgemm_cn_batched(cn, 1.0, 0.0, p->proj_part, p->proj_part_bytes, s, ev, 3);
  const int64_t total = int64_t(k1 - k0) * np * nbnd;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(k_apply_d, dim3(blocks), dim3(256), 0, s, P, Q, p->dmat, p->drange, np, nbnd,
                     total);
  QM_HIP(hipGetLastError());
  if (ev) ev->mark(5);
  zgemm_ex_batched(ex, 1.0, 1.0, s);
  if (ev) ev->mark(6);
}

void launch_nonlocal(qm_hpsi_plan* p, int k0, int k1, int nbnd, const void* psi, void* hpsi,
                     hipStream_t s, qm_prec prec, StageEvents* ev) {
  (void)prec;
  launch_nonlocal_fp64(p, k0, k1, nbnd, psi, hpsi, s, ev);
}

void convert_beta(qm_hpsi_plan*, qm_prec, hipStream_t) {}

}  // namespace qm
