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

void launch_nonlocal_t(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi,
                       void* hpsi, hipStream_t s, StageEvents* ev, int lp) {
  if (p->nproj == 0) return;
  const int np = p->nproj;
  double2* P = reinterpret_cast<double2*>(p->proj_q);
  double2* Q = P + int64_t(p->nk) * np * p->nbnd_max;
  std::vector<GemmCN> cn;
  std::vector<GemmEX> ex;
  int64_t off = 0;
  for (const KSlice& x : sl) {
    const KInfo& ki = p->kinfo[x.k];
    const char* bbase = reinterpret_cast<const char*>(lp == 0 ? p->beta64 : p->beta_lp);
    const size_t esz = lp == 0 ? 16 : (lp == 1 ? 8 : 4);
    const void* bk = bbase + size_t(ki.beta_off) * esz;
    const double2* pk = reinterpret_cast<const double2*>(psi) + x.psi_off;
    double2* hk = reinterpret_cast<double2*>(hpsi) + x.hpsi_off;
    cn.push_back(GemmCN{bk, pk, P + off, np, x.nb, ki.npw, ki.npw, ki.npw, x.nb});
    ex.push_back(GemmEX{Q + off, bk, hk, x.nb, ki.npw, np, x.nb, ki.npw, ki.npw});
    off += int64_t(np) * x.nb;
  }
  zgemm_cn_batched(cn, 1.0, 0.0, p->proj_part, p->proj_part_bytes, s, ev, 3, lp);
  // D acts on each slice's [np][nb] block; blocks are packed back to back
  int64_t base = 0;
  for (const KSlice& x : sl) {
    const int64_t total = int64_t(np) * x.nb;
    const int blocks = int(std::min<int64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL(k_apply_d, dim3(blocks), dim3(256), 0, s, P + base, Q + base, p->dmat,
                       p->drange, np, x.nb, total);
    QM_HIP(hipGetLastError());
    base += total;
  }
  if (ev) ev->mark(5);
  zgemm_ex_batched(ex, 1.0, 1.0, s, lp);
  if (ev) ev->mark(6);
}

void launch_nonlocal(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                     hipStream_t s, qm_prec prec, StageEvents* ev) {
  const int lp = prec == QM_PREC_FP64 ? 0 : (prec == QM_PREC_FP32 ? 1 : 2);
  if (lp != 0 && p->beta_lp_kind != lp) convert_beta(p, prec, s);
  launch_nonlocal_t(p, sl, psi, hpsi, s, ev, lp);
}

// low-precision copy of beta for the FP32 (c64) or MIXED (bf16 pairs) projector GEMMs
void convert_beta(qm_hpsi_plan* p, qm_prec prec, hipStream_t s) {
  if (p->nproj == 0 || prec == QM_PREC_FP64) return;
  const int lp = prec == QM_PREC_FP32 ? 1 : 2;
  if (p->beta_lp_kind == lp) return;
  const int64_t n = int64_t(p->nproj) * p->npw_total;
  if (!p->beta_lp) QM_HIP(hipMalloc(&p->beta_lp, size_t(n) * 8));
  convert_beta_lp(p->beta64, p->beta_lp, n, lp, s);
  p->beta_lp_kind = lp;
}

}  // namespace qm
