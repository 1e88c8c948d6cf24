// Block Davidson for the lowest bands of H(k), all k-points of a call batched
// (Sec. 5 'dft' module: a Davidson that only needs H applied to trial blocks).
//
// Per iteration and active k:  corrections t_n = K(x) r_n for the unconverged
// bands (Teter-Payne-Allan, or the learned gain network), restart V = X when
// the basis would overflow, two block Gram-Schmidt passes against V and two
// CholQR passes, H t, extend the projected matrix by its new columns,
// Hermitian eigenproblem on the GPU (tridiagonalisation + bisection + inverse
// iteration), Ritz vectors X = V Y, HX = HV Y, residuals.  Convergence is the
// plain residual norm max_n ||H x_n - theta_n x_n|| <= tol.  The host only
// reads the per-band residual norms and Ritz values once per iteration.
#include <chrono>
#include <cmath>
#include <cstring>

#include <string>
#include <thread>

#include "dense.h"

namespace qm {

void mlp_precondition(qm_hpsi_plan* p, const DJobs& jobs, const void* weights, hipStream_t s,
                      const double2* R, double2* V, const int32_t* unconv, const double* tkin,
                      const double* theta, const double* resn, const int64_t* goff);

struct DavState {
  int nb = 0, mb = 0, k0 = 0, k1 = 0, nk = 0;
  int nwant = 0;             // bands returned and tested for convergence (nb minus buffer bands)
  int64_t g0 = 0, npl = 0;   // G offset of k0 and plane waves of k0..k1-1 (band block base)
  ProjScratch ps;            // own projector scratch (lanes only; else the plan's)
  bool ready = false;
  bool lowp = false;
  bool sub32 = false;        // float32-arithmetic subspace products while lowp
  double2 *V = nullptr, *HV = nullptr, *X = nullptr, *HX = nullptr, *R = nullptr, *TS = nullptr;
  double2 *Hs = nullptr, *Aw = nullptr, *Z = nullptr, *tau = nullptr, *Cw = nullptr, *G = nullptr,
          *W = nullptr;
  double *theta = nullptr, *d = nullptr, *e = nullptr, *resn = nullptr, *tkin = nullptr,
         *yw = nullptr, *fw = nullptr;
  int32_t *unconv = nullptr, *info = nullptr;
  double* cgs_ovl = nullptr;     // [k] overlap left after the first Gram-Schmidt pass
  int64_t* goff = nullptr;
  TrdWork trd{};
  EigWork ew{};
  double* chol_dmax = nullptr;   // [k] largest Gram diagonal (Cholesky pivot test)
  double2* chol_ld = nullptr;    // [k][nb / 16 rounded up][16][16] diagonal blocks of L
  double2* bt_t = nullptr;       // [k][mb / 32 rounded up][32][32] T factors of the back-transform
  void* work = nullptr;
  int64_t work_bytes = 0;
  double *h_resn = nullptr, *h_theta = nullptr;
  int32_t *h_unconv = nullptr, *h_info = nullptr;
  double* h_cgs_ovl = nullptr;
  std::vector<int> m, it, done;
  // qm_davidson_solve: Ritz vectors, H Ritz vectors and residuals only for the bands being
  // corrected (the rest before a restart, a precision switch, a convergence verdict and the
  // return); stale[k]: some rows of X and HX predate the last Rayleigh-Ritz step of k, whose
  // refreshed bands are lastact[k]
  bool lazy = false;
  std::vector<char> stale;
  std::vector<std::vector<int32_t>> lastact;
  int32_t* slist = nullptr;      // [k][nb] device list of the stale bands being completed
  int32_t* h_slist = nullptr;
  int64_t n_hpsi = 0, n_hpsi_lowp = 0;
  int64_t n_cgs = 0, n_cgs2 = 0;   // Gram-Schmidt calls per k, and those that took a second pass
  double tol = 1e-8;
  std::vector<double> hist;  // max residual per step (precision-ladder stagnation test)
  double* estar = nullptr;   // converged eigenvalues for training-pair generation
  double t_hpsi = 0, t_sub = 0, t_eig = 0;
  hipEvent_t ev[8] = {};     // 0-1 H application, 2-3 eigenproblem, 4-5 orthonormalisation,
                             // 6-7 Ritz vectors and residuals
};

static void dav_release(DavState* d) {
  void* dev[] = {d->V, d->HV, d->X, d->HX, d->R, d->TS, d->Hs, d->Aw, d->Z, d->tau, d->Cw, d->G,
                 d->W, d->theta, d->d, d->e, d->resn, d->tkin, d->yw, d->fw, d->unconv, d->info,
                 d->goff, d->work, d->estar, d->ps.part, d->trd.v, d->trd.w, d->trd.part, d->trd.cnt, d->trd.bcnt, d->trd.prow,
                 d->ew.sc, d->ew.nrm, d->chol_dmax, d->chol_ld, d->bt_t, d->cgs_ovl, d->slist};
  for (void* q : dev)
    if (q) (void)hipFree(q);
  void* host[] = {d->h_resn, d->h_theta, d->h_unconv, d->h_info, d->h_cgs_ovl, d->h_slist};
  for (void* q : host)
    if (q) (void)hipHostFree(q);
  for (hipEvent_t& e : d->ev)
    if (e) (void)hipEventDestroy(e);
  delete d;
}

void davidson_free(qm_hpsi_plan* p) {
  if (p->dav) dav_release(p->dav);
  p->dav = nullptr;
  for (DavState* d : p->dav_lanes)
    if (d) dav_release(d);
  p->dav_lanes.clear();
  for (hipStream_t q : p->lane_streams)
    if (q) (void)hipStreamDestroy(q);
  p->lane_streams.clear();
}

template <typename T>
static T* dalloc(size_t n) {
  T* q = nullptr;
  QM_HIP(hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
  return q;
}

static DavState* dav_create(qm_hpsi_plan* p, int k0, int k1, int nb, int mb, bool own_scratch) {
  DavState* d = new DavState();
  try {
    d->nb = nb;
    d->mb = mb;
    d->k0 = k0;
    d->k1 = k1;
    d->nk = p->nk;
    d->g0 = p->kinfo[k0].g_off;
    d->npl = p->kinfo[k1 - 1].g_off + p->kinfo[k1 - 1].npw - d->g0;
    const size_t np = size_t(d->npl), nk = size_t(p->nk);
    if (own_scratch && p->proj_part_bytes > 0) {
      d->ps.bytes = p->proj_part_bytes;
      d->ps.part = dalloc<char>(size_t(d->ps.bytes));
    }
    d->V = dalloc<double2>(size_t(mb) * np);
    d->HV = dalloc<double2>(size_t(mb) * np);
    d->X = dalloc<double2>(size_t(nb) * np);
    d->HX = dalloc<double2>(size_t(nb) * np);
    d->R = dalloc<double2>(size_t(nb) * np);
    d->TS = dalloc<double2>(size_t(nb) * np);
    d->Hs = dalloc<double2>(nk * mb * mb);
    d->Aw = dalloc<double2>(nk * mb * mb);
    d->Z = dalloc<double2>(nk * mb * nb);
    d->tau = dalloc<double2>(nk * mb);
    d->Cw = dalloc<double2>(nk * mb * nb);
    d->G = dalloc<double2>(nk * nb * nb);
    d->W = dalloc<double2>(nk * nb * nb);
    d->theta = dalloc<double>(nk * mb);
    d->d = dalloc<double>(nk * mb);
    d->e = dalloc<double>(nk * mb);
    d->resn = dalloc<double>(nk * nb);
    d->tkin = dalloc<double>(nk * nb);
    d->yw = dalloc<double>(nk * nb * mb);
    d->fw = dalloc<double>(nk * nb * 3 * mb);
    d->unconv = dalloc<int32_t>(nk * nb);
    d->info = dalloc<int32_t>(nk);
    d->cgs_ovl = dalloc<double>(nk);
    d->goff = dalloc<int64_t>(nk);
    QM_REQUIRE(mb <= kTrdMaxBasis, QM_E_ARG, "max_basis above the tridiagonalisation limit (2048)");
    d->trd.v = dalloc<double2>(nk * 2 * mb);
    d->trd.w = dalloc<double2>(nk * mb);
    d->trd.ptiles = trd_tile_slots(mb);
    d->trd.part = dalloc<double2>(nk * size_t(d->trd.ptiles) * 2 * kTrdTile);
    d->trd.cnt = dalloc<uint32_t>(nk);
    d->trd.nblk = (mb + kTrdTile - 1) / kTrdTile;
    d->trd.bcnt = dalloc<uint32_t>(nk * size_t(d->trd.nblk));
    d->trd.prow = dalloc<double2>(nk * mb);
    d->trd.fin_min = p->trd_fin_min;
    d->ew.sc = dalloc<double>(nk * nb);
    d->ew.nrm = dalloc<double>(nk);
    d->chol_dmax = dalloc<double>(nk);
    d->chol_ld = dalloc<double2>(nk * size_t((nb + kCholBlk - 1) / kCholBlk) * kCholBlk * kCholBlk);
    d->bt_t = dalloc<double2>(nk * size_t((mb + kBtBlk - 1) / kBtBlk) * kBtBlk * kBtBlk);
    std::vector<int64_t> go(nk);
    for (size_t k = 0; k < nk; ++k) go[k] = p->kinfo[k].g_off;
    QM_HIP(hipMemcpy(d->goff, go.data(), nk * sizeof(int64_t), hipMemcpyHostToDevice));
    d->work_bytes = int64_t(16) * int64_t(nk) * mb * nb * int64_t(sizeof(double2));
    d->work = dalloc<char>(size_t(d->work_bytes));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_resn), nk * nb * 2 * sizeof(double)));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_theta), nk * mb * sizeof(double)));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_unconv), nk * nb * sizeof(int32_t)));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_info), nk * sizeof(int32_t)));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_cgs_ovl), nk * sizeof(double)));
    QM_HIP(hipHostMalloc(reinterpret_cast<void**>(&d->h_slist), nk * nb * sizeof(int32_t)));
    d->slist = dalloc<int32_t>(nk * nb);
    for (hipEvent_t& e : d->ev) QM_HIP(hipEventCreate(&e));
    const void* big[] = {reinterpret_cast<const void*>(&k_tridiag), reinterpret_cast<const void*>(&k_eig_vals),
                         reinterpret_cast<const void*>(&k_chol_inv_cols),
                         reinterpret_cast<const void*>(&k_bt_apply)};
    for (const void* f : big) QM_HIP(allow_full_lds(f));
    d->m.assign(nk, 0);
    d->it.assign(nk, 0);
    d->done.assign(nk, 0);
    d->stale.assign(nk, 0);
    d->lastact.assign(nk, {});
  } catch (...) {
    dav_release(d);
    throw;
  }
  return d;
}

static double2* vrow(DavState* d, double2* base, const DJob& j, int row) {
  return base + j.voff + int64_t(row) * j.npw;
}

static void timed_apply(qm_hpsi_plan* p, DavState* d, const std::vector<KSlice>& sl, const void* in,
                        void* out, hipStream_t s, bool lowp) {
  QM_HIP(hipEventRecord(d->ev[0], s));
  apply_h_slices(p, sl, in, out, s, lowp ? p->prec : QM_PREC_FP64, nullptr, d->ps.part ? &d->ps : nullptr,
                 nullptr, false);
  QM_HIP(hipEventRecord(d->ev[1], s));
  QM_HIP(hipEventSynchronize(d->ev[1]));
  float ms = 0.f;
  QM_HIP(hipEventElapsedTime(&ms, d->ev[0], d->ev[1]));
  d->t_hpsi += ms;
  int64_t nb = 0;
  for (const KSlice& x : sl) nb += x.nb;
  d->n_hpsi += nb;
  if (lowp && p->prec != QM_PREC_FP64) d->n_hpsi_lowp += nb;
}

// Cholesky G = L L^H of every job's Gram matrix and W = conj(Linv)^T: blocked on many
// workgroups when the inverse's column block fits in LDS, else one workgroup per job.
static void cholesky_inverse(qm_hpsi_plan* p, DavState* d, const DJobs& jobs, hipStream_t s) {
  if (d->nb > kCholMaxBlocked || p->chol_forced == 1) {
    hipLaunchKernelGGL(k_chol_inv, dim3(jobs.n), dim3(1024), 0, s, jobs, d->G, d->W, d->info);
    QM_HIP(hipGetLastError());
    return;
  }
  int numax = 0;
  for (int i = 0; i < jobs.n; ++i) numax = std::max(numax, jobs.j[i].nu);
  const int nblk = (numax + kCholBlk - 1) / kCholBlk;
  hipLaunchKernelGGL(k_chol_prep, dim3(jobs.n), dim3(256), 0, s, jobs, d->G, d->chol_dmax);
  for (int jb = 0; jb < nblk; ++jb)
    hipLaunchKernelGGL(k_chol_col, dim3(nblk - jb, jobs.n), dim3(256), 0, s, jobs, jb, d->G,
                       d->chol_ld, d->chol_dmax, d->info);
  hipLaunchKernelGGL(k_chol_inv_cols, dim3(nblk, jobs.n), dim3(256),
                     size_t(nblk) * kCholBlk * kCholBlk * sizeof(double2), s, jobs, d->G, d->chol_ld,
                     d->W, d->info);
  QM_HIP(hipGetLastError());
}

// Subspace products (Gram-Schmidt, CholQR, projected matrix, Ritz vectors) run in float64
// unless the caller opts in (qm_dav_opts.subspace_fp32) to float32 arithmetic on the float64
// basis while H itself runs in reduced precision: there the basis only has to be accurate
// to the reduced-precision H.  From the switch on they are float64 either way.
static int subspace_lp(const DavState* d) { return (d->lowp && d->sub32) ? 3 : 0; }

// T = rows [m - nu, m) of V (unit columns); orthogonalise against rows [0, m - nu) by
// classical Gram-Schmidt and orthonormalise (two CholQR passes).  The second Gram-Schmidt
// pass runs for the k-points where the first one removed more than half of some column's
// squared norm (Kahan-Parlett "twice is enough": a column that keeps at least 1/sqrt 2 of its
// norm is orthogonal to the basis to working precision after one pass), and always in the
// float32-arithmetic subspace mode.  Returns false if a Gram matrix was not positive definite.
static bool orthonormalise(qm_hpsi_plan* p, DavState* d, const DJobs& jobs, hipStream_t s) {
  const int lp = subspace_lp(d);
  std::vector<GemmCN> cn;
  std::vector<GemmEX> ex;
  QM_HIP(hipEventRecord(d->ev[4], s));
  // cleared once here and only ever set by a failed pivot, so a failure in the first CholQR
  // pass is still reported after the second
  QM_HIP(hipMemsetAsync(d->info, 0, sizeof(int32_t) * d->nk, s));
  DJobs again = jobs;   // the jobs of the second pass
  for (int pass = 0; pass < 2; ++pass) {
    const DJobs& js = pass == 0 ? jobs : again;
    cn.clear();
    ex.clear();
    for (int i = 0; i < js.n; ++i) {
      const DJob& j = js.j[i];
      const int base = j.m - j.nu;
      if (base == 0) continue;
      double2* T = vrow(d, d->V, j, base);
      double2* C = d->Cw + int64_t(j.k) * d->mb * d->nb;
      cn.push_back(GemmCN{vrow(d, d->V, j, 0), T, C, base, j.nu, j.npw, j.npw, j.npw, d->nb});
      ex.push_back(GemmEX{C, vrow(d, d->V, j, 0), T, j.nu, j.npw, base, d->nb, j.npw, j.npw});
    }
    if (cn.empty()) break;
    zgemm_cn_batched(cn, 1.0, 0.0, d->work, d->work_bytes, s, nullptr, 0, lp);
    if (pass == 0 && lp == 0) {
      hipLaunchKernelGGL(k_cgs_overlap, dim3(jobs.n), dim3(256), 0, s, jobs, d->Cw, d->cgs_ovl);
      QM_HIP(hipGetLastError());
      QM_HIP(hipMemcpyAsync(d->h_cgs_ovl, d->cgs_ovl, sizeof(double) * d->nk, hipMemcpyDeviceToHost, s));
    }
    zgemm_ex_batched(ex, -1.0, 1.0, s, lp);
    if (pass == 0 && lp == 0) {
      QM_HIP(hipStreamSynchronize(s));
      again.n = 0;
      for (int i = 0; i < jobs.n; ++i) {
        const DJob& j = jobs.j[i];
        if (j.m - j.nu > 0 && !(d->h_cgs_ovl[j.k] <= 0.5)) again.j[again.n++] = j;
      }
      d->n_cgs2 += again.n;
      d->n_cgs += jobs.n;
    }
  }
  for (int pass = 0; pass < 2; ++pass) {
    cn.clear();
    ex.clear();
    for (int i = 0; i < jobs.n; ++i) {
      const DJob& j = jobs.j[i];
      double2* T = pass == 0 ? vrow(d, d->V, j, j.m - j.nu) : d->TS + j.xoff;
      double2* O = pass == 0 ? d->TS + j.xoff : vrow(d, d->V, j, j.m - j.nu);
      double2* Gk = d->G + int64_t(j.k) * d->nb * d->nb;
      double2* Wk = d->W + int64_t(j.k) * d->nb * d->nb;
      cn.push_back(GemmCN{T, T, Gk, j.nu, j.nu, j.npw, j.npw, j.npw, d->nb});
      ex.push_back(GemmEX{Wk, T, O, j.nu, j.npw, j.nu, d->nb, j.npw, j.npw});
    }
    zgemm_cn_batched(cn, 1.0, 0.0, d->work, d->work_bytes, s, nullptr, 0, lp);
    cholesky_inverse(p, d, jobs, s);
    zgemm_ex_batched(ex, 1.0, 0.0, s, lp);
  }
  QM_HIP(hipEventRecord(d->ev[5], s));
  QM_HIP(hipMemcpyAsync(d->h_info, d->info, sizeof(int32_t) * d->nk, hipMemcpyDeviceToHost, s));
  QM_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  QM_HIP(hipEventElapsedTime(&ms, d->ev[4], d->ev[5]));
  d->t_sub += ms;
  for (int i = 0; i < jobs.n; ++i)
    if (d->h_info[jobs.j[i].k] != 0) return false;
  return true;
}

// Basis size from which the tridiagonalisation runs on many workgroups per k-point (one
// launch per step) instead of one workgroup per k-point.
constexpr int kTrdMultiMin = 192;

static void tridiagonalise(qm_hpsi_plan* p, DavState* d, const DJobs& jobs, hipStream_t s) {
  int mmax = 0;
  for (int i = 0; i < jobs.n; ++i) mmax = std::max(mmax, jobs.j[i].m);
  const bool multi = p->trd_forced == 2 || mmax > kTridiagMaxM ||
                     (p->trd_forced != 1 && mmax >= kTrdMultiMin);
  if (!multi) {
    hipLaunchKernelGGL(k_tridiag, dim3(jobs.n), dim3(1024), size_t(20) * mmax * sizeof(double2), s,
                       jobs, d->Aw, d->d, d->e, d->tau, mmax);
    QM_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(k_trd_start, dim3(jobs.n), dim3(256), 0, s, jobs, d->Aw, d->d, d->e, d->tau,
                     d->trd);
  QM_HIP(hipGetLastError());
  for (int j = 0; j <= mmax - 2; ++j) {
    int gx = 0;
    for (int i = 0; i < jobs.n; ++i) {
      const int m = jobs.j[i].m;
      if (j >= m - 1) continue;
      const int nt = (m - 1) / kTrdTile - (j + 1) / kTrdTile + 1;
      gx = std::max(gx, nt * (nt + 1) / 2);
    }
    hipLaunchKernelGGL(k_trd_step, dim3(gx, jobs.n), dim3(256), 0, s, jobs, j, d->Aw, d->d, d->e,
                       d->tau, d->trd);
  }
  QM_HIP(hipGetLastError());
}

// Projected matrix columns [m_old, m), eigenproblem, Ritz vectors and residuals.
// lazy: X, HX and the residuals only for each job's nu bands listed in d->unconv (the bands
// being corrected this step); the other rows of X and HX are left as they were (stale)
static void rayleigh_ritz(qm_hpsi_plan* p, DavState* d, const DJobs& jobs, hipStream_t s,
                          bool lazy = false) {
  const int lp = subspace_lp(d);
  std::vector<GemmCN> cn;
  QM_HIP(hipEventRecord(d->ev[6], s));
  for (int i = 0; i < jobs.n; ++i) {
    const DJob& j = jobs.j[i];
    double2* Hk = d->Hs + int64_t(j.k) * d->mb * d->mb;
    cn.push_back(GemmCN{vrow(d, d->V, j, 0), vrow(d, d->HV, j, j.m_old), Hk + j.m_old, j.m,
                        j.m - j.m_old, j.npw, j.npw, j.npw, d->mb});
  }
  zgemm_cn_batched(cn, 1.0, 0.0, d->work, d->work_bytes, s, nullptr, 0, lp);
  hipLaunchKernelGGL(k_hs_fill, dim3(64, jobs.n), dim3(256), 0, s, jobs, d->Hs);
  hipLaunchKernelGGL(k_hs_copy, dim3(64, jobs.n), dim3(256), 0, s, jobs, d->Hs, d->Aw);
  QM_HIP(hipGetLastError());
  QM_HIP(hipEventRecord(d->ev[2], s));
  tridiagonalise(p, d, jobs, s);
  int mmax = 0;
  for (int i = 0; i < jobs.n; ++i) mmax = std::max(mmax, jobs.j[i].m);
  const int nw = std::min(d->nb, mmax);
  hipLaunchKernelGGL(k_eig_vals, dim3((nw + 3) / 4, jobs.n), dim3(256), size_t(3) * d->mb * sizeof(double),
                     s, jobs, d->d, d->e, d->theta, d->ew);
  QM_HIP(hipGetLastError());
  for (int step = 0; step < 3; ++step) {   // inverse iteration, clusters re-orthogonalised
    hipLaunchKernelGGL(k_eig_inviter, dim3((nw + 63) / 64, jobs.n), dim3(64),
                       size_t(2) * d->mb * sizeof(double), s, jobs, d->d, d->e, d->theta, d->yw,
                       d->fw, d->ew, step);
    hipLaunchKernelGGL(k_eig_orth, dim3(nw, jobs.n), dim3(256), 0, s, jobs, d->theta, d->yw, d->ew);
  }
  QM_HIP(hipGetLastError());
  // blocked back-transform: T factors of every 32-reflector block, then the eigenvector
  // slices (Z slice, partial sums and W must fit in the 160 KiB of LDS next to the 17 KiB T)
  const int nblk_bt = (mmax - 1 + kBtBlk - 1) / kBtBlk;
  if (nblk_bt > 0)
    hipLaunchKernelGGL(k_bt_tfactor, dim3(nblk_bt, jobs.n), dim3(256), 0, s, jobs, d->Aw, d->tau, d->bt_t);
  const int64_t per_col = (int64_t(d->mb) + 9 * kBtBlk) * int64_t(sizeof(double2));
  const int cols = std::max(1, std::min<int>(8, int((160 * 1024 - 18 * 1024) / per_col)));
  hipLaunchKernelGGL(k_bt_apply, dim3((d->nb + cols - 1) / cols, jobs.n), dim3(256),
                     size_t(per_col) * cols, s, jobs, d->Aw, d->bt_t, d->yw, d->ew.sc, d->Z, cols);
  QM_HIP(hipGetLastError());
  QM_HIP(hipEventRecord(d->ev[3], s));
  std::vector<GemmEX> ex;
  for (int i = 0; i < jobs.n; ++i) {
    const DJob& j = jobs.j[i];
    double2* Zk = d->Z + int64_t(j.k) * d->mb * d->nb;
    const int32_t* rows = lazy ? d->unconv + int64_t(j.k) * d->nb : nullptr;
    const int nr = lazy ? j.nu : d->nb;
    ex.push_back(GemmEX{Zk, vrow(d, d->V, j, 0), d->X + j.xoff, nr, j.npw, j.m, d->nb, j.npw, j.npw, rows});
    ex.push_back(GemmEX{Zk, vrow(d, d->HV, j, 0), d->HX + j.xoff, nr, j.npw, j.m, d->nb, j.npw, j.npw, rows});
    if (lazy) {
      d->lastact[j.k].assign(d->h_unconv + int64_t(j.k) * d->nb, d->h_unconv + int64_t(j.k) * d->nb + j.nu);
      d->stale[j.k] = j.nu < d->nb;
    } else {
      d->stale[j.k] = 0;
    }
  }
  zgemm_ex_batched(ex, 1.0, 0.0, s, lp);
  hipLaunchKernelGGL(k_residual, dim3(d->nb, jobs.n), dim3(256), 0, s, jobs, d->X, d->HX, d->R,
                     d->theta, p->g.kin, d->goff, d->resn, d->tkin, lazy ? d->unconv : nullptr);
  QM_HIP(hipGetLastError());
  QM_HIP(hipEventRecord(d->ev[7], s));
  QM_HIP(hipMemcpyAsync(d->h_resn, d->resn, sizeof(double) * d->nk * d->nb, hipMemcpyDeviceToHost, s));
  QM_HIP(hipMemcpyAsync(d->h_theta, d->theta, sizeof(double) * d->nk * d->mb, hipMemcpyDeviceToHost, s));
  QM_HIP(hipStreamSynchronize(s));
  float ms = 0.f, ms_h = 0.f, ms_r = 0.f;
  QM_HIP(hipEventElapsedTime(&ms, d->ev[2], d->ev[3]));
  QM_HIP(hipEventElapsedTime(&ms_h, d->ev[6], d->ev[2]));
  QM_HIP(hipEventElapsedTime(&ms_r, d->ev[3], d->ev[7]));
  d->t_eig += ms;
  d->t_sub += ms_h + ms_r;
}

static DJob make_job(qm_hpsi_plan* p, DavState* d, int k) {
  DJob j{};
  j.k = k;
  j.npw = p->kinfo[k].npw;
  j.voff = int64_t(d->mb) * (p->kinfo[k].g_off - d->g0);
  j.xoff = int64_t(d->nb) * (p->kinfo[k].g_off - d->g0);
  return j;
}

// Bring the stale rows of X and HX of the k-points ks up to date with their last
// Rayleigh-Ritz step (whose Z, V and HV are still in place), and with resid their residuals
// too (host copy of the norms refreshed).
static void complete_ritz(qm_hpsi_plan* p, DavState* d, const std::vector<int>& ks, bool resid,
                          hipStream_t s) {
  DJobs cj{};
  cj.nb = d->nb;
  cj.mb = d->mb;
  std::vector<char> mark(size_t(d->nb));
  for (int k : ks) {
    if (!d->stale[k]) continue;
    std::fill(mark.begin(), mark.end(), 0);
    for (int32_t b : d->lastact[k]) mark[size_t(b)] = 1;
    int cnt = 0;
    for (int b = 0; b < d->nb; ++b)
      if (!mark[size_t(b)]) d->h_slist[int64_t(k) * d->nb + cnt++] = b;
    DJob j = make_job(p, d, k);
    j.m = d->m[k];
    j.nu = cnt;
    cj.j[cj.n++] = j;
    d->stale[k] = 0;
  }
  if (cj.n == 0) return;
  QM_HIP(hipMemcpyAsync(d->slist, d->h_slist, sizeof(int32_t) * d->nk * d->nb, hipMemcpyHostToDevice, s));
  std::vector<GemmEX> ex;
  for (int i = 0; i < cj.n; ++i) {
    const DJob& j = cj.j[i];
    double2* Zk = d->Z + int64_t(j.k) * d->mb * d->nb;
    const int32_t* rows = d->slist + int64_t(j.k) * d->nb;
    ex.push_back(GemmEX{Zk, vrow(d, d->V, j, 0), d->X + j.xoff, j.nu, j.npw, j.m, d->nb, j.npw, j.npw, rows});
    ex.push_back(GemmEX{Zk, vrow(d, d->HV, j, 0), d->HX + j.xoff, j.nu, j.npw, j.m, d->nb, j.npw, j.npw, rows});
  }
  zgemm_ex_batched(ex, 1.0, 0.0, s, 0);
  if (resid) {
    hipLaunchKernelGGL(k_residual, dim3(d->nb, cj.n), dim3(256), 0, s, cj, d->X, d->HX, d->R,
                       d->theta, p->g.kin, d->goff, d->resn, d->tkin, d->slist);
    QM_HIP(hipGetLastError());
    QM_HIP(hipMemcpyAsync(d->h_resn, d->resn, sizeof(double) * d->nk * d->nb, hipMemcpyDeviceToHost, s));
  }
  QM_HIP(hipStreamSynchronize(s));   // (h_slist is rewritten by the next call)
}

// copy X (and HX) of the job's k into basis rows [0, nb) after re-orthonormalising X by CholQR
static bool restart_basis(qm_hpsi_plan* p, DavState* d, std::vector<DJob>& js, hipStream_t s) {
  for (DJob& j : js) {
    QM_HIP(hipMemcpyAsync(vrow(d, d->V, j, 0), d->X + j.xoff, sizeof(double2) * d->nb * j.npw,
                          hipMemcpyDeviceToDevice, s));
    QM_HIP(hipMemcpyAsync(vrow(d, d->HV, j, 0), d->HX + j.xoff, sizeof(double2) * d->nb * j.npw,
                          hipMemcpyDeviceToDevice, s));
  }
  (void)p;
  return true;
}

struct StepResult {
  int n_unconv = 0;
  double max_res = 0.0;
  bool nan = false;
};

// Every unconverged band (buffer bands too) is listed for correction; only the wanted ones
// count towards convergence and the reported maximum.
static void collect(qm_hpsi_plan* p, DavState* d, double tol, StepResult& r) {
  (void)p;
  for (int k = d->k0; k < d->k1; ++k) {
    if (d->done[k]) continue;
    int nu = 0, nuw = 0;
    for (int n = 0; n < d->nb; ++n) {
      const double x = d->h_resn[int64_t(k) * d->nb + n];
      if (!std::isfinite(x)) r.nan = true;
      if (n < d->nwant) r.max_res = std::max(r.max_res, x);
      if (!(x <= tol)) {
        d->h_unconv[int64_t(k) * d->nb + nu++] = n;
        if (n < d->nwant) ++nuw;
      }
    }
    r.n_unconv += nuw;
    if (nuw == 0) d->done[k] = 1;
  }
}

static void write_outputs(qm_hpsi_plan* p, DavState* d, void* psi, double* eig, double* resnorm,
                          hipStream_t s) {
  const int64_t g0 = p->kinfo[d->k0].g_off;
  for (int k = d->k0; k < d->k1; ++k) {
    const KInfo& ki = p->kinfo[k];
    if (psi)
      QM_HIP(hipMemcpyAsync(reinterpret_cast<double2*>(psi) + int64_t(d->nwant) * (ki.g_off - g0),
                            d->X + int64_t(d->nb) * (ki.g_off - g0), sizeof(double2) * d->nwant * ki.npw,
                            hipMemcpyDeviceToDevice, s));
    for (int n = 0; n < d->nwant; ++n) {
      if (eig) eig[int64_t(k - d->k0) * d->nwant + n] = d->h_theta[int64_t(k) * d->mb + n];
      if (resnorm) resnorm[int64_t(k - d->k0) * d->nwant + n] = d->h_resn[int64_t(k) * d->nb + n];
    }
  }
  QM_HIP(hipStreamSynchronize(s));
}

// One Davidson iteration on k-points k0..k1-1 with the state in *slot (created or rebuilt as
// needed).  psi points at k0's first band, eig and resnorm at k0's first entry.
static qm_status dav_step_range(qm_hpsi_plan* p, DavState** slot, bool own_scratch, int k0, int k1,
                                void* psi, double* eig, double* resnorm, int nwant,
                                const qm_dav_opts* o, int32_t* n_unconv, hipStream_t s,
                                bool lazy = false) {
  QM_REQUIRE(nwant >= 1, QM_E_ARG, "need nbnd >= 1");
  QM_REQUIRE(!o || o->extra_bands >= 0, QM_E_ARG, "extra_bands must be >= 0");
  QM_REQUIRE(!o || o->subspace_fp32 == 0 || o->subspace_fp32 == 1, QM_E_ARG,
             "subspace_fp32 must be 0 or 1");
  const int nb = nwant + (o ? o->extra_bands : 0);   // block size: wanted + buffer bands
  QM_REQUIRE(nb <= p->nbnd_max, QM_E_ARG, "need nbnd + extra_bands <= nbnd_max");
  QM_REQUIRE(k0 >= 0 && k0 < k1 && k1 <= p->nk, QM_E_ARG, "k out of range");
  QM_REQUIRE(psi, QM_E_ARG, "psi must be non-NULL");
  const double tol = (o && o->tol > 0) ? o->tol : 1e-8;
  int mb = (o && o->max_basis > 0) ? o->max_basis : 4 * nb;
  QM_REQUIRE(mb >= 2 * nb, QM_E_ARG, "max_basis must be at least 2 nbnd");
  QM_REQUIRE(mb <= 2000, QM_E_ARG, "max_basis above 2000 is not supported");
  const int precond = o ? o->precond : QM_PRECOND_TETER;
  QM_REQUIRE(precond == QM_PRECOND_TETER || (precond == QM_PRECOND_MLP && o->mlp_weights),
             QM_E_ARG, "QM_PRECOND_MLP needs mlp_weights");
  QM_REQUIRE(k1 - k0 <= kMaxSlices, QM_E_ARG, "at most 32 k-points per Davidson call");
  DavState* d = *slot;
  const bool fresh = !d || !d->ready || (o && o->restart) || d->k0 != k0 || d->k1 != k1 ||
                     d->nb != nb || d->mb != mb || d->nwant != nwant;
  if (fresh) {
    if (!d || d->k0 != k0 || d->k1 != k1 || d->nb != nb || d->mb != mb) {
      if (d) dav_release(d);
      *slot = d = nullptr;
      *slot = d = dav_create(p, k0, k1, nb, mb, own_scratch);
    }
    d->ready = false;
    d->nwant = nwant;
    std::fill(d->m.begin(), d->m.end(), 0);
    std::fill(d->it.begin(), d->it.end(), 0);
    std::fill(d->done.begin(), d->done.end(), 0);
    d->n_hpsi = d->n_hpsi_lowp = 0;
    d->n_cgs = d->n_cgs2 = 0;
    d->t_hpsi = d->t_sub = d->t_eig = 0;
    d->lowp = o && o->switch_resid > 0.0 && p->prec != QM_PREC_FP64;
    d->sub32 = o && o->subspace_fp32 != 0;
    std::fill(d->stale.begin(), d->stale.end(), 0);
  }
  d->lazy = lazy;
  DJobs jobs{};
  jobs.nb = nb;
  jobs.mb = mb;
  std::vector<KSlice> sl;
  if (!d->ready) {
    const int64_t g0 = p->kinfo[k0].g_off;
    for (int kk = k0; kk < k1; ++kk) {
      DJob j = make_job(p, d, kk);
      QM_HIP(hipMemcpyAsync(vrow(d, d->V, j, 0),
                            reinterpret_cast<const double2*>(psi) + int64_t(nwant) * (p->kinfo[kk].g_off - g0),
                            sizeof(double2) * nwant * j.npw, hipMemcpyDeviceToDevice, s));
      j.m = nb;
      j.m_old = 0;
      j.nu = nb;
      jobs.j[jobs.n++] = j;
      sl.push_back(KSlice{kk, nb, j.voff, j.voff});
    }
    if (nb > nwant) {   // buffer bands: a fixed pseudo-random start
      hipLaunchKernelGGL(k_start_block, dim3(nb - nwant, jobs.n), dim3(256), 0, s, jobs, d->V, nwant);
      QM_HIP(hipGetLastError());
    }
    if (!orthonormalise(p, d, jobs, s)) throw Error(QM_E_NOT_SPD, "start block is linearly dependent");
    timed_apply(p, d, sl, d->V, d->HV, s, d->lowp);
    rayleigh_ritz(p, d, jobs, s);
    for (int i = 0; i < jobs.n; ++i) d->m[jobs.j[i].k] = nb;
    d->ready = true;
  } else {
    // precision ladder: leave the reduced-precision H once the residual is small enough,
    // rebuilding the basis from the Ritz vectors with float64 H
    double maxres = 0.0;
    for (int kk = k0; kk < k1; ++kk)
      for (int n = 0; n < nwant; ++n) maxres = std::max(maxres, d->h_resn[int64_t(kk) * nb + n]);
    // switch when below switch_resid, or when the reduced-precision H stops making progress
    // (max residual not down by 20% over the last four iterations)
    bool stagnant = false;
    const size_t nh = d->hist.size();
    if (nh >= 5) stagnant = d->hist[nh - 1] > 0.8 * d->hist[nh - 5];
    const bool refresh = d->lowp && o && (maxres <= o->switch_resid || stagnant);
    if (refresh) {
      d->lowp = false;
      {
        std::vector<int> ks;
        for (int kk = k0; kk < k1; ++kk)
          if (!d->done[kk]) ks.push_back(kk);
        complete_ritz(p, d, ks, false, s);   // the new basis is every Ritz vector
      }
      for (int kk = k0; kk < k1; ++kk) {
        if (d->done[kk]) continue;
        DJob j = make_job(p, d, kk);
        QM_HIP(hipMemcpyAsync(vrow(d, d->V, j, 0), d->X + j.xoff, sizeof(double2) * nb * j.npw,
                              hipMemcpyDeviceToDevice, s));
        j.m = nb;
        j.m_old = 0;
        j.nu = nb;
        jobs.j[jobs.n++] = j;
        sl.push_back(KSlice{kk, nb, j.voff, j.voff});
      }
      if (jobs.n) {
        if (!orthonormalise(p, d, jobs, s)) throw Error(QM_E_NOT_SPD, "Ritz block lost rank");
        timed_apply(p, d, sl, d->V, d->HV, s, false);
        rayleigh_ritz(p, d, jobs, s);
        for (int i = 0; i < jobs.n; ++i) {
          d->m[jobs.j[i].k] = nb;
          d->it[jobs.j[i].k] += 1;
        }
      }
    } else {
      {   // the k-points that restart from their Ritz vectors need every row of X and HX
        std::vector<int> ks;
        for (int kk = k0; kk < k1; ++kk) {
          if (d->done[kk] || !d->stale[kk]) continue;
          int nu = 0;
          for (int n = 0; n < nb; ++n)
            if (!(d->h_resn[int64_t(kk) * nb + n] <= tol)) ++nu;
          if (d->m[kk] + nu > mb) ks.push_back(kk);
        }
        complete_ritz(p, d, ks, false, s);
      }
      std::vector<DJob> restart;
      for (int kk = k0; kk < k1; ++kk) {
        if (d->done[kk]) continue;
        int nu = 0;
        for (int n = 0; n < nb; ++n)
          if (!(d->h_resn[int64_t(kk) * nb + n] <= tol)) ++nu;
        DJob j = make_job(p, d, kk);
        if (d->m[kk] + nu > mb) {
          restart.push_back(j);
          d->m[kk] = nb;
          j.m_old = 0;
        } else {
          j.m_old = d->m[kk];
        }
        j.m = d->m[kk] + nu;
        j.nu = nu;
        jobs.j[jobs.n++] = j;
        sl.push_back(KSlice{kk, nu, j.voff + int64_t(j.m - nu) * j.npw, j.voff + int64_t(j.m - nu) * j.npw});
      }
      if (jobs.n) {
        if (!restart.empty()) restart_basis(p, d, restart, s);
        QM_HIP(hipMemcpyAsync(d->unconv, d->h_unconv, sizeof(int32_t) * d->nk * nb,
                              hipMemcpyHostToDevice, s));
        if (precond == QM_PRECOND_MLP) {
          mlp_precondition(p, jobs, o->mlp_weights, s, d->R, d->V, d->unconv, d->tkin, d->theta,
                           d->resn, d->goff);
        } else {
          hipLaunchKernelGGL(k_teter, dim3(nb, jobs.n), dim3(256), 0, s, jobs, d->R, d->V, d->unconv,
                             d->tkin, p->g.kin, d->goff);
          QM_HIP(hipGetLastError());
        }
        if (!orthonormalise(p, d, jobs, s)) throw Error(QM_E_NOT_SPD, "correction block lost rank");
        timed_apply(p, d, sl, d->V, d->HV, s, d->lowp);
        const bool lazy_now = d->lazy && subspace_lp(d) == 0;
        rayleigh_ritz(p, d, jobs, s, lazy_now);
        for (int i = 0; i < jobs.n; ++i) {
          d->m[jobs.j[i].k] = jobs.j[i].m;
          d->it[jobs.j[i].k] += 1;
        }
        if (lazy_now) {   // before a k-point is declared converged, every band is checked
          std::vector<int> ks;
          for (int i = 0; i < jobs.n; ++i) {
            const int kk = jobs.j[i].k;
            if (!d->stale[kk]) continue;
            bool open = false;
            for (int n = 0; n < nwant; ++n)
              if (!(d->h_resn[int64_t(kk) * nb + n] <= tol)) open = true;
            if (!open) ks.push_back(kk);
          }
          complete_ritz(p, d, ks, true, s);
        }
      }
    }
  }
  StepResult r;
  d->tol = tol;
  collect(p, d, tol, r);
  if (fresh || r.max_res < 0) d->hist.clear();
  d->hist.push_back(r.max_res);
  write_outputs(p, d, psi, eig, resnorm, s);
  if (n_unconv) *n_unconv = r.n_unconv;
  if (r.nan) throw Error(QM_E_NAN, "non-finite residual norm");
  return QM_OK;
}

static qm_status dav_step(qm_hpsi_plan* p, int k, void* psi, double* eig, double* resnorm, int nb,
                          const qm_dav_opts* o, int32_t* n_unconv, hipStream_t s) {
  QM_REQUIRE(k >= -1 && k < p->nk, QM_E_ARG, "k out of range");
  const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? p->nk : k + 1;
  return dav_step_range(p, &p->dav, false, k0, k1, psi, eig, resnorm, nb, o, n_unconv, s);
}

DavState* dav_of(qm_hpsi_plan* p) { return p->dav; }

// keep C[m][n] only where |e*_m - e*_n| <= ctol (the degenerate level of band n)
__global__ void k_mask_cluster(DJobs jobs, double2* __restrict__ C, const double* __restrict__ estar,
                               double ctol) {
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb;
  double2* Ck = C + int64_t(J.k) * nb * nb;
  const double* e = estar + int64_t(J.k) * nb;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nb * nb; t += gridDim.x * blockDim.x) {
    const int m = t / nb, n = t % nb;
    if (fabs(e[m] - e[n]) > ctol) Ck[t] = make_double2(0.0, 0.0);
  }
}

struct PairArgs { int64_t rowbase[kMaxSlices]; };

// rows of (features, residual, target) for unconverged band j of each job
__global__ void __launch_bounds__(256) k_pairs(DJobs jobs, PairArgs pa, const double2* __restrict__ X,
                                               const double2* __restrict__ P, const double2* __restrict__ Rr,
                                               const int32_t* __restrict__ unconv,
                                               const double* __restrict__ tkin,
                                               const double* __restrict__ theta,
                                               const double* __restrict__ resn,
                                               const double* __restrict__ kin_all,
                                               const int64_t* __restrict__ goff, float* __restrict__ feat,
                                               float* __restrict__ resid, float* __restrict__ target) {
  __shared__ double red[16];
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb, j = blockIdx.x;
  if (j >= J.nu) return;
  const int n = unconv[int64_t(J.k) * nb + j];
  const double2* x = X + J.xoff + int64_t(n) * J.npw;
  const double2* pn = P + J.xoff + int64_t(n) * J.npw;
  const double2* r = Rr + J.xoff + int64_t(n) * J.npw;
  const double* kin = kin_all + goff[J.k];
  double pp = 0.0;
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) pp += pn[g].x * pn[g].x + pn[g].y * pn[g].y;
  // block reduction (same order on every thread)
  for (int o = 32; o > 0; o >>= 1) pp += __shfl_down(pp, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pp;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < int(blockDim.x >> 6); ++i) s += red[i];
  const double ip = 1.0 / sqrt(s);
  const double tn = tkin[int64_t(J.k) * nb + n];
  const double th = theta[int64_t(J.k) * jobs.mb + n];
  const double rs = sqrt(double(J.npw)) / resn[int64_t(J.k) * nb + n];
  const int64_t row0 = pa.rowbase[blockIdx.y] + int64_t(j) * J.npw;
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const int64_t row = row0 + g;
    const double2 rv = r[g];
    float f[QM_MLP_NIN];
    make_feat(kin[g], tn, th, sqrt(rv.x * rv.x + rv.y * rv.y) * rs, f);
#pragma unroll
    for (int i = 0; i < QM_MLP_NIN; ++i) feat[row * QM_MLP_NIN + i] = f[i];
    resid[2 * row] = float(rv.x);
    resid[2 * row + 1] = float(rv.y);
    target[2 * row] = float(pn[g].x * ip - x[g].x);
    target[2 * row + 1] = float(pn[g].y * ip - x[g].y);
  }
}

static void training_pairs(qm_hpsi_plan* p, const void* xstar, const double* estar, double ctol,
                           float* feat, float* resid, float* target, int32_t* band_ptr,
                           int64_t cap_rows, int32_t cap_bands, int64_t* nrows, int32_t* nbands,
                           hipStream_t s) {
  DavState* d = p->dav;
  QM_REQUIRE(d && d->ready, QM_E_STATE, "no Davidson state: call qm_davidson_step first");
  // x_star and eig_star are laid out [nk][nbnd] like psi: a state with buffer bands holds
  // rows the caller's arrays do not have
  QM_REQUIRE(d->nb == d->nwant, QM_E_STATE,
             "training pairs need a Davidson state without buffer bands (extra_bands = 0)");
  QM_REQUIRE(xstar && estar && feat && resid && target && band_ptr && nrows && nbands, QM_E_ARG,
             "NULL argument");
  if (!d->estar) d->estar = dalloc<double>(size_t(d->nk) * d->nb);
  std::vector<double> eh(size_t(d->nk) * d->nb, 0.0);
  DJobs jobs{};
  jobs.nb = d->nb;
  jobs.mb = d->mb;
  PairArgs pa{};
  std::vector<int32_t> bp;
  int64_t rows = 0;
  std::vector<GemmCN> cn;
  std::vector<GemmEX> ex;
  const int64_t g0 = p->kinfo[d->k0].g_off;
  for (int kk = d->k0; kk < d->k1; ++kk) {
    for (int n = 0; n < d->nb; ++n) eh[size_t(kk) * d->nb + n] = estar[size_t(kk - d->k0) * d->nb + n];
    if (d->done[kk]) continue;
    int nu = 0;
    for (int n = 0; n < d->nb; ++n)
      if (!(d->h_resn[int64_t(kk) * d->nb + n] <= d->tol)) ++nu;
    if (nu == 0) continue;
    DJob j = make_job(p, d, kk);
    j.nu = nu;
    j.m = d->m[kk];
    pa.rowbase[jobs.n] = rows;
    for (int q = 0; q < nu; ++q) bp.push_back(int32_t(rows + int64_t(q) * j.npw));
    rows += int64_t(nu) * j.npw;
    jobs.j[jobs.n++] = j;
    const double2* xs = reinterpret_cast<const double2*>(xstar) + int64_t(d->nb) * (p->kinfo[kk].g_off - g0);
    double2* C = d->G + int64_t(kk) * d->nb * d->nb;
    cn.push_back(GemmCN{xs, d->X + j.xoff, C, d->nb, d->nb, j.npw, j.npw, j.npw, d->nb});
    ex.push_back(GemmEX{C, xs, d->TS + j.xoff, d->nb, j.npw, d->nb, d->nb, j.npw, j.npw});
  }
  bp.push_back(int32_t(rows));
  QM_REQUIRE(rows <= cap_rows && int64_t(bp.size()) - 1 <= cap_bands, QM_E_ARG,
             "training-pair buffers too small");
  QM_REQUIRE(rows < (int64_t(1) << 31), QM_E_ARG, "too many rows");
  *nrows = rows;
  *nbands = int32_t(bp.size()) - 1;
  QM_HIP(hipMemcpy(d->estar, eh.data(), sizeof(double) * eh.size(), hipMemcpyHostToDevice));
  QM_HIP(hipMemcpy(band_ptr, bp.data(), sizeof(int32_t) * bp.size(), hipMemcpyHostToDevice));
  if (jobs.n == 0) return;
  zgemm_cn_batched(cn, 1.0, 0.0, d->work, d->work_bytes, s);
  hipLaunchKernelGGL(k_mask_cluster, dim3(32, jobs.n), dim3(256), 0, s, jobs, d->G, d->estar, ctol);
  QM_HIP(hipGetLastError());
  zgemm_ex_batched(ex, 1.0, 0.0, s);
  QM_HIP(hipMemcpyAsync(d->unconv, d->h_unconv, sizeof(int32_t) * d->nk * d->nb, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_pairs, dim3(d->nb, jobs.n), dim3(256), 0, s, jobs, pa, d->X, d->TS, d->R, d->unconv,
                     d->tkin, d->theta, d->resn, p->g.kin, d->goff, feat, resid, target);
  QM_HIP(hipGetLastError());
  QM_HIP(hipStreamSynchronize(s));
}

}  // namespace qm

namespace qm {

struct SolveResult {
  qm_status st = QM_OK;
  int32_t nun = 0;
  std::string err;
};

// the Davidson loop on k0..k1-1 with the state in *slot: a restart step, then steps until
// every band of the range has converged or max_iter is reached
static SolveResult solve_range(qm_hpsi_plan* p, DavState** slot, bool own_scratch, int k0, int k1,
                               void* psi, double* eig, double* resnorm, int nb, qm_dav_opts o,
                               hipStream_t s) {
  SolveResult r;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  auto step = [&]() {
    try {
      r.st = dav_step_range(p, slot, own_scratch, k0, k1, psi, eig, resnorm, nb, &o, &r.nun, s, true);
    } catch (const Error& e) {
      r.err = e.what();
      r.st = e.code;
    } catch (const std::exception& e) {
      r.err = e.what();
      r.st = QM_E_STATE;
    }
    if (r.st != QM_OK && *slot) (*slot)->ready = false;
  };
  o.restart = 1;
  step();
  o.restart = 0;
  for (int iter = 0; r.st == QM_OK && r.nun > 0 && iter < max_iter; ++iter) step();
  // stopped at max_iter: the returned vectors and norms are completed for every band
  DavState* d = *slot;
  if (r.st == QM_OK && d && d->ready) {
    try {
      std::vector<int> ks;
      for (int kk = k0; kk < k1; ++kk)
        if (d->stale[kk]) ks.push_back(kk);
      if (!ks.empty()) {
        complete_ritz(p, d, ks, true, s);
        write_outputs(p, d, psi, eig, resnorm, s);
      }
    } catch (const Error& e) {
      r.err = e.what();
      r.st = e.code;
    }
  }
  return r;
}

}  // namespace qm

using namespace qm;

extern "C" {

qm_status qm_davidson_step(qm_hpsi_plan* plan, int32_t k, void* psi, double* eig, double* resnorm,
                           int32_t nbnd, const qm_dav_opts* opts, int32_t* n_unconverged,
                           void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    return dav_step(plan, k, psi, eig, resnorm, nbnd, opts, n_unconverged,
                    reinterpret_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    plan->err = e.what();
    if (plan->dav) plan->dav->ready = false;
    return e.code;
  } catch (const std::exception& e) {
    plan->err = e.what();
    if (plan->dav) plan->dav->ready = false;
    return QM_E_STATE;
  }
}

qm_status qm_davidson_solve(qm_hpsi_plan* plan, int32_t k, void* psi, double* eig, double* resnorm,
                            int32_t nbnd, const qm_dav_opts* opts, qm_dav_stats* stats,
                            void* stream) {
  if (!plan) return QM_E_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  qm_dav_opts o{};
  if (opts) o = *opts;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (k < -1 || k >= plan->nk) {
    plan->err = "k out of range";
    return QM_E_ARG;
  }
  const int nlanes = (k < 0 && o.lanes >= 2) ? std::min<int>(o.lanes, plan->nk) : 1;
  std::vector<int> kb(nlanes + 1);
  for (int i = 0; i <= nlanes; ++i) kb[i] = k < 0 ? (i * plan->nk) / nlanes : (i == 0 ? k : k + 1);
  std::vector<SolveResult> res(nlanes);
  try {
    if (nlanes == 1) {
      res[0] = solve_range(plan, &plan->dav, false, kb[0], kb[1], psi, eig, resnorm, nbnd, o, s);
    } else {
      // every lane reads the reduced-precision beta: convert it before they start
      if (o.switch_resid > 0.0 && plan->prec != QM_PREC_FP64) convert_beta(plan, plan->prec, s);
      plan->dav_lanes.resize(nlanes, nullptr);
      plan->lane_streams.resize(nlanes, nullptr);
      for (hipStream_t& q : plan->lane_streams)
        if (!q) QM_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      hipEvent_t ready;
      QM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      QM_HIP(hipEventRecord(ready, s));  // psi and earlier work on the caller's stream
      for (hipStream_t q : plan->lane_streams) QM_HIP(hipStreamWaitEvent(q, ready, 0));
      std::vector<std::thread> th;
      const int64_t gbase = plan->kinfo[0].g_off;
      for (int i = 0; i < nlanes; ++i) {
        double2* lp = reinterpret_cast<double2*>(psi) + int64_t(nbnd) * (plan->kinfo[kb[i]].g_off - gbase);
        th.emplace_back([&, i, lp]() {
          res[i] = solve_range(plan, &plan->dav_lanes[i], true, kb[i], kb[i + 1], lp,
                               eig ? eig + int64_t(kb[i]) * nbnd : nullptr,
                               resnorm ? resnorm + int64_t(kb[i]) * nbnd : nullptr, nbnd, o,
                               plan->lane_streams[i]);
        });
      }
      for (std::thread& t : th) t.join();
      (void)hipEventDestroy(ready);
    }
  } catch (const Error& e) {
    plan->err = e.what();
    return e.code;
  }
  qm_status st = QM_OK;
  int32_t nun = 0;
  for (const SolveResult& r : res) {
    if (r.st != QM_OK && st == QM_OK) {
      st = r.st;
      plan->err = r.err;
    }
    nun += r.nun;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    double mr = 0.0, th = 0.0, te = 0.0, ts = 0.0;
    int itmax = 0;
    for (int i = 0; i < nlanes; ++i) {
      const DavState* d = nlanes == 1 ? plan->dav : plan->dav_lanes[i];
      if (!d) continue;
      for (int kk = d->k0; kk < d->k1; ++kk) {
        itmax = std::max(itmax, d->it[kk]);
        for (int n = 0; n < d->nwant; ++n) mr = std::max(mr, d->h_resn[int64_t(kk) * d->nb + n]);
      }
      stats->n_hpsi_bands += d->n_hpsi;
      stats->n_hpsi_bands_lowp += d->n_hpsi_lowp;
      stats->n_gs += d->n_cgs;
      stats->n_gs_second += d->n_cgs2;
      th = std::max(th, d->t_hpsi);   // lanes overlap in time: the slowest lane's phases
      te = std::max(te, d->t_eig);
      ts = std::max(ts, d->t_sub);
    }
    stats->iterations = itmax;
    stats->converged = (st == QM_OK && nun == 0) ? 1 : 0;
    stats->max_resnorm = mr;
    stats->t_hpsi_ms = th;
    stats->t_eig_ms = te;
    stats->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->t_subspace_ms = ts;
  }
  if (st == QM_OK && nun > 0) {
    plan->err = "Davidson did not converge within max_iter";
    return QM_E_NOT_CONVERGED;
  }
  return st;
}

qm_status qm_dav_training_pairs(qm_hpsi_plan* plan, const void* x_star, const double* eig_star,
                                double cluster_tol, float* feat, float* resid, float* target,
                                int32_t* band_ptr, int64_t cap_rows, int32_t cap_bands, int64_t* nrows,
                                int32_t* nbands, void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    training_pairs(plan, x_star, eig_star, cluster_tol > 0 ? cluster_tol : 1e-6, feat, resid, target,
                   band_ptr, cap_rows, cap_bands, nrows, nbands, reinterpret_cast<hipStream_t>(stream));
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
