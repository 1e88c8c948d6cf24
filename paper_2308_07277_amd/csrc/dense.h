// Davidson job descriptors shared by the subspace kernels.
#pragma once
#include "qm_internal.h"

namespace qm {

// One active k-point of a Davidson step.
struct DJob {
  int32_t k;      // k index (selects the per-k blocks of every buffer)
  int32_t m;      // basis size after this step's expansion
  int32_t m_old;  // basis columns whose projected matrix entries are already known
  int32_t nu;     // new columns in this step (corrections)
  int32_t npw;
  int32_t pad;
  int64_t voff;   // element offset of the k's basis block V/HV ([mb][npw])
  int64_t xoff;   // element offset of the k's band blocks X/HX/R ([nb][npw])
};
struct DJobs {
  DJob j[kMaxSlices];
  int32_t n, nb, mb, pad;
};
// Scratch of the many-workgroup tridiagonalisation, per k (mb = basis capacity).
constexpr int kTrdTile = 64;       // tile edge of a step launch
constexpr int kTrdMaxBasis = 2048; // rows of a column one 256-thread workgroup holds in registers
struct TrdWork {
  double2* v;      // [k][2][mb] reflectors of the current and the previous step (slot j & 1)
  double2* w;      // [k][mb]    w of the previous step (the pending rank-2 update is v w^H + w v^H)
  double2* part;   // [k][ptiles][2][kTrdTile] each tile's share of A v: its 64 row sums and
                   //            its 64 column sums, summed in a fixed order by the last workgroup
  uint32_t* cnt;   // [k]        workgroups (or, with row-block finishers, row blocks) of the
                   //            current step that have finished
  uint32_t* bcnt;  // [k][nblk]  per row block: slots of the current step written
  double2* prow;   // [k][mb]    A v per row, summed by the row block's finisher
  int32_t ptiles;  // tile slots per k: nt (nt + 1) / 2 with nt = ceil(mb / kTrdTile)
  int32_t nblk;    // row blocks per k: ceil(mb / kTrdTile)
  int32_t fin_min; // steps with at least this many slots per row (nt + 1) use row-block finishers
};
inline int trd_tile_slots(int mb) {
  const int nt = (mb + kTrdTile - 1) / kTrdTile;
  return nt * (nt + 1) / 2;
}

// Scratch of the tridiagonal eigensolver, per k.
struct EigWork {
  double* sc;    // [k][nb] scale of each stored eigenvector (true vector = Y[.][n] * sc[n])
  double* nrm;   // [k]     norm estimate of the tridiagonal
};

// Input features of the learned preconditioner at one (G, band): x = T(G)/T_n, log(1 + x),
// (theta_n - T_n)/T_n, the residual amplitude |r_n(G)| sqrt(npw)/||r_n|| (passed in as ramp)
// and T(G) = 1/2|k+G|^2, computed in float64 and stored as float32.  The one definition used
// by inference inside the Davidson and by the training-row generation.
__device__ __forceinline__ void make_feat(double kin, double tn, double theta, double ramp,
                                          float f[QM_MLP_NIN]) {
  const double x = kin / tn;
  f[0] = float(x);
  f[1] = float(log1p(x));
  f[2] = float((theta - tn) / tn);
  f[3] = float(ramp);
  f[4] = float(kin);
}

}  // namespace qm

namespace qm {
__global__ void k_hs_fill(DJobs jobs, double2* Hs);
__global__ void k_hs_copy(DJobs jobs, const double2* Hs, double2* Aw);
__global__ void k_tridiag(DJobs jobs, double2* Aw, double* dd, double* ee, double2* tau, int ms);
// largest basis the one-workgroup reduction takes: 4 + 16 vectors of m complex entries in LDS
constexpr int kTridiagMaxM = (160 * 1024 - 2048) / (20 * 16);
__global__ void k_trd_start(DJobs jobs, double2* Aw, double* dd, double* ee, double2* tau, TrdWork tw);
__global__ void k_trd_step(DJobs jobs, int j, double2* Aw, double* dd, double* ee, double2* tau,
                           TrdWork tw);
__global__ void k_eig_vals(DJobs jobs, const double* dd, const double* ee, double* theta, EigWork ew);
__global__ void k_eig_inviter(DJobs jobs, const double* dd, const double* ee, const double* theta,
                              double* yw, double* fw, EigWork ew, int step);
__global__ void k_eig_orth(DJobs jobs, const double* theta, double* yw, EigWork ew);
__global__ void k_bt_tfactor(DJobs jobs, const double2* Aw, const double2* tau, double2* Tw);
__global__ void k_bt_apply(DJobs jobs, const double2* Aw, const double2* Tw, const double* yw,
                           const double* scw, double2* Zout, int cols);
constexpr int kBtBlk = 32;   // reflectors per block of the blocked back-transform
__global__ void k_chol_inv(DJobs jobs, double2* Gm, double2* Wm, int32_t* info);
constexpr int kCholBlk = 16;        // block size of the many-workgroup Cholesky
// largest band count whose Linv column block fits in LDS next to the kernel's static
// 13 KiB: 36 blocks of 16 x 16 complex (147 KiB)
constexpr int kCholMaxBlocked = 576;
__global__ void k_chol_prep(DJobs jobs, const double2* Gm, double* dmax);
__global__ void k_chol_col(DJobs jobs, int jb, double2* Gm, double2* Ldw, const double* dmaxw,
                           int32_t* info);
__global__ void k_chol_inv_cols(DJobs jobs, const double2* Gm, const double2* Ldw, double2* Wm,
                                const int32_t* info);
__global__ void k_residual(DJobs jobs, const double2* X, const double2* HX, double2* Rr,
                           const double* theta, const double* kin_all, const int64_t* goff,
                           double* resn, double* tkin, const int32_t* list);
__global__ void k_start_block(DJobs jobs, double2* V, int first);
__global__ void k_cgs_overlap(DJobs jobs, const double2* Cw, double* ovl);
__global__ void k_teter(DJobs jobs, const double2* Rr, double2* V, const int32_t* unconv,
                        const double* tkin, const double* kin_all, const int64_t* goff);
}  // namespace qm
