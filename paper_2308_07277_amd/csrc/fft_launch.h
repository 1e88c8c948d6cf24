// Host dispatch of the local-part kernels over the supported FFT lengths.
#pragma once
#include "fft_kernels.h"

namespace qm {

constexpr int kZTile = 32;  // sticks per z-kernel tile (the plan's tile tables use it)


// Kernel arguments of the local-part kernels for the slices sl; nblk_z / npair receive the
// z-kernel block count and the number of (k, band) pairs.
template <typename R>
LocalArgs make_local_args(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi,
                          void* hpsi, const HpsiWork* wk, int64_t& nblk_z, int64_t& npair) {
  LocalArgs a{};
  QM_REQUIRE(!sl.empty() && sl.size() <= size_t(kMaxSlices), QM_E_STATE, "bad slice count");
  a.kinfo = p->g.kinfo;
  a.nsl = int32_t(sl.size());
  a.N3 = p->N3;
  nblk_z = 0;
  npair = 0;
  for (size_t i = 0; i < sl.size(); ++i) {
    a.sl[i] = sl[i];
    a.blk_z[i] = int32_t(nblk_z);
    a.pair0[i] = int32_t(npair);
    nblk_z += int64_t(sl[i].nb) * p->kinfo[sl[i].k].ntile;
    npair += sl[i].nb;
  }
  a.blk_z[sl.size()] = int32_t(nblk_z);
  a.pair0[sl.size()] = int32_t(npair);
  a.psi = reinterpret_cast<const double2*>(psi);
  a.hpsi = reinterpret_cast<double2*>(hpsi);
  a.sbuf = wk ? wk->sbuf : p->sbuf;
  a.sbuf_per_k = wk ? 0 : 1;
  a.ent_g = p->g.ent_g;
  a.ent_sz = p->g.ent_sz;
  a.tile_ptr = p->g.tile_ptr;
  a.stick_pos = p->g.stick_pos;
  a.col_of_i1 = p->g.col_of_i1;
  a.stick_at = p->g.stick_at;
  a.sat_stride = p->nax_max;
  a.kin = p->g.kin;
  a.vplan = sizeof(R) == 8 ? p->vplan64 : p->vplan32;
  a.tw_z = p->tw_z;
  a.tw_x = p->tw_x;
  a.ts = kZTile;
  a.nax_stride = p->nax_max | 1;
  a.xy_stride = xy_row_stride(p->N1, p->nax_max, false);
  a.zero_mid = p->zero_mid;
  QM_REQUIRE(nblk_z < (int64_t(1) << 31), QM_E_SHAPE, "launch too large");
  return a;
}

// scatter + inverse z transform of every slice into the stick buffer
template <typename R>
void launch_zinv_t(const LocalArgs& a, int64_t nblk_z, int N3, hipStream_t s) {
#define QM_ZINV_ONLY(n)                                                                     \
  case n:                                                                                   \
    hipLaunchKernelGGL((k_zinv<R, n, kZTile>), dim3(unsigned(nblk_z)),                      \
                       dim3(kZTile * Split<n>::R2), 0, s, a);                               \
    break;
  switch (N3) {
    QM_FOR_EACH_FFT_LEN(QM_ZINV_ONLY)
    default: throw Error(QM_E_SHAPE, "unsupported N3");
  }
#undef QM_ZINV_ONLY
  QM_HIP(hipGetLastError());
}

template <typename R>
void launch_local_t(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                    hipStream_t s, StageEvents* ev, const HpsiWork* wk) {
  int64_t nblk_z = 0, npair = 0;
  LocalArgs a = make_local_args<R>(p, sl, psi, hpsi, wk, nblk_z, npair);
  const int64_t nblk_xy = npair * p->N3;
  QM_REQUIRE(nblk_xy < (int64_t(1) << 31), QM_E_SHAPE, "launch too large");
  const int NX = p->N1;
  const int xy_mode = xy_pick(p, sizeof(R) == 8 ? 0 : 1);
  const bool own = xy_mode == 3;
  if (own) a.xy_stride = xy_row_stride(NX, p->nax_max, true);
  const size_t smem_xy = xy_lds_bytes(NX, a.xy_stride, sizeof(R), own);
  QM_REQUIRE(smem_xy <= 160 * 1024, QM_E_SHAPE, "xy-plane does not fit in LDS for this grid/precision");
#define QM_ZINV(n)                                                                          \
  case n:                                                                                   \
    hipLaunchKernelGGL((k_zinv<R, n, kZTile>), dim3(unsigned(nblk_z)),                      \
                       dim3(kZTile * Split<n>::R2), 0, s, a);                               \
    break;
#define QM_ZFWD(n)                                                                          \
  case n:                                                                                   \
    hipLaunchKernelGGL((k_zfwd<R, n, kZTile>), dim3(unsigned(nblk_z)),                      \
                       dim3(kZTile * Split<n>::R2), 0, s, a);                               \
    break;
#define QM_XY(n)                                                                            \
  case n: {                                                                                 \
    static bool attr_set[2] = {false, false};                                               \
    const void* fn = own ? reinterpret_cast<const void*>(&k_xy<R, n, true>)                 \
                         : reinterpret_cast<const void*>(&k_xy<R, n, false>);               \
    if (!attr_set[own]) {                                                                   \
      QM_HIP(allow_full_lds(fn));                                                           \
      attr_set[own] = true;                                                                 \
    }                                                                                       \
    if (own)                                                                                \
      hipLaunchKernelGGL((k_xy<R, n, true>), dim3(unsigned(nblk_xy)), dim3(256), smem_xy, s, a); \
    else                                                                                    \
      hipLaunchKernelGGL((k_xy<R, n, false>), dim3(unsigned(nblk_xy)), dim3(256), smem_xy, s, a); \
  } break;
  switch (p->N3) {
    QM_FOR_EACH_FFT_LEN(QM_ZINV)
    default: throw Error(QM_E_SHAPE, "unsupported N3");
  }
  QM_HIP(hipGetLastError());
  if (ev) ev->mark(0);
  if (xy_mode == 2) {
    const size_t smem_p = sizeof(cplx<R>) * (size_t(NX) * a.nax_stride + NX) + sizeof(int) * NX;
#define QM_XYP(n, l)                                                                        \
  case n: {                                                                                 \
    static bool attr_p = false;                                                             \
    if (!attr_p) {                                                                          \
      QM_HIP(allow_full_lds(reinterpret_cast<const void*>(&k_xy_group<R, n, l>)));         \
      attr_p = true;                                                                        \
    }                                                                                       \
    hipLaunchKernelGGL((k_xy_group<R, n, l>), dim3(unsigned(nblk_xy)), dim3(l * n), smem_p, s, a); \
  } break;
    switch (NX) {
      QM_XYP(20, 2) QM_XYP(40, 2) QM_XYP(72, 8)
      default: throw Error(QM_E_SHAPE, "unsupported N1");
    }
#undef QM_XYP
  } else {
    switch (NX) {
      QM_FOR_EACH_FFT_LEN(QM_XY)
      default: throw Error(QM_E_SHAPE, "unsupported N1");
    }
  }
  QM_HIP(hipGetLastError());
  if (ev) ev->mark(1);
  switch (p->N3) {
    QM_FOR_EACH_FFT_LEN(QM_ZFWD)
    default: throw Error(QM_E_SHAPE, "unsupported N3");
  }
  QM_HIP(hipGetLastError());
  if (ev) ev->mark(2);
#undef QM_ZINV
#undef QM_ZFWD
#undef QM_XY
}

}  // namespace qm
