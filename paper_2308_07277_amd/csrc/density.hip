// Electron density, Hartree potential and a Hartree-only SCF cycle (Sec. 2.1: the density
// n(r) = sum_i f_i |psi_i(r)|^2 of the Kohn-Sham equations, the Hartree term of the
// auxiliary potential, and the self-consistency cycle n -> V -> {psi} -> n_out, mixed until
// n_out = n).
//
// Density: the bands' coefficients are scattered and transformed along z into the plan's
// stick buffer by the same kernel H|psi> uses; k_density_xy then runs the inverse y and x
// transforms of every (k, band) pair of one z-plane and accumulates w_k f_kn |psi(r)|^2 in
// registers.  The pairs are split into groups, one workgroup per (plane, group), each group
// writing its own partial plane; k_density_reduce adds the groups in a fixed order, so the
// result does not depend on scheduling (no atomics).
// Hartree: the periodic Poisson equation in G, V_H(G) = 4 pi n(G) / |G|^2 (G != 0, zero
// average), with the full-grid 3-D FFT done as three passes of batched line transforms.
#include <chrono>
#include <cmath>
#include <cstring>

#include "cplx.h"
#include "fft_kernels.h"
#include "qm_internal.h"

namespace qm {

// ---------------------------------------------------------------- density
struct DensArgs {
  const KInfo* kinfo;
  int32_t slk[kMaxSlices];          // k of each slice
  int32_t pair0[kMaxSlices + 1];    // prefix of band counts over the slices
  int32_t nsl, N3, npair, ngroups;
  const double2* sbuf;              // the plan's stick buffer (float64)
  const int32_t* stick_at;          // [nk][NX i2][sat_stride] stick index or -1
  const int32_t* col_of_i1;
  const double2* tw_x;
  const double* wf;                 // [npair] w_k f_kn / Omega
  double* part;                     // [ngroups][N3 slot][NX i2][NX i1]
  int32_t nax_stride;               // LDS row stride: active columns plus a zero slot
  int32_t sat_stride;
  int32_t zero_mid;                 // the plan's zero middle band (LocalArgs::zero_mid)
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup per (z-plane slot p, pair group g).  For every pair of the group the
// plane's active columns go through the two inverse y passes in LDS, the first gathering its
// input straight from the plane's sticks (raw buffer loads; absent sticks read zero), then
// every row through the inverse x transform: lanes q < R1 of a row take the R2-point DFTs
// over the row's samples q + R1 n2 (inactive columns read the row's zero slot), the row
// scratch exchanges them (lane q writes slots q R2 + k2 and reads slots n1 R2 + q: odd lane
// strides, different LDS banks), and lane q ends with the row's values at i1 = q + R2 k1,
// whose squared moduli it accumulates with weight w_k f_kn.  Lane (wave, q, row slot rs)
// keeps the same rows for every pair, so the sums stay in registers until the partial plane
// is written.
template <int NX>
__global__ void __launch_bounds__(256) k_density_xy(DensArgs a) {
  using R = double;
  constexpr int R1 = Split<NX>::R1, R2 = Split<NX>::R2;
  constexpr int RG = 256 / R2, RW = 64 / R2, NXP = NX + 1;
  constexpr int NRND = (NX + 4 * RW - 1) / (4 * RW);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ns = a.nax_stride;
  cplx<R>* L = reinterpret_cast<cplx<R>*>(smem_raw);  // [NX positions][ns]
  cplx<R>* X = L + NX * ns;                              // [RG rows][NX + 1]
  cplx<R>* tw = X + NXP * RG;                            // [NX]
  int* col = reinterpret_cast<int*>(tw + NX);            // [NX]
  const int tid = threadIdx.x, p = blockIdx.x, g = blockIdx.y, N3 = a.N3;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int ZF = zero_mid_f(R2);
  const bool zm = ZF > 0 && a.zero_mid;
  auto in_zm = [](int n) { return ZF > 0 && n >= ZF && n < 2 * ZF; };
  const int q = lane % R2, rs = lane / R2;
  cplx<R>* Xr = X + (wave * RW + (rs < RW ? rs : 0)) * NXP;
  for (int i = tid; i < NX; i += 256) {
    const double2 w = a.tw_x[i];
    tw[i] = {w.x, w.y};
    L[i * ns + ns - 1] = {R(0), R(0)};   // the zero slot of every row (no pass writes it)
  }
  R acc[NRND][R1];
#pragma unroll
  for (int r = 0; r < NRND; ++r)
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) acc[r][k1] = R(0);
  int kprev = -1;
  int cr[R2];
  cplx<R> tq[R2];
  for (int kb = g; kb < a.npair; kb += a.ngroups) {
    int si = 0;
    while (si < a.nsl - 1 && kb >= a.pair0[si + 1]) ++si;
    const int k = a.slk[si], band = kb - a.pair0[si];
    const KInfo ki = a.kinfo[k];
    const int nax = ki.nax;
    __syncthreads();   // the previous pair's reads of L and col are done; tw is written
    if (k != kprev) {
      for (int i = tid; i < NX; i += 256) col[i] = a.col_of_i1[int64_t(k) * NX + i];
      __syncthreads();
      // per-lane constants of every row: the slots of the samples i1 = q + R1 j (the zero
      // slot for inactive columns) and the twiddles w^{q j} (exponents below NX)
#pragma unroll
      for (int j = 0; j < R2; ++j) {
        const int c = col[min(q, R1 - 1) + R1 * j];
        cr[j] = c >= 0 ? c : ns - 1;
        tq[j] = tw[min(q * j, NX - 1)];
      }
    }
    kprev = k;
    const double2* plane = a.sbuf + ki.sbuf_off + (int64_t(band) * N3 + p) * ki.nstick;
    const __amdgpu_buffer_rsrc_t prs = stick_rsrc<R>(reinterpret_cast<const cplx<R>*>(plane), ki.nstick);
    const int32_t* sat = a.stick_at + int64_t(k) * NX * a.sat_stride;
    const int sts = a.sat_stride;
    // y-pass items w = ia + nax j, walked without a division per item (256 = dj nax + dia)
    const int ia0 = tid % nax, j0 = tid / nax, dj = 256 / nax, dia = 256 - dj * nax;
    // inverse y, pass 1 (R2-point, stride R1), input gathered from the sticks
    for (int w = tid, ia = ia0, n1 = j0; w < nax * R1; w += 256, ia += dia, n1 += dj) {
      if (ia >= nax) {
        ia -= nax;
        ++n1;
      }
      int sx[R2];
      cplx<R> x[R2];
      if (ZF > 0 && zm) {   // rows of the zero middle band hold no stick (as in k_xy)
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2)
          if (!in_zm(n2)) sx[n2] = sat[(n1 + R1 * n2) * sts + ia];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2)
          x[n2] = in_zm(n2) ? cplx<R>{R(0), R(0)} : stick_load(prs, sx[n2], R(0));
        dft_zm<R2, +1, R, (ZF > 0)>(x);
      } else {
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) sx[n2] = sat[(n1 + R1 * n2) * sts + ia];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) x[n2] = stick_load(prs, sx[n2], R(0));
        Dft<R2, +1, R>::run(x);
      }
#pragma unroll
      for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tw[n1 * k2]);   // n1 k2 < NX
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) L[(n1 + R1 * k2) * ns + ia] = x[k2];
    }
    __syncthreads();
    // pass 2 (R1-point on contiguous runs): y frequency k2 + R2 k1 at position k1 + R1 k2
    for (int w = tid, ia = ia0, k2 = j0; w < nax * R2; w += 256, ia += dia, k2 += dj) {
      if (ia >= nax) {
        ia -= nax;
        ++k2;
      }
      cplx<R> y[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) y[n1] = L[(n1 + R1 * k2) * ns + ia];
      Dft<R1, +1, R>::run(y);
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) L[(n1 + R1 * k2) * ns + ia] = y[n1];
    }
    __syncthreads();
    const R wf = a.wf[kb];
#pragma unroll
    for (int rnd = 0; rnd < NRND; ++rnd) {
      const int i2 = wave * RW + 4 * RW * rnd + rs;
      const bool act = rs < RW && i2 < NX;
      const int lrow = act ? (i2 / R2) + R1 * (i2 % R2) : 0;
      if (act && q < R1) {
        cplx<R> x[R2];
        inverse_first_pass<R2, R, ZF>(x, L + lrow * ns, cr, zm);
#pragma unroll
        for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tq[k2]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Xr[q * R2 + k2] = x[k2];
      }
      wave_sync_lds();
      if (act) {
        cplx<R> y[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) y[n1] = Xr[n1 * R2 + q];
        Dft<R1, +1, R>::run(y);   // y[k1]: the row at i1 = q + R2 k1
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) acc[rnd][k1] += wf * (y[k1].re * y[k1].re + y[k1].im * y[k1].im);
      }
      wave_sync_lds();
    }
  }
  double* out = a.part + (int64_t(g) * N3 + p) * NX * NX;
#pragma unroll
  for (int rnd = 0; rnd < NRND; ++rnd) {
    const int i2 = wave * RW + 4 * RW * rnd + rs;
    if (rs < RW && i2 < NX) {
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) out[int64_t(i2) * NX + q + R2 * k1] = acc[rnd][k1];
    }
  }
}

// rho[i1][i2][i3] (C order) = sum over groups, in group order, of part[g][slot(i3)][i2][i1]
// with slot(i3) = i3 / R2 + R1 (i3 % R2), the z order the inverse z transform leaves.
__global__ void k_density_reduce(const double* __restrict__ part, int ngroups, int NX, int N3,
                                 int R1z, int R2z, double* __restrict__ rho) {
  const int64_t nr = int64_t(NX) * NX * N3;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nr;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int i3 = int(t % N3);
    const int64_t r = t / N3;
    const int i2 = int(r % NX), i1 = int(r / NX);
    const int slot = i3 / R2z + R1z * (i3 % R2z);
    const int64_t o = (int64_t(slot) * NX + i2) * NX + i1;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += part[int64_t(g) * nr + o];
    rho[t] = s;
  }
}

template <int NX>
static void launch_density_xy(const DensArgs& a, hipStream_t s) {
  constexpr int R2 = Split<NX>::R2, RG = 256 / R2;
  const size_t smem = sizeof(double2) * (size_t(NX) * a.nax_stride + size_t(NX + 1) * RG + NX) +
                      sizeof(int) * NX;
  QM_REQUIRE(smem <= 160 * 1024, QM_E_SHAPE, "density plane does not fit in LDS for this grid");
  static bool attr = false;
  if (!attr) {
    QM_HIP(allow_full_lds(reinterpret_cast<const void*>(&k_density_xy<NX>)));
    attr = true;
  }
  hipLaunchKernelGGL(k_density_xy<NX>, dim3(unsigned(a.N3), unsigned(a.ngroups)), dim3(256), smem, s, a);
  QM_HIP(hipGetLastError());
}

static double cell_volume(const qm_hpsi_plan* p) {
  const double* a = p->cell;
  return std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                   a[2] * (a[3] * a[7] - a[4] * a[6]));
}

template <typename T>
static T* grow(T*& buf, int64_t& have, int64_t need) {
  if (have < need) {
    if (buf) QM_HIP(hipFree(buf));
    buf = nullptr;
    have = 0;
    QM_HIP(hipMalloc(&buf, size_t(need) * sizeof(T)));
    have = need;
  }
  return buf;
}

void density_free(qm_hpsi_plan* p) {
  void* ptrs[] = {p->rho_part, p->dens_wf, p->grid_c, p->grid_sum};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  p->rho_part = nullptr;
  p->dens_wf = nullptr;
  p->grid_c = nullptr;
  p->grid_sum = nullptr;
  p->rho_part_bytes = p->dens_wf_n = 0;
}

static void density(qm_hpsi_plan* p, int k, const void* psi, int nbnd, const double* weights,
                    const double* occ, double* rho, hipStream_t s) {
  QM_REQUIRE(psi && weights && occ && rho, QM_E_ARG, "psi, weights, occ and rho must be non-NULL");
  QM_REQUIRE(nbnd >= 1 && nbnd <= p->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
  QM_REQUIRE(k >= -1 && k < p->nk, QM_E_ARG, "k out of range");
  const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? p->nk : k + 1;
  QM_REQUIRE(k1 - k0 <= kMaxSlices, QM_E_ARG, "at most 32 k-points per density call");
  const int NX = p->N1, N3 = p->N3;
  const int64_t nr = int64_t(NX) * NX * N3;
  const double vol = cell_volume(p);
  std::vector<KSlice> sl = contiguous_slices(p, k0, k1, nbnd);
  std::vector<double> wf;
  DensArgs a{};
  a.kinfo = p->g.kinfo;
  a.nsl = int32_t(sl.size());
  a.N3 = N3;
  for (size_t i = 0; i < sl.size(); ++i) {
    a.slk[i] = sl[i].k;
    a.pair0[i] = int32_t(wf.size());
    for (int n = 0; n < nbnd; ++n) {
      const double f = occ[int64_t(i) * nbnd + n];
      QM_REQUIRE(std::isfinite(f) && std::isfinite(weights[i]), QM_E_ARG, "non-finite weight or occupation");
      wf.push_back(weights[i] * f / vol);
    }
  }
  a.pair0[sl.size()] = int32_t(wf.size());
  a.npair = int32_t(wf.size());
  // enough (plane, group) workgroups to fill the chip, each group with at least one pair
  a.ngroups = int32_t(std::max<int64_t>(1, std::min<int64_t>(a.npair, (2048 + N3 - 1) / N3)));
  grow(p->dens_wf, p->dens_wf_n, int64_t(wf.size()));
  QM_HIP(hipMemcpy(p->dens_wf, wf.data(), wf.size() * sizeof(double), hipMemcpyHostToDevice));
  int64_t have = p->rho_part_bytes / int64_t(sizeof(double));
  grow(p->rho_part, have, int64_t(a.ngroups) * nr);
  p->rho_part_bytes = have * int64_t(sizeof(double));
  a.sbuf = reinterpret_cast<const double2*>(p->sbuf);
  a.stick_at = p->g.stick_at;
  a.sat_stride = p->nax_max;
  a.col_of_i1 = p->g.col_of_i1;
  a.tw_x = p->tw_x;
  a.wf = p->dens_wf;
  a.part = p->rho_part;
  a.nax_stride = (p->nax_max + 1) | 1;
  a.zero_mid = p->zero_mid;
  launch_zinv_f64(p, sl, psi, s);
#define QM_DXY(n)                       \
  case n:                               \
    launch_density_xy<n>(a, s);         \
    break;
  switch (NX) {
    QM_FOR_EACH_FFT_LEN(QM_DXY)
    default: throw Error(QM_E_SHAPE, "unsupported N1");
  }
#undef QM_DXY
  const int blocks = int(std::min<int64_t>((nr + 255) / 256, 8192));
  hipLaunchKernelGGL(k_density_reduce, dim3(blocks), dim3(256), 0, s, p->rho_part, a.ngroups, NX, N3,
                     fft_split_r1(N3), fft_split_r2(N3), rho);
  QM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- Poisson solve
// Length-N transforms of LT lines of nbatch complex grids [N1][N2][N3] (consecutive in
// memory) along one axis, sign S (unnormalised: sum_n x_n e^{S 2 pi i n k / N}).  Lines go
// through an LDS tile; the transform is the two-factor split N = R1 R2: R2-point DFTs over n2
// of x[n1 + R1 n2], twiddle w_N^{S n1 k2}, then R1-point DFTs over n1, giving X[k2 + R2 k1].
template <int N, int S>
__global__ void __launch_bounds__(256) k_fft_lines(double2* __restrict__ c, int axis, int N1, int N2,
                                                   int N3, const double2* __restrict__ twp, int64_t nbatch) {
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2, LT = 16;
  __shared__ cplx<double> tile[LT][N + 1];
  __shared__ cplx<double> tws[N];
  const int tid = threadIdx.x;
  const int64_t ngrid = axis == 2 ? int64_t(N1) * N2 : (axis == 1 ? int64_t(N1) * N3 : int64_t(N2) * N3);
  const int64_t nlines = ngrid * nbatch, nr = int64_t(N1) * N2 * N3;
  const int64_t stride = axis == 2 ? 1 : (axis == 1 ? int64_t(N3) : int64_t(N2) * N3);
  auto base = [&](int64_t lb) -> int64_t {
    const int64_t b = lb / ngrid, l = lb - b * ngrid;
    if (axis == 2) return b * nr + l * N3;
    if (axis == 1) return b * nr + (l / N3) * int64_t(N2) * N3 + l % N3;
    return b * nr + l;
  };
  const int64_t l0 = int64_t(blockIdx.x) * LT;
  for (int i = tid; i < N; i += 256) {
    const double2 w = twp[i];
    tws[i] = {w.x, S > 0 ? w.y : -w.y};
  }
  for (int e = tid; e < LT * N; e += 256) {
    const int line = stride == 1 ? e / N : e % LT, j = stride == 1 ? e % N : e / LT;
    const int64_t l = l0 + line;
    if (l < nlines) {
      const double2 v = c[base(l) + j * stride];
      tile[line][j] = {v.x, v.y};
    }
  }
  __syncthreads();
  for (int w = tid; w < LT * R1; w += 256) {
    const int line = w % LT, n1 = w / LT;
    cplx<double> x[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) x[n2] = tile[line][n1 + R1 * n2];
    Dft<R2, S, double>::run(x);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tws[(n1 * k2) % N]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) tile[line][n1 + R1 * k2] = x[k2];
  }
  __syncthreads();
  for (int w = tid; w < LT * R2; w += 256) {
    const int line = w % LT, k2 = w / LT;
    const int64_t l = l0 + line;
    cplx<double> y[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n1] = tile[line][n1 + R1 * k2];
    Dft<R1, S, double>::run(y);
    if (l < nlines) {
      const int64_t b = base(l);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) c[b + (k2 + R2 * k1) * stride] = make_double2(y[k1].re, y[k1].im);
    }
  }
}

template <int S>
static void fft_axis(qm_hpsi_plan* p, double2* c, int axis, hipStream_t s, int64_t nbatch = 1) {
  const int N = axis == 2 ? p->N3 : p->N1;
  const double2* tw = axis == 2 ? p->tw_z : p->tw_x;
  const int64_t nlines = nbatch * (axis == 2 ? int64_t(p->N1) * p->N2
                                             : (axis == 1 ? int64_t(p->N1) * p->N3 : int64_t(p->N2) * p->N3));
  QM_REQUIRE((nlines + 15) / 16 < (int64_t(1) << 31), QM_E_SHAPE, "too many grid lines");
  const unsigned blocks = unsigned((nlines + 15) / 16);
#define QM_FL(n)                                                                                   \
  case n:                                                                                          \
    hipLaunchKernelGGL((k_fft_lines<n, S>), dim3(blocks), dim3(256), 0, s, c, axis, p->N1, p->N2,  \
                       p->N3, tw, nbatch);                                                         \
    break;
  switch (N) {
    QM_FOR_EACH_FFT_LEN(QM_FL)
    default: throw Error(QM_E_SHAPE, "unsupported grid length");
  }
#undef QM_FL
  QM_HIP(hipGetLastError());
}

// modes of the elementwise grid kernel
enum { kToComplex = 0, kPoisson = 1, kRealPart = 2, kAdd = 3, kMix = 4, kFill = 5 };
struct GridOp {
  int mode;
  int N1, N2, N3;
  double b[9];      // reciprocal rows (Poisson)
  double scale;     // Poisson: 4 pi / N_r; mix: alpha; fill: value
};

// elementwise: to complex (x -> c), Poisson in G (c *= 4 pi / (|G|^2 N_r), 0 at G = 0, m in
// the centred range), real part (c -> y), y = x + z, y += alpha (x - y), y = value
__global__ void k_grid_op(GridOp op, const double* __restrict__ x, const double* __restrict__ z,
                          double* __restrict__ y, double2* __restrict__ c) {
  const int64_t nr = int64_t(op.N1) * op.N2 * op.N3;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nr;
       t += int64_t(gridDim.x) * blockDim.x) {
    switch (op.mode) {
      case kToComplex: c[t] = make_double2(x[t], 0.0); break;
      case kPoisson: {
        const int i3 = int(t % op.N3);
        const int64_t r = t / op.N3;
        const int i2 = int(r % op.N2), i1 = int(r / op.N2);
        const double m1 = i1 < (op.N1 + 1) / 2 ? i1 : i1 - op.N1;
        const double m2 = i2 < (op.N2 + 1) / 2 ? i2 : i2 - op.N2;
        const double m3 = i3 < (op.N3 + 1) / 2 ? i3 : i3 - op.N3;
        const double gx = m1 * op.b[0] + m2 * op.b[3] + m3 * op.b[6];
        const double gy = m1 * op.b[1] + m2 * op.b[4] + m3 * op.b[7];
        const double gz = m1 * op.b[2] + m2 * op.b[5] + m3 * op.b[8];
        const double g2 = gx * gx + gy * gy + gz * gz;
        const double f = (i1 == 0 && i2 == 0 && i3 == 0) ? 0.0 : op.scale / g2;
        c[t] = make_double2(c[t].x * f, c[t].y * f);
      } break;
      case kRealPart: y[t] = c[t].x; break;
      case kAdd: y[t] = x[t] + z[t]; break;
      case kMix: y[t] += op.scale * (x[t] - y[t]); break;
      default: y[t] = op.scale; break;
    }
  }
}

// one workgroup: out[0] = sum_t x[t] y[t] (mode 0) or sum_t (x[t] - y[t])^2 (mode 1), each
// thread over a fixed stride, then a fixed-order tree
__global__ void __launch_bounds__(1024) k_grid_sum(const double* __restrict__ x, const double* __restrict__ y,
                                                   int64_t n, int mode, double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 1024) {
    const double a = x[t], b = y[t];
    s += mode == 0 ? a * b : (a - b) * (a - b);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

static GridOp grid_op(const qm_hpsi_plan* p, int mode, double scale) {
  GridOp op{};
  op.mode = mode;
  op.N1 = p->N1;
  op.N2 = p->N2;
  op.N3 = p->N3;
  std::memcpy(op.b, p->recip, sizeof(op.b));
  op.scale = scale;
  return op;
}

static void run_grid_op(const qm_hpsi_plan* p, int mode, double scale, const double* x, const double* z,
                        double* y, double2* c, hipStream_t s) {
  const int64_t nr = int64_t(p->N1) * p->N2 * p->N3;
  const int blocks = int(std::min<int64_t>((nr + 255) / 256, 8192));
  hipLaunchKernelGGL(k_grid_op, dim3(blocks), dim3(256), 0, s, grid_op(p, mode, scale), x, z, y, c);
  QM_HIP(hipGetLastError());
}

void fft3_batched(qm_hpsi_plan* p, double2* c, int64_t nbatch, int sign, hipStream_t s) {
  for (int ax = 0; ax < 3; ++ax) {
    if (sign > 0)
      fft_axis<+1>(p, c, ax, s, nbatch);
    else
      fft_axis<-1>(p, c, ax, s, nbatch);
  }
}

void grid_add(qm_hpsi_plan* p, const double* x, const double* z, double* y, hipStream_t s) {
  run_grid_op(p, kAdd, 0.0, x, z, y, nullptr, s);
}

// sum_t x y (mode 0) or sum_t (x - y)^2 (mode 1), synchronous
static double grid_sum(qm_hpsi_plan* p, const double* x, const double* y, int mode, hipStream_t s) {
  if (!p->grid_sum) QM_HIP(hipMalloc(&p->grid_sum, 2 * sizeof(double)));
  const int64_t nr = int64_t(p->N1) * p->N2 * p->N3;
  hipLaunchKernelGGL(k_grid_sum, dim3(1), dim3(1024), 0, s, x, y, nr, mode, p->grid_sum);
  QM_HIP(hipGetLastError());
  double out = 0.0;
  QM_HIP(hipMemcpyAsync(&out, p->grid_sum, sizeof(double), hipMemcpyDeviceToHost, s));
  QM_HIP(hipStreamSynchronize(s));
  return out;
}

static void hartree(qm_hpsi_plan* p, const double* rho, double* vh, double* e_h, hipStream_t s) {
  QM_REQUIRE(rho && vh, QM_E_ARG, "rho and vh must be non-NULL");
  QM_REQUIRE(rho != vh, QM_E_ARG, "vh must not alias rho");
  const int64_t nr = int64_t(p->N1) * p->N2 * p->N3;
  if (!p->grid_c) QM_HIP(hipMalloc(&p->grid_c, size_t(nr) * sizeof(double2)));
  double2* c = reinterpret_cast<double2*>(p->grid_c);
  run_grid_op(p, kToComplex, 0.0, rho, nullptr, nullptr, c, s);
  for (int ax = 0; ax < 3; ++ax) fft_axis<-1>(p, c, ax, s);
  run_grid_op(p, kPoisson, 4.0 * 3.14159265358979323846 / double(nr), nullptr, nullptr, nullptr, c, s);
  for (int ax = 0; ax < 3; ++ax) fft_axis<+1>(p, c, ax, s);
  run_grid_op(p, kRealPart, 0.0, nullptr, nullptr, vh, c, s);
  if (e_h) *e_h = 0.5 * cell_volume(p) / double(nr) * grid_sum(p, vh, rho, 0, s);
}

// ---------------------------------------------------------------- Hartree-only SCF
static qm_status scf_hartree(qm_hpsi_plan* p, const double* vext, const double* kw, int nocc, void* psi,
                             int nbnd, const qm_scf_opts* o, double* eig, double* rho, double* vh,
                             qm_scf_stats* st, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  QM_REQUIRE(vext && kw && psi && rho && vh, QM_E_ARG, "vext, kweights, psi, rho and vh must be non-NULL");
  QM_REQUIRE(nocc >= 1 && nocc <= nbnd, QM_E_ARG, "need 1 <= nocc <= nbnd");
  QM_REQUIRE(p->nk <= kMaxSlices, QM_E_ARG, "at most 32 k-points");
  const double alpha = (o && o->alpha > 0) ? o->alpha : 0.7;
  const double tol = (o && o->tol > 0) ? o->tol : 1e-9;
  const int max_iter = (o && o->max_iter > 0) ? o->max_iter : 100;
  qm_dav_opts dav{};
  if (o) dav = o->dav;
  if (!(dav.tol > 0)) dav.tol = 1e-10;
  const int64_t nr = int64_t(p->N1) * p->N2 * p->N3;
  const double vol = cell_volume(p);
  double wsum = 0.0;
  for (int k = 0; k < p->nk; ++k) wsum += kw[k];
  const double nel = 2.0 * nocc * wsum;
  double* rho_out = nullptr;
  double* vtot = nullptr;
  QM_HIP(hipMalloc(&rho_out, size_t(nr) * sizeof(double)));
  qm_status status = QM_OK;
  qm_scf_stats stats{};
  try {
    QM_HIP(hipMalloc(&vtot, size_t(nr) * sizeof(double)));
    std::vector<double> occ(size_t(p->nk) * nbnd, 0.0), res(size_t(p->nk) * nbnd);
    for (int k = 0; k < p->nk; ++k)
      for (int n = 0; n < nocc; ++n) occ[size_t(k) * nbnd + n] = 2.0;
    run_grid_op(p, kFill, nel / vol, nullptr, nullptr, rho, nullptr, s);   // uniform start
    double r = 0.0;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
      hartree(p, rho, vh, nullptr, s);
      run_grid_op(p, kAdd, 0.0, vext, vh, vtot, nullptr, s);
      launch_vplan(p, vtot, s);
      qm_dav_stats ds{};
      const qm_status dst = qm_davidson_solve(p, -1, psi, eig, res.data(), nbnd, &dav, &ds, s);
      stats.dav_iterations += ds.iterations;
      stats.n_hpsi_bands += ds.n_hpsi_bands;
      if (dst != QM_OK) {
        status = dst;
        break;
      }
      density(p, -1, psi, nbnd, kw, occ.data(), rho_out, s);
      r = std::sqrt(vol / double(nr) * grid_sum(p, rho_out, rho, 1, s));
      if (r <= tol) {
        QM_HIP(hipMemcpyAsync(rho, rho_out, size_t(nr) * sizeof(double), hipMemcpyDeviceToDevice, s));
        break;
      }
      run_grid_op(p, kMix, alpha, rho_out, nullptr, rho, nullptr, s);
    }
    stats.iterations = std::min(it, max_iter);
    stats.residual = r;
    stats.converged = (status == QM_OK && r <= tol) ? 1 : 0;
    if (status == QM_OK) hartree(p, rho, vh, &stats.e_hartree, s);
    QM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipFree(rho_out);
    if (vtot) (void)hipFree(vtot);
    throw;
  }
  (void)hipFree(rho_out);
  (void)hipFree(vtot);
  stats.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if (status == QM_OK && !stats.converged) {
    p->err = "SCF did not converge within max_iter";
    return QM_E_NOT_CONVERGED;
  }
  return status;
}

}  // namespace qm

using namespace qm;

#define QM_DENS_GUARD(plan, ...)          \
  if (!plan) return QM_E_ARG;             \
  try {                                   \
    __VA_ARGS__;                          \
  } catch (const Error& e) {              \
    plan->err = e.what();                 \
    return e.code;                        \
  } catch (const std::exception& e) {     \
    plan->err = e.what();                 \
    return QM_E_STATE;                    \
  }

extern "C" {

qm_status qm_density(qm_hpsi_plan* plan, int32_t k, const void* psi, int32_t nbnd, const double* weights,
                     const double* occ, double* rho, void* stream) {
  QM_DENS_GUARD(plan, {
    density(plan, k, psi, nbnd, weights, occ, rho, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  })
}

qm_status qm_hartree(qm_hpsi_plan* plan, const double* rho, double* vh, double* e_hartree, void* stream) {
  QM_DENS_GUARD(plan, {
    hartree(plan, rho, vh, e_hartree, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  })
}

qm_status qm_hpsi_plan_set_vloc(qm_hpsi_plan* plan, const double* vloc_r, void* stream) {
  QM_DENS_GUARD(plan, {
    QM_REQUIRE(vloc_r, QM_E_ARG, "vloc_r must be non-NULL");
    launch_vplan(plan, vloc_r, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  })
}

qm_status qm_scf_hartree(qm_hpsi_plan* plan, const double* vext_r, const double* kweights, int32_t nocc,
                         void* psi, int32_t nbnd, const qm_scf_opts* opts, double* eig, double* rho,
                         double* vh, qm_scf_stats* stats, void* stream) {
  QM_DENS_GUARD(plan, {
    return scf_hartree(plan, vext_r, kweights, nocc, psi, nbnd, opts, eig, rho, vh, stats,
                       reinterpret_cast<hipStream_t>(stream));
  })
}

}  // extern "C"
