// Plane-wave matrix elements of the GW polarizability (Sec. 5, 'gw' module, matrix
// elements of the Epsilon class): M_nn'(k, q, G) = <n k+q| e^{i(q+G).r} |n' k>, computed the
// way the paper describes - both band sets to real space by inverse FFT, the product
// conj(u_{n,k+q}) u_{n',k}, and one more inverse FFT of every product, read at the requested
// G vectors.  All transforms are full-grid batched line FFTs in float64.
#include <cstring>

#include "qm_internal.h"

namespace qm {

// zero the grids, then u_b(G) at the grid index of every G of the sphere (m mod N)
__global__ void k_scatter_grid(const double2* __restrict__ c, const int32_t* __restrict__ flat, int npw,
                               int nb, int64_t nr, double2* __restrict__ u) {
  const int64_t total = int64_t(nb) * npw;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t / npw;
    const int g = int(t - b * npw);
    u[b * nr + flat[g]] = c[t];
  }
}

// f[b'] = conj(ua) u[b'] over nb grids of nr points
__global__ void k_conj_product(const double2* __restrict__ ua, const double2* __restrict__ u, int nb,
                               int64_t nr, double2* __restrict__ f) {
  const int64_t total = int64_t(nb) * nr;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const double2 a = ua[t % nr], b = u[t];
    f[t] = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
  }
}

// out[b'][g] = f[b'][gidx[g]] / nr
__global__ void k_gather_g(const double2* __restrict__ f, const int32_t* __restrict__ gidx, int ng, int nb,
                           int64_t nr, double2* __restrict__ out) {
  const int64_t total = int64_t(nb) * ng;
  const double s = 1.0 / double(nr);
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t / ng;
    const int g = int(t - b * ng);
    const double2 v = f[b * nr + gidx[g]];
    out[t] = make_double2(v.x * s, v.y * s);
  }
}

static int blocks_for(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 16384)); }

static void mtxel(qm_hpsi_plan* p, int kq, const void* psi_kq, int nb1, int k, const void* psi_k, int nb2,
                  const int32_t* miller_g, int ng, void* out, hipStream_t s) {
  QM_REQUIRE(psi_kq && psi_k && miller_g && out, QM_E_ARG, "NULL argument");
  QM_REQUIRE(kq >= 0 && kq < p->nk && k >= 0 && k < p->nk, QM_E_ARG, "k out of range");
  QM_REQUIRE(nb1 >= 1 && nb2 >= 1 && ng >= 1, QM_E_ARG, "need nb1, nb2, ng >= 1");
  const int Ns[3] = {p->N1, p->N2, p->N3};
  std::vector<int32_t> gidx(ng);
  for (int g = 0; g < ng; ++g) {
    int ii[3];
    for (int d = 0; d < 3; ++d) {
      const int v = miller_g[3 * g + d];
      QM_REQUIRE(2 * std::abs(int64_t(v)) < Ns[d], QM_E_ARG, "G outside the FFT grid (need 2|m_i| < N_i)");
      ii[d] = ((v % Ns[d]) + Ns[d]) % Ns[d];
    }
    gidx[g] = (ii[0] * Ns[1] + ii[1]) * Ns[2] + ii[2];
  }
  const int64_t nr = int64_t(Ns[0]) * Ns[1] * Ns[2];
  const KInfo& a = p->kinfo[kq];
  const KInfo& b = p->kinfo[k];
  double2 *u1 = nullptr, *u2 = nullptr, *f = nullptr;
  int32_t* gdev = nullptr;
  auto release = [&]() {
    void* q[] = {u1, u2, f, gdev};
    for (void* x : q)
      if (x) (void)hipFree(x);
  };
  try {
    QM_HIP(hipMalloc(&u1, size_t(nb1) * nr * sizeof(double2)));
    QM_HIP(hipMalloc(&u2, size_t(nb2) * nr * sizeof(double2)));
    QM_HIP(hipMalloc(&f, size_t(nb2) * nr * sizeof(double2)));
    QM_HIP(hipMalloc(&gdev, size_t(ng) * sizeof(int32_t)));
    QM_HIP(hipMemcpyAsync(gdev, gidx.data(), size_t(ng) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    QM_HIP(hipMemsetAsync(u1, 0, size_t(nb1) * nr * sizeof(double2), s));
    QM_HIP(hipMemsetAsync(u2, 0, size_t(nb2) * nr * sizeof(double2), s));
    hipLaunchKernelGGL(k_scatter_grid, dim3(blocks_for(int64_t(nb1) * a.npw)), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(psi_kq), p->g.flat + a.g_off, a.npw, nb1, nr, u1);
    hipLaunchKernelGGL(k_scatter_grid, dim3(blocks_for(int64_t(nb2) * b.npw)), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(psi_k), p->g.flat + b.g_off, b.npw, nb2, nr, u2);
    QM_HIP(hipGetLastError());
    fft3_batched(p, u1, nb1, +1, s);   // u(r) = sum_G c(G) e^{iG.r}
    fft3_batched(p, u2, nb2, +1, s);
    for (int n = 0; n < nb1; ++n) {
      hipLaunchKernelGGL(k_conj_product, dim3(blocks_for(int64_t(nb2) * nr)), dim3(256), 0, s,
                         u1 + int64_t(n) * nr, u2, nb2, nr, f);
      QM_HIP(hipGetLastError());
      fft3_batched(p, f, nb2, +1, s);
      hipLaunchKernelGGL(k_gather_g, dim3(blocks_for(int64_t(nb2) * ng)), dim3(256), 0, s, f, gdev, ng, nb2,
                         nr, reinterpret_cast<double2*>(out) + int64_t(n) * nb2 * ng);
      QM_HIP(hipGetLastError());
    }
    QM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    release();
    throw;
  }
  release();
}

}  // namespace qm

using namespace qm;

extern "C" qm_status qm_mtxel(qm_hpsi_plan* plan, int32_t kq, const void* psi_kq, int32_t nb1, int32_t k,
                              const void* psi_k, int32_t nb2, const int32_t* miller_g, int32_t ng, void* mtx,
                              void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    mtxel(plan, kq, psi_kq, nb1, k, psi_k, nb2, miller_g, ng, mtx, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  } catch (const Error& e) {
    plan->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    plan->err = e.what();
    return QM_E_STATE;
  }
}
