// Learned residual -> correction preconditioner for the Davidson (an extension of
// the paper's solver, Sec. 5 'dft' module): a per-(G, band) network with shared
// weights, 5 inputs -> 128 SiLU -> 2 outputs o, a complex gain
//   g = K(x) [exp(2 tanh o_0) + 0.5 i tanh o_1],   K(x) the Teter-Payne-Allan factor,
// and the correction t_n(G) = g(G, n) r_n(G).  The network only reshapes Teter, by a
// real factor in [e^-2, e^2]; with a zero output layer it is Teter exactly.  Features:
//   x = T(G)/T_n, log(1 + x), (theta_n - T_n)/T_n, |r_n(G)| sqrt(npw)/||r_n||, T(G)
// with T(G) = 1/2|k+G|^2 and T_n = <x_n|T|x_n>.  Weights are float32:
// W1[128][5], b1[128], W2[2][128], b2[2].
//
// Kernels: inference inside the Davidson (Teter factor where the network output
// is not finite), batched inference, loss + gradient of the per-band cosine loss
// 1 - |<t, delta>|^2/(|t|^2 |delta|^2) (rows grouped by band; deterministic
// fixed-order reductions), Adam, and the generation of (features, residual,
// target) training rows from a Davidson state and converged eigenvectors.
#include <cmath>

#include "dense.h"

namespace qm {

constexpr int NIN = QM_MLP_NIN, NH = QM_MLP_NHID, NPAR = QM_MLP_NPARAM;
constexpr int OW1 = 0, OB1 = NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + 2 * NH;

// z sigmoid(z) with the hardware reciprocal (about 1 ulp): exp(-z) -> inf gives -0, -> 0 gives z
__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float teter_k(float x) {
  const float num = 27.0f + x * (18.0f + x * (12.0f + 8.0f * x));
  return num / (num + 16.0f * x * x * x * x);
}

// raw network outputs o_0, o_1
__device__ __forceinline__ void mlp_out(const float* __restrict__ w, const float f[NIN], float& g0,
                                        float& g1) {
  float a0 = w[OB2], a1 = w[OB2 + 1];
#pragma unroll 8
  for (int u = 0; u < NH; ++u) {
    float z = w[OB1 + u];
#pragma unroll
    for (int i = 0; i < NIN; ++i) z += w[OW1 + u * NIN + i] * f[i];
    const float h = silu_f(z);
    a0 += w[OW2 + u] * h;
    a1 += w[OW2 + NH + u] * h;
  }
  g0 = a0;
  g1 = a1;
}

// gain (re, im) from the features (f[0] = x)
__device__ __forceinline__ void mlp_fwd(const float* __restrict__ w, const float f[NIN], float& g0,
                                        float& g1) {
  float o0, o1;
  mlp_out(w, f, o0, o1);
  const float k = teter_k(f[0]);
  g0 = k * __expf(2.0f * tanhf(o0));
  g1 = 0.5f * k * tanhf(o1);
}

__device__ double block_sum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < int(blockDim.x >> 6); ++i) s += red[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- Davidson correction
__global__ void __launch_bounds__(256) k_mlp_precond(DJobs jobs, const double2* __restrict__ Rr,
                                                     double2* __restrict__ V,
                                                     const int32_t* __restrict__ unconv,
                                                     const double* __restrict__ tkin,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ resn,
                                                     const double* __restrict__ kin_all,
                                                     const int64_t* __restrict__ goff,
                                                     const float* __restrict__ weights) {
  // the weights are read at wave-uniform addresses straight from the read-only argument
  // (scalar loads), so the hidden-layer loop issues no LDS traffic
  const float* __restrict__ w = weights;
  __shared__ double red[16];
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb, j = blockIdx.x;
  if (j >= J.nu) return;
  const int n = unconv[int64_t(J.k) * nb + j];
  const double tn = tkin[int64_t(J.k) * nb + n];
  const double th = theta[int64_t(J.k) * jobs.mb + n];
  const double rs = sqrt(double(J.npw)) / resn[int64_t(J.k) * nb + n];
  const double* kin = kin_all + goff[J.k];
  const double2* r = Rr + J.xoff + int64_t(n) * J.npw;
  double2* t = V + J.voff + int64_t(J.m - J.nu + j) * J.npw;
  double ss = 0.0;
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const double2 rv = r[g];
    float f[NIN];
    make_feat(kin[g], tn, th, sqrt(rv.x * rv.x + rv.y * rv.y) * rs, f);
    float g0, g1;
    mlp_fwd(w, f, g0, g1);
    double gr = g0, gi = g1;
    if (!isfinite(gr) || !isfinite(gi)) {  // Teter fallback
      const double x = kin[g] / tn;
      const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
      gr = num / (num + 16.0 * x * x * x * x);
      gi = 0.0;
    }
    const double2 v = make_double2(gr * rv.x - gi * rv.y, gr * rv.y + gi * rv.x);
    t[g] = v;
    ss += v.x * v.x + v.y * v.y;
  }
  ss = block_sum_d(ss, red);
  const double s = 1.0 / sqrt(ss);
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const double2 v = t[g];
    t[g] = make_double2(v.x * s, v.y * s);
  }
}

// ---------------------------------------------------------------- batched inference
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ weights,
                                                     const float* __restrict__ feat,
                                                     float* __restrict__ gain, int64_t n) {
  __shared__ float w[NPAR];
  for (int i = threadIdx.x; i < NPAR; i += blockDim.x) w[i] = weights[i];
  __syncthreads();
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < n;
       r += int64_t(gridDim.x) * blockDim.x) {
    float f[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) f[i] = feat[r * NIN + i];
    float g0, g1;
    mlp_fwd(w, f, g0, g1);
    gain[2 * r] = g0;
    gain[2 * r + 1] = g1;
  }
}

// ---------------------------------------------------------------- loss and gradient
// One workgroup (256 threads) per band.  Pass 1: a = sum conj(t) delta, |t|^2, |delta|^2.
// Pass 2: chunks of 64 rows, one row per thread, backprop; the per-parameter sums over a
// chunk's rows are done by all threads in fixed order.  part[b][NPAR] and lossb[b] out.
constexpr int CH = 64;
__global__ void __launch_bounds__(256) k_mlp_loss_grad(const float* __restrict__ weights,
                                                       const float* __restrict__ feat,
                                                       const float* __restrict__ resid,
                                                       const float* __restrict__ target,
                                                       const int32_t* __restrict__ band_ptr,
                                                       int nbands, float* __restrict__ part,
                                                       double* __restrict__ lossb) {
  __shared__ float w[NPAR];
  __shared__ float sdz[CH][NH + 1];
  __shared__ float sh[CH][NH + 1];
  __shared__ float sf[CH][NIN];
  __shared__ float sdg[CH][2];
  __shared__ double red[16];
  const int b = blockIdx.x;
  const int r0 = band_ptr[b], r1 = band_ptr[b + 1];
  const int tid = threadIdx.x;
  for (int i = tid; i < NPAR; i += blockDim.x) w[i] = weights[i];
  __syncthreads();
  double ar = 0.0, ai = 0.0, tt = 0.0, dd = 0.0;
  for (int r = r0 + tid; r < r1; r += blockDim.x) {
    float f[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) f[i] = feat[int64_t(r) * NIN + i];
    float g0, g1;
    mlp_fwd(w, f, g0, g1);
    const double rr = resid[2 * int64_t(r)], ri = resid[2 * int64_t(r) + 1];
    const double tr = g0 * rr - g1 * ri, ti = g0 * ri + g1 * rr;
    const double dr = target[2 * int64_t(r)], di = target[2 * int64_t(r) + 1];
    ar += tr * dr + ti * di;   // conj(t) delta
    ai += tr * di - ti * dr;
    tt += tr * tr + ti * ti;
    dd += dr * dr + di * di;
  }
  ar = block_sum_d(ar, red);
  ai = block_sum_d(ai, red);
  tt = block_sum_d(tt, red);
  dd = block_sum_d(dd, red);
  const double a2 = ar * ar + ai * ai;
  const double c = a2 / (tt * dd);
  if (tid == 0) lossb[b] = 1.0 - c;
  // dL/dt = -(1/nbands) [2 conj(a) delta/(tt dd) - 2 |a|^2 t/(tt^2 dd)]
  const double s1 = 2.0 / (tt * dd), s2 = 2.0 * a2 / (tt * tt * dd), inv = 1.0 / nbands;
  float acc[5] = {0, 0, 0, 0, 0};  // up to ceil(NPAR / 256) = 5 parameters per thread
  for (int c0 = r0; c0 < r1; c0 += CH) {
    const int r = c0 + tid;
    if (tid < CH && r < r1) {
      float f[NIN];
#pragma unroll
      for (int i = 0; i < NIN; ++i) {
        f[i] = feat[int64_t(r) * NIN + i];
        sf[tid][i] = f[i];
      }
      float o0 = w[OB2], o1 = w[OB2 + 1];
      for (int u = 0; u < NH; ++u) {
        float z = w[OB1 + u];
#pragma unroll
        for (int i = 0; i < NIN; ++i) z += w[OW1 + u * NIN + i] * f[i];
        const float sg = 1.0f / (1.0f + __expf(-z));
        const float h = z * sg;
        sh[tid][u] = h;
        sdz[tid][u] = sg * (1.0f + z * (1.0f - sg));  // silu'(z), scaled by dh below
        o0 += w[OW2 + u] * h;
        o1 += w[OW2 + NH + u] * h;
      }
      const float kx = teter_k(f[0]), th0 = tanhf(o0), th1 = tanhf(o1);
      const float e0 = __expf(2.0f * th0);
      const float g0 = kx * e0, g1 = 0.5f * kx * th1;
      const double rr = resid[2 * int64_t(r)], ri = resid[2 * int64_t(r) + 1];
      const double tr = g0 * rr - g1 * ri, ti = g0 * ri + g1 * rr;
      const double dr = target[2 * int64_t(r)], di = target[2 * int64_t(r) + 1];
      // conj(a) delta = (ar - i ai)(dr + i di)
      const double cr = ar * dr + ai * di, ci = ar * di - ai * dr;
      const double dtr = -inv * (s1 * cr - s2 * tr), dti = -inv * (s1 * ci - s2 * ti);
      // dL/dg_re = Re(conj(dt) r), dL/dg_im = -Im(conj(dt) r); then through the output map
      const float dg0 = float(dtr * rr + dti * ri) * kx * e0 * 2.0f * (1.0f - th0 * th0);
      const float dg1 = float(-(dtr * ri - dti * rr)) * 0.5f * kx * (1.0f - th1 * th1);
      sdg[tid][0] = dg0;
      sdg[tid][1] = dg1;
      for (int u = 0; u < NH; ++u) {
        const float dh = w[OW2 + u] * dg0 + w[OW2 + NH + u] * dg1;
        sdz[tid][u] *= dh;
      }
    } else if (tid < CH) {
      sdg[tid][0] = sdg[tid][1] = 0.0f;
      for (int i = 0; i < NIN; ++i) sf[tid][i] = 0.0f;
      for (int u = 0; u < NH; ++u) sdz[tid][u] = sh[tid][u] = 0.0f;
    }
    __syncthreads();
    const int nrow = min(CH, r1 - c0);
    for (int q = 0; q < 5; ++q) {
      const int pidx = tid + q * 256;
      if (pidx >= NPAR) break;
      float s = 0.0f;
      if (pidx < OB1) {
        const int u = pidx / NIN, i = pidx - u * NIN;
        for (int rr = 0; rr < nrow; ++rr) s += sdz[rr][u] * sf[rr][i];
      } else if (pidx < OW2) {
        const int u = pidx - OB1;
        for (int rr = 0; rr < nrow; ++rr) s += sdz[rr][u];
      } else if (pidx < OB2) {
        const int cc = (pidx - OW2) / NH, u = (pidx - OW2) % NH;
        for (int rr = 0; rr < nrow; ++rr) s += sdg[rr][cc] * sh[rr][u];
      } else {
        const int cc = pidx - OB2;
        for (int rr = 0; rr < nrow; ++rr) s += sdg[rr][cc];
      }
      acc[q] += s;
    }
    __syncthreads();
  }
  for (int q = 0; q < 5; ++q) {
    const int pidx = tid + q * 256;
    if (pidx < NPAR) part[int64_t(b) * NPAR + pidx] = acc[q];
  }
}

__global__ void k_mlp_sum_parts(const float* __restrict__ part, int nbands, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  double s = 0.0;
  for (int b = 0; b < nbands; ++b) s += part[int64_t(b) * NPAR + p];
  grad[p] = float(s);
}

__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int t, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  const float gg = g[p];
  const float mm = b1 * m[p] + (1.0f - b1) * gg;
  const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.0f - powf(b1, float(t)));
  const float vh = vv / (1.0f - powf(b2, float(t)));
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

void mlp_precondition(qm_hpsi_plan* p, const DJobs& jobs, const void* weights, hipStream_t s,
                      const double2* R, double2* V, const int32_t* unconv, const double* tkin,
                      const double* theta, const double* resn, const int64_t* goff) {
  hipLaunchKernelGGL(k_mlp_precond, dim3(jobs.nb, jobs.n), dim3(256), 0, s, jobs, R, V, unconv, tkin,
                     theta, resn, p->g.kin, goff, reinterpret_cast<const float*>(weights));
  QM_HIP(hipGetLastError());
}

}  // namespace qm

using namespace qm;

extern "C" {

qm_status qm_mlp_forward(const float* weights, const float* feat, float* gain, int64_t n, void* stream) {
  if (!weights || !feat || !gain || n < 0) return QM_E_ARG;
  if (n == 0) return QM_OK;
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     weights, feat, gain, n);
  return hipGetLastError() == hipSuccess ? QM_OK : QM_E_HIP;
}

qm_status qm_mlp_loss_grad(const float* weights, const float* feat, const float* resid,
                           const float* target, const int32_t* band_ptr, int32_t nbands, float* grad,
                           double* loss, void* stream) {
  if (!weights || !feat || !resid || !target || !band_ptr || !grad || nbands < 1) return QM_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* part = nullptr;
  double* lb = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&part), sizeof(float) * size_t(nbands) * NPAR, s) != hipSuccess)
    return QM_E_NOMEM;
  if (hipMallocAsync(reinterpret_cast<void**>(&lb), sizeof(double) * size_t(nbands), s) != hipSuccess) {
    (void)hipFreeAsync(part, s);
    return QM_E_NOMEM;
  }
  hipLaunchKernelGGL(k_mlp_loss_grad, dim3(nbands), dim3(256), 0, s, weights, feat, resid, target,
                     band_ptr, nbands, part, lb);
  hipLaunchKernelGGL(k_mlp_sum_parts, dim3((NPAR + 255) / 256), dim3(256), 0, s, part, nbands, grad);
  std::vector<double> hl(nbands);
  qm_status st = QM_OK;
  if (hipMemcpyAsync(hl.data(), lb, sizeof(double) * nbands, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    st = QM_E_HIP;
  (void)hipFreeAsync(part, s);
  (void)hipFreeAsync(lb, s);
  if (loss) {
    double t = 0.0;
    for (double x : hl) t += x;
    *loss = t / nbands;
  }
  return st;
}

qm_status qm_mlp_adam(float* weights, const float* grad, float* m, float* v, int32_t t, float lr,
                      float beta1, float beta2, float eps, void* stream) {
  if (!weights || !grad || !m || !v || t < 1) return QM_E_ARG;
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), weights, grad, m, v, t, lr, beta1, beta2, eps);
  return hipGetLastError() == hipSuccess ? QM_OK : QM_E_HIP;
}

}  // extern "C"
