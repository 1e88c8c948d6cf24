// Small dense float64 linear algebra for the Davidson subspace, one workgroup
// per k-point (all active k-points in one launch):
//   k_hs_fill     complete the Hermitian projected matrix from its new columns
//   k_tridiag     Householder reduction of the complex Hermitian projected matrix
//                 to a real symmetric tridiagonal one (H = I - tau v v^H, with the
//                 reflector chosen so the off-diagonal comes out real)
//   k_trd_start/k_trd_step  the same reduction spread over many workgroups, one
//                 launch per step (used from a basis of a few hundred columns)
//   k_eig_vals, k_eig_inviter, k_eig_orth  lowest nb eigenvalues by Sturm-count
//                 multisection, eigenvectors by inverse iteration (re-orthogonalised
//                 inside clusters of close eigenvalues, so degenerate levels get
//                 orthonormal vectors)
//   k_bt_tfactor, k_bt_apply  eigenvectors back through the reflectors, 32 at a time
//                 (compact WY form)
//   k_chol_inv    Cholesky G = L L^H of a Gram matrix and W = conj(L^-1)^T for the
//                 CholQR update T <- L^-1 T
//   k_residual    r = HX - theta X, ||r||, band kinetic energy <x|T|x>
//   k_teter       Teter-Payne-Allan correction t = K(T(G)/T_n) r, normalised
// These take the place of the LAPACK / cuSOLVER calls of a library-based Davidson.
#include "dense.h"

namespace qm {

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// block-wide sum (blockDim.x a multiple of 64, <= 1024); identical result on every thread
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// two block-wide sums at once (red holds 2 * waves values)
__device__ void block_sum2(double& a, double& b, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[w] = a;
    red[nw + w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < nw; ++i) {
    sa += red[i];
    sb += red[nw + i];
  }
  __syncthreads();
  a = sa;
  b = sb;
}

// ---------------------------------------------------------------- Hermitian fill
__global__ void k_hs_fill(DJobs jobs, double2* __restrict__ Hs) {
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb;
  double2* H = Hs + int64_t(J.k) * mb * mb;
  const int nnew = J.m - J.m_old;
  const int64_t total = int64_t(J.m) * nnew;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t / nnew), j = J.m_old + int(t % nnew);
    if (i < J.m_old) {
      H[int64_t(j) * mb + i] = cconj(H[int64_t(i) * mb + j]);
    } else if (i < j) {
      const double2 a = H[int64_t(i) * mb + j], b = H[int64_t(j) * mb + i];
      const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      H[int64_t(i) * mb + j] = h;
      H[int64_t(j) * mb + i] = cconj(h);
    } else if (i == j) {
      H[int64_t(i) * mb + i] = make_double2(H[int64_t(i) * mb + i].x, 0.0);
    }
  }
}

// copy Hs[0:m][0:m] -> Aw (eigensolver workspace)
__global__ void k_hs_copy(DJobs jobs, const double2* __restrict__ Hs, double2* __restrict__ Aw) {
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb;
  const int64_t total = int64_t(J.m) * J.m;
  const int64_t base = int64_t(J.k) * mb * mb;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(t / J.m), j = int(t % J.m);
    Aw[base + int64_t(i) * mb + j] = Hs[base + int64_t(i) * mb + j];
  }
}

// ---------------------------------------------------------------- tridiagonalisation
// Householder reduction with the rank-2 update of step j-1 applied lazily: step j first
// brings column j up to date, builds its reflector, then makes one pass over the lower
// triangle of the trailing block that applies the pending update and accumulates
// p = tau A v at the same time (one read and one write per stored element and step).
// A stored element a_rc (c < r) serves both halves of the Hermitian product: a_rc v_c
// goes to p_r (summed in the wave that owns row r) and conj(a_rc) v_r to p_c (summed in
// a column-sum slice of the wave's own, and the slices added in wave order, so the result
// does not depend on the order the waves ran in).  A (row-major, stride mb) holds the
// Hermitian matrix in its lower triangle (the upper one is never read) and is destroyed;
// column j below the subdiagonal receives v_j (v_j[j+1] = 1 implicit).
// Dynamic LDS: 4 + 16 vectors of ms >= m complex entries (ms = the launch's largest m).
__global__ void __launch_bounds__(1024) k_tridiag(DJobs jobs, double2* __restrict__ Aw,
                                                  double* __restrict__ dd, double* __restrict__ ee,
                                                  double2* __restrict__ tau, int ms) {
  extern __shared__ double2 sh[];   // vA, vB, pA, pB, then the 16 waves' column sums: [ms] each
  const DJob& J = jobs.j[blockIdx.x];
  const int mb = jobs.mb, m = J.m;
  double2* A = Aw + int64_t(J.k) * mb * mb;
  double* d = dd + int64_t(J.k) * mb;
  double* e = ee + int64_t(J.k) * mb;
  double2* tk = tau + int64_t(J.k) * mb;
  __shared__ double red[32];
  __shared__ double2 s_tau, s_scale, s_alpha;
  __shared__ double s_beta, s_dj;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double2* colsum = sh + int64_t(4 + wave) * ms;   // this wave's column sums
  for (int i = tid; i < (4 + nw) * ms; i += blockDim.x) sh[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int j = 0; j < m - 1; ++j) {
    double2* vc = sh + (j & 1 ? ms : 0);          // this step's reflector
    double2* pc = sh + 2 * ms + (j & 1 ? ms : 0);  // this step's p, then w
    const double2* vq = sh + (j & 1 ? 0 : ms);     // pending reflector (step j-1)
    const double2* wq = sh + 2 * ms + (j & 1 ? 0 : ms);  // pending w
    // column j, rows >= j, brought up to date and kept in registers (m <= 2 blockDim)
    const double2 vqj = vq[j], wqj = wq[j];
    double2 colv[2];
    double xs = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = j + tid + q * int(blockDim.x);
      colv[q] = make_double2(0.0, 0.0);
      if (r < m) {
        double2 a = A[int64_t(r) * mb + j];
        a = csub2(a, cmul2(vq[r], cconj(wqj)));
        a = csub2(a, cmul2(wq[r], cconj(vqj)));
        colv[q] = a;
        if (r == j) s_dj = a.x;
        else if (r == j + 1) s_alpha = a;
        else xs += a.x * a.x + a.y * a.y;
      }
    }
    xs = block_sum(xs, red);   // its barriers also publish s_dj and s_alpha
    if (tid == 0) {
      const double2 alpha = s_alpha;
      if (xs == 0.0 && alpha.y == 0.0) {
        s_tau = make_double2(0.0, 0.0);
        s_beta = alpha.x;
        s_scale = make_double2(0.0, 0.0);
      } else {
        double beta = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xs);
        if (alpha.x >= 0.0) beta = -beta;
        s_tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);
        const double dn = den.x * den.x + den.y * den.y;
        s_scale = make_double2(den.x / dn, -den.y / dn);
        s_beta = beta;
      }
      d[j] = s_dj;
      e[j] = s_beta;
      tk[j] = s_tau;
    }
    __syncthreads();
    const double2 t = s_tau;
    const bool refl = !(t.x == 0.0 && t.y == 0.0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = j + tid + q * int(blockDim.x);
      if (r > j && r < m) {
        double2 x = make_double2(0.0, 0.0);
        if (refl) {
          x = r == j + 1 ? make_double2(1.0, 0.0) : cmul2(colv[q], s_scale);
          if (r > j + 1) A[int64_t(r) * mb + j] = x;
        }
        vc[r] = x;
      }
    }
    for (int i = tid; i < nw * ms; i += blockDim.x) sh[4 * ms + i] = make_double2(0.0, 0.0);
    if (tid == 0) vc[j] = make_double2(0.0, 0.0);
    __syncthreads();
    // fused pass over the lower triangle of [j+1, m): pending update, then A v.  A wave
    // takes four rows at a time so the reflector values it reads from LDS serve four rows.
    // Row groups go to waves in snake order (the lower triangle's rows grow in length).
    const int ngroups = (m - j - 1 + 3) / 4;
    for (int rd = 0; rd * nw < ngroups; ++rd) {
      const int g = rd * nw + ((rd & 1) ? nw - 1 - wave : wave);
      if (g >= ngroups) continue;
      const int r0 = j + 1 + 4 * g;
      double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
      double2 vr[4], wr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = min(r0 + q, m - 1);
        vr[q] = vq[r];
        wr[q] = wq[r];
      }
      const int rmax = min(r0 + 3, m - 1);
      for (int c = j + 1 + lane; c <= rmax; c += 64) {
        const double2 vqc = cconj(vq[c]), wqc = cconj(wq[c]), b = vc[c];
        double tr = 0.0, ti = 0.0;   // sum over this wave's rows r > c of conj(a_rc) v_r
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = r0 + q;
          if (r > rmax || c > r) continue;
          double2* ap = A + int64_t(r) * mb + c;
          double2 a = *ap;
          a = csub2(a, cmul2(vr[q], wqc));
          a = csub2(a, cmul2(wr[q], vqc));
          *ap = a;
          sr[q] += a.x * b.x - a.y * b.y;
          si[q] += a.x * b.y + a.y * b.x;
          if (c < r) {
            const double2 br = vc[r];   // same address on every lane: an LDS broadcast
            tr += a.x * br.x + a.y * br.y;
            ti += a.x * br.y - a.y * br.x;
          }
        }
        if (c < rmax) {   // lanes of a wave hold distinct c: a plain update of its own slice
          colsum[c].x += tr;
          colsum[c].y += ti;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        for (int o = 32; o > 0; o >>= 1) {
          sr[q] += __shfl_down(sr[q], o, 64);
          si[q] += __shfl_down(si[q], o, 64);
        }
        if (lane == 0 && r0 + q < m) pc[r0 + q] = make_double2(sr[q], si[q]);
      }
    }
    if (tid == 0) pc[j] = make_double2(0.0, 0.0);
    __syncthreads();
    double pr = 0.0, pi = 0.0;   // p = tau (row part + column part); p^H v
    for (int c = j + 1 + tid; c < m; c += blockDim.x) {
      double2 cs = pc[c];
      for (int w = 0; w < nw; ++w) cs = cadd2(cs, sh[int64_t(4 + w) * ms + c]);
      const double2 pv = cmul2(t, cs), vv = vc[c];
      pc[c] = pv;
      pr += pv.x * vv.x + pv.y * vv.y;
      pi += pv.x * vv.y - pv.y * vv.x;
    }
    block_sum2(pr, pi, red);
    const double2 aw = cmul2(make_double2(-0.5 * t.x, -0.5 * t.y), make_double2(pr, pi));
    for (int c = j + 1 + tid; c < m; c += blockDim.x) pc[c] = cadd2(pc[c], cmul2(aw, vc[c]));
    __syncthreads();
  }
  if (tid == 0) {
    const int j = m - 1;  // pending update of step m-2 on the last diagonal element
    const double2* vq = sh + ((m - 2) & 1 ? ms : 0);
    const double2* wq = sh + 2 * ms + ((m - 2) & 1 ? ms : 0);
    double a = A[int64_t(j) * mb + j].x;
    if (m >= 2) a -= 2.0 * (vq[j].x * wq[j].x + vq[j].y * wq[j].y);
    d[j] = a;
    e[j] = 0.0;
    tk[j] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------- tridiagonalisation, many CUs
// The same reduction (same reflectors, same lazy rank-2 update) spread over the whole GPU:
// one launch per step j, one 256-thread workgroup per 64 x 64 tile of the lower triangle of
// the trailing block [j+1, m).  A tile applies the pending update of step j-1 to its
// elements and writes its share of A v_j to a slot of its own: 64 row sums (a_rc v_c) and
// 64 column sums (conj(a_rc) v_r).  The workgroup that finishes last (arrival counter) adds
// the slots in a fixed order (for a row block: the row sums of the tiles left of the
// diagonal, left to right, then the column sums of the tiles below it, top to bottom), so
// the result does not depend on which workgroup ran when, forms p = tau A v and
// w = p - (tau/2)(p^H v) v, brings column j+1 up to date and builds the next reflector, so
// the following launch can start at once.  Only the order of the floating-point additions
// into p differs from the one-workgroup kernel.
// Cross-workgroup traffic inside a launch goes through agent-scope atomics only, so no
// workgroup needs a memory fence (an agent-scope release writes back the whole L2 and costs
// ~70 ns per workgroup, serialised): a tile writes its slot with atomic exchanges, whose
// returned values it waits for before its counter increment, and the last workgroup reads
// the slots with agent-scope atomic loads.  Column j+1 is never stored by the tiles (it is
// dead after this step): the last workgroup rebuilds it from the values of the previous
// launch with both pending updates.
constexpr int kTrdRows = kTrdMaxBasis / 256;   // column rows per tail thread

// v where ok, else 0 (two scalar selects: a select between double2 values can be compiled
// into a load through a pointer to a zero kept in private memory)
__device__ __forceinline__ double2 keep(double2 v, bool ok) {
  return make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
}

// Column jc (rows jc + tid + 256 q in register q, q < kTrdRows) -> d[jc], e[jc], tau[jc] and
// the reflector v (vout[r], r in (jc, m); stored in A below the subdiagonal too).
__device__ void trd_reflector(int jc, int m, int mb, double2* A, double2 (&a)[kTrdRows],
                              double2* vout, double* d, double* e, double2* tk, double* red) {
  __shared__ double2 s_alpha, s_tau, s_scale;
  __shared__ double s_dj, s_beta;
  const int tid = threadIdx.x;
  double xs = 0.0;
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = jc + tid + q * 256;
    if (r >= m) continue;
    if (r == jc) s_dj = a[q].x;
    else if (r == jc + 1) s_alpha = a[q];
    else xs += a[q].x * a[q].x + a[q].y * a[q].y;
  }
  xs = block_sum(xs, red);   // its barriers publish s_dj and s_alpha
  if (tid == 0) {
    if (jc == m - 1) {       // last column: no reflector
      s_tau = make_double2(0.0, 0.0);
      s_beta = 0.0;
      s_scale = make_double2(0.0, 0.0);
    } else {
      const double2 alpha = s_alpha;
      if (xs == 0.0 && alpha.y == 0.0) {
        s_tau = make_double2(0.0, 0.0);
        s_beta = alpha.x;
        s_scale = make_double2(0.0, 0.0);
      } else {
        double beta = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xs);
        if (alpha.x >= 0.0) beta = -beta;
        s_tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);
        const double dn = den.x * den.x + den.y * den.y;
        s_scale = make_double2(den.x / dn, -den.y / dn);
        s_beta = beta;
      }
    }
    d[jc] = s_dj;
    e[jc] = s_beta;
    tk[jc] = s_tau;
  }
  __syncthreads();
  const double2 t = s_tau, sc = s_scale;
  const bool refl = !(t.x == 0.0 && t.y == 0.0);
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = jc + tid + q * 256;
    if (r <= jc || r >= m) continue;
    double2 x = make_double2(0.0, 0.0);
    if (refl) {
      x = r == jc + 1 ? make_double2(1.0, 0.0) : cmul2(a[q], sc);
      if (r > jc + 1) A[int64_t(r) * mb + jc] = x;
    }
    vout[r] = x;
  }
}

// First reflector (column 0) and a zero accumulator; one workgroup per job.
__global__ void __launch_bounds__(256) k_trd_start(DJobs jobs, double2* __restrict__ Aw,
                                                   double* __restrict__ dd, double* __restrict__ ee,
                                                   double2* __restrict__ tau, TrdWork tw) {
  __shared__ double red[32];
  const DJob& J = jobs.j[blockIdx.x];
  const int mb = jobs.mb, m = J.m, k = J.k;
  double2* A = Aw + int64_t(k) * mb * mb;
  if (threadIdx.x == 0) tw.cnt[k] = 0u;
  for (int b = threadIdx.x; b < tw.nblk; b += 256) tw.bcnt[int64_t(k) * tw.nblk + b] = 0u;
  double2 a[kTrdRows];
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = threadIdx.x + q * 256;
    a[q] = keep(A[int64_t(min(r, m - 1)) * mb], r < m);
  }
  trd_reflector(0, m, mb, A, a, tw.v + int64_t(k) * 2 * mb, dd + int64_t(k) * mb,
                ee + int64_t(k) * mb, tau + int64_t(k) * mb, red);
}

// Step j (0 <= j <= m - 2).  Grid (tiles of the largest job, jobs); 256 threads.
__global__ void __launch_bounds__(256) k_trd_step(DJobs jobs, int j, double2* __restrict__ Aw,
                                                  double* __restrict__ dd, double* __restrict__ ee,
                                                  double2* __restrict__ tau, TrdWork tw) {
  constexpr int T = kTrdTile;
  __shared__ double2 s_col[4][T];
  __shared__ double2 s_row[T];
  __shared__ double2 s_vec[6][T];
  __shared__ double red[32];
  __shared__ unsigned s_last, s_fin;
  __shared__ double2 s_wj1, s_vj1;
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, m = J.m, k = J.k;
  if (j >= m - 1) return;
  const int j1 = j + 1;
  const int b0 = j1 / T, nt = (m - 1) / T - b0 + 1, ntiles = nt * (nt + 1) / 2;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  int ti = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int R0 = (b0 + ti) * T, C0 = (b0 + tj) * T;
  double2* A = Aw + int64_t(k) * mb * mb;
  const double2* vj = tw.v + (int64_t(k) * 2 + (j & 1)) * mb;        // this step's reflector
  const double2* vp = tw.v + (int64_t(k) * 2 + ((j + 1) & 1)) * mb;  // pending: v_{j-1}
  double2* W = tw.w + int64_t(k) * mb;                                // pending: w_{j-1}
  double* PS = reinterpret_cast<double*>(tw.part + int64_t(k) * tw.ptiles * 2 * T);
  const bool pend = j > 0;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15, lane = tid & 63, wave = tid >> 6;
  const double2 z = make_double2(0.0, 0.0);
  // Every load reads an in-bounds address (indices clamped to m - 1) and masked values are
  // replaced afterwards: a conditional load would be compiled into a load through a
  // selected pointer (flat addressing, split, serialised waits).
  // The tile's slices of v_j, v_{j-1}, w_{j-1} (rows and columns) go through LDS, one load
  // per entry; the tile itself is loaded at the same time.  Every load reads an in-bounds
  // address (indices clamped to m - 1) and masked values are replaced afterwards: a
  // conditional load would be compiled into a load through a selected pointer.
  double2 a[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rc = min(R0 + 4 * tr + q, m - 1);
#pragma unroll
    for (int u = 0; u < 4; ++u) a[q][u] = A[int64_t(rc) * mb + min(C0 + 4 * tc + u, rc)];
  }
  {
    const int wv = __builtin_amdgcn_readfirstlane(wave), i = lane;
    const int r = R0 + i, c = C0 + i, rr = min(r, m - 1), cc = min(c, m - 1);
    const bool okr = r >= j1 && r < m, okc = c >= j1 && c < m;
    if (wv == 0) {          // wave 0: v_j rows, v_{j-1} columns
      const double2 x = vj[rr], y = vp[cc];
      s_vec[0][i] = keep(x, okr);
      s_vec[4][i] = keep(y, okc && pend);
    } else if (wv == 1) {   // wave 1: v_{j-1} rows, w_{j-1} columns
      const double2 x = vp[rr], y = W[cc];
      s_vec[1][i] = keep(x, okr && pend);
      s_vec[5][i] = keep(y, okc && pend);
    } else if (wv == 2) {   // wave 2: w_{j-1} rows
      const double2 x = W[rr];
      s_vec[2][i] = keep(x, okr && pend);
    } else {                // wave 3: v_j columns
      const double2 x = vj[cc];
      s_vec[3][i] = keep(x, okc);
    }
  }
  __syncthreads();
  double2 vr[4], vpr[4], wpr[4], vc[4], vpc[4], wpc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    vr[q] = s_vec[0][4 * tr + q];
    vpr[q] = s_vec[1][4 * tr + q];
    wpr[q] = s_vec[2][4 * tr + q];
    vc[q] = s_vec[3][4 * tc + q];
    vpc[q] = s_vec[4][4 * tc + q];
    wpc[q] = s_vec[5][4 * tc + q];
  }
  double2 racc[4], cacc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) racc[q] = cacc[q] = z;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = R0 + 4 * tr + q;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = C0 + 4 * tc + u;
      if (!(r < m && c >= j1 && c <= r)) continue;
      double2 x = a[q][u];
      if (pend) {
        x = csub2(x, cmul2(vpr[q], cconj(wpc[u])));
        x = csub2(x, cmul2(wpr[q], cconj(vpc[u])));
        if (c != j1) A[int64_t(r) * mb + c] = x;
      }
      racc[q] = cadd2(racc[q], cmul2(x, vc[u]));
      if (c < r) cacc[u] = cadd2(cacc[u], cmul2(cconj(x), vr[q]));
    }
  }
  // row parts summed over the 16 column groups (lane bits 0-3), column parts over the 16 row
  // groups (lane bits 4-5, then the four waves, in order); then one round of exchanges into
  // the tile's slot, 64 row and 64 column entries (zero where the row or column is outside
  // the block, or for a diagonal tile's last column).  chk collects the values the exchanges
  // return, so a thread cannot pass the barrier below before its writes are done.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (int o = 1; o < 16; o <<= 1) {
      racc[q].x += __shfl_xor(racc[q].x, o, 64);
      racc[q].y += __shfl_xor(racc[q].y, o, 64);
    }
    for (int o = 16; o < 64; o <<= 1) {
      cacc[q].x += __shfl_xor(cacc[q].x, o, 64);
      cacc[q].y += __shfl_xor(cacc[q].y, o, 64);
    }
    if (tc == 0) s_row[4 * tr + q] = racc[q];
    if (lane < 16) s_col[wave][4 * tc + q] = cacc[q];
  }
  __syncthreads();
  double chk = 0.0;
  if (tid < T) {
    const int r = R0 + tid;
    const double2 s = keep(s_row[tid], r >= j1 && r < m);
    chk += __hip_atomic_exchange(&PS[(int64_t(t) * 2 * T + tid) * 2], s.x, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    chk += __hip_atomic_exchange(&PS[(int64_t(t) * 2 * T + tid) * 2 + 1], s.y, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  } else if (tid < 2 * T) {
    const int i = tid - T, c = C0 + i;
    const double2 s = keep(cadd2(cadd2(s_col[0][i], s_col[1][i]), cadd2(s_col[2][i], s_col[3][i])),
                           c >= j1 && c < m && c < R0 + T - 1);
    chk += __hip_atomic_exchange(&PS[(int64_t(t) * 2 * T + tid) * 2], s.x, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    chk += __hip_atomic_exchange(&PS[(int64_t(t) * 2 * T + tid) * 2 + 1], s.y, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  }
  if (chk == 1.0e300) s_last = 2u;   // never true; makes the thread wait for its additions
  const int nall = nt + 1;
  const bool blockfin = nall >= tw.fin_min;
  constexpr int kCohLoad = 16;   // cache-policy bits of a buffer load: sc1 (see the gather below)
  if (!blockfin) {
    // the last workgroup of this job to finish carries on
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&tw.cnt[k], 1u) == unsigned(ntiles - 1) ? 1u : 0u;
    __syncthreads();
    if (s_last != 1u) return;
  } else {
    // Row-block finishers: a tile counts its row sums on its row block's counter and its
    // column sums on its column block's counter.  The tile that completes a block adds that
    // block's nt + 1 slots per row: four quarters of the slot list in turn (one quarter per
    // wave, in slot order), then the quarters in order, so the sums do not depend on which
    // tile finishes.  It stores A v of the block's rows (agent-scope exchanges, waited for)
    // and counts the block on the job's counter; the workgroup that completes the last block
    // carries on and reads A v per row.
    uint32_t* bc = tw.bcnt + int64_t(k) * tw.nblk;
    __syncthreads();
    if (tid == 0) {
      unsigned f = 0u;
      if (ti == tj) {
        if (atomicAdd(&bc[ti], 2u) == unsigned(nall - 2)) f = 1u;
      } else {
        if (atomicAdd(&bc[ti], 1u) == unsigned(nall - 1)) f |= 1u;
        if (atomicAdd(&bc[tj], 1u) == unsigned(nall - 1)) f |= 2u;
      }
      s_fin = f;
    }
    __syncthreads();
    const unsigned fin = s_fin;
    if (fin == 0u) return;
    const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
        PS, (short)0, tw.ptiles * 2 * T * int(sizeof(double2)), 0x00020000);
    double2* prow = tw.prow + int64_t(k) * mb;
    const int g = tid >> 6, i = lane;
    const int Q = (nall + 3) / 4;   // slots per quarter (at most 9: nt <= 32)
    const int c0 = g * Q, c1 = min(nall, c0 + Q);
    double chk2 = 0.0;
    unsigned nfin = 0u;
    for (int h = 0; h < 2; ++h) {
      if (!(fin & (1u << h))) continue;
      const int ib = h == 0 ? ti : tj, nrow = ib + 1;
      constexpr int kQMax = (kTrdMaxBasis / kTrdTile + 4) / 4;
      double2 gl[kQMax];
#pragma unroll
      for (int u = 0; u < kQMax; ++u) {
        const int c = min(c0 + u, nall - 1);
        const int slot = c < nrow ? (ib * (ib + 1) / 2 + c) * 2
                                  : ((ib + c - nrow) * (ib + c - nrow + 1) / 2 + ib) * 2 + 1;
        gl[u] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                                srs, (slot * T + i) * int(sizeof(double2)), 0, kCohLoad));
      }
      double2 acc = z;
#pragma unroll
      for (int u = 0; u < kQMax; ++u)
        if (c0 + u < c1) acc = cadd2(acc, gl[u]);
      s_col[g][i] = acc;
      __syncthreads();
      if (g == 0) {
        const double2 pr = cadd2(cadd2(cadd2(s_col[0][i], s_col[1][i]), s_col[2][i]), s_col[3][i]);
        const int r = (b0 + ib) * T + i;
        if (r >= j1 && r < m) {
          chk2 += __hip_atomic_exchange(&prow[r].x, pr.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          chk2 += __hip_atomic_exchange(&prow[r].y, pr.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (tid == 0) __hip_atomic_store(&bc[ib], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      ++nfin;
    }
    if (chk2 == 1.0e300) s_last = 2u;   // never true; waits for the exchanges
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&tw.cnt[k], nfin) + nfin == unsigned(nt) ? 1u : 0u;
    __syncthreads();
    if (s_last != 1u) return;
  }
  double* d = dd + int64_t(k) * mb;
  double* e = ee + int64_t(k) * mb;
  double2* tk = tau + int64_t(k) * mb;
  const double2 tj_ = tk[j];
  // (A v)_r for row r of block ib: row sums of tiles (ib, 0..ib), then column sums of tiles
  // (ib..nt-1, ib), always in this order.  The slots are read with 16-byte loads under the
  // same cache policy as the agent-scope atomic loads (sc1: served by the coherent level, not
  // by this CU's cache), kTrdGather slots of every row of the thread in flight at once, so the
  // whole gather costs about (nt + 1) / kTrdGather round trips to memory.
  constexpr int kTrdGather = 4;
  const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
      PS, (short)0, tw.ptiles * 2 * T * int(sizeof(double2)), 0x00020000);
  int ibq[kTrdRows], iq[kTrdRows];
  double2 pq[kTrdRows];
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = j1 + tid + q * 256;
    ibq[q] = r / T - b0;
    iq[q] = r - (b0 + ibq[q]) * T;
    pq[q] = z;
  }
  if (blockfin) {   // A v per row from the row-block finishers (rows past m read row m - 1)
    const __amdgpu_buffer_rsrc_t rrs = __builtin_amdgcn_make_buffer_rsrc(
        tw.prow + int64_t(k) * mb, (short)0, mb * int(sizeof(double2)), 0x00020000);
#pragma unroll
    for (int q = 0; q < kTrdRows; ++q) {
      if (j1 + q * 256 >= m) break;
      const int r = min(j1 + tid + q * 256, m - 1);
      pq[q] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(
                                              rrs, r * int(sizeof(double2)), 0, kCohLoad));
    }
  }
  for (int c0 = 0; c0 < (blockfin ? 0 : nall); c0 += kTrdGather) {
    double2 g[kTrdRows][kTrdGather];
#pragma unroll
    for (int q = 0; q < kTrdRows; ++q) {
      if (j1 + q * 256 >= m) break;   // no row of this q in the job (uniform)
      const int ib = ibq[q], nrow = ib + 1;
#pragma unroll
      for (int u = 0; u < kTrdGather; ++u) {
        const int c = min(c0 + u, nall - 1);
        const int slot = c < nrow ? (ib * (ib + 1) / 2 + c) * 2
                                  : ((ib + c - nrow) * (ib + c - nrow + 1) / 2 + ib) * 2 + 1;
        // rows past m read a clamped slot; their sums are discarded below
        const int off = (min(slot, tw.ptiles * 2 - 1) * T + iq[q]) * int(sizeof(double2));
        g[q][u] = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(prs, off, 0, kCohLoad));
      }
    }
#pragma unroll
    for (int q = 0; q < kTrdRows; ++q) {
      if (j1 + q * 256 >= m) break;
#pragma unroll
      for (int u = 0; u < kTrdGather; ++u)
        if (c0 + u < nall) pq[q] = cadd2(pq[q], g[q][u]);
    }
  }
  // column j+1 as the previous launch left it, with the update of step j-1 applied
  const double2 wpj1c = keep(cconj(W[j1]), pend), vpj1c = keep(cconj(vp[j1]), pend);
  double2 vq[kTrdRows], col[kTrdRows], vpq[kTrdRows], wpq[kTrdRows];
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int rc = min(j1 + tid + q * 256, m - 1);
    col[q] = A[int64_t(rc) * mb + j1];
    vq[q] = vj[rc];
    vpq[q] = vp[rc];
    wpq[q] = W[rc];
  }
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const bool ok = j1 + tid + q * 256 < m;
    pq[q] = keep(pq[q], ok);
    col[q] = keep(col[q], ok);
    vq[q] = keep(vq[q], ok);
    vpq[q] = keep(vpq[q], ok && pend);
    wpq[q] = keep(wpq[q], ok && pend);
    col[q] = csub2(col[q], cmul2(vpq[q], wpj1c));
    col[q] = csub2(col[q], cmul2(wpq[q], vpj1c));
    pq[q] = cmul2(tj_, pq[q]);
    sr += pq[q].x * vq[q].x + pq[q].y * vq[q].y;
    si += pq[q].x * vq[q].y - pq[q].y * vq[q].x;
  }
  block_sum2(sr, si, red);   // its barriers also separate the reads of W above from the writes below
  const double2 aw = cmul2(make_double2(-0.5 * tj_.x, -0.5 * tj_.y), make_double2(sr, si));
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = j1 + tid + q * 256;
    if (r < m) {
      pq[q] = cadd2(pq[q], cmul2(aw, vq[q]));   // w_j
      W[r] = pq[q];
      if (r == j1) {
        s_wj1 = pq[q];
        s_vj1 = vq[q];
      }
    }
  }
  __syncthreads();
  if (tid == 0) tw.cnt[k] = 0u;
  if (j == m - 2) {   // only the last diagonal element is left: apply the update of step j
    if (tid == 0) {
      d[m - 1] = col[0].x - 2.0 * (s_vj1.x * s_wj1.x + s_vj1.y * s_wj1.y);
      e[m - 1] = 0.0;
      tk[m - 1] = z;
    }
    return;
  }
  // column j+1, rows [j+1, m), with the update of step j applied
  const double2 wj1c = cconj(s_wj1), vj1c = cconj(s_vj1);
#pragma unroll
  for (int q = 0; q < kTrdRows; ++q) {
    const int r = j1 + tid + q * 256;
    if (r < m) {
      col[q] = csub2(col[q], cmul2(vq[q], wj1c));
      col[q] = csub2(col[q], cmul2(pq[q], vj1c));
    }
  }
  trd_reflector(j1, m, mb, A, col, tw.v + (int64_t(k) * 2 + (j1 & 1)) * mb, d, e, tk, red);
}

// ---------------------------------------------------------------- tridiagonal eigenpairs
// Lowest nwant = min(nb, m) eigenpairs of the real symmetric tridiagonal (d, e), spread over
// the GPU in three kernels:
//   k_eig_vals     eigenvalues: one wave per eigenvalue, 64-section on Sturm counts (the 64
//                  lanes cut the bracket into 65 parts per round)
//   k_eig_inviter  one step of inverse iteration, one lane per eigenvector (64 per
//                  workgroup); vectors are stored unnormalised with their scale 1/||y||
//   k_eig_orth     one workgroup per cluster of close eigenvalues (gap <= ortol): block
//                  classical Gram-Schmidt, twice, then unit norm, so that degenerate levels
//                  get orthonormal vectors
// The host runs k_eig_vals once and (k_eig_inviter, k_eig_orth) three times.
// Y[k][i][n] (n fastest: the lanes of an inverse-iteration wave touch consecutive addresses),
// true vector n = Y[.][n] * sc[k][n].

// 1/q from the hardware reciprocal refined by two Newton steps (relative error of a few
// ulps): a Sturm count tolerates that as a relative perturbation of e^2 of the same size,
// and it is half the dependent chain of a correctly rounded division.
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double t = fma(-q, r, 1.0);
  r = fma(r, t, r);
  t = fma(-q, r, 1.0);
  return fma(r, t, r);
}

// Number of eigenvalues of the tridiagonal (diagonal d, squared off-diagonal e2) below x.
__device__ int sturm_count(const double* d, const double* e2, int m, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < m; ++i) {
    q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// deterministic start vector of inverse iteration, entries in [0.5, 1.5)
__device__ __forceinline__ double inviter_start(int i, int n) {
  uint32_t h = uint32_t(i + 1) * 0x9E3779B1u ^ uint32_t(n + 1) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return 0.5 + double(h) * 2.3283064365386963e-10;
}

__device__ __forceinline__ double wave_sum_all(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr double kEps = 2.220446049250313e-16;

// Gershgorin interval and the norm estimate max_i |d_i| + |e_{i-1}| + |e_i| of (d, e) in LDS,
// identical on every thread of the block.
__device__ void gershgorin(const double* sd, const double* se, int m, double* red, double& lo,
                           double& hi, double& nrm) {
  double l = 1e300, h = -1e300, nr = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double r = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i < m - 1 ? fabs(se[i]) : 0.0);
    l = fmin(l, sd[i] - r);
    h = fmax(h, sd[i] + r);
    nr = fmax(nr, fabs(sd[i]) + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_xor(l, o, 64));
    h = fmax(h, __shfl_xor(h, o, 64));
    nr = fmax(nr, __shfl_xor(nr, o, 64));
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = l;
    red[nw + w] = h;
    red[2 * nw + w] = nr;
  }
  __syncthreads();
  lo = red[0];
  hi = red[nw];
  nrm = red[2 * nw];
  for (int i = 1; i < nw; ++i) {
    lo = fmin(lo, red[i]);
    hi = fmax(hi, red[nw + i]);
    nrm = fmax(nrm, red[2 * nw + i]);
  }
  nrm = fmax(nrm, 1e-300);
  __syncthreads();
}

// Grid (ceil(nwant / 4), jobs), 256 threads: wave w finds eigenvalue 4 blockIdx.x + w.
__global__ void __launch_bounds__(256) k_eig_vals(DJobs jobs, const double* __restrict__ dd,
                                                  const double* __restrict__ ee,
                                                  double* __restrict__ theta, EigWork ew) {
  extern __shared__ double sde[];  // d [mb], e [mb], e^2 [mb]
  __shared__ double red[12];
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, m = J.m, k = J.k, nwant = min(jobs.nb, m);
  if (blockIdx.x * 4 >= nwant) return;
  double* sd = sde;
  double* se = sd + mb;
  double* se2 = se + mb;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double ev = ee[int64_t(k) * mb + i];
    sd[i] = dd[int64_t(k) * mb + i];
    se[i] = ev;
    se2[i] = ev * ev;
  }
  __syncthreads();
  double glo, ghi, nrm;
  gershgorin(sd, se, m, red, glo, ghi, nrm);
  if (blockIdx.x == 0 && threadIdx.x == 0) ew.nrm[k] = nrm;
  const int lane = threadIdx.x & 63, n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= nwant) return;
  const double pivmin = fmax(1e-290, kEps * kEps * nrm * nrm * 1e-6);
  const double atol = 1e-3 * kEps * nrm;
  double lo = glo - 4 * kEps * nrm, hi = ghi + 4 * kEps * nrm;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= fmax(2.0 * kEps * fmax(fabs(lo), fabs(hi)), atol)) break;
    const double w = (hi - lo) / 65.0;
    const bool below = sturm_count(sd, se2, m, lo + w * double(lane + 1), pivmin) <= n;
    // the lanes whose point lies at or below lambda_n form a prefix
    const int j = __popcll(__ballot(below));
    const double nlo = j == 0 ? lo : lo + w * double(j);
    const double nhi = j == 64 ? hi : lo + w * double(j + 1);
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) theta[int64_t(k) * mb + n] = 0.5 * (lo + hi);
}

// Inverse-iteration shift of eigenvalue n: inside a cluster (gaps <= ortol) the shifts are
// nudged apart by 10 eps ||T|| so that no two coincide.
__device__ double inviter_shift(const double* th, int n, double ortol, double tiny) {
  int n0 = n;
  while (n0 > 0 && th[n0] - th[n0 - 1] <= ortol) --n0;
  double prev = th[n0];
  for (int t = n0 + 1; t <= n; ++t) {
    const double x = th[t];
    prev = x - prev < 10.0 * tiny ? prev + 10.0 * tiny : x;
  }
  return prev;
}

constexpr int kInvBlk = 8;   // rows whose right-hand side is loaded ahead in the forward sweep
constexpr int kBwdBlk = 8;   // and whose factors are loaded ahead in the back substitution

// One inverse-iteration step (T - lambda_n I) y_new = y for 64 eigenvectors per workgroup
// (one lane each; grid (ceil(nwant / 64), jobs)).  The sweep that eliminates the right-hand
// side (partial pivoting) also produces the factors, so it never reads what it writes; it
// stores 1/pivot so the back substitution only multiplies.  fw: [k][3][mb][nb] (1/pivot and
// the two superdiagonals of U), same interleaving as Y.
__global__ void __launch_bounds__(64) k_eig_inviter(DJobs jobs, const double* __restrict__ dd,
                                                    const double* __restrict__ ee,
                                                    const double* __restrict__ theta,
                                                    double* __restrict__ yw, double* __restrict__ fw,
                                                    EigWork ew, int step) {
  extern __shared__ double sde[];  // d [mb], e [mb]
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, nb = jobs.nb, m = J.m, k = J.k, nwant = min(nb, m);
  if (blockIdx.x * 64 >= nwant) return;
  double* sd = sde;
  double* se = sd + mb;
  for (int i = threadIdx.x; i < m; i += 64) {
    sd[i] = dd[int64_t(k) * mb + i];
    se[i] = ee[int64_t(k) * mb + i];
  }
  __syncthreads();
  const int n = blockIdx.x * 64 + threadIdx.x;
  if (n >= nwant) return;
  const double nrm = ew.nrm[k];
  const double tiny = kEps * nrm, ortol = 1e-5 * nrm;
  const double* th = theta + int64_t(k) * mb;
  const double lam = inviter_shift(th, n, ortol, tiny);
  const int64_t st = nb;  // stride between consecutive elements of one vector
  double* y = yw + int64_t(k) * nb * mb + n;
  double* RD = fw + int64_t(k) * nb * 3 * mb + n;
  double* U1 = RD + int64_t(mb) * nb;
  double* U2 = U1 + int64_t(mb) * nb;
  double* scp = ew.sc + int64_t(k) * nb + n;
  const double s_in = step == 0 ? 1.0 : *scp;
  auto rhs = [&](int r) {
    if (r >= m) return 0.0;
    return step == 0 ? inviter_start(r, n) : y[r * st] * s_in;
  };
  auto safe = [&](double p) { return fabs(p) < tiny ? (p < 0.0 ? -tiny : tiny) : p; };
  double dcur = sd[0] - lam, u1 = m > 1 ? se[0] : 0.0;
  double bcur = rhs(0);
  double bq[kInvBlk];
#pragma unroll
  for (int q = 0; q < kInvBlk; ++q) bq[q] = rhs(q + 1);
  for (int ib = 0; ib < m - 1; ib += kInvBlk) {
    double bn[kInvBlk];
#pragma unroll
    for (int q = 0; q < kInvBlk; ++q) bn[q] = rhs(ib + kInvBlk + q + 1);   // ahead of the stores
#pragma unroll
    for (int q = 0; q < kInvBlk; ++q) {
      const int i = ib + q;
      if (i >= m - 1) break;
      const double sub = se[i];
      const double anext = sd[i + 1] - lam;
      const double enext = i + 1 < m - 1 ? se[i + 1] : 0.0;
      const double bnext = bq[q];
      if (fabs(dcur) >= fabs(sub)) {
        const double piv = safe(dcur), rp = rcp_nr(piv);
        const double f = sub * rp;
        RD[i * st] = rp;
        U1[i * st] = u1;
        U2[i * st] = 0.0;
        y[i * st] = bcur;
        bcur = bnext - f * bcur;
        dcur = anext - f * u1;
        u1 = enext;
      } else {
        const double piv = safe(sub), rp = rcp_nr(piv);
        const double f = dcur * rp;
        RD[i * st] = rp;
        U1[i * st] = anext;
        U2[i * st] = enext;
        y[i * st] = bnext;
        bcur = bcur - f * bnext;
        dcur = u1 - f * anext;
        u1 = -f * enext;
      }
    }
#pragma unroll
    for (int q = 0; q < kInvBlk; ++q) bq[q] = bn[q];
  }
  // back substitution with U (rows m-1 .. 0), a block of rows loaded ahead; the norm of the
  // solution accumulates on the way
  double y1 = bcur * rcp_nr(safe(dcur)), y2 = 0.0;
  double ss = y1 * y1;
  y[(m - 1) * st] = y1;
  double pz[kBwdBlk], pu1[kBwdBlk], pu2[kBwdBlk], pd[kBwdBlk];
#pragma unroll
  for (int q = 0; q < kBwdBlk; ++q) {
    const int i = max(m - 2 - q, 0);
    pz[q] = y[i * st];
    pu1[q] = U1[i * st];
    pu2[q] = U2[i * st];
    pd[q] = RD[i * st];
  }
  for (int ib = m - 2; ib >= 0; ib -= kBwdBlk) {
    double nz[kBwdBlk], nu1[kBwdBlk], nu2[kBwdBlk], nd[kBwdBlk];
#pragma unroll
    for (int q = 0; q < kBwdBlk; ++q) {
      const int i = max(ib - kBwdBlk - q, 0);
      nz[q] = y[i * st];
      nu1[q] = U1[i * st];
      nu2[q] = U2[i * st];
      nd[q] = RD[i * st];
    }
#pragma unroll
    for (int q = 0; q < kBwdBlk; ++q) {
      const int i = ib - q;
      if (i < 0) break;
      const double yi = (pz[q] - pu1[q] * y1 - pu2[q] * y2) * pd[q];
      y[i * st] = yi;
      ss += yi * yi;
      y2 = y1;
      y1 = yi;
    }
#pragma unroll
    for (int q = 0; q < kBwdBlk; ++q) {
      pz[q] = nz[q];
      pu1[q] = nu1[q];
      pu2[q] = nu2[q];
      pd[q] = nd[q];
    }
  }
  *scp = 1.0 / sqrt(ss);
}

// Grid (nwant, jobs), 256 threads: workgroup n0 orthonormalises the cluster that starts at
// eigenvalue n0 if it has two or more members (others return at once).  Vectors in order:
// two passes of block classical Gram-Schmidt against the finished ones (16 at a time, one
// batched reduction per block), then unit norm; rows i = tid + 256 r.
constexpr int kOrthBlk = 16;
__global__ void __launch_bounds__(256) k_eig_orth(DJobs jobs, const double* __restrict__ theta,
                                                  double* __restrict__ yw, EigWork ew) {
  __shared__ double red[4][kOrthBlk];
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, nb = jobs.nb, m = J.m, k = J.k, nwant = min(nb, m);
  const int n0 = blockIdx.x;
  if (n0 >= nwant) return;
  const double* th = theta + int64_t(k) * mb;
  const double ortol = 1e-5 * ew.nrm[k];
  if (n0 > 0 && th[n0] - th[n0 - 1] <= ortol) return;   // not the first of its cluster
  int n1 = n0 + 1;
  while (n1 < nwant && th[n1] - th[n1 - 1] <= ortol) ++n1;
  if (n1 - n0 < 2) return;
  double* Y = yw + int64_t(k) * nb * mb;
  double* sc = ew.sc + int64_t(k) * nb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int R = kTrdMaxBasis / 256;   // rows per thread
  for (int n = n0; n < n1; ++n) {
    double yn[R];
    const double s0 = sc[n];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 256 * r;
      yn[r] = i < m ? Y[int64_t(i) * nb + n] * s0 : 0.0;
    }
    for (int pass = 0; pass < 2; ++pass) {
      for (int qb = n0; qb < n; qb += kOrthBlk) {
        const int nq = min(kOrthBlk, n - qb);
        double part[kOrthBlk];
#pragma unroll
        for (int q = 0; q < kOrthBlk; ++q) part[q] = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = tid + 256 * r;
          if (i >= m) break;
#pragma unroll
          for (int q = 0; q < kOrthBlk; ++q)
            if (q < nq) part[q] += Y[int64_t(i) * nb + qb + q] * yn[r];
        }
#pragma unroll
        for (int q = 0; q < kOrthBlk; ++q) {
          for (int o = 32; o > 0; o >>= 1) part[q] += __shfl_xor(part[q], o, 64);
          if (lane == 0) red[wave][q] = part[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kOrthBlk; ++q) part[q] = red[0][q] + red[1][q] + red[2][q] + red[3][q];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = tid + 256 * r;
          if (i >= m) break;
#pragma unroll
          for (int q = 0; q < kOrthBlk; ++q)
            if (q < nq) yn[r] -= part[q] * Y[int64_t(i) * nb + qb + q];
        }
      }
    }
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) ss += yn[r] * yn[r];
    ss = wave_sum_all(ss);
    if (lane == 0) red[wave][0] = ss;
    __syncthreads();
    const double s = 1.0 / sqrt(red[0][0] + red[1][0] + red[2][0] + red[3][0]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 256 * r;
      if (i < m) Y[int64_t(i) * nb + n] = yn[r] * s;
    }
    if (tid == 0) sc[n] = 1.0;
  }
}

// Blocked back-transform (compact WY form of 32 reflectors at a time):
//   H_j0 ... H_j0+b-1 = I - V T V^H  (V: the b reflectors as columns, T upper triangular,
//   T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] (V[:, 0:i]^H v_i)),
// applied to the eigenvector block from the last block to the first: Z -= V (T (V^H Z)).
// Reflector q of a block (global j = j0 + q) is v[j+1] = 1, v[r] = A[r][j] below, 0 above.
constexpr int kBtB = kBtBlk;

__device__ __forceinline__ double2 bt_v(const double2* A, int mb, int r, int j) {
  const double2 x = A[int64_t(max(r, j + 1)) * mb + j];   // clamped: r >= j + 1 always exists
  return make_double2(r > j + 1 ? x.x : (r == j + 1 ? 1.0 : 0.0), r > j + 1 ? x.y : 0.0);
}

// T of every block: grid (blocks, jobs), 256 threads.
__global__ void __launch_bounds__(256) k_bt_tfactor(DJobs jobs, const double2* __restrict__ Aw,
                                                    const double2* __restrict__ tau,
                                                    double2* __restrict__ Tw) {
  constexpr int B = kBtB;
  __shared__ double2 sV[B][B + 1];   // a chunk of 32 rows of the block's reflectors
  __shared__ double2 sG[B][B + 1];   // Gram V^H V
  __shared__ double2 sT[B][B + 1];
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, m = J.m, k = J.k, nref = m - 1;
  const int j0 = blockIdx.x * B;
  if (j0 >= nref) return;
  const int bb = min(B, nref - j0);
  const double2* A = Aw + int64_t(k) * mb * mb;
  const int tid = threadIdx.x;
  // thread (p, q) pairs: p = tid / 8 .. in steps; 4 entries of G each
  double2 g[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) g[e] = make_double2(0.0, 0.0);
  for (int r0 = j0 + 1; r0 < m; r0 += B) {
    for (int e = tid; e < B * B; e += 256) {
      const int rr = e / B, q = e % B, r = min(r0 + rr, m - 1);
      sV[rr][q] = keep(bt_v(A, mb, r, j0 + min(q, bb - 1)), r0 + rr < m && q < bb);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 256 * e, p = idx / B, q = idx % B;
#pragma unroll 8
      for (int rr = 0; rr < B; ++rr) g[e] = cadd2(g[e], cmul2(cconj(sV[rr][p]), sV[rr][q]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 256 * e;
    sG[idx / B][idx % B] = g[e];
  }
  for (int e = tid; e < B * B; e += 256) sT[e / B][e % B] = make_double2(0.0, 0.0);
  __syncthreads();
  const double2* tk = tau + int64_t(k) * mb;
  if (tid == 0) sT[0][0] = tk[j0];
  __syncthreads();
  for (int i = 1; i < bb; ++i) {
    const double2 ti = tk[j0 + i];
    double2 s = make_double2(0.0, 0.0);
    if (tid < i) {
      for (int q = tid; q < i; ++q) s = cadd2(s, cmul2(sT[tid][q], sG[q][i]));
    }
    __syncthreads();
    if (tid < i) sT[tid][i] = cmul2(make_double2(-ti.x, -ti.y), s);
    if (tid == i) sT[i][i] = ti;
    __syncthreads();
  }
  const int nblk_all = (jobs.mb + B - 1) / B;
  double2* T = Tw + (int64_t(k) * nblk_all + blockIdx.x) * B * B;
  for (int e = tid; e < B * B; e += 256) T[e] = sT[e / B][e % B];
}

// Z = Q y for a slice of cols columns per workgroup: grid (column slices, jobs), 256 threads,
// dynamic LDS [mb][cols] slice + [8][32][cols] partial sums + [32][cols] W.
__global__ void __launch_bounds__(256) k_bt_apply(DJobs jobs, const double2* __restrict__ Aw,
                                                  const double2* __restrict__ Tw,
                                                  const double* __restrict__ yw,
                                                  const double* __restrict__ scw,
                                                  double2* __restrict__ Zout, int cols) {
  constexpr int B = kBtB;
  extern __shared__ double2 shz[];
  __shared__ double2 sT[B][B + 1];
  const DJob& J = jobs.j[blockIdx.y];
  const int mb = jobs.mb, nb = jobs.nb, m = J.m, k = J.k, nref = m - 1;
  const int c0 = blockIdx.x * cols;
  if (c0 >= min(nb, m)) return;
  const int nc = min(cols, min(nb, m) - c0);
  const double2* A = Aw + int64_t(k) * mb * mb;
  const double* Y = yw + int64_t(k) * nb * mb;
  double2* Z = Zout + int64_t(k) * mb * nb;
  double2* zs = shz;                                   // [m][cols]
  double2* part = zs + int64_t(mb) * cols;             // [8][B][cols]
  double2* sW = part + 8 * B * cols;                   // [B][cols]
  const int tid = threadIdx.x;
  for (int t = tid; t < m * cols; t += 256) {
    const int i = t / cols, c = t % cols, cl = min(c, nc - 1);
    const double yv = Y[int64_t(i) * nb + c0 + cl] * scw[int64_t(k) * nb + c0 + cl];
    zs[t] = make_double2(c < nc ? yv : 0.0, 0.0);
  }
  const int nblk = (nref + B - 1) / B, nblk_all = (mb + B - 1) / B;
  const int q = tid & (B - 1), grp = tid >> 5;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = blk * B, bb = min(B, nref - j0);
    const double2* T = Tw + (int64_t(k) * nblk_all + blk) * B * B;
    for (int e = tid; e < B * B; e += 256) sT[e / B][e % B] = T[e];
    __syncthreads();   // also orders the previous block's Z update before the reads below
    // W = V^H Z: thread (q, group) sums rows r = j0 + 1 + group + 8 t
    double2 acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = make_double2(0.0, 0.0);
    const int qc = j0 + min(q, bb - 1);
    int r = j0 + 1 + grp;
    for (; r + 24 < m; r += 32) {   // four rows per trip: their loads are in flight together
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = cconj(keep(bt_v(A, mb, r + 8 * u, qc), q < bb));
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < cols) acc[c] = cadd2(acc[c], cmul2(v[u], zs[(r + 8 * u) * cols + c]));
    }
    for (; r < m; r += 8) {
      const double2 v = cconj(keep(bt_v(A, mb, r, qc), q < bb));
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < cols) acc[c] = cadd2(acc[c], cmul2(v, zs[r * cols + c]));
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < cols) part[(grp * B + q) * cols + c] = acc[c];
    __syncthreads();
    // W' = T W (T upper triangular)
    for (int e = tid; e < B * cols; e += 256) {
      const int p = e / cols, c = e % cols;
      double2 w = make_double2(0.0, 0.0);
      for (int qq = p; qq < bb; ++qq) {
        double2 s = part[qq * cols + c];
        for (int g2 = 1; g2 < 8; ++g2) s = cadd2(s, part[(g2 * B + qq) * cols + c]);
        w = cadd2(w, cmul2(sT[p][qq], s));
      }
      sW[p * cols + c] = w;
    }
    __syncthreads();
    // Z -= V W', one row per thread (its 32 reflector entries loaded once for all columns)
    for (int r = j0 + 1 + tid; r < m; r += 256) {
      double2 sacc[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) sacc[c] = make_double2(0.0, 0.0);
      for (int qq = 0; qq < bb; ++qq) {
        const double2 v = bt_v(A, mb, r, j0 + qq);
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < cols) sacc[c] = cadd2(sacc[c], cmul2(v, sW[qq * cols + c]));
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < cols) zs[r * cols + c] = csub2(zs[r * cols + c], sacc[c]);
    }
    __syncthreads();
  }
  for (int t = tid; t < m * cols; t += 256) {
    const int i = t / cols, c = t % cols;
    if (c < nc) Z[int64_t(i) * nb + c0 + c] = zs[t];
  }
}

// ---------------------------------------------------------------- Cholesky + inverse
// G [k][nb][nb] (leading nu x nu, Hermitian PD) -> W[k][i][n] = conj(Linv[n][i]);
// info[k] is left as it is on success and set to j+1 if pivot j failed; a non-zero info[k]
// on entry skips the job (the caller clears info once per orthonormalisation, so a failure
// stays visible through its later passes).  Right-looking, one workgroup.
__global__ void __launch_bounds__(1024) k_chol_inv(DJobs jobs, double2* __restrict__ Gm,
                                                   double2* __restrict__ Wm, int32_t* __restrict__ info) {
  const DJob& J = jobs.j[blockIdx.x];
  const int nb = jobs.nb, n = J.nu;
  double2* G = Gm + int64_t(J.k) * nb * nb;
  double2* W = Wm + int64_t(J.k) * nb * nb;
  __shared__ int s_fail;
  __shared__ double s_dmax;
  const int tid = threadIdx.x;
  if (info[J.k] != 0) return;   // an earlier factorisation of this orthonormalisation failed
  if (tid == 0) {
    s_fail = 0;
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, G[int64_t(i) * nb + i].x);
    s_dmax = mx;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    __shared__ double s_piv;
    if (tid == 0) {
      const double djj = G[int64_t(j) * nb + j].x;
      if (!(djj > 1e-14 * s_dmax) || !(djj < 1e300)) s_fail = j + 1;
      s_piv = s_fail ? 1.0 : sqrt(djj);
      G[int64_t(j) * nb + j] = make_double2(s_piv, 0.0);
    }
    __syncthreads();
    if (s_fail) break;
    const double inv = 1.0 / s_piv;
    for (int r = j + 1 + tid; r < n; r += blockDim.x) {
      const double2 a = G[int64_t(r) * nb + j];
      G[int64_t(r) * nb + j] = make_double2(a.x * inv, a.y * inv);
    }
    __syncthreads();
    // trailing lower update: G[r][c] -= L[r][j] conj(L[c][j]) for c <= r
    const int nn = n - j - 1;
    for (int64_t t = tid; t < int64_t(nn) * nn; t += blockDim.x) {
      const int r = j + 1 + int(t / nn), c = j + 1 + int(t % nn);
      if (c > r) continue;
      const double2 lr = G[int64_t(r) * nb + j], lc = G[int64_t(c) * nb + j];
      G[int64_t(r) * nb + c] = csub2(G[int64_t(r) * nb + c], cmul2(lr, cconj(lc)));
    }
    __syncthreads();
  }
  if (s_fail) {
    if (tid == 0) info[J.k] = s_fail;
    return;
  }
  // Linv column c by forward substitution; W[i][c'] = conj(Linv[c'][i])  (i <= c')
  for (int c = tid; c < n; c += blockDim.x) {
    // x = Linv[:, c]: x[r] = 0 for r < c
    W[int64_t(c) * nb + c] = make_double2(1.0 / G[int64_t(c) * nb + c].x, 0.0);  // conj of real
    for (int r = c + 1; r < n; ++r) {
      double sr = 0.0, si = 0.0;
      for (int q = c; q < r; ++q) {
        const double2 l = G[int64_t(r) * nb + q];
        const double2 x = cconj(W[int64_t(c) * nb + q]);   // Linv[q][c] = conj(W[c][q])
        sr += l.x * x.x - l.y * x.y;
        si += l.x * x.y + l.y * x.x;
      }
      const double lrr = G[int64_t(r) * nb + r].x;
      // Linv[r][c] = -s / L[r][r]; W[c][r] = conj(Linv[r][c])
      W[int64_t(c) * nb + r] = make_double2(-sr / lrr, si / lrr);
    }
    for (int r = 0; r < c; ++r) W[int64_t(c) * nb + r] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------- blocked Cholesky + inverse
// The same factorisation and inverse on many workgroups, in blocks of kCholB = 16:
//   k_chol_prep      largest diagonal entry (pivot test); info is cleared by the caller once
//                    per orthonormalisation and only ever set by a failed pivot
//   k_chol_col       block column jb of L (Crout order, one launch per block column): the
//                    workgroup of row block ib forms [S_jj; S_ib,j] = G - (finished columns)
//                    through LDS tiles, factors S_jj itself (every workgroup of the launch
//                    does, identically, so none waits for another) and solves its own block.
//                    The diagonal blocks of L go to Ld: the other workgroups of the launch
//                    still read that block of G, and no later block column needs them
//   k_chol_inv_cols  one workgroup per column block of Linv, walking down the block rows
//                    with the finished part of its column block kept in LDS
// Output: the off-diagonal blocks of L in the lower triangle of G, its diagonal blocks in
// Ld [k][block][16][16], W[i][n] = conj(Linv[n][i]) as from k_chol_inv.
constexpr int kCholB = kCholBlk;

__global__ void __launch_bounds__(256) k_chol_prep(DJobs jobs, const double2* __restrict__ Gm,
                                                   double* __restrict__ dmax) {
  __shared__ double red[4];
  const DJob& J = jobs.j[blockIdx.x];
  const int nb = jobs.nb, n = J.nu;
  const double2* G = Gm + int64_t(J.k) * nb * nb;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, G[int64_t(i) * nb + i].x);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) dmax[J.k] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Grid (row blocks from jb on, jobs), 256 threads: thread (r = tid / 16, c = tid % 16).
__global__ void __launch_bounds__(256) k_chol_col(DJobs jobs, int jb, double2* __restrict__ Gm,
                                                  double2* __restrict__ Ldw,
                                                  const double* __restrict__ dmaxw,
                                                  int32_t* __restrict__ info) {
  constexpr int B = kCholB;
  __shared__ double2 sL[2 * B][B + 1];
  __shared__ double2 sS[2 * B][B + 1];
  __shared__ double s_piv;
  __shared__ int s_fail;
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb, n = J.nu, k = J.k;
  const int ib = jb + blockIdx.x;
  if (jb * B >= n || ib * B >= n) return;
  if (info[k] != 0) return;   // an earlier block column failed
  double2* G = Gm + int64_t(k) * nb * nb;
  const int tid = threadIdx.x, r = tid >> 4, c = tid & 15;
  const int rj = jb * B + r, ri = ib * B + r, cj = jb * B + c;
  const double2 z = make_double2(0.0, 0.0);
  // S = G - sum over the finished columns q < jb B of L[row][q] conj(L[cj][q])
  double2 acc0 = z, acc1 = z;
  for (int k0 = 0; k0 < jb * B; k0 += B) {
    for (int e = tid; e < 2 * B * B; e += 256) {
      const int rr = e / B, qq = e % B;
      const int row = rr < B ? jb * B + rr : ib * B + rr - B;
      sL[rr][qq] = keep(G[int64_t(min(row, n - 1)) * nb + k0 + qq], row < n);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const double2 lc = cconj(sL[c][q]);
      acc0 = cadd2(acc0, cmul2(sL[r][q], lc));
      acc1 = cadd2(acc1, cmul2(sL[B + r][q], lc));
    }
    __syncthreads();
  }
  {
    const bool ok0 = rj < n && cj < n && c <= r;
    const double2 g0 = G[int64_t(min(rj, n - 1)) * nb + min(cj, n - 1)];
    sS[r][c] = keep(csub2(g0, acc0), ok0);
    if (ib != jb) {
      const bool ok1 = ri < n && cj < n;
      const double2 g1 = G[int64_t(min(ri, n - 1)) * nb + min(cj, n - 1)];
      sS[B + r][c] = keep(csub2(g1, acc1), ok1);
    }
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();
  // Cholesky of S_jj in LDS (rows past n: identity)
  const double dmax = dmaxw[k];
  for (int q = 0; q < B; ++q) {
    if (tid == 0) {
      double piv = 1.0;
      if (jb * B + q < n) {
        const double djj = sS[q][q].x;
        if (!(djj > 1e-14 * dmax) || !(djj < 1e300)) s_fail = jb * B + q + 1;
        else piv = sqrt(djj);
      }
      s_piv = piv;
      sS[q][q] = make_double2(piv, 0.0);
    }
    __syncthreads();
    if (s_fail) break;
    if (tid > q && tid < B) {
      const double inv = 1.0 / s_piv;
      sS[tid][q] = make_double2(sS[tid][q].x * inv, sS[tid][q].y * inv);
    }
    __syncthreads();
    if (r > q && c > q && c <= r) sS[r][c] = csub2(sS[r][c], cmul2(sS[r][q], cconj(sS[c][q])));
    __syncthreads();
  }
  if (s_fail) {
    if (ib == jb && tid == 0) info[k] = s_fail;
    return;
  }
  if (ib == jb) {
    const int nblk_all = (nb + B - 1) / B;
    Ldw[((int64_t(k) * nblk_all + jb) * B + r) * B + c] = keep(sS[r][c], c <= r);
    return;
  }
  // L_ib,j = S_ib,j L_jj^-H: row r solves x L_jj^H = s column by column
  for (int cc = 0; cc < B; ++cc) {
    if (tid < B) {
      double2 s = sS[B + tid][cc];
      for (int q = 0; q < cc; ++q) s = csub2(s, cmul2(sS[B + tid][q], cconj(sS[cc][q])));
      const double inv = 1.0 / sS[cc][cc].x;
      sS[B + tid][cc] = make_double2(s.x * inv, s.y * inv);
    }
    __syncthreads();
  }
  if (ri < n && cj < n) G[int64_t(ri) * nb + cj] = sS[B + r][c];
}

// Grid (column blocks, jobs), 256 threads, dynamic LDS [n rounded up to B][B] complex.
__global__ void __launch_bounds__(256) k_chol_inv_cols(DJobs jobs, const double2* __restrict__ Gm,
                                                       const double2* __restrict__ Ldw,
                                                       double2* __restrict__ Wm,
                                                       const int32_t* __restrict__ info) {
  constexpr int B = kCholB;
  extern __shared__ double2 sX[];          // rows [jb B, n) of column block jb of Linv, [.][B]
  __shared__ double2 sLc[B][B + 1];
  __shared__ double2 sD[B][B + 1];
  __shared__ double2 sY[B][B + 1];
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb, n = J.nu, k = J.k;
  const int jb = blockIdx.x;
  if (jb * B >= n || info[k] != 0) return;
  const double2* G = Gm + int64_t(k) * nb * nb;
  double2* W = Wm + int64_t(k) * nb * nb;
  const int tid = threadIdx.x, r = tid >> 4, c = tid & 15;
  const int cj = jb * B + c;
  const double2 z = make_double2(0.0, 0.0);
  const int nblk = (n + B - 1) / B;
  // the other triangle of W's rows for this column block
  for (int e = tid; e < B * jb * B; e += 256) {
    const int cc = e / (jb * B), rr = e % (jb * B);
    if (jb * B + cc < n) W[int64_t(jb * B + cc) * nb + rr] = z;
  }
  for (int ib = jb; ib < nblk; ++ib) {
    // acc = sum over q in [jb B, ib B) of L[ib B + r][q] X[q][c]
    double2 acc = z;
    for (int q0 = jb * B; q0 < ib * B; q0 += B) {
      const int row = ib * B + r;
      sLc[r][c] = keep(G[int64_t(min(row, n - 1)) * nb + q0 + c], row < n);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < B; ++q) acc = cadd2(acc, cmul2(sLc[r][q], sX[(q0 - jb * B + q) * B + c]));
      __syncthreads();
    }
    // diagonal block of L and the right-hand side (identity on the diagonal block)
    {
      const int row = ib * B + r, col = ib * B + c;
      const bool ok = row < n && col < n && c <= r;
      sD[r][c] = keep(Ldw[((int64_t(k) * ((nb + B - 1) / B) + ib) * B + r) * B + c], ok);
      if (row >= n && r == c) sD[r][c] = make_double2(1.0, 0.0);
      const double2 id = make_double2(ib == jb && r == c ? 1.0 : 0.0, 0.0);
      sY[r][c] = csub2(id, acc);
    }
    __syncthreads();
    // forward substitution L_ii Y = rhs, one row at a time (16 columns in parallel)
    for (int rr = 0; rr < B; ++rr) {
      if (tid < B) {
        double2 s = sY[rr][tid];
        for (int q = 0; q < rr; ++q) s = csub2(s, cmul2(sD[rr][q], sY[q][tid]));
        const double inv = 1.0 / sD[rr][rr].x;
        sY[rr][tid] = make_double2(s.x * inv, s.y * inv);
      }
      __syncthreads();
    }
    const int row = ib * B + r;
    sX[(ib * B - jb * B + r) * B + c] = sY[r][c];
    if (row < n && cj < n) W[int64_t(cj) * nb + row] = cconj(sY[r][c]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- buffer-band start
// Basis rows [first, first + gridDim.x) of every job (V row-major [row][npw_k] at J.voff)
// filled with a fixed pseudo-random complex block, entries in [-0.5, 0.5)^2: the start
// vectors of buffer bands, orthonormalised against the caller's block afterwards.
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h;
}
__global__ void __launch_bounds__(256) k_start_block(DJobs jobs, double2* __restrict__ V, int first) {
  const DJob& J = jobs.j[blockIdx.y];
  const int row = first + blockIdx.x;
  double2* v = V + J.voff + int64_t(row) * J.npw;
  const uint32_t base = mix32(uint32_t(J.k) * 0x9E3779B1u + uint32_t(row) * 0x85EBCA77u + 0x165667B1u);
  for (int g = threadIdx.x; g < J.npw; g += 256) {
    const uint32_t h1 = mix32(base ^ uint32_t(2 * g + 1)), h2 = mix32(base ^ uint32_t(2 * g + 2) * 0xC2B2AE3Du);
    v[g] = make_double2(double(h1) * 2.3283064365386963e-10 - 0.5, double(h2) * 2.3283064365386963e-10 - 0.5);
  }
}

// ---------------------------------------------------------------- residuals
// One workgroup per (job, band): r = HX - theta X into R, ||r||, <x|T|x>/<x|x>.  With a
// list, workgroup x < J.nu of a job takes band list[k][x] (the others return).
__global__ void __launch_bounds__(256) k_residual(DJobs jobs, const double2* __restrict__ X,
                                                  const double2* __restrict__ HX,
                                                  double2* __restrict__ Rr,
                                                  const double* __restrict__ theta,
                                                  const double* __restrict__ kin_all,
                                                  const int64_t* __restrict__ goff,
                                                  double* __restrict__ resn,
                                                  double* __restrict__ tkin,
                                                  const int32_t* __restrict__ list) {
  __shared__ double red[16];
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb;
  if (list ? int(blockIdx.x) >= J.nu : int(blockIdx.x) >= nb) return;
  const int n = list ? list[int64_t(J.k) * nb + blockIdx.x] : int(blockIdx.x);
  const double th = theta[int64_t(J.k) * jobs.mb + n];
  const int64_t off = J.xoff + int64_t(n) * J.npw;
  const double* kin = kin_all + goff[J.k];
  double rr = 0.0, xt = 0.0, xx = 0.0;
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const double2 x = X[off + g], h = HX[off + g];
    const double2 r = make_double2(h.x - th * x.x, h.y - th * x.y);
    Rr[off + g] = r;
    rr += r.x * r.x + r.y * r.y;
    const double p = x.x * x.x + x.y * x.y;
    xx += p;
    xt += p * kin[g];
  }
  rr = block_sum(rr, red);
  xt = block_sum(xt, red);
  xx = block_sum(xx, red);
  if (threadIdx.x == 0) {
    resn[int64_t(J.k) * nb + n] = sqrt(rr);
    tkin[int64_t(J.k) * nb + n] = xt / xx;
  }
}

// One workgroup per (job, j < nu): band n = unconv[k][j]; t = K(kin/T_n) r_n normalised,
// written to row (m - nu + j) of the basis block V.
// Largest squared norm, over the correction columns c of a job, of their overlap with the old
// basis after a Gram-Schmidt pass: ovl[k] = max_c sum_{i < m - nu} |C(i, c)|^2, C = V^H T.
// The corrections are unit vectors, so 1 - ovl[k] is the smallest squared column norm left
// by the pass.  Fixed-order sums and a max: the same result on every run.
__global__ void __launch_bounds__(256) k_cgs_overlap(DJobs jobs, const double2* __restrict__ Cw,
                                                     double* __restrict__ ovl) {
  __shared__ double red[4];
  const DJob& J = jobs.j[blockIdx.x];
  const int nb = jobs.nb, base = J.m - J.nu;
  const double2* C = Cw + int64_t(J.k) * jobs.mb * nb;
  double mx = 0.0;
  for (int c = threadIdx.x; c < J.nu; c += blockDim.x) {
    double sq = 0.0;
    for (int i = 0; i < base; ++i) {
      const double2 v = C[int64_t(i) * nb + c];
      sq += v.x * v.x + v.y * v.y;
    }
    mx = fmax(mx, sq);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) ovl[J.k] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void __launch_bounds__(256) k_teter(DJobs jobs, const double2* __restrict__ Rr,
                                               double2* __restrict__ V,
                                               const int32_t* __restrict__ unconv,
                                               const double* __restrict__ tkin,
                                               const double* __restrict__ kin_all,
                                               const int64_t* __restrict__ goff) {
  __shared__ double red[16];
  const DJob& J = jobs.j[blockIdx.y];
  const int nb = jobs.nb, j = blockIdx.x;
  if (j >= J.nu) return;
  const int n = unconv[int64_t(J.k) * nb + j];
  const double tn = tkin[int64_t(J.k) * nb + n];
  const double* kin = kin_all + goff[J.k];
  const double2* r = Rr + J.xoff + int64_t(n) * J.npw;
  double2* t = V + J.voff + int64_t(J.m - J.nu + j) * J.npw;
  double ss = 0.0;
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const double x = kin[g] / tn;
    const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
    const double k = num / (num + 16.0 * x * x * x * x);
    const double2 v = make_double2(k * r[g].x, k * r[g].y);
    t[g] = v;
    ss += v.x * v.x + v.y * v.y;
  }
  ss = block_sum(ss, red);
  const double s = 1.0 / sqrt(ss);
  for (int g = threadIdx.x; g < J.npw; g += blockDim.x) {
    const double2 v = t[g];
    t[g] = make_double2(v.x * s, v.y * s);
  }
}

}  // namespace qm
