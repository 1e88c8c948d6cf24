// Complex GEMMs on the gfx950 matrix cores.
//
// Two shapes cover the whole path:
//   CN:  C(i,j) = sum_g conj(A(i,g)) B(j,g)        projection P = beta^dagger psi
//        (Sec. 2.3 <beta_j|psi>), Davidson overlaps <v_i|H v_j>, <v_i|t_n>
//        (the ZGEMM-based vdot of Sec. 4.4).  K = g is contiguous for both operands;
//        tall-skinny (K up to 1e5), so K is split across workgroups and the
//        partial sums are reduced in a fixed order (deterministic).
//   EX:  Y(j,g) = alpha sum_i W(i,j) A(i,g) + beta Y   expansion beta (D P)
//        accumulated into H psi, Ritz updates X = V Y, Gram-Schmidt and CholQR
//        updates.
// Complex products in float64 and float32 are three real MFMAs (v_mfma_f64_16x16x4f64,
// v_mfma_f32_16x16x4f32) by Gauss's three-multiplication form: with t1 = sum ar br,
// t2 = sum ai bi and t3 = sum (ar + s ai)(br + s' bi) for the signs of the product, the real
// and imaginary parts are t1 -+ t2 and t3 - t1 +- t2 (the sums of the operand parts are
// formed once per element read from LDS).  bfloat16 operands (v_mfma_f32_16x16x32_bf16,
// float32 accumulation) use four: those kernels are bound by memory traffic.  Workgroup tile 64x64, four waves of
// 32x32 (2x2 MFMA tiles), K staged through LDS 16 (32 for bf16) at a time.
#include <hip/hip_bf16.h>

#include <type_traits>

#include "cplx.h"
#include "qm_internal.h"

namespace qm {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4v type; };
template <> struct Acc<float> { typedef f4v type; };

__device__ __forceinline__ d4v mfma4(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Output row of accumulator element r held by a lane (column = lane % 16), as measured on
// gfx950: the float64 16x16x4 MFMA interleaves rows (lane/16 + 4r), the float32 ones block
// them (4 (lane/16) + r).
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

// storage -> compute conversion of one complex element
template <typename T> __device__ __forceinline__ cplx<T> cv(double2 v) { return {T(v.x), T(v.y)}; }
template <typename T> __device__ __forceinline__ cplx<T> cv(float2 v) { return {T(v.x), T(v.y)}; }
// Ties a prefetched register value to this point of the program: the conversion and
// masking that follow are not moved up to the load, where the wave would wait for it.
__device__ __forceinline__ void pin(double2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
__device__ __forceinline__ void pin(float2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

struct CNDev {
  const void* A; const void* B;
  int32_t M, N, K, tm, tn, blk0;
  int64_t lda, ldb;
  int64_t work_off;   // complex elements
};
struct EXDev {
  const void* W; const void* A; void* Y;
  int32_t M, N, K, tm, tn, blk0;
  int64_t ldw, lda, ldy;
  const int32_t* rows;    // nullptr, or the W column / Y row of each product row
};

constexpr int MAXP = 24; // problems per launch (descriptors travel as kernel arguments)
struct CNBatch { CNDev p[MAXP]; int32_t n; };
struct EXBatch { EXDev p[MAXP]; int32_t n; };
struct CNOut;

constexpr int BT = 64;   // tile edge
constexpr int KC = 16;   // K chunk (complex elements)

// Workgroups are handed to the 8 XCDs round-robin (block b to XCD b % 8), and each XCD has
// its own L2.  This maps the hardware block index to a logical tile index so that every
// XCD works through one contiguous range of logical tiles; tiles that share an operand
// slab are numbered consecutively and so run on the same XCD at about the same time.
__device__ __forceinline__ int xcd_logical_block(int bid, int nblk) {
  const int full = nblk >> 3, rem = nblk & 7, x = bid & 7;
  return x * full + min(x, rem) + (bid >> 3);
}

template <typename B>
__device__ __forceinline__ int find_prob(const B& b, int bid) {
  int pi = 0;
  while (pi < b.n - 1 && bid >= b.p[pi + 1].blk0) ++pi;
  return pi;
}

// ------------------------------------------------------------------ CN, split-K partials
// Output tile TM x TN: 64 x 64, or 128 x 32 when the column count is a multiple of 32 but
// not of 64 (e.g. 160 bands: no padded columns); four waves of 32 x 32 each.
template <typename T, typename SA, typename SB, int TM, int TN>
__global__ void __launch_bounds__(256, 2) k_cgemm_cn(const CNBatch batch, int nsplit,
                                                  cplx<T>* __restrict__ work) {
  typedef typename Acc<T>::type AV;
  constexpr int NAE = TM * KC / 256, NBE = TN * KC / 256;   // K values per thread and chunk
  constexpr int WM = TM / 32;                               // waves along the rows
  __shared__ cplx<T> As[TM][KC + 1];
  __shared__ cplx<T> Bs[TN][KC + 1];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int pi = find_prob(batch, lb);
  const CNDev& P = batch.p[pi];
  // the tiles of one K split are numbered consecutively (column tiles fastest), so each of
  // its A and B slabs is fetched from memory once and shared through the XCD's L2
  const int bid = lb - P.blk0, per_split = P.tm * P.tn;
  const int split = bid / per_split, tile = bid - split * per_split;
  const int i0 = (tile / P.tn) * TM, j0 = (tile % P.tn) * TN;
  const int nch = (P.K + KC - 1) / KC;
  const int per = (nch + nsplit - 1) / nsplit;
  const int c0 = split * per, c1 = min(nch, c0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave % WM) * 32, wj = (wave / WM) * 32;
  const int larow = tid / (KC / NAE), laseg = (tid % (KC / NAE)) * NAE;
  const int lbrow = tid / (KC / NBE), lbseg = (tid % (KC / NBE)) * NBE;
  const SA* A = reinterpret_cast<const SA*>(P.A);
  const SB* B = reinterpret_cast<const SB*>(P.B);
  AV t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = AV{0, 0, 0, 0};
      t2[a][b] = AV{0, 0, 0, 0};
      t3[a][b] = AV{0, 0, 0, 0};
    }
  const bool arow = (i0 + larow) < P.M, brow = (j0 + lbrow) < P.N;
  // rows past the matrix read row i0 / j0 (which exists) and are zeroed after the load
  const SA* Ar = A + int64_t(arow ? i0 + larow : i0) * P.lda;
  const SB* Br = B + int64_t(brow ? j0 + lbrow : j0) * P.ldb;
  // the next chunk's operands are loaded into registers, in their storage type, while this
  // chunk's MFMAs run; they are converted, and the rows past the matrix zeroed, when they are
  // stored to LDS (work on them right after the load would wait for it there)
  SA pa[NAE];
  SB pb[NBE];
  auto fetch = [&](int c) {
    const int ka = c * KC + laseg, kb = c * KC + lbseg;
    // the test is the same for the whole workgroup, so the interior loads are not followed
    // by lane-masked writes of the same registers (which would wait for them)
    const bool inner = (c + 1) * KC <= P.K;
    if (inner) {   // the whole chunk inside K: no element tests
#pragma unroll
      for (int q = 0; q < NAE; ++q) pa[q] = Ar[ka + q];
#pragma unroll
      for (int q = 0; q < NBE; ++q) pb[q] = Br[kb + q];
    } else {
#pragma unroll
      for (int q = 0; q < NAE; ++q) pa[q] = ka + q < P.K ? Ar[ka + q] : SA{0, 0};
#pragma unroll
      for (int q = 0; q < NBE; ++q) pb[q] = kb + q < P.K ? Br[kb + q] : SB{0, 0};
    }
  };
  if (c0 < c1) fetch(c0);
  for (int c = c0; c < c1; ++c) {
#pragma unroll
    for (int q = 0; q < NAE; ++q) {
      pin(pa[q]);
      As[larow][laseg + q] = arow ? cv<T>(pa[q]) : cplx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < NBE; ++q) {
      pin(pb[q]);
      Bs[lbrow][lbseg + q] = brow ? cv<T>(pb[q]) : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    if (c + 1 < c1) fetch(c + 1);
    // LDS fragments of two K steps: the next step's are read while this step's MFMAs run
    // (the scheduling barrier keeps the reads ahead of the MFMAs). Not in the float64
    // 128 x 32 tile, where reading ahead measured slower.
    constexpr bool AHEAD = !(std::is_same<T, double>::value && TM == 128);
    cplx<T> fa[2][2], fb[2][2];
    auto rd = [&](int kk, int u) {
      const int kq = kk * 4 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[u][t] = As[wi + t * 16 + (lane & 15)][kq];
        fb[u][t] = Bs[wj + t * 16 + (lane & 15)][kq];
      }
    };
    if constexpr (AHEAD) rd(0, 0);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int u = AHEAD ? (kk & 1) : 0;
      if constexpr (AHEAD) {
        if (kk + 1 < KC / 4) rd(kk + 1, u ^ 1);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        rd(kk, 0);
      }
      const cplx<T>* a = fa[u];
      const cplx<T>* b = fb[u];
      // conj(a) b = (ar br + ai bi) + i (ar bi - ai br); (ar - ai)(br + bi) = t1 - t2 + im
      T sa[2], sb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        sa[t] = a[t].re - a[t].im;
        sb[t] = b[t].re + b[t].im;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          t1[ti][tj] = mfma4(a[ti].re, b[tj].re, t1[ti][tj]);
          t2[ti][tj] = mfma4(a[ti].im, b[tj].im, t2[ti][tj]);
          t3[ti][tj] = mfma4(sa[ti], sb[tj], t3[ti][tj]);
        }
    }
    __syncthreads();
  }
  cplx<T>* W = work + P.work_off + int64_t(split) * P.M * P.N;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + ti * 16 + acc_row<T>(lane, r);
        const int j = j0 + wj + tj * 16 + (lane & 15);
        const T x1 = t1[ti][tj][r], x2 = t2[ti][tj][r];
        if (i < P.M && j < P.N) W[int64_t(i) * P.N + j] = cplx<T>{x1 + x2, t3[ti][tj][r] - x1 + x2};
      }
}

// C = alpha * sum_s part_s + beta * C  (c128 output, row-major ldc)
struct CNOut { void* C; int32_t M, N; int64_t ldc, work_off, elem0; };
struct CNOutBatch { CNOut p[MAXP]; int32_t n; };
template <typename T>
__global__ void k_cn_reduce(const CNOutBatch outs, int nsplit,
                            const cplx<T>* __restrict__ work, double alpha, double beta,
                            int64_t total) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    int pi = 0;
    while (pi < outs.n - 1 && t >= outs.p[pi + 1].elem0) ++pi;
    const CNOut& o = outs.p[pi];
    const int64_t e = t - o.elem0;
    const int i = int(e / o.N), j = int(e % o.N);
    double sr = 0, si = 0;
    const cplx<T>* w = work + o.work_off + e;
    for (int s = 0; s < nsplit; ++s) {
      sr += double(w[int64_t(s) * o.M * o.N].re);
      si += double(w[int64_t(s) * o.M * o.N].im);
    }
    double2* c = reinterpret_cast<double2*>(o.C) + int64_t(i) * o.ldc + j;
    double2 old = beta != 0.0 ? *c : make_double2(0.0, 0.0);
    *c = make_double2(alpha * sr + beta * old.x, alpha * si + beta * old.y);
  }
}

// ------------------------------------------------------------------ EX
// Makes a loaded value live in registers at this point, so that its load is not moved into
// a later conditional block.
__device__ __forceinline__ void hold(double x) { asm volatile("" ::"v"(x)); }

// Y = alpha * acc + beta * Y for a wave's 2 x 2 accumulator tiles (element r of a lane at
// row acc_row, column lane % 16).  With beta != 0 the eight old values of one tile row are
// loaded together, from addresses clamped into the matrix, and held in registers before
// the guarded stores: a load under each element's guard had compiled to one memory round
// trip per element.
template <typename T, typename AV, bool ROWS = false>
__device__ __forceinline__ void store_ex_tile(const EXDev& P, int m0, int n0, int wi, int wj, int lane,
                                              const AV (&cr)[2][2], const AV (&ci)[2][2], double alpha,
                                              double beta) {
  double2* Y = reinterpret_cast<double2*>(P.Y);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti) {
    double ore[8], oim[8];
    if (beta != 0.0) {
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = min(m0 + wi + ti * 16 + acc_row<T>(lane, r), P.M - 1);
          const int n = min(n0 + wj + tj * 16 + (lane & 15), P.N - 1);
          const int mr = (ROWS && P.rows) ? P.rows[m] : m;
          const double2 o = Y[int64_t(mr) * P.ldy + n];
          ore[tj * 4 + r] = o.x;
          oim[tj * 4 + r] = o.y;
        }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hold(ore[e]);
        hold(oim[e]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) ore[e] = oim[e] = 0.0;
    }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wi + ti * 16 + acc_row<T>(lane, r);
        const int n = n0 + wj + tj * 16 + (lane & 15);
        if (m < P.M && n < P.N)
          Y[int64_t((ROWS && P.rows) ? P.rows[m] : m) * P.ldy + n] =
              make_double2(alpha * double(cr[ti][tj][r]) + beta * ore[tj * 4 + r],
                           alpha * double(ci[ti][tj][r]) + beta * oim[tj * 4 + r]);
      }
  }
}

// Output tile TM x TN (64 x 64, or 32 x 128 when the row count is a multiple of 32 but not
// of 64, e.g. 160 bands: no padded rows); four waves of 32 x 32 each.
// ROWS: the problems may carry row lists (EXDev::rows); the other instantiations ignore them
template <typename T, typename SW, typename SA, int TM, int TN, bool ROWS = false>
__global__ void __launch_bounds__(256, 2) k_cgemm_ex(const EXBatch batch, double alpha, double beta) {
  typedef typename Acc<T>::type AV;
  constexpr int NWE = KC * TM / 256, NAE = KC * TN / 256;   // elements per thread and chunk
  constexpr int WM = TM / 32;                               // waves along the rows
  __shared__ cplx<T> Ws[KC][TM + 1];
  __shared__ cplx<T> As[KC][TN + 1];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int pi = find_prob(batch, lb);
  const EXDev& P = batch.p[pi];
  // row tiles fastest: the row tiles of one column tile share the A slab
  const int tile = lb - P.blk0;
  const int m0 = (tile % P.tm) * TM, n0 = (tile / P.tm) * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave % WM) * 32, wj = (wave / WM) * 32;
  const int lrw = tid / (TM / NWE), lcw = (tid % (TM / NWE)) * NWE;
  const int lra = tid / (TN / NAE), lca = (tid % (TN / NAE)) * NAE;
  const SW* Wp = reinterpret_cast<const SW*>(P.W);
  const SA* Ap = reinterpret_cast<const SA*>(P.A);
  AV t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = AV{0, 0, 0, 0};
      t2[a][b] = AV{0, 0, 0, 0};
      t3[a][b] = AV{0, 0, 0, 0};
    }
  const int nch = (P.K + KC - 1) / KC;
  // the next chunk's operands are loaded into registers, in their storage type, while this
  // chunk's MFMAs run, and converted when they are stored to LDS
  SW pw[NWE];
  SA pa[NAE];
  // with a row list, this thread's W columns (-1 past M), fixed for the whole K loop
  int wcol[ROWS ? NWE : 1];
  if constexpr (ROWS) {
#pragma unroll
    for (int q = 0; q < NWE; ++q) {
      const int m = m0 + lcw + q;
      wcol[q] = m < P.M ? (P.rows ? P.rows[m] : m) : -1;
    }
  }
  auto fetch = [&](int c) {
    const int iw = c * KC + lrw, ia = c * KC + lra;
    // the interior tests are the same for the whole workgroup, so the interior loads are not
    // followed by lane-masked writes of the same registers (which would wait for them)
    const bool inner_k = (c + 1) * KC <= P.K;
    if (ROWS && P.rows) {   // clamped loads; columns past M and rows past K zeroed in the store
#pragma unroll
      for (int q = 0; q < NWE; ++q)
        pw[q] = Wp[int64_t(min(iw, P.K - 1)) * P.ldw + max(wcol[ROWS ? q : 0], 0)];
    } else if (inner_k && m0 + TM <= P.M) {   // interior: no element tests
#pragma unroll
      for (int q = 0; q < NWE; ++q) pw[q] = Wp[int64_t(iw) * P.ldw + m0 + lcw + q];
    } else {
#pragma unroll
      for (int q = 0; q < NWE; ++q) {
        const int m = m0 + lcw + q;
        pw[q] = (iw < P.K && m < P.M) ? Wp[int64_t(iw) * P.ldw + m] : SW{0, 0};
      }
    }
    if (inner_k && n0 + TN <= P.N) {
#pragma unroll
      for (int q = 0; q < NAE; ++q) pa[q] = Ap[int64_t(ia) * P.lda + n0 + lca + q];
    } else {
#pragma unroll
      for (int q = 0; q < NAE; ++q) {
        const int n = n0 + lca + q;
        pa[q] = (ia < P.K && n < P.N) ? Ap[int64_t(ia) * P.lda + n] : SA{0, 0};
      }
    }
  };
  if (nch > 0) fetch(0);
  for (int c = 0; c < nch; ++c) {
#pragma unroll
    for (int q = 0; q < NWE; ++q) {
      if constexpr (ROWS) {
        const bool ok = !P.rows || (c * KC + lrw < P.K && wcol[q] >= 0);
        Ws[lrw][lcw + q] = ok ? cv<T>(pw[q]) : cplx<T>{T(0), T(0)};
      } else {
        Ws[lrw][lcw + q] = cv<T>(pw[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NAE; ++q) As[lra][lca + q] = cv<T>(pa[q]);
    __syncthreads();
    if (c + 1 < nch) fetch(c + 1);
    // LDS fragments of two K steps: the next step's are read while this step's MFMAs run
    // (the scheduling barrier keeps the reads ahead of the MFMAs)
    constexpr bool AHEAD = true;
    cplx<T> fa[2][2], fb[2][2];
    auto rd = [&](int kk, int u) {
      const int kq = kk * 4 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[u][t] = Ws[kq][wi + t * 16 + (lane & 15)];
        fb[u][t] = As[kq][wj + t * 16 + (lane & 15)];
      }
    };
    if constexpr (AHEAD) rd(0, 0);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int u = AHEAD ? (kk & 1) : 0;
      if constexpr (AHEAD) {
        if (kk + 1 < KC / 4) rd(kk + 1, u ^ 1);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        rd(kk, 0);
      }
      const cplx<T>* a = fa[u];
      const cplx<T>* b = fb[u];
      // w a = (wr ar - wi ai) + i (wr ai + wi ar); (wr + wi)(ar + ai) = t1 + t2 + im
      T sa[2], sb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        sa[t] = a[t].re + a[t].im;
        sb[t] = b[t].re + b[t].im;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          t1[ti][tj] = mfma4(a[ti].re, b[tj].re, t1[ti][tj]);
          t2[ti][tj] = mfma4(a[ti].im, b[tj].im, t2[ti][tj]);
          t3[ti][tj] = mfma4(sa[ti], sb[tj], t3[ti][tj]);
        }
    }
    __syncthreads();
  }
  AV cr[2][2], ci[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      cr[ti][tj] = t1[ti][tj] - t2[ti][tj];
      ci[ti][tj] = t3[ti][tj] - t1[ti][tj] - t2[ti][tj];
    }
  store_ex_tile<T, AV, ROWS>(P, m0, n0, wi, wj, lane, cr, ci, alpha, beta);
}


// ------------------------------------------------------------------ bfloat16 operands
// v_mfma_f32_16x16x32_bf16: lane l supplies A[i = l%16][k = 8(l/16) .. +7] and
// B[k = 8(l/16) .. +7][j = l%16]; the four float32 accumulators follow the float32
// 16x16 layout.  Complex operands are staged in LDS as separate re/im planes with K
// contiguous so each lane reads its eight K values with one 16-byte load.
typedef unsigned short u16;
struct bf2 { u16 re, im; };   // bfloat16 complex storage (round to nearest even)

__device__ __forceinline__ u16 f2bf(float x) {
  __bf16 b = (__bf16)x;
  return *reinterpret_cast<u16*>(&b);
}
__device__ __forceinline__ bf8v ld8(const u16* p) {
  typedef u16 u16x8 __attribute__((ext_vector_type(8)));
  u16x8 v = *reinterpret_cast<const u16x8*>(p);
  return *reinterpret_cast<bf8v*>(&v);
}
__device__ __forceinline__ bf8v neg8(bf8v a) {
  typedef u16 u16x8 __attribute__((ext_vector_type(8)));
  u16x8 v = *reinterpret_cast<u16x8*>(&a);
  v ^= (u16)0x8000;
  return *reinterpret_cast<bf8v*>(&v);
}
__device__ __forceinline__ f4v mfma32(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
// two floats -> two bfloat16 (round to nearest even) packed low, high
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi) {
  bf2v b = __builtin_convertvector((f2v){lo, hi}, bf2v);
  return *reinterpret_cast<uint32_t*>(&b);
}
// eight stored bf16 complex (re | im << 16) -> the re plane and the im plane, 16 bytes each
__device__ __forceinline__ void split_bf2(const uint32_t* v, uint4& re, uint4& im) {
  re = make_uint4((v[0] & 0xffffu) | (v[1] << 16), (v[2] & 0xffffu) | (v[3] << 16),
                  (v[4] & 0xffffu) | (v[5] << 16), (v[6] & 0xffffu) | (v[7] << 16));
  im = make_uint4((v[0] >> 16) | (v[1] & 0xffff0000u), (v[2] >> 16) | (v[3] & 0xffff0000u),
                  (v[4] >> 16) | (v[5] & 0xffff0000u), (v[6] >> 16) | (v[7] & 0xffff0000u));
}
// eight c128 -> bfloat16 re plane and im plane
__device__ __forceinline__ void pack_c128(const double2* v, uint4& re, uint4& im) {
  re = make_uint4(pk_bf16(float(v[0].x), float(v[1].x)), pk_bf16(float(v[2].x), float(v[3].x)),
                  pk_bf16(float(v[4].x), float(v[5].x)), pk_bf16(float(v[6].x), float(v[7].x)));
  im = make_uint4(pk_bf16(float(v[0].y), float(v[1].y)), pk_bf16(float(v[2].y), float(v[3].y)),
                  pk_bf16(float(v[4].y), float(v[5].y)), pk_bf16(float(v[6].y), float(v[7].y)));
}

constexpr int KB = 32;       // K chunk of the bf16 kernels (complex elements)
constexpr int KBP = KB + 8;  // padded LDS row (bf16 elements), keeps 16-byte alignment

// CN with A = bf16 complex (beta), B = c128 (psi, converted on load); float32 partials
__global__ void __launch_bounds__(256) k_cgemm_cn_bf16(const CNBatch batch, int nsplit,
                                                       cplx<float>* __restrict__ work) {
  __shared__ __align__(16) u16 Ar[BT][KBP], Ai[BT][KBP], Br[BT][KBP], Bi[BT][KBP];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int pi = find_prob(batch, lb);
  const CNDev& P = batch.p[pi];
  // the tiles of one K split are numbered consecutively (column tiles fastest), so each of
  // its A and B slabs is fetched from memory once and shared through the XCD's L2
  const int bid = lb - P.blk0, per_split = P.tm * P.tn;
  const int split = bid / per_split, tile = bid - split * per_split;
  const int i0 = (tile / P.tn) * BT, j0 = (tile % P.tn) * BT;
  const int nch = (P.K + KB - 1) / KB;
  const int per = (nch + nsplit - 1) / nsplit;
  const int c0 = split * per, c1 = min(nch, c0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
  const int lrow = tid >> 2, lseg = (tid & 3) * 8;   // 64 rows x 4 segments of 8
  const bf2* A = reinterpret_cast<const bf2*>(P.A);
  const double2* B = reinterpret_cast<const double2*>(P.B);
  f4v cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = f4v{0, 0, 0, 0};
      ci[a][b] = f4v{0, 0, 0, 0};
    }
  const bool arow = (i0 + lrow) < P.M, brow = (j0 + lrow) < P.N;
  // rows past the matrix read row i0 / j0 (which exists) and are zeroed after the load
  const bf2* Arow = A + int64_t(arow ? i0 + lrow : i0) * P.lda;
  const double2* Brow = B + int64_t(brow ? j0 + lrow : j0) * P.ldb;
  // raw operands of the next two chunks are in flight while this chunk's MFMAs run
  // (two register sets, used alternately); converted and stored to LDS as 16-byte re and
  // im runs of eight K values
  uint32_t pa0[8], pa1[8];
  double2 pb0[8], pb1[8];
  auto fetch = [&](uint32_t* pa, double2* pb, int c) {
    const int kb = c * KB + lseg;
    if (kb + 8 <= P.K) {   // whole run inside K: one bounds test per row
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t av = *reinterpret_cast<const uint32_t*>(Arow + kb + q);
        const double2 bv = Brow[kb + q];
        pa[q] = arow ? av : 0u;
        pb[q] = brow ? bv : make_double2(0.0, 0.0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int g = kb + q;
        pa[q] = (arow && g < P.K) ? *reinterpret_cast<const uint32_t*>(Arow + g) : 0u;
        pb[q] = (brow && g < P.K) ? Brow[g] : make_double2(0.0, 0.0);
      }
    }
  };
  auto stage = [&](const uint32_t* pa, const double2* pb) {
    uint4 re, im;
    split_bf2(pa, re, im);
    *reinterpret_cast<uint4*>(&Ar[lrow][lseg]) = re;
    *reinterpret_cast<uint4*>(&Ai[lrow][lseg]) = im;
    pack_c128(pb, re, im);
    *reinterpret_cast<uint4*>(&Br[lrow][lseg]) = re;
    *reinterpret_cast<uint4*>(&Bi[lrow][lseg]) = im;
  };
  auto compute = [&]() {
    const int ko = 8 * (lane >> 4);
    bf8v ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      ar[t] = ld8(&Ar[wi + t * 16 + (lane & 15)][ko]);
      ai[t] = ld8(&Ai[wi + t * 16 + (lane & 15)][ko]);
      nai[t] = neg8(ai[t]);
      br[t] = ld8(&Br[wj + t * 16 + (lane & 15)][ko]);
      bi[t] = ld8(&Bi[wj + t * 16 + (lane & 15)][ko]);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        cr[ti][tj] = mfma32(ar[ti], br[tj], cr[ti][tj]);
        cr[ti][tj] = mfma32(ai[ti], bi[tj], cr[ti][tj]);
        ci[ti][tj] = mfma32(ar[ti], bi[tj], ci[ti][tj]);
        ci[ti][tj] = mfma32(nai[ti], br[tj], ci[ti][tj]);
      }
  };
  if (c0 < c1) fetch(pa0, pb0, c0);
  if (c0 + 1 < c1) fetch(pa1, pb1, c0 + 1);
  for (int c = c0; c < c1; c += 2) {
    stage(pa0, pb0);
    __syncthreads();
    if (c + 2 < c1) fetch(pa0, pb0, c + 2);
    compute();
    __syncthreads();
    if (c + 1 >= c1) break;
    stage(pa1, pb1);
    __syncthreads();
    if (c + 3 < c1) fetch(pa1, pb1, c + 3);
    compute();
    __syncthreads();
  }
  cplx<float>* W = work + P.work_off + int64_t(split) * P.M * P.N;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + ti * 16 + acc_row<float>(lane, r);
        const int j = j0 + wj + tj * 16 + (lane & 15);
        if (i < P.M && j < P.N) W[int64_t(i) * P.N + j] = cplx<float>{cr[ti][tj][r], ci[ti][tj][r]};
      }
}

// EX with W = c128 (Q, converted on load), A = bf16 complex (beta); Y c128 accumulated
__global__ void __launch_bounds__(256) k_cgemm_ex_bf16(const EXBatch batch, double alpha, double beta) {
  __shared__ __align__(16) u16 Wr[BT][KBP], Wi[BT][KBP], Ar[BT][KBP], Ai[BT][KBP];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int pi = find_prob(batch, lb);
  const EXDev& P = batch.p[pi];
  // row tiles fastest: the row tiles of one column tile share the A slab
  const int tile = lb - P.blk0;
  const int m0 = (tile % P.tm) * BT, n0 = (tile / P.tm) * BT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
  const double2* Wp = reinterpret_cast<const double2*>(P.W);
  const bf2* Ap = reinterpret_cast<const bf2*>(P.A);
  f4v cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = f4v{0, 0, 0, 0};
      ci[a][b] = f4v{0, 0, 0, 0};
    }
  const int nch = (P.K + KB - 1) / KB;
  // staging: thread t takes column t%64 of both tiles and the eight K rows 8 (t/64) .. +7,
  // so its values form the K-contiguous run one LDS row needs (16-byte stores); lanes hold
  // consecutive columns, so every global load is coalesced.  The next chunk is loaded
  // while this chunk's MFMAs run.
  const int col = tid & 63, kg = (tid >> 6) * 8;
  const bool wcol = m0 + col < P.M, acol = n0 + col < P.N;
  // columns past the matrix read column m0 / n0 (which exists) and are zeroed after the load
  const int wc = wcol ? m0 + col : m0, ac = acol ? n0 + col : n0;
  double2 pw[8];
  uint32_t pa[8];
  auto fetch = [&](int c) {
    const int i0 = c * KB + kg;
    if ((c + 1) * KB <= P.K) {   // the whole chunk inside K (a workgroup-uniform test)
#pragma unroll
      for (int q = 0; q < 8; ++q) {   // columns past the matrix are zeroed when staged
        pw[q] = Wp[int64_t(i0 + q) * P.ldw + wc];
        pa[q] = *reinterpret_cast<const uint32_t*>(Ap + int64_t(i0 + q) * P.lda + ac);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q;
        pw[q] = (i < P.K && wcol) ? Wp[int64_t(i) * P.ldw + m0 + col] : make_double2(0.0, 0.0);
        pa[q] = (i < P.K && acol) ? *reinterpret_cast<const uint32_t*>(Ap + int64_t(i) * P.lda + n0 + col)
                                  : 0u;
      }
    }
  };
  if (nch > 0) fetch(0);
  for (int c = 0; c < nch; ++c) {
    {
      double2 w8[8];
      uint32_t a8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        w8[q] = wcol ? pw[q] : make_double2(0.0, 0.0);
        a8[q] = acol ? pa[q] : 0u;
      }
      uint4 re, im;
      pack_c128(w8, re, im);
      *reinterpret_cast<uint4*>(&Wr[col][kg]) = re;
      *reinterpret_cast<uint4*>(&Wi[col][kg]) = im;
      split_bf2(a8, re, im);
      *reinterpret_cast<uint4*>(&Ar[col][kg]) = re;
      *reinterpret_cast<uint4*>(&Ai[col][kg]) = im;
    }
    __syncthreads();
    if (c + 1 < nch) fetch(c + 1);
    const int ko = 8 * (lane >> 4);
    bf8v wr[2], wim[2], nwi[2], ar[2], ai[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      wr[t] = ld8(&Wr[wi + t * 16 + (lane & 15)][ko]);
      wim[t] = ld8(&Wi[wi + t * 16 + (lane & 15)][ko]);
      nwi[t] = neg8(wim[t]);
      ar[t] = ld8(&Ar[wj + t * 16 + (lane & 15)][ko]);
      ai[t] = ld8(&Ai[wj + t * 16 + (lane & 15)][ko]);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        cr[ti][tj] = mfma32(wr[ti], ar[tj], cr[ti][tj]);
        cr[ti][tj] = mfma32(nwi[ti], ai[tj], cr[ti][tj]);
        ci[ti][tj] = mfma32(wr[ti], ai[tj], ci[ti][tj]);
        ci[ti][tj] = mfma32(wim[ti], ar[tj], ci[ti][tj]);
      }
    __syncthreads();
  }
  store_ex_tile<float>(P, m0, n0, wi, wj, lane, cr, ci, alpha, beta);
}

// beta (c128) -> float32 or bfloat16 complex copy
__global__ void k_beta_lp(const double2* __restrict__ in, void* __restrict__ out, int64_t n, int kind) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const double2 v = in[t];
    if (kind == 1) {
      reinterpret_cast<float2*>(out)[t] = make_float2(float(v.x), float(v.y));
    } else {
      reinterpret_cast<bf2*>(out)[t] = bf2{f2bf(float(v.x)), f2bf(float(v.y))};
    }
  }
}

void convert_beta_lp(const void* beta64, void* out, int64_t n, int kind, hipStream_t s) {
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(k_beta_lp, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(beta64),
                     out, n, kind);
  QM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ host side
static int choose_splits(int64_t tiles, int64_t maxK) {
  int s = 1;
  while (tiles * s < 1024 && (maxK / (KC * (s * 2))) >= 8 && s < 64) s *= 2;
  return s;
}

int64_t zgemm_cn_work_bytes(const std::vector<GemmCN>& probs) {
  int64_t tiles = 0, maxK = 0, mn = 0;
  for (const GemmCN& g : probs) {
    tiles += int64_t((g.M + BT - 1) / BT) * ((g.N + BT - 1) / BT);
    maxK = std::max<int64_t>(maxK, g.K);
    mn += int64_t(g.M) * g.N;
  }
  return int64_t(choose_splits(tiles, maxK)) * mn * int64_t(sizeof(cplx<double>));
}

void zgemm_cn_batched(const std::vector<GemmCN>& probs, double alpha, double beta_c, void* work,
                      int64_t work_bytes, hipStream_t s, StageEvents* ev, int stage0, int lp,
                      int force_split) {
  for (size_t base = 0; base < probs.size(); base += MAXP) {
    const size_t n = std::min<size_t>(MAXP, probs.size() - base);
    std::vector<GemmCN> sub(probs.begin() + base, probs.begin() + base + n);
    CNBatch d{};
    CNOutBatch o{};
    d.n = o.n = int32_t(n);
    // tile shape: 128 x 32 where it pads fewer output elements than 64 x 64 (bf16: 64 x 64)
    int64_t pad64 = 0, padw = 0;
    for (const GemmCN& g : sub) {
      pad64 += int64_t((g.M + 63) / 64 * 64) * ((g.N + 63) / 64 * 64);
      padw += int64_t((g.M + 127) / 128 * 128) * ((g.N + 31) / 32 * 32);
    }
    const bool wide = lp != 2 && padw * 20 < pad64 * 19;   // at least 5% less padded work
    const int tm_ = wide ? 128 : 64, tn_ = wide ? 32 : 64;
    int64_t tiles = 0, maxK = 0;
    for (const GemmCN& g : sub) {
      tiles += int64_t((g.M + tm_ - 1) / tm_) * ((g.N + tn_ - 1) / tn_);
      maxK = std::max<int64_t>(maxK, g.K);
    }
    int64_t mn = 0;
    for (const GemmCN& g : sub) mn += int64_t(g.M) * g.N;
    int nsplit = force_split > 0 ? force_split : choose_splits(tiles, maxK);
    while (nsplit > 1 && int64_t(nsplit) * mn * int64_t(sizeof(cplx<double>)) > work_bytes) nsplit /= 2;
    int64_t blk = 0, woff = 0, e0 = 0;
    for (size_t i = 0; i < n; ++i) {
      const GemmCN& g = sub[i];
      CNDev& x = d.p[i];
      x.A = g.A; x.B = g.B;
      x.M = g.M; x.N = g.N; x.K = g.K;
      x.tm = (g.M + tm_ - 1) / tm_; x.tn = (g.N + tn_ - 1) / tn_;
      x.blk0 = int32_t(blk);
      x.lda = g.lda; x.ldb = g.ldb;
      x.work_off = woff;
      o.p[i] = CNOut{g.C, g.M, g.N, g.ldc, woff, e0};
      blk += int64_t(x.tm) * x.tn * nsplit;
      woff += int64_t(nsplit) * g.M * g.N;
      e0 += int64_t(g.M) * g.N;
    }
    if (e0 == 0) continue;
    QM_REQUIRE(woff * int64_t(sizeof(cplx<double>)) <= work_bytes, QM_E_STATE,
               "GEMM split-K workspace too small");
    const int rb = int(std::min<int64_t>((e0 + 255) / 256, 8192));
    if (lp == 0) {
      if (wide)
        hipLaunchKernelGGL((k_cgemm_cn<double, double2, double2, 128, 32>), dim3(unsigned(blk)), dim3(256),
                           0, s, d, nsplit, reinterpret_cast<cplx<double>*>(work));
      else
        hipLaunchKernelGGL((k_cgemm_cn<double, double2, double2, 64, 64>), dim3(unsigned(blk)), dim3(256),
                           0, s, d, nsplit, reinterpret_cast<cplx<double>*>(work));
      QM_HIP(hipGetLastError());
      if (ev) ev->mark(stage0);
      hipLaunchKernelGGL(k_cn_reduce<double>, dim3(rb), dim3(256), 0, s, o, nsplit,
                         reinterpret_cast<const cplx<double>*>(work), alpha, beta_c, e0);
    } else {
      if (lp == 1)
        if (wide)
          hipLaunchKernelGGL((k_cgemm_cn<float, float2, double2, 128, 32>), dim3(unsigned(blk)), dim3(256),
                             0, s, d, nsplit, reinterpret_cast<cplx<float>*>(work));
        else
          hipLaunchKernelGGL((k_cgemm_cn<float, float2, double2, 64, 64>), dim3(unsigned(blk)), dim3(256),
                             0, s, d, nsplit, reinterpret_cast<cplx<float>*>(work));
      else if (lp == 3)
        if (wide)
          hipLaunchKernelGGL((k_cgemm_cn<float, double2, double2, 128, 32>), dim3(unsigned(blk)), dim3(256),
                             0, s, d, nsplit, reinterpret_cast<cplx<float>*>(work));
        else
          hipLaunchKernelGGL((k_cgemm_cn<float, double2, double2, 64, 64>), dim3(unsigned(blk)), dim3(256),
                             0, s, d, nsplit, reinterpret_cast<cplx<float>*>(work));
      else
        hipLaunchKernelGGL(k_cgemm_cn_bf16, dim3(unsigned(blk)), dim3(256), 0, s, d, nsplit,
                           reinterpret_cast<cplx<float>*>(work));
      QM_HIP(hipGetLastError());
      if (ev) ev->mark(stage0);
      hipLaunchKernelGGL(k_cn_reduce<float>, dim3(rb), dim3(256), 0, s, o, nsplit,
                         reinterpret_cast<const cplx<float>*>(work), alpha, beta_c, e0);
    }
    QM_HIP(hipGetLastError());
    if (ev) ev->mark(stage0 + 1);
  }
}

void zgemm_ex_batched(const std::vector<GemmEX>& probs, double alpha, double beta_y, hipStream_t s,
                      int lp) {
  for (size_t base = 0; base < probs.size(); base += MAXP) {
    const size_t n = std::min<size_t>(MAXP, probs.size() - base);
    // tile shape: 32 x 128 where it pads fewer output elements than 64 x 64 (bf16: 64 x 64)
    int64_t pad64 = 0, pad32 = 0;
    for (size_t i = 0; i < n; ++i) {
      const GemmEX& g = probs[base + i];
      pad64 += int64_t((g.M + 63) / 64 * 64) * ((g.N + 63) / 64 * 64);
      pad32 += int64_t((g.M + 31) / 32 * 32) * ((g.N + 127) / 128 * 128);
    }
    const bool narrow = lp != 2 && pad32 * 20 < pad64 * 19;   // at least 5% less padded work
    const int tm_ = narrow ? 32 : 64, tn_ = narrow ? 128 : 64;
    EXBatch d{};
    d.n = int32_t(n);
    int64_t blk = 0;
    for (size_t i = 0; i < n; ++i) {
      const GemmEX& g = probs[base + i];
      EXDev& x = d.p[i];
      x.W = g.W; x.A = g.A; x.Y = g.Y;
      x.rows = g.rows;

      x.M = g.M; x.N = g.N; x.K = g.K;
      x.tm = (g.M + tm_ - 1) / tm_; x.tn = (g.N + tn_ - 1) / tn_;
      x.blk0 = int32_t(blk);
      x.ldw = g.ldw; x.lda = g.lda; x.ldy = g.ldy;
      blk += int64_t(x.tm) * x.tn;
    }
    if (blk == 0) continue;
    bool rows = false;
    for (size_t i = 0; i < n; ++i) rows = rows || probs[base + i].rows;
    QM_REQUIRE(!rows || lp == 0, QM_E_STATE, "row lists need the float64 expansion kernels");
    if (rows && narrow)
      hipLaunchKernelGGL((k_cgemm_ex<double, double2, double2, 32, 128, true>), dim3(unsigned(blk)), dim3(256),
                         0, s, d, alpha, beta_y);
    else if (rows)
      hipLaunchKernelGGL((k_cgemm_ex<double, double2, double2, 64, 64, true>), dim3(unsigned(blk)), dim3(256),
                         0, s, d, alpha, beta_y);
    else if (lp == 0 && narrow)
      hipLaunchKernelGGL((k_cgemm_ex<double, double2, double2, 32, 128>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else if (lp == 0)
      hipLaunchKernelGGL((k_cgemm_ex<double, double2, double2, 64, 64>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else if (lp == 1 && narrow)
      hipLaunchKernelGGL((k_cgemm_ex<float, double2, float2, 32, 128>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else if (lp == 1)
      hipLaunchKernelGGL((k_cgemm_ex<float, double2, float2, 64, 64>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else if (lp == 3 && narrow)
      hipLaunchKernelGGL((k_cgemm_ex<float, double2, double2, 32, 128>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else if (lp == 3)
      hipLaunchKernelGGL((k_cgemm_ex<float, double2, double2, 64, 64>), dim3(unsigned(blk)), dim3(256), 0,
                         s, d, alpha, beta_y);
    else
      hipLaunchKernelGGL(k_cgemm_ex_bf16, dim3(unsigned(blk)), dim3(256), 0, s, d, alpha, beta_y);
    QM_HIP(hipGetLastError());
  }
}

}  // namespace qm
