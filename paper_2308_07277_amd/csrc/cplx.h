// Complex arithmetic and in-register small DFTs for the gfx950 kernels.
//
// A DFT of length N with sign S computes X[k] = sum_n x[n] exp(S 2 pi i n k / N);
// S = +1 is the inverse transform of the plane-wave basis (g2r, e^{+iG.r}),
// S = -1 the forward one (r2g), matching the transform pair of Sec. 4.3.
// Roots of unity are compile-time constants: a constexpr sine/cosine built
// from the Taylor series after reducing the angle to [0, pi/4], evaluated in
// double precision when the templates are instantiated.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qm {

template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.re * s, a.im * s}; }
// multiply by S*i
template <int S, typename R>
__device__ __forceinline__ cplx<R> cmul_si(cplx<R> a) {
  return S > 0 ? cplx<R>{-a.im, a.re} : cplx<R>{a.im, -a.re};
}

// ---------------------------------------------------------------- constexpr trig
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi p / q for integers, exact octant reduction on the integers
constexpr void sincos_frac(long p, long q, double& c, double& s) {
  p %= q;
  if (p < 0) p += q;
  // angle = 2 pi p / q ; use 8 p / q to find the octant with integer arithmetic
  long e = 8 * p;
  int oct = int(e / q);          // 0..7
  // residual angle within octant, in units of (2 pi / q): r = p - oct*q/8
  double r = (double(e - long(oct) * q) / double(8 * q)) * 2.0 * kPi;  // in [0, pi/4)
  double sr = taylor_sin(r), cr = taylor_cos(r);
  // angle = oct * pi/4 + r
  double q4s = 0, q4c = 0;
  switch (oct) {
    case 0: q4c = cr; q4s = sr; break;
    case 1: { double a = kPi / 4 - r; q4c = taylor_sin(a); q4s = taylor_cos(a); } break;
    case 2: q4c = -sr; q4s = cr; break;
    case 3: { double a = kPi / 4 - r; q4c = -taylor_cos(a); q4s = taylor_sin(a); } break;
    case 4: q4c = -cr; q4s = -sr; break;
    case 5: { double a = kPi / 4 - r; q4c = -taylor_sin(a); q4s = -taylor_cos(a); } break;
    case 6: q4c = sr; q4s = -cr; break;
    default: { double a = kPi / 4 - r; q4c = taylor_cos(a); q4s = -taylor_sin(a); } break;
  }
  c = q4c;
  s = q4s;
}
constexpr double cos_frac(long p, long q) { double c = 0, s = 0; sincos_frac(p, q, c, s); return c; }
constexpr double sin_frac(long p, long q) { double c = 0, s = 0; sincos_frac(p, q, c, s); return s; }
}  // namespace ct

// ---------------------------------------------------------------- small DFTs
template <int N, int S, typename R>
struct Dft;

template <int S, typename R>
struct Dft<1, S, R> {
  __device__ __forceinline__ static void run(cplx<R>*) {}
};

template <int S, typename R>
struct Dft<2, S, R> {
  __device__ __forceinline__ static void run(cplx<R>* a) {
    cplx<R> t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <int S, typename R>
struct Dft<3, S, R> {
  __device__ __forceinline__ static void run(cplx<R>* a) {
    const R h = R(0.866025403784438646763723170752936183);  // sqrt(3)/2
    cplx<R> s = cadd(a[1], a[2]);
    cplx<R> d = csub(a[1], a[2]);
    cplx<R> m = {a[0].re - R(0.5) * s.re, a[0].im - R(0.5) * s.im};
    cplx<R> t = cmul_si<S>(cscale(d, h));
    a[0] = cadd(a[0], s);
    a[1] = cadd(m, t);
    a[2] = csub(m, t);
  }
};

template <int S, typename R>
struct Dft<4, S, R> {
  __device__ __forceinline__ static void run(cplx<R>* a) {
    cplx<R> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    cplx<R> s13 = cadd(a[1], a[3]), d13 = cmul_si<S>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

// odd prime N: symmetric/antisymmetric pair form
template <int N, int S, typename R>
struct DftOddPrime {
  __device__ __forceinline__ static void run(cplx<R>* a) {
    constexpr int H = (N - 1) / 2;
    cplx<R> sp[H], dm[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      sp[j - 1] = cadd(a[j], a[N - j]);
      dm[j - 1] = csub(a[j], a[N - j]);
    }
    cplx<R> x0 = a[0];
    cplx<R> tot = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) tot = cadd(tot, sp[j]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cplx<R> p = x0, q = {R(0), R(0)};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const R c = R(ct::cos_frac(long(j) * k, N));
        const R s = R(ct::sin_frac(long(j) * k, N));
        p.re += c * sp[j - 1].re;
        p.im += c * sp[j - 1].im;
        q.re += s * dm[j - 1].re;
        q.im += s * dm[j - 1].im;
      }
      cplx<R> iq = cmul_si<S>(q);
      a[k] = cadd(p, iq);
      a[N - k] = csub(p, iq);
    }
    a[0] = tot;
  }
};
template <int S, typename R> struct Dft<5, S, R> : DftOddPrime<5, S, R> {};
template <int S, typename R> struct Dft<7, S, R> : DftOddPrime<7, S, R> {};

// 3-point DFT of (a0, 0, a2): the middle input is known to be zero and is not read
template <int S, typename R>
struct Dft3ZeroMid {
  __device__ __forceinline__ static void run(cplx<R>* a) {
    const R h = R(0.866025403784438646763723170752936183);  // sqrt(3)/2
    const cplx<R> x0 = a[0], x2 = a[2];
    cplx<R> m = {x0.re - R(0.5) * x2.re, x0.im - R(0.5) * x2.im};
    cplx<R> t = cmul_si<S>(cscale(x2, -h));
    a[0] = cadd(x0, x2);
    a[1] = cadd(m, t);
    a[2] = csub(m, t);
  }
};

// composite N = F * M in registers: x[n1 + F n2] -> DFT_M over n2, twiddle, DFT_F over n1.
// ZM (M = 3 only): the inputs [F, 2F) (n2 = 1 of every inner DFT) are known to be zero.
template <int N, int F, int S, typename R, bool ZM = false>
struct DftComposite {
  static constexpr int M = N / F;
  static_assert(!ZM || M == 3, "zero-middle pruning needs M = 3");
  __device__ __forceinline__ static void run(cplx<R>* a) {
    cplx<R> y[F][M];
#pragma unroll
    for (int n1 = 0; n1 < F; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < M; ++n2) y[n1][n2] = (ZM && n2 == 1) ? cplx<R>{R(0), R(0)} : a[n1 + F * n2];
      if constexpr (ZM) Dft3ZeroMid<S, R>::run(y[n1]);
      else Dft<M, S, R>::run(y[n1]);
#pragma unroll
      for (int k2 = 1; k2 < M; ++k2) {
        if (n1 == 0) continue;
        const long e = long(n1) * k2;
        if ((4 * e) % N == 0) {   // quarter turns are exact: S i, -1, -S i
          const long q = (4 * e / N) % 4;
          if (q == 1) y[n1][k2] = cmul_si<S>(y[n1][k2]);
          else if (q == 2) y[n1][k2] = {-y[n1][k2].re, -y[n1][k2].im};
          else if (q == 3) y[n1][k2] = cmul_si<-S>(y[n1][k2]);
          continue;
        }
        const R c = R(ct::cos_frac(e, N));
        const R s = R(S * ct::sin_frac(e, N));
        y[n1][k2] = cmul(y[n1][k2], cplx<R>{c, s});
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
      cplx<R> z[F];
#pragma unroll
      for (int n1 = 0; n1 < F; ++n1) z[n1] = y[n1][k2];
      Dft<F, S, R>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < F; ++k1) a[k2 + M * k1] = z[k1];
    }
  }
};
template <int S, typename R> struct Dft<6, S, R> : DftComposite<6, 2, S, R> {};
template <int S, typename R> struct Dft<8, S, R> : DftComposite<8, 2, S, R> {};
template <int S, typename R> struct Dft<9, S, R> : DftComposite<9, 3, S, R> {};
template <int S, typename R> struct Dft<10, S, R> : DftComposite<10, 2, S, R> {};
template <int S, typename R> struct Dft<12, S, R> : DftComposite<12, 4, S, R> {};
template <int S, typename R> struct Dft<14, S, R> : DftComposite<14, 2, S, R> {};
template <int S, typename R> struct Dft<15, S, R> : DftComposite<15, 3, S, R> {};
template <int S, typename R> struct Dft<16, S, R> : DftComposite<16, 4, S, R> {};
template <int S, typename R> struct Dft<18, S, R> : DftComposite<18, 2, S, R> {};
template <int S, typename R> struct Dft<20, S, R> : DftComposite<20, 4, S, R> {};
template <int S, typename R> struct Dft<24, S, R> : DftComposite<24, 4, S, R> {};
template <int S, typename R> struct Dft<32, S, R> : DftComposite<32, 4, S, R> {};
template <int S, typename R> struct Dft<36, S, R> : DftComposite<36, 4, S, R> {};
template <int S, typename R> struct Dft<40, S, R> : DftComposite<40, 8, S, R> {};
template <int S, typename R> struct Dft<48, S, R> : DftComposite<48, 4, S, R> {};
template <int S, typename R> struct Dft<64, S, R> : DftComposite<64, 8, S, R> {};
template <int S, typename R> struct Dft<72, S, R> : DftComposite<72, 8, S, R> {};
template <int S, typename R> struct Dft<27, S, R> : DftComposite<27, 3, S, R> {};
template <int S, typename R> struct Dft<54, S, R> : DftComposite<54, 6, S, R> {};

// DFTs of length N = 3F whose inputs [F, 2F) are zero (the middle third of a line whose
// nonzero samples lie within a third of the length of index 0, taken modulo N); zero_mid_f(N)
// is that F, or 0 where no such pruned form exists.
template <int N, int S, typename R> struct DftZM;
template <int S, typename R> struct DftZM<6, S, R> : DftComposite<6, 2, S, R, true> {};
template <int S, typename R> struct DftZM<9, S, R> : DftComposite<9, 3, S, R, true> {};
template <int S, typename R> struct DftZM<12, S, R> : DftComposite<12, 4, S, R, true> {};
__host__ __device__ constexpr int zero_mid_f(int n) { return n == 6 ? 2 : n == 9 ? 3 : n == 12 ? 4 : 0; }

// Two-factor split used by the LDS line transforms: N = R1 * R2 with R1 <= R2.
template <int N> struct Split;
#define QM_SPLIT(n, a, b) template <> struct Split<n> { static constexpr int R1 = a, R2 = b; };
QM_SPLIT(12, 3, 4)
QM_SPLIT(16, 4, 4)
QM_SPLIT(18, 3, 6)
QM_SPLIT(20, 4, 5)
QM_SPLIT(24, 4, 6)
QM_SPLIT(27, 3, 9)
QM_SPLIT(28, 4, 7)
QM_SPLIT(30, 5, 6)
QM_SPLIT(32, 4, 8)
QM_SPLIT(36, 6, 6)
QM_SPLIT(40, 5, 8)
QM_SPLIT(45, 5, 9)
QM_SPLIT(48, 6, 8)
QM_SPLIT(54, 6, 9)
QM_SPLIT(56, 7, 8)
QM_SPLIT(60, 6, 10)
QM_SPLIT(64, 8, 8)
QM_SPLIT(72, 8, 9)
QM_SPLIT(80, 8, 10)
QM_SPLIT(81, 9, 9)
QM_SPLIT(90, 9, 10)
QM_SPLIT(96, 8, 12)
QM_SPLIT(100, 10, 10)
QM_SPLIT(108, 9, 12)
QM_SPLIT(120, 10, 12)
QM_SPLIT(128, 8, 16)
QM_SPLIT(144, 12, 12)
#undef QM_SPLIT

// every supported FFT length, for host-side dispatch
#define QM_FOR_EACH_FFT_LEN(X) \
  X(12) X(16) X(18) X(20) X(24) X(27) X(28) X(30) X(32) X(36) X(40) X(45) X(48) X(54) \
  X(56) X(60) X(64) X(72) X(80) X(81) X(90) X(96) X(100) X(108) X(120) X(128) X(144)

}  // namespace qm
