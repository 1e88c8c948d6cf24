// Stick-pruned batched 3-D FFT with the local potential fused in (gfx950).
//
// Local part of H|psi> for every (k, band) of a launch (Sec. 4.3: inverse
// FFT of the sphere, multiply by V(r), forward FFT, keep the sphere; with the
// stick pruning of "Optimizing FFT operations for G-Space"):
//
//   k_zinv  scatter the sphere coefficients of a tile of z-sticks into LDS
//           (only sticks holding a G exist), inverse z-transform, write the
//           tile to the stick buffer, plane-slot major ([slot][stick]).
//   k_xy    one (k, band, z-plane) per workgroup, the plane staged in LDS
//           restricted to the active x-columns: inverse y-transform on the
//           active columns, then per y-row the inverse x-transform, the
//           multiplication by V(r)/N_r and the forward x-transform chained in
//           registers (only active columns written back), forward
//           y-transform, write the plane back in place.
//   k_zfwd  forward z-transform of a stick tile, then gather the sphere and
//           add the kinetic term 1/2|k+G|^2 c(G) (computed in float64).
//
// Each 1-D transform of length N = R1*R2 is done in two in-place passes
// (R2-point then R1-point register DFTs, twiddles between) by a group of
// threads.  The inverse leaves its output in R1 x R2 transposed order and the
// forward transform uses the swapped factorisation, which consumes exactly
// that order and produces natural order, so no transposition pass exists
// anywhere; V(r) is stored in the plan in the same permuted plane order.
#pragma once
#include <type_traits>
#include "cplx.h"
#include "qm_internal.h"

namespace qm {

struct LocalArgs {
  const KInfo* kinfo;
  KSlice sl[kMaxSlices];    // k-point band blocks of this launch
  int32_t blk_z[kMaxSlices + 1];  // prefix of nb * ntile over slices (z kernels)
  int32_t pair0[kMaxSlices + 1];  // prefix of nb over slices (xy kernel)
  int32_t nsl, N3;
  const double2* psi;       // c128 base
  double2* hpsi;            // c128 base
  void* sbuf;               // cplx<R>
  const int32_t* ent_g;
  const int32_t* ent_sz;
  const int32_t* tile_ptr;
  const int32_t* stick_pos;
  const int32_t* col_of_i1;
  const int32_t* stick_at;  // [nk][N2][sat_stride] stick index of (i2, active column), or -1
  int32_t sat_stride;
  const double* kin;
  const void* vplan;        // R [slot][i1][i2]
  const double2* tw_z;      // exp(+2 pi i m / N3), m < N3
  const double2* tw_x;      // exp(+2 pi i m / N1)
  int32_t ts;               // sticks per tile
  int32_t nax_stride;       // row stride of the lane-group xy-plane buffer (elements)
  int32_t xy_stride;        // row stride of the two-pass xy-plane buffer (elements)
  int32_t sbuf_per_k;       // 1: k's stick block at sbuf + kinfo[k].sbuf_off; 0: at sbuf (one slice)
  int32_t zero_mid;         // 1: no stick of any k has i1 or i2 in [R1 F, 2 R1 F) (F = zero_mid_f(R2)
                            // of the N1 = N2 split), so those inputs of the inverse x and y
                            // transforms are zero and those outputs of the forward ones unused
};

// This k's stick buffer.  In the plan's buffer its region starts at the same byte offset
// (sbuf_off complex double elements) whatever the working precision, so k-points that run in
// different precisions at the same time (concurrent Davidson lanes) never share bytes.  A
// caller-given buffer holds the one slice of its launch from its start.
template <typename R>
__device__ __forceinline__ cplx<R>* stick_base(const LocalArgs& a, const KInfo& ki) {
  return reinterpret_cast<cplx<R>*>(reinterpret_cast<char*>(a.sbuf) +
                                    (a.sbuf_per_k ? ki.sbuf_off * int64_t(16) : int64_t(0)));
}

// slice holding z-kernel block bid; bid becomes the block index within the slice
__device__ __forceinline__ int locate_tile_block(const LocalArgs& a, int& bid) {
  int s = 0;
  while (s < a.nsl - 1 && bid >= a.blk_z[s + 1]) ++s;
  bid -= a.blk_z[s];
  return s;
}

// Loops over table entries keep kUnroll of them in flight per thread: the loads of a group
// are all issued before any is used, so a workgroup waits for one round trip to memory per
// group instead of one per entry.  Indices past the end are clamped to the last valid entry.
// Where the loop only moves a value to the place its entry names, the clamped copies store
// the same value at the same place again, which needs no guard; a guard would let the
// compiler sink each load into its guarded store and serialise the group again.
constexpr int kUnroll = 4;

// Makes a loaded value live in registers at this point, so that its load is not moved into
// a later conditional block.
__device__ __forceinline__ void pin(int x) { asm volatile("" ::"v"(x)); }
__device__ __forceinline__ void pin(double x) { asm volatile("" ::"v"(x)); }
__device__ __forceinline__ void pin(double2 x) {
  pin(x.x);
  pin(x.y);
}

// plane[s] -> L at the stick's (row, active column) position, s < nstick
template <typename R, int NT>
__device__ __forceinline__ void sticks_to_lds(const cplx<R>* plane, const int32_t* spos, int nstick,
                                              cplx<R>* L, int ns, int tid) {
  for (int s0 = tid; s0 < nstick; s0 += kUnroll * NT) {
    int ps[kUnroll];
    cplx<R> v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int s = min(s0 + u * NT, nstick - 1);
      ps[u] = spos[s];
      v[u] = plane[s];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) L[(ps[u] & 0xffff) * ns + (ps[u] >> 16)] = v[u];
  }
}

// L at the stick's position -> plane[s], s < nstick
template <typename R, int NT>
__device__ __forceinline__ void lds_to_sticks(cplx<R>* plane, const int32_t* spos, int nstick,
                                              const cplx<R>* L, int ns, int tid) {
  for (int s0 = tid; s0 < nstick; s0 += kUnroll * NT) {
    int s[kUnroll], ps[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      s[u] = min(s0 + u * NT, nstick - 1);
      ps[u] = spos[s[u]];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) plane[s[u]] = L[(ps[u] & 0xffff) * ns + (ps[u] >> 16)];
  }
}

// ------------------------------------------------------------------ z inverse + scatter
template <typename R, int N3, int TS>
__global__ void __launch_bounds__(TS * Split<N3>::R2) k_zinv(LocalArgs a) {
  constexpr int R1 = Split<N3>::R1, R2 = Split<N3>::R2, NT = TS * R2;
  __shared__ cplx<R> tile[N3 * TS];
  __shared__ cplx<R> tw[N3];
  const int tid = threadIdx.x;
  int bid = blockIdx.x;
  const int si = locate_tile_block(a, bid);
  const KSlice& ks = a.sl[si];
  const KInfo ki = a.kinfo[ks.k];
  const int band = bid / ki.ntile, t = bid - band * ki.ntile;
  const int s0 = t * TS;
  const int cnt = min(TS, ki.nstick - s0);
  for (int i = tid; i < N3; i += NT) {
    double2 w = a.tw_z[i];
    tw[i] = {R(w.x), R(w.y)};
  }
  for (int i = tid; i < N3 * TS; i += NT) tile[i] = {R(0), R(0)};
  __syncthreads();
  const int32_t* tp = a.tile_ptr + ki.tile_off;
  const int e0 = tp[t], e1 = tp[t + 1];
  const double2* psi_b = a.psi + ks.psi_off + int64_t(band) * ki.npw;
  const int32_t* eg = a.ent_g + ki.g_off;
  const int32_t* esz = a.ent_sz + ki.g_off;
  for (int eb = e0 + tid; eb < e1; eb += kUnroll * NT) {
    int sz[kUnroll];
    double2 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = min(eb + u * NT, e1 - 1);
      sz[u] = esz[e];
      v[u] = psi_b[eg[e]];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int s = sz[u] / N3, z = sz[u] - s * N3;
      tile[z * TS + (s - s0)] = {R(v[u].x), R(v[u].y)};
    }
  }
  __syncthreads();
  const int sl = tid % TS, j = tid / TS;
  if (j < R1) {
    cplx<R> x[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) x[n2] = tile[(j + R1 * n2) * TS + sl];
    Dft<R2, +1, R>::run(x);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tw[(j * k2) % N3]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) tile[(j + R1 * k2) * TS + sl] = x[k2];
  }
  __syncthreads();
  if (sl < cnt) {
    cplx<R> y[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n1] = tile[(n1 + R1 * j) * TS + sl];
    Dft<R1, +1, R>::run(y);
    cplx<R>* out = stick_base<R>(a, ki) +
                   int64_t(band) * N3 * ki.nstick + s0 + sl;
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) out[int64_t(k1 + R1 * j) * ki.nstick] = y[k1];
  }
}

// ------------------------------------------------------------------ stick access by index
// Raw buffer loads and stores on one plane's sticks (a buffer resource of nstick elements):
// an index s < 0 puts the byte offset past the resource's range, where the hardware returns
// zero for a load and drops a store, so absent sticks need no select and no branch.
constexpr int kBufferConfig = 0x00020000;   // gfx9 buffer resource word 3 (32-bit data format)
template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stick_rsrc(const cplx<R>* plane, int nstick) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cplx<R>*>(plane), (short)0,
                                           nstick * int(sizeof(cplx<R>)), kBufferConfig);
}
// the builtins' data types: vectors of 32-bit words (moved in and out by bit casts)
typedef unsigned int qm_w4 __attribute__((vector_size(16)));
typedef unsigned int qm_w2 __attribute__((vector_size(8)));
__device__ __forceinline__ cplx<double> stick_load(__amdgpu_buffer_rsrc_t r, int s, double) {
  return __builtin_bit_cast(cplx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, s * 16, 0, 0));
}
__device__ __forceinline__ cplx<float> stick_load(__amdgpu_buffer_rsrc_t r, int s, float) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, s * 8, 0, 0));
}
__device__ __forceinline__ void stick_store(__amdgpu_buffer_rsrc_t r, int s, cplx<double> z) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(qm_w4, z), r, s * 16, 0, 0);
}
__device__ __forceinline__ void stick_store(__amdgpu_buffer_rsrc_t r, int s, cplx<float> z) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qm_w2, z), r, s * 8, 0, 0);
}

// ------------------------------------------------------------------ xy plane
// Orders the LDS accesses of one wave: every lane's earlier LDS writes are complete and
// visible to the other lanes of the wave before any later LDS access.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waves per SIMD the two-pass xy kernel is compiled for.  Without the row scratch a float64
// plane of up to 80 points takes at most 53 KB of LDS, so three workgroups fit on a CU if the
// registers allow it.
template <typename R, int NX, bool OWN>
constexpr int xy_min_waves() { return OWN && sizeof(R) == 8 && NX <= 80 ? 3 : 1; }

// the N-point DFT, pruned (inputs [N/3, 2N/3) known zero) when Z
template <int N, int S, typename R, bool Z>
__device__ __forceinline__ void dft_zm(cplx<R>* x) {
  if constexpr (Z) DftZM<N, S, R>::run(x);
  else Dft<N, S, R>::run(x);
}

// x[n2] = row[cr[n2]], then the inverse R2-point DFT; with zm the inputs n2 in [ZF, 2 ZF) are
// known zeros (not read, pruned DFT)
template <int R2, typename R, int ZF>
__device__ __forceinline__ void inverse_first_pass(cplx<R> (&x)[R2], const cplx<R>* row,
                                                   const int (&cr)[R2], bool zm) {
  if constexpr (ZF > 0) {
    if (zm) {
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2)
        x[n2] = (n2 >= ZF && n2 < 2 * ZF) ? cplx<R>{R(0), R(0)} : row[cr[n2]];
      DftZM<R2, +1, R>::run(x);
      return;
    }
  }
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) x[n2] = row[cr[n2]];
  Dft<R2, +1, R>::run(x);
}

// OWN = false: the x-row exchanges go through a row scratch of NX + 1 slots per row in flight
// (4 R_W rows).  OWN = true: they go through the rows' own ns slots in two rounds each, which
// leaves the plane as the only large LDS buffer (more workgroups per CU, more LDS operations);
// float64 then forms its x-row twiddles w^{q j} from w^q at each use instead of holding them
// in VGPRs.
template <typename R, int NX, bool OWN>
__global__ void __launch_bounds__(256, (xy_min_waves<R, NX, OWN>())) k_xy(LocalArgs a) {
  constexpr int R1 = Split<NX>::R1, R2 = Split<NX>::R2;
  constexpr int RW = 64 / R2, NXP = NX + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ns = a.xy_stride;
  constexpr bool kTwReg = !OWN || sizeof(R) == 4;
  cplx<R>* L = reinterpret_cast<cplx<R>*>(smem_raw);  // [NX positions][ns]
  cplx<R>* X = L + NX * ns;                              // [4 R_W rows][NX + 1] (OWN = false)
  cplx<R>* tw = X + (OWN ? 0 : 4 * RW * NXP);            // [NX]
  int* col = reinterpret_cast<int*>(tw + NX);            // [NX]
  const int tid = threadIdx.x;
  const int N3 = a.N3;
  // (k, band) pair and z-slot; each XCD keeps a fixed eighth of the slots when N3 % 8 == 0
  int bid = blockIdx.x, kb, p;
  if ((N3 & 7) == 0) {
    const int xcd = bid & 7, jj = bid >> 3, per = N3 >> 3;
    kb = jj / per;
    p = xcd * per + (jj - kb * per);
  } else {
    kb = bid / N3;
    p = bid - kb * N3;
  }
  int si = 0;
  while (si < a.nsl - 1 && kb >= a.pair0[si + 1]) ++si;
  const int k = a.sl[si].k, band = kb - a.pair0[si];
  const KInfo ki = a.kinfo[k];
  const int nax = ki.nax;
  cplx<R>* plane = stick_base<R>(a, ki) +
                   (int64_t(band) * N3 + p) * ki.nstick;
  // stick index of (row i2, active column ia) at sat[i2 * sat_stride + ia], -1 where the
  // sphere has no stick: the y passes read and write the plane's sticks directly in memory
  const int32_t* sat = a.stick_at + int64_t(k) * NX * a.sat_stride;
  const int sts = a.sat_stride;
  const __amdgpu_buffer_rsrc_t prs = stick_rsrc<R>(plane, ki.nstick);
  for (int i = tid; i < NX; i += 256) {
    double2 w = a.tw_x[i];
    tw[i] = {R(w.x), R(w.y)};
    col[i] = a.col_of_i1[int64_t(k) * NX + i];
    L[i * ns + ns - 1] = {R(0), R(0)};   // the zero slot of every row
  }
  __syncthreads();
  // y-pass items w = ia + nax j: thread tid starts at (tid % nax, tid / nax) and steps by
  // 256 = dj nax + dia, so each pass walks its items without a division per item
  const int ia0 = tid % nax, j0 = tid / nax, dj = 256 / nax, dia = 256 - dj * nax;
  // zero middle band: with a.zero_mid the samples n1 + R1 n2, n2 in [ZF, 2 ZF), of every
  // x-row and y-column hold no stick, so the inverse R2-point passes skip those inputs (no
  // load, pruned DFT) and the forward y pass skips those outputs' stores
  constexpr int ZF = zero_mid_f(R2);
  const bool zm = ZF > 0 && a.zero_mid;
  auto in_zm = [](int n) { return ZF > 0 && n >= ZF && n < 2 * ZF; };
  // ---- inverse y on active columns: pass 1 (R2-point, stride R1), input gathered from the
  // sticks (rows without a stick read zero)
  auto ypass1 = [&](auto zmc) {
    constexpr bool Z = decltype(zmc)::value;
    for (int w = tid, ia = ia0, n1 = j0; w < nax * R1; w += 256, ia += dia, n1 += dj) {
      if (ia >= nax) {
        ia -= nax;
        ++n1;
      }
      int si[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2)
        if (!(Z && in_zm(n2))) si[n2] = sat[(n1 + R1 * n2) * sts + ia];
      cplx<R> x[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2)
        x[n2] = (Z && in_zm(n2)) ? cplx<R>{R(0), R(0)} : stick_load(prs, si[n2], R(0));
      dft_zm<R2, +1, R, Z && (ZF > 0)>(x);
      // twiddle exponents n1 k2 <= (R1 - 1)(R2 - 1) < NX: no reduction modulo NX needed
#pragma unroll
      for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tw[n1 * k2]);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) L[(n1 + R1 * k2) * ns + ia] = x[k2];
    }
  };
  if (zm) ypass1(std::integral_constant<bool, (ZF > 0)>{});
  else ypass1(std::false_type{});
  __syncthreads();
  // pass 2 (R1-point on contiguous runs); output X[k2 + R2 k1] at position k1 + R1 k2
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
  // ---- x rows: inverse x, * V / N_r, forward x; active columns only written back.
  const R* V = reinterpret_cast<const R*>(a.vplan) + int64_t(p) * NX * NX;  // [i2][i1]
  if constexpr (OWN) {
  // Each wave owns R_W = 64 / R2 consecutive rows of L at a time (R2 lanes per row, lanes over
  // the intra-row index q).  The two exchanges between the passes of a row's transform pair go
  // through the row's own ns slots, in two rounds each (ns holds half of the R1 R2 values), so
  // the plane is the only large LDS buffer and only wave-level ordering is required.
  // L row lr holds plane row i2 = R2 (lr % R1) + lr / R1 (the y-pass order).
  // inverse exchange: values of n1 < HA in the first round, value (n1, k2) at slot
  // (n1 - round start) PA + k2; forward exchange: values of n < HB in the first round, value
  // (n, k2) at slot k2 QB + (n - round start).  PA and QB are odd, so the lanes of a row that
  // write (inverse) or read (forward) one value each fall on different LDS banks.
  constexpr int HA = (R1 + 1) / 2, PA = R2 | 1;
  constexpr int HB = (R2 + 1) / 2, QB = HB | 1;
  {
    const int wave = tid >> 6, lane = tid & 63;
    const int q = lane % R2, rs = lane / R2;
    // per-lane constants of every row: the slots of the row samples i1 = q + R1 j (read by
    // the inverse pass, written by the forward one; inactive columns read the row's last
    // slot, which no y pass writes, so it holds zero until the row's exchanges start) and the
    // twiddles w^{q j}, used for j < R2 by lanes q < R1 (inverse pass 1) and for j < R1 by
    // lanes q < R2 (forward pass): those exponents stay below NX, so no reduction modulo NX
    // is needed; the other (unused) combinations are clamped into the table
    // (float64 forms them at each use instead: held in registers they would cost 4 R2 VGPRs
    // and a wave slot per SIMD)
    int cr[R2];  // active columns are below nax < ns - 1, so cr[j] != ns - 1 marks them
    cplx<R> tq[kTwReg ? R2 : 1];
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      const int c = col[min(q, R1 - 1) + R1 * j];
      cr[j] = c >= 0 ? c : ns - 1;
      if (kTwReg) tq[j] = tw[min(q * j, NX - 1)];
    }
    // without the register table: w^{q j} = w^{q (j - 1)} w^q, one product per use (rounding
    // grows like j, below 10 ulp for j < R2); the empty asm keeps the compiler from hoisting
    // the powers out of the row loop, which would hold them in VGPRs after all
    const cplx<R> w1 = tw[min(q, NX - 1)];
    auto base = [&]() {
      cplx<R> b = w1;
      asm volatile("" : "+v"(b.re), "+v"(b.im));
      return b;
    };
    for (int r0 = wave * RW; r0 < NX; r0 += 4 * RW) {
      const int lr = r0 + rs;
      const bool act = rs < RW && lr < NX;
      const int i2 = act ? R2 * (lr % R1) + lr / R1 : 0;
      // this row's V(r) values, loaded before the row's LDS exchanges (whose wave-level
      // fences the loads could not be moved across); idle lanes read row 0
      R vr[R1];
      {
        const R* Vrow = V + i2 * NX;
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) vr[k1] = Vrow[q + R2 * k1];
      }
      cplx<R>* Lr = L + (act ? lr : 0) * ns;
      // inverse pass 1: lanes q < R1 (n1 = q), R2-point DFT over n2 of x[q + R1 n2], twiddle
      cplx<R> x[R2];
      if (act && q < R1) {
        inverse_first_pass<R2, R, ZF>(x, Lr, cr, zm);
        if constexpr (kTwReg) {
#pragma unroll
          for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tq[k2]);
        } else {
          const cplx<R> b = base();
          cplx<R> t = b;
#pragma unroll
          for (int k2 = 1; k2 < R2; ++k2) {
            x[k2] = cmul(x[k2], t);
            if (k2 + 1 < R2) t = cmul(t, b);
          }
        }
      }
      wave_lds_sync();
      // inverse exchange; lane q collects k2 = q
      cplx<R> y[R1];
      if (act && q < HA) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Lr[q * PA + k2] = x[k2];
      }
      wave_lds_sync();
      if (act) {
#pragma unroll
        for (int n1 = 0; n1 < HA; ++n1) y[n1] = Lr[n1 * PA + q];
      }
      wave_lds_sync();
      if (act && q >= HA && q < R1) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Lr[(q - HA) * PA + k2] = x[k2];
      }
      wave_lds_sync();
      if (act) {
#pragma unroll
        for (int n1 = HA; n1 < R1; ++n1) y[n1] = Lr[(n1 - HA) * PA + q];
        Dft<R1, +1, R>::run(y);  // y[k1] is the row value at i1 = q + R2 k1
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) y[k1] = cscale(y[k1], vr[k1]);
        Dft<R1, -1, R>::run(y);  // forward, factorisation (R2, R1): first pass over n = k1
        if constexpr (kTwReg) {
#pragma unroll
          for (int k2 = 1; k2 < R1; ++k2) y[k2] = cmul(y[k2], cplx<R>{tq[k2].re, -tq[k2].im});
        } else {
          const cplx<R> b = base();
          cplx<R> t = {b.re, -b.im};
#pragma unroll
          for (int k2 = 1; k2 < R1; ++k2) {
            y[k2] = cmul(y[k2], t);
            if (k2 + 1 < R1) t = cmul(t, cplx<R>{b.re, -b.im});
          }
        }
      }
      wave_lds_sync();
      // forward exchange; lane q < R1 collects k2 = q
      cplx<R> z[R2];
      if (act && q < HB) {
#pragma unroll
        for (int k2 = 0; k2 < R1; ++k2) Lr[k2 * QB + q] = y[k2];
      }
      wave_lds_sync();
      if (act && q < R1) {
#pragma unroll
        for (int n = 0; n < HB; ++n) z[n] = Lr[q * QB + n];
      }
      wave_lds_sync();
      if (act && q >= HB) {
#pragma unroll
        for (int k2 = 0; k2 < R1; ++k2) Lr[k2 * QB + (q - HB)] = y[k2];
      }
      wave_lds_sync();
      if (act && q < R1) {
#pragma unroll
        for (int n = HB; n < R2; ++n) z[n] = Lr[q * QB + (n - HB)];
        Dft<R2, -1, R>::run(z);  // natural output at i1 = q + R1 k1
      }
      wave_lds_sync();
      if (act && q < R1) {
#pragma unroll
        for (int k1 = 0; k1 < R2; ++k1)
          if (cr[k1] != ns - 1) Lr[cr[k1]] = z[k1];
      }
    }
  }
  } else {
  // Each wave owns whole rows (R2 lanes per row, R_W rows at a time) and its own row scratch,
  // so the exchanges between the two passes of a row need only wave-level ordering.  Lanes run
  // over the intra-row index q (consecutive LDS columns, consecutive V entries).  In the
  // inverse exchange lane q < R1 writes its R2 values at slots q R2 + k2 and lane q reads
  // slots n1 R2 + q; in the forward one lane q writes slots q + R2 k2 and lane q < R1 reads
  // slots n + R2 q: odd strides between lanes, so a row's lanes fall on different LDS banks.
    const int wave = tid >> 6, lane = tid & 63;
    const int q = lane % R2, rs = lane / R2;
    cplx<R>* Xr = X + (wave * RW + (rs < RW ? rs : 0)) * NXP;
    // per-lane constants of every row: the slots of the row samples i1 = q + R1 j (read by
    // the inverse pass, written by the forward one; inactive columns read the row's last slot,
    // which no pass writes) and the twiddles w^{q j} (exponents below NX, as above)
    int cr[R2];
    cplx<R> tq[R2];
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      const int c = col[min(q, R1 - 1) + R1 * j];
      cr[j] = c >= 0 ? c : ns - 1;
      tq[j] = tw[min(q * j, NX - 1)];
    }
    for (int r0 = wave * RW; r0 < NX; r0 += 4 * RW) {
      const int i2 = r0 + rs;
      const bool act = rs < RW && i2 < NX;
      const int lrow = act ? (i2 / R2) + R1 * (i2 % R2) : 0;
      R vr[R1];
      {
        const R* Vrow = V + (act ? i2 : 0) * NX;
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) vr[k1] = Vrow[q + R2 * k1];
      }
      cplx<R>* Lrow = L + lrow * ns;
      if (act && q < R1) {
        cplx<R> x[R2];
        inverse_first_pass<R2, R, ZF>(x, Lrow, cr, zm);
#pragma unroll
        for (int k2 = 1; k2 < R2; ++k2) x[k2] = cmul(x[k2], tq[k2]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Xr[q * R2 + k2] = x[k2];
      }
      wave_lds_sync();
      cplx<R> y[R1];
      if (act) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) y[n1] = Xr[n1 * R2 + q];
        Dft<R1, +1, R>::run(y);  // y[k1] is the row value at i1 = q + R2 k1
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) y[k1] = cscale(y[k1], vr[k1]);
        Dft<R1, -1, R>::run(y);  // forward, factorisation (R2, R1): first pass over n = k1
#pragma unroll
        for (int k2 = 1; k2 < R1; ++k2) y[k2] = cmul(y[k2], cplx<R>{tq[k2].re, -tq[k2].im});
      }
      wave_lds_sync();
      if (act) {
#pragma unroll
        for (int k2 = 0; k2 < R1; ++k2) Xr[q + R2 * k2] = y[k2];
      }
      wave_lds_sync();
      if (act && q < R1) {
        cplx<R> z[R2];
#pragma unroll
        for (int n = 0; n < R2; ++n) z[n] = Xr[n + R2 * q];
        Dft<R2, -1, R>::run(z);  // natural output at i1 = q + R1 k1
#pragma unroll
        for (int k1 = 0; k1 < R2; ++k1)
          if (cr[k1] != ns - 1) Lrow[cr[k1]] = z[k1];
      }
      wave_lds_sync();
    }
  }
  __syncthreads();
  // ---- forward y on active columns, input in the transposed order left above
  for (int w = tid, ia = ia0, n1 = j0; w < nax * R2; w += 256, ia += dia, n1 += dj) {  // n1 < R2
    if (ia >= nax) {
      ia -= nax;
      ++n1;
    }
    cplx<R> x[R1];
#pragma unroll
    for (int n2 = 0; n2 < R1; ++n2) x[n2] = L[(n2 + R1 * n1) * ns + ia];
    Dft<R1, -1, R>::run(x);
#pragma unroll
    for (int k2 = 1; k2 < R1; ++k2) {   // n1 k2 <= (R2 - 1)(R1 - 1) < NX
      const cplx<R> t = tw[n1 * k2];
      x[k2] = cmul(x[k2], cplx<R>{t.re, -t.im});
    }
#pragma unroll
    for (int k2 = 0; k2 < R1; ++k2) L[(k2 + R1 * n1) * ns + ia] = x[k2];
  }
  __syncthreads();
  for (int w = tid, ia = ia0, k2 = j0; w < nax * R1; w += 256, ia += dia, k2 += dj) {  // k2 < R1
    if (ia >= nax) {
      ia -= nax;
      ++k2;
    }
    // rows of the zero middle band hold no stick: with zm neither their stick indices are
    // read nor their (dropped) stores issued
    int si[R2];
#pragma unroll
    for (int k1 = 0; k1 < R2; ++k1) si[k1] = (zm && in_zm(k1)) ? -1 : sat[(k2 + R1 * k1) * sts + ia];
    cplx<R> z[R2];
#pragma unroll
    for (int n1 = 0; n1 < R2; ++n1) z[n1] = L[(k2 + R1 * n1) * ns + ia];
    Dft<R2, -1, R>::run(z);
    // row i2 = k2 + R1 k1 of the plane: written back where it has a stick
#pragma unroll
    for (int k1 = 0; k1 < R2; ++k1)
      if (!(zm && in_zm(k1))) stick_store(prs, si[k1], z[k1]);
  }
}

// ------------------------------------------------------------------ xy plane, lane-group lines
// Lines of length NX split over L lanes of a wave (H = NX/L complex per lane, in registers).
// Inverse = decimation in time: lane t holds x[L n + t], runs an H-point DFT, twiddles by
// w_NX^{t k}, then an L-point DFT across the lane group (xor shuffles) leaves X[H t + k].
// Forward = decimation in frequency: lane q holds x[H q + n]; the L-point DFT across the group
// comes first, then the twiddle w_NX^{-t n} and an H-point DFT leave X[L k + t].  The inverse's
// output distribution is exactly the forward's input distribution, so the x-row transform pair
// with V(r) in between never leaves registers.  For L = 8 the cross-lane DFT is three radix-2
// stages of xor shuffles: decimation in frequency for the inverse (natural order in, lane l
// ends with block rev3(l)) and decimation in time for the forward (block rev3(l) in, natural
// order out), so the bit-reversed block order only shows where the data is addressed.
template <typename R>
__device__ __forceinline__ cplx<R> shflx(cplx<R> v, int m) {
  return {__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64)};
}
// v * (S i)^e for e in 0..3, branch free: (S i)^e = c + i s with c, s in {-1, 0, 1}
template <int S, typename R>
__device__ __forceinline__ cplx<R> mul_ipow(cplx<R> v, int e) {
  e &= 3;
  const R c = R((e == 0) - (e == 2));
  const R s = R(S * ((e == 1) - (e == 3)));
  return {c * v.re - s * v.im, c * v.im + s * v.re};
}
// lane t of an L-group: out = sum_{t'} z_{t'} w_L^{S t' t}
template <int S, int L, typename R>
__device__ __forceinline__ cplx<R> cross_dft(cplx<R> z, int t) {
  if (L == 2) {
    const cplx<R> p = shflx(z, 1);
    return t ? csub(p, z) : cadd(z, p);
  } else {  // L == 4: gather the group, w_4 = S i
    cplx<R> acc = z;
#pragma unroll
    for (int x = 1; x < 4; ++x) {
      const cplx<R> v = shflx(z, x);
      acc = cadd(acc, mul_ipow<S>(v, (t ^ x) * t));
    }
    return acc;
  }
}

// v * w_8^{S j} for j in 0..3, branch free
template <int S, typename R>
__device__ __forceinline__ cplx<R> mul_w8(cplx<R> v, int j) {
  const R r = R(0.707106781186547524400844362104849039);
  const R c = R(j == 0) + r * R((j == 1) - (j == 3));
  const R sn = R(S) * (R(j == 2) + r * R((j == 1) + (j == 3)));
  return {c * v.re - sn * v.im, c * v.im + sn * v.re};
}
// twiddle w_{2h}^{S j} of a radix-2 stage across lanes (h = 1, 2, 4)
template <int S, typename R>
__device__ __forceinline__ cplx<R> stage_tw(cplx<R> v, int h, int j) {
  return h == 4 ? mul_w8<S>(v, j) : (h == 2 ? mul_ipow<S>(v, j) : v);
}
// 8-lane DFT, decimation in frequency: natural input, lane l ends with output rev3(l)
template <int S, typename R>
__device__ __forceinline__ cplx<R> cross_dif8(cplx<R> z, int t) {
#pragma unroll
  for (int h = 4; h >= 1; h >>= 1) {
    const cplx<R> p = shflx(z, h);
    z = (t & h) ? stage_tw<S>(csub(p, z), h, t & (h - 1)) : cadd(z, p);
  }
  return z;
}
// 8-lane DFT, decimation in time: lane l holds input rev3(l), natural output
template <int S, typename R>
__device__ __forceinline__ cplx<R> cross_dit8(cplx<R> z, int t) {
#pragma unroll
  for (int h = 1; h <= 4; h <<= 1) {
    const cplx<R> zt = (t & h) ? stage_tw<S>(z, h, t & (h - 1)) : z;
    const cplx<R> p = shflx(zt, h);
    z = (t & h) ? csub(p, zt) : cadd(z, p);
  }
  return z;
}
// output block held by lane t after group_inverse (and expected by group_forward)
template <int L>
__device__ __forceinline__ int lane_block(int t) {
  return L == 8 ? (((t & 1) << 2) | (t & 2) | ((t >> 2) & 1)) : t;
}

template <typename R, int NX, int L>
__device__ __forceinline__ void group_inverse(cplx<R>* y, int t, const cplx<R>* tw) {
  constexpr int H = NX / L;
  Dft<H, +1, R>::run(y);
#pragma unroll
  for (int k = 1; k < H; ++k) y[k] = cmul(y[k], tw[(t * k) % NX]);
#pragma unroll
  for (int k = 0; k < H; ++k) y[k] = L == 8 ? cross_dif8<+1>(y[k], t) : cross_dft<+1, L>(y[k], t);
}

template <typename R, int NX, int L>
__device__ __forceinline__ void group_forward(cplx<R>* y, int t, const cplx<R>* tw) {
  constexpr int H = NX / L;
#pragma unroll
  for (int n = 0; n < H; ++n) {
    const cplx<R> a = L == 8 ? cross_dit8<-1>(y[n], t) : cross_dft<-1, L>(y[n], t);
    const cplx<R> w = tw[(t * n) % NX];
    y[n] = n ? cmul(a, cplx<R>{w.re, -w.im}) : a;
  }
  Dft<H, -1, R>::run(y);
}

template <typename R, int NX, int L>
__global__ void __launch_bounds__(L * NX) k_xy_group(LocalArgs a) {
  constexpr int H = NX / L, NT = L * NX, LPW = 64 / L;  // lines per wave
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ns = a.nax_stride;
  cplx<R>* Lp = reinterpret_cast<cplx<R>*>(smem_raw);  // [NX rows i2][ns]
  cplx<R>* tw = Lp + NX * ns;                           // [NX]
  int* col = reinterpret_cast<int*>(tw + NX);           // [NX]
  const int tid = threadIdx.x, t = tid % L, line = tid / L, tb = lane_block<L>(t);
  const int N3 = a.N3;
  int bid = blockIdx.x, kb, p;
  if ((N3 & 7) == 0) {
    const int xcd = bid & 7, jj = bid >> 3, per = N3 >> 3;
    kb = jj / per;
    p = xcd * per + (jj - kb * per);
  } else {
    kb = bid / N3;
    p = bid - kb * N3;
  }
  int si = 0;
  while (si < a.nsl - 1 && kb >= a.pair0[si + 1]) ++si;
  const int k = a.sl[si].k, band = kb - a.pair0[si];
  const KInfo ki = a.kinfo[k];
  const int nax = ki.nax;
  for (int i = tid; i < NX; i += NT) {
    double2 w = a.tw_x[i];
    tw[i] = {R(w.x), R(w.y)};
    col[i] = a.col_of_i1[int64_t(k) * NX + i];
  }
  for (int i = tid; i < NX * ns; i += NT) Lp[i] = {R(0), R(0)};
  __syncthreads();
  cplx<R>* plane = stick_base<R>(a, ki) +
                   (int64_t(band) * N3 + p) * ki.nstick;
  const int32_t* spos = a.stick_pos + ki.stick_off;
  sticks_to_lds<R, NT>(plane, spos, ki.nstick, Lp, ns, tid);
  __syncthreads();
  // whole waves take part in the cross-lane steps (lines rounded up to a wave)
  const int nax_w = ((nax + LPW - 1) / LPW) * LPW;
  cplx<R> y[H];
  // inverse y on active columns
  if (line < nax_w) {
    const bool live = line < nax;
#pragma unroll
    for (int n = 0; n < H; ++n) y[n] = live ? Lp[(L * n + t) * ns + line] : cplx<R>{R(0), R(0)};
    group_inverse<R, NX, L>(y, t, tw);
    if (live) {
#pragma unroll
      for (int k2 = 0; k2 < H; ++k2) Lp[(H * tb + k2) * ns + line] = y[k2];
    }
  }
  __syncthreads();
  // x rows: inverse, * V / N_r, forward
  {
    const int i2 = line;
    cplx<R>* row = Lp + i2 * ns;
#pragma unroll
    for (int n = 0; n < H; ++n) {
      const int c = col[L * n + t];
      y[n] = c >= 0 ? row[c] : cplx<R>{R(0), R(0)};
    }
    group_inverse<R, NX, L>(y, t, tw);
    const R* Vrow = reinterpret_cast<const R*>(a.vplan) + (int64_t(p) * NX + i2) * NX + H * tb;
#pragma unroll
    for (int n = 0; n < H; ++n) y[n] = cscale(y[n], Vrow[n]);
    group_forward<R, NX, L>(y, t, tw);
#pragma unroll
    for (int k2 = 0; k2 < H; ++k2) {
      const int c = col[L * k2 + t];
      if (c >= 0) row[c] = y[k2];
    }
  }
  __syncthreads();
  // forward y on active columns
  if (line < nax_w) {
    const bool live = line < nax;
#pragma unroll
    for (int n = 0; n < H; ++n) y[n] = live ? Lp[(H * tb + n) * ns + line] : cplx<R>{R(0), R(0)};
    group_forward<R, NX, L>(y, t, tw);
    if (live) {
#pragma unroll
      for (int k2 = 0; k2 < H; ++k2) Lp[(L * k2 + t) * ns + line] = y[k2];
    }
  }
  __syncthreads();
  lds_to_sticks<R, NT>(plane, spos, ki.nstick, Lp, ns, tid);
}

// ------------------------------------------------------------------ z forward + gather + kinetic
template <typename R, int N3, int TS>
__global__ void __launch_bounds__(TS * Split<N3>::R2) k_zfwd(LocalArgs a) {
  constexpr int R1 = Split<N3>::R1, R2 = Split<N3>::R2, NT = TS * R2;
  __shared__ cplx<R> tile[N3 * TS];
  __shared__ cplx<R> tw[N3];
  const int tid = threadIdx.x;
  int bid = blockIdx.x;
  const int si = locate_tile_block(a, bid);
  const KSlice& ks = a.sl[si];
  const KInfo ki = a.kinfo[ks.k];
  const int band = bid / ki.ntile, t = bid - band * ki.ntile;
  const int s0 = t * TS;
  const int cnt = min(TS, ki.nstick - s0);
  for (int i = tid; i < N3; i += NT) {
    double2 w = a.tw_z[i];
    tw[i] = {R(w.x), R(w.y)};
  }
  __syncthreads();
  const int sl = tid % TS, j = tid / TS;  // j in [0, R2)
  {
    const cplx<R>* in = static_cast<const cplx<R>*>(stick_base<R>(a, ki)) +
                        int64_t(band) * N3 * ki.nstick + s0 + sl;
    cplx<R> x[R1];
#pragma unroll
    for (int n2 = 0; n2 < R1; ++n2)
      x[n2] = sl < cnt ? in[int64_t(n2 + R1 * j) * ki.nstick] : cplx<R>{R(0), R(0)};
    Dft<R1, -1, R>::run(x);
#pragma unroll
    for (int k2 = 1; k2 < R1; ++k2) {
      const cplx<R> w = tw[(j * k2) % N3];
      x[k2] = cmul(x[k2], cplx<R>{w.re, -w.im});
    }
#pragma unroll
    for (int k2 = 0; k2 < R1; ++k2) tile[(k2 + R1 * j) * TS + sl] = x[k2];
  }
  __syncthreads();
  if (j < R1) {
    cplx<R> z[R2];
#pragma unroll
    for (int n1 = 0; n1 < R2; ++n1) z[n1] = tile[(j + R1 * n1) * TS + sl];
    Dft<R2, -1, R>::run(z);
#pragma unroll
    for (int k1 = 0; k1 < R2; ++k1) tile[(j + R1 * k1) * TS + sl] = z[k1];
  }
  __syncthreads();
  const int32_t* tp = a.tile_ptr + ki.tile_off;
  const int e0 = tp[t], e1 = tp[t + 1];
  const double2* psi_b = a.psi + ks.psi_off + int64_t(band) * ki.npw;
  double2* out_b = a.hpsi + ks.hpsi_off + int64_t(band) * ki.npw;
  const int32_t* eg = a.ent_g + ki.g_off;
  const int32_t* esz = a.ent_sz + ki.g_off;
  const double* kin = a.kin + ki.g_off;
  for (int eb = e0 + tid; eb < e1; eb += kUnroll * NT) {
    int sz[kUnroll], g[kUnroll];
    double2 ps[kUnroll];
    double kv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = min(eb + u * NT, e1 - 1);
      sz[u] = esz[e];
      g[u] = eg[e];
      ps[u] = psi_b[g[u]];
      kv[u] = kin[g[u]];
    }
    // each G is read and written by the one entry that owns it, so the stores stay guarded
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      pin(sz[u]);
      pin(ps[u]);
      pin(kv[u]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (eb + u * NT < e1) {
        const int s = sz[u] / N3, z = sz[u] - s * N3;
        const cplx<R> v = tile[z * TS + (s - s0)];
        out_b[g[u]] = make_double2(kv[u] * ps[u].x + double(v.re), kv[u] * ps[u].y + double(v.im));
      }
    }
  }
}

}  // namespace qm
