// Plan-side helpers of the local part: supported lengths, V(r) re-layout.
#include <algorithm>
#include "cplx.h"
#include "qm_internal.h"

namespace qm {

void launch_local_f64(qm_hpsi_plan*, const std::vector<KSlice>&, const void*, void*, hipStream_t,
                      StageEvents*, const HpsiWork*);
void launch_local_f32(qm_hpsi_plan*, const std::vector<KSlice>&, const void*, void*, hipStream_t,
                      StageEvents*, const HpsiWork*);

bool fft_len_supported(int n) {
  switch (n) {
#define QM_CASE(x) case x:
    QM_FOR_EACH_FFT_LEN(QM_CASE)
#undef QM_CASE
    return true;
    default:
      return false;
  }
}
int fft_split_r1(int n) {
  switch (n) {
#define QM_CASE(x) case x: return Split<x>::R1;
    QM_FOR_EACH_FFT_LEN(QM_CASE)
#undef QM_CASE
    default:
      return 0;
  }
}
int fft_split_r2(int n) {
  switch (n) {
#define QM_CASE(x) case x: return Split<x>::R2;
    QM_FOR_EACH_FFT_LEN(QM_CASE)
#undef QM_CASE
    default:
      return 0;
  }
}

int xy_row_stride(int n, int nax_max, bool own) {
  const int r2 = fft_split_r2(n), r1 = r2 ? n / r2 : 0;
  // one slot past the active columns reads as zero; odd, so that rows at this stride fall on
  // different LDS banks; with the exchanges in the rows' own slots each round of the x-row
  // transform pair holds half of the row's values
  int ns = nax_max + 1;
  if (own) ns = std::max({ns, (r1 + 1) / 2 * (r2 | 1), r1 * ((r2 + 1) / 2 | 1)});
  return ns | 1;
}

size_t xy_lds_bytes(int n, int ns, size_t real_bytes, bool own) {
  const int r2 = fft_split_r2(n);
  size_t cplx_elems = size_t(n) * ns + n;            // plane + twiddles
  if (!own) cplx_elems += size_t(4 * (64 / r2)) * (n + 1);   // row scratch
  return 2 * real_bytes * cplx_elems + sizeof(int) * n;
}

void launch_hpsi_local(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                       hipStream_t s, bool fp32, StageEvents* ev, const HpsiWork* wk) {
  if (fp32)
    launch_local_f32(p, sl, psi, hpsi, s, ev, wk);
  else
    launch_local_f64(p, sl, psi, hpsi, s, ev, wk);
}

int xy_group_lanes(int nx) { return nx == 20 || nx == 40 ? 2 : (nx == 72 ? 8 : 0); }

int xy_pick(const qm_hpsi_plan* p, int rt) {
  const bool group_ok = xy_group_lanes(p->N1) > 0;
  const int forced = p->xy_forced, v = p->xy_variant[rt];
  if (forced == 1 || forced == 3) return forced;
  if (forced == 2) return group_ok ? 2 : 1;
  if (v == 2 && group_ok) return 2;
  if (v == 1 || v == 3) return v;
  // built-in choice, as measured on the workloads: lane pairs for float64 20 and 40; for other
  // float64 grids the own-slot exchanges where they fit more workgroups on a CU
  if (rt == 0 && (p->N1 == 20 || p->N1 == 40)) return 2;
  if (rt == 0) {
    const size_t lds = 160 * 1024;
    const size_t b1 = xy_lds_bytes(p->N1, xy_row_stride(p->N1, p->nax_max, false), 8, false);
    const size_t b3 = xy_lds_bytes(p->N1, xy_row_stride(p->N1, p->nax_max, true), 8, true);
    if (b3 <= lds && (b1 > lds || lds / b3 > lds / b1)) return 3;
  }
  return 1;
}

std::vector<KSlice> contiguous_slices(const qm_hpsi_plan* p, int k0, int k1, int nbnd) {
  std::vector<KSlice> out;
  const int64_t g0 = p->kinfo[k0].g_off;
  for (int k = k0; k < k1; ++k) {
    const int64_t off = int64_t(nbnd) * (p->kinfo[k].g_off - g0);
    out.push_back(KSlice{k, nbnd, off, off});
  }
  return out;
}

bool side_stream_wanted(const qm_hpsi_plan* p, qm_prec prec) {
  const int lp = prec == QM_PREC_FP64 ? 0 : (prec == QM_PREC_FP32 ? 1 : 2);
  const int ovl = p->overlap_forced >= 0 ? p->overlap_forced : p->overlap_tuned[lp];
  return ovl && p->nproj > 0;
}

// The side stream is created on first use: every stream of the process takes one of the few
// hardware queues in turn, so a stream that is never used would still change which streams
// share a queue (the Davidson lanes, for one).
void ensure_side_stream(qm_hpsi_plan* p) {
  if (p->side_stream) return;
  QM_HIP(hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking));
  QM_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  QM_HIP(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
}

void apply_h_slices(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                    hipStream_t s, qm_prec prec, StageEvents* ev, const ProjScratch* ps,
                    const HpsiWork* wk, bool side_ok) {
  QM_REQUIRE(!wk || sl.size() == 1, QM_E_STATE, "caller-given working memory takes one slice");
  for (size_t b = 0; b < sl.size(); b += kMaxSlices) {
    std::vector<KSlice> chunk(sl.begin() + b, sl.begin() + std::min(sl.size(), b + kMaxSlices));
    std::vector<KSlice> nz;
    for (const KSlice& x : chunk)
      if (x.nb > 0) nz.push_back(x);
    if (nz.empty()) continue;
    // the projection on the side stream, concurrent with the local part; calls with stage
    // events, their own split-K scratch or caller-given working memory, and the Davidson's
    // (side_ok = false: its lanes are streams of their own) stay on one stream.  The side stream first waits for everything before on s (the previous
    // call's expansion still reads Q), and s waits for it before the expansion.
    if (side_ok && side_stream_wanted(p, prec) && !ev && !ps && !wk) {
      ensure_side_stream(p);
      convert_beta(p, prec, s);   // (a no-op unless the precision changed)
      QM_HIP(hipEventRecord(p->ev_fork, s));
      QM_HIP(hipStreamWaitEvent(p->side_stream, p->ev_fork, 0));
      launch_nonlocal(p, nz, psi, hpsi, p->side_stream, prec, nullptr, nullptr, nullptr, kNlProject);
      QM_HIP(hipEventRecord(p->ev_join, p->side_stream));
      launch_hpsi_local(p, nz, psi, hpsi, s, prec != QM_PREC_FP64, nullptr, nullptr);
      QM_HIP(hipStreamWaitEvent(s, p->ev_join, 0));
      launch_nonlocal(p, nz, psi, hpsi, s, prec, nullptr, nullptr, nullptr, kNlExpand);
      continue;
    }
    launch_hpsi_local(p, nz, psi, hpsi, s, prec != QM_PREC_FP64, ev, wk);
    launch_nonlocal(p, nz, psi, hpsi, s, prec, ev, ps, wk);
  }
}

// V(r) [i1][i2][i3] (float64, C order) -> plan layout [slot][i2][i1] scaled by 1/N_r, where
// slot p = k1 + R1 k2 holds plane i3 = k2 + R2 k1 (order left by the inverse z-transform).
__global__ void k_vplan(const double* __restrict__ v, double* __restrict__ v64, float* __restrict__ v32,
                        int N1, int N2, int N3, int R1, int R2, double scale) {
  const int64_t n = int64_t(N1) * N2 * N3;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int i1 = int(t % N1);
    const int64_t r = t / N1;
    const int i2 = int(r % N2);
    const int p = int(r / N2);
    const int k1 = p % R1, k2 = p / R1;
    const int i3 = k2 + R2 * k1;
    const double val = v[(int64_t(i1) * N2 + i2) * N3 + i3] * scale;
    v64[t] = val;
    v32[t] = float(val);
  }
}

void launch_vplan(qm_hpsi_plan* p, const double* vloc_r, hipStream_t s) {
  const int64_t n = int64_t(p->N1) * p->N2 * p->N3;
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(k_vplan, dim3(blocks), dim3(256), 0, s, vloc_r,
                     reinterpret_cast<double*>(p->vplan64), reinterpret_cast<float*>(p->vplan32),
                     p->N1, p->N2, p->N3, fft_split_r1(p->N3), fft_split_r2(p->N3), 1.0 / double(n));
  QM_HIP(hipGetLastError());
}

}  // namespace qm
