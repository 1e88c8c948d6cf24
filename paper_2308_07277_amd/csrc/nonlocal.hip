// Kleinman-Bylander non-local term of H|psi> (Sec. 2.3, separable form
// sum_ij |beta_i> D_ij <beta_j|):  P = beta^dagger psi (CN GEMM),
// Q = D P (banded row ranges of D), H psi += beta Q (EX GEMM, accumulating).
#include "cplx.h"
#include "qm_internal.h"

namespace qm {

// Q[k](i, j) = sum_{l in range(i)} D(i, l) P[k](l, j); P, Q c128 [nproj][nbnd] per k
__global__ void k_apply_d(const double2* __restrict__ P, double2* __restrict__ Q,
                          const double* __restrict__ D, const int32_t* __restrict__ drange,
                          int nproj, int nbnd, int64_t total) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(t % nbnd);
    const int64_t r = t / nbnd;
    const int i = int(r % nproj);
    const int64_t kb = (r / nproj) * int64_t(nproj) * nbnd;
    const int lo = drange[2 * i], hi = drange[2 * i + 1];
    double sr = 0, si = 0;
    for (int l = lo; l < hi; ++l) {
      const double d = D[int64_t(i) * nproj + l];
      const double2 p = P[kb + int64_t(l) * nbnd + j];
      sr += d * p.x;
      si += d * p.y;
    }
    Q[t] = make_double2(sr, si);
  }
}

void launch_nonlocal_t(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi,
                       void* hpsi, hipStream_t s, StageEvents* ev, int lp, const ProjScratch* ps,
                       const HpsiWork* wk, int parts) {
  if (p->nproj == 0) return;
  const int np = p->nproj;
  double2* P = wk ? wk->P : reinterpret_cast<double2*>(p->proj_q);
  double2* Q = wk ? wk->Q : P + int64_t(p->nk) * np * p->nbnd_max;
  // P and Q blocks of slice x: at k nproj nbnd_max in the plan's buffers, at 0 in the caller's
  auto pq_off = [&](const KSlice& x) { return wk ? int64_t(0) : int64_t(x.k) * np * p->nbnd_max; };
  std::vector<GemmCN> cn;
  std::vector<GemmEX> ex;
  for (const KSlice& x : sl) {
    const int64_t off = pq_off(x);
    const KInfo& ki = p->kinfo[x.k];
    const char* bbase = reinterpret_cast<const char*>(lp == 0 ? p->beta64 : p->beta_lp);
    const size_t esz = lp == 0 ? 16 : (lp == 1 ? 8 : 4);
    const void* bk = bbase + size_t(ki.beta_off) * esz;
    const double2* pk = reinterpret_cast<const double2*>(psi) + x.psi_off;
    double2* hk = reinterpret_cast<double2*>(hpsi) + x.hpsi_off;
    cn.push_back(GemmCN{bk, pk, P + off, np, x.nb, ki.npw, ki.npw, ki.npw, x.nb});
    ex.push_back(GemmEX{Q + off, bk, hk, x.nb, ki.npw, np, x.nb, ki.npw, ki.npw});
  }
  if (parts == kNlExpand) {
    zgemm_ex_batched(ex, 1.0, 1.0, s, lp);
    return;
  }
  void* part = wk ? wk->part : (ps ? ps->part : p->proj_part);
  const int64_t part_bytes = wk ? wk->part_bytes : (ps ? ps->bytes : p->proj_part_bytes);
  zgemm_cn_batched(cn, 1.0, 0.0, part, part_bytes, s, ev, 3, lp, p->tuned_splits[lp]);
  // D acts on each slice's [np][nb] block
  for (const KSlice& x : sl) {
    const int64_t base = pq_off(x);
    const int64_t total = int64_t(np) * x.nb;
    const int blocks = int(std::min<int64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL(k_apply_d, dim3(blocks), dim3(256), 0, s, P + base, Q + base, p->dmat,
                       p->drange, np, x.nb, total);
    QM_HIP(hipGetLastError());
  }
  if (ev) ev->mark(5);
  if (parts == kNlProject) return;
  zgemm_ex_batched(ex, 1.0, 1.0, s, lp);
  if (ev) ev->mark(6);
}

void launch_nonlocal(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                     hipStream_t s, qm_prec prec, StageEvents* ev, const ProjScratch* ps,
                     const HpsiWork* wk, int parts) {
  const int lp = prec == QM_PREC_FP64 ? 0 : (prec == QM_PREC_FP32 ? 1 : 2);
  if (lp != 0 && p->beta_lp_kind != lp) {
    QM_REQUIRE(!wk, QM_E_STATE, "the reduced-precision copy of beta is not built");
    convert_beta(p, prec, s);
  }
  launch_nonlocal_t(p, sl, psi, hpsi, s, ev, lp, ps, wk, parts);
}

// low-precision copy of beta for the FP32 (c64) or MIXED (bf16 pairs) projector GEMMs
void convert_beta(qm_hpsi_plan* p, qm_prec prec, hipStream_t s) {
  if (p->nproj == 0 || prec == QM_PREC_FP64) return;
  const int lp = prec == QM_PREC_FP32 ? 1 : 2;
  if (p->beta_lp_kind == lp) return;
  const int64_t n = int64_t(p->nproj) * p->npw_total;
  if (!p->beta_lp) QM_HIP(hipMalloc(&p->beta_lp, size_t(n) * 8));
  convert_beta_lp(p->beta64, p->beta_lp, n, lp, s);
  p->beta_lp_kind = lp;
}

}  // namespace qm

// ---------------------------------------------------------------- autotuning
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>

namespace qm {

static std::map<std::string, int> load_cache(const char* path) {
  std::map<std::string, int> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {  // one "key": value per line
    const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find(':', b);
    if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
    m[line.substr(a + 1, b - a - 1)] = std::atoi(line.c_str() + c + 1);
  }
  return m;
}

static void save_cache(const char* path, const std::map<std::string, int>& m) {
  if (!path) return;
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
  f << "}\n";
}

// time the projector GEMM of every k at nbnd bands for each split-K candidate
void autotune_projection(qm_hpsi_plan* p, int nbnd, hipStream_t s, int lp, double* best_ms) {
  if (p->nproj == 0) return;
  if (lp != 0) convert_beta(p, lp == 1 ? QM_PREC_FP32 : QM_PREC_MIXED, s);
  std::ostringstream key;
  key << "cn/" << lp << "/" << p->nproj << "x" << nbnd << "/" << p->nk << "/" << p->npw_total;
  const char* path = std::getenv("QM_AUTOTUNE_CACHE");
  std::map<std::string, int> cache = load_cache(path);
  auto it = cache.find(key.str());
  if (it != cache.end()) {
    p->tuned_splits[lp] = it->second;
    if (best_ms) *best_ms = -1.0;
    return;
  }
  void* psi = nullptr;
  QM_HIP(hipMalloc(&psi, size_t(nbnd) * size_t(p->npw_total) * 16));
  QM_HIP(hipMemsetAsync(psi, 0, size_t(nbnd) * size_t(p->npw_total) * 16, s));
  double2* P = reinterpret_cast<double2*>(p->proj_q);
  std::vector<GemmCN> cn;
  int64_t off = 0;
  for (int k = 0; k < p->nk; ++k) {
    const KInfo& ki = p->kinfo[k];
    const char* bbase = reinterpret_cast<const char*>(lp == 0 ? p->beta64 : p->beta_lp);
    const size_t esz = lp == 0 ? 16 : (lp == 1 ? 8 : 4);
    cn.push_back(GemmCN{bbase + size_t(ki.beta_off) * esz,
                        reinterpret_cast<const double2*>(psi) + int64_t(nbnd) * ki.g_off, P + off,
                        p->nproj, nbnd, ki.npw, ki.npw, ki.npw, nbnd});
    off += int64_t(p->nproj) * nbnd;
  }
  hipEvent_t e0, e1;
  QM_HIP(hipEventCreate(&e0));
  QM_HIP(hipEventCreate(&e1));
  int best = 0;
  double bms = 1e30;
  for (int sp = 1; sp <= 64; sp *= 2) {
    if (int64_t(sp) * off * 16 > p->proj_part_bytes) break;
    zgemm_cn_batched(cn, 1.0, 0.0, p->proj_part, p->proj_part_bytes, s, nullptr, 0, lp, sp);  // warm
    QM_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r)
      zgemm_cn_batched(cn, 1.0, 0.0, p->proj_part, p->proj_part_bytes, s, nullptr, 0, lp, sp);
    QM_HIP(hipEventRecord(e1, s));
    QM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QM_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms / 3.0 < bms) {
      bms = ms / 3.0;
      best = sp;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(psi);
  p->tuned_splits[lp] = best;
  if (best_ms) *best_ms = bms;
  cache[key.str()] = best;
  save_cache(path, cache);
}

// time the local part (scatter, FFTs, V, gather) of min(nk, 32) k-points at nbnd bands with
// each xy-plane kernel, per real type; keep the faster one
static void autotune_xy(qm_hpsi_plan* p, int nbnd, hipStream_t s) {
  if (p->xy_forced != 0) return;
  const char* path = std::getenv("QM_AUTOTUNE_CACHE");
  std::map<std::string, int> cache = load_cache(path);
  const int k1 = std::min(p->nk, kMaxSlices);
  const std::vector<KSlice> sl = contiguous_slices(p, 0, k1, nbnd);
  const int64_t npw = p->kinfo[k1 - 1].g_off + p->kinfo[k1 - 1].npw - p->kinfo[0].g_off;
  void* psi = nullptr;
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool dirty = false;
  for (int rt = 0; rt < 2; ++rt) {
    std::ostringstream key;
    key << "xy/" << rt << "/" << p->N1 << "x" << p->N2 << "x" << p->N3 << "/" << nbnd << "/" << k1
        << "/" << npw;
    auto it = cache.find(key.str());
    if (it != cache.end()) {
      p->xy_variant[rt] = it->second;
      continue;
    }
    if (!psi) {
      QM_HIP(hipMalloc(&psi, size_t(nbnd) * size_t(npw) * 16));
      QM_HIP(hipMalloc(&out, size_t(nbnd) * size_t(npw) * 16));
      QM_HIP(hipMemsetAsync(psi, 0, size_t(nbnd) * size_t(npw) * 16, s));
      QM_HIP(hipEventCreate(&e0));
      QM_HIP(hipEventCreate(&e1));
    }
    int best = 1;
    double bms = 1e30;
    for (int v = 1; v <= 3; ++v) {
      if (v == 2 && xy_group_lanes(p->N1) == 0) continue;
      const size_t real_bytes = rt == 0 ? 8 : 4;
      if (v != 2 && xy_lds_bytes(p->N1, xy_row_stride(p->N1, p->nax_max, v == 3), real_bytes,
                                 v == 3) > 160 * 1024)
        continue;
      p->xy_variant[rt] = v;
      launch_hpsi_local(p, sl, psi, out, s, rt == 1, nullptr);  // warm
      QM_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch_hpsi_local(p, sl, psi, out, s, rt == 1, nullptr);
      QM_HIP(hipEventRecord(e1, s));
      QM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QM_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < bms) {
        bms = ms;
        best = v;
      }
    }
    p->xy_variant[rt] = best;
    cache[key.str()] = best;
    dirty = true;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (psi) (void)hipFree(psi);
  if (out) (void)hipFree(out);
  if (dirty) save_cache(path, cache);
}

// time whole H applications of every k at nbnd bands with the projection on the side stream
// and with everything on the caller's stream, per precision, launched as qm_apply_h launches
// them (graph replays when the plan uses graphs); keep the faster
static void autotune_overlap(qm_hpsi_plan* p, int nbnd, hipStream_t s) {
  if (p->overlap_forced >= 0 || p->nproj == 0) return;
  const qm_prec saved = p->prec;
  auto drop_graphs = [&]() {
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    p->graphs.clear();
  };
  const char* path = std::getenv("QM_AUTOTUNE_CACHE");
  std::map<std::string, int> cache = load_cache(path);
  const std::vector<KSlice> sl = contiguous_slices(p, 0, p->nk, nbnd);
  void* psi = nullptr;
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool dirty = false;
  for (int lp = 0; lp < 3; ++lp) {
    std::ostringstream key;
    key << "ovl/" << lp << "/" << p->N1 << "x" << p->N2 << "x" << p->N3 << "/" << p->nproj << "x"
        << nbnd << "/" << p->nk << "/" << p->npw_total;
    auto it = cache.find(key.str());
    if (it != cache.end()) {
      p->overlap_tuned[lp] = it->second;
      continue;
    }
    if (!psi) {
      const size_t bytes = size_t(nbnd) * size_t(p->npw_total) * 16;
      QM_HIP(hipMalloc(&psi, bytes));
      QM_HIP(hipMalloc(&out, bytes));
      QM_HIP(hipMemsetAsync(psi, 0, bytes, s));
      QM_HIP(hipEventCreate(&e0));
      QM_HIP(hipEventCreate(&e1));
    }
    const qm_prec prec = lp == 0 ? QM_PREC_FP64 : (lp == 1 ? QM_PREC_FP32 : QM_PREC_MIXED);
    p->prec = prec;
    auto run = [&]() {
      if (p->use_graphs && p->nk <= kMaxSlices) apply_graph(p, -1, psi, out, nbnd, s);
      else apply_h_slices(p, sl, psi, out, s, prec);
    };
    float ms[2] = {0.f, 0.f};
    for (int v = 1; v >= 0; --v) {
      p->overlap_tuned[lp] = v;
      drop_graphs();
      run();   // warm (and capture)
      QM_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) run();
      QM_HIP(hipEventRecord(e1, s));
      QM_HIP(hipEventSynchronize(e1));
      QM_HIP(hipEventElapsedTime(&ms[v], e0, e1));
    }
    // the side stream only where it gains at least 1% (one stream keeps each kernel's
    // duration its own)
    const int best = ms[1] < 0.99f * ms[0] ? 1 : 0;
    p->overlap_tuned[lp] = best;
    cache[key.str()] = best;
    dirty = true;
  }
  p->prec = saved;
  drop_graphs();   // they name the tuning buffers
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (psi) (void)hipFree(psi);
  if (out) (void)hipFree(out);
  if (dirty) save_cache(path, cache);
}

}  // namespace qm

extern "C" qm_status qm_hpsi_plan_autotune(qm_hpsi_plan* plan, int32_t nbnd, void* stream) {
  if (!plan) return QM_E_ARG;
  try {
    QM_REQUIRE(nbnd >= 1 && nbnd <= plan->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
    for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
    plan->graphs.clear();
    for (int lp = 0; lp < 3; ++lp)
      qm::autotune_projection(plan, nbnd, reinterpret_cast<hipStream_t>(stream), lp, nullptr);
    qm::autotune_xy(plan, nbnd, reinterpret_cast<hipStream_t>(stream));
    qm::autotune_overlap(plan, nbnd, reinterpret_cast<hipStream_t>(stream));
    return QM_OK;
  } catch (const qm::Error& e) {
    plan->err = e.what();
    return e.code;
  }
}
