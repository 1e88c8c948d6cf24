// Plan creation (G-space tables, uploads), H|psi> orchestration and the C ABI.
//
// The plan turns the caller's k-points and Miller lists into the tables the
// kernels use: for each k the z-sticks holding at least one sphere point
// (the pruning of Sec. 4.3, "Optimizing FFT operations for G-Space"),
// sorted by (i2, i1), the active x-columns, the sphere entries grouped by
// stick, the stick tiles of the z kernels and the kinetic energies
// 1/2|k+G|^2.  V(r) is re-laid out per z-slot and scaled by 1/N_r, beta and
// D are copied.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <memory>

#include "cplx.h"
#include "qm_internal.h"

namespace qm {

constexpr int kTileSticks = 32;  // must match the z kernels' tile (fft_launch.h)

static thread_local std::string g_create_err;

template <typename T>
static T* upload(const std::vector<T>& v, hipStream_t s) {
  T* d = nullptr;
  if (v.empty()) return nullptr;
  QM_HIP(hipMalloc(&d, v.size() * sizeof(T)));
  (void)s;
  QM_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

static void plan_free(qm_hpsi_plan* p) {
  if (!p) return;
  davidson_free(p);
  density_free(p);
  td_free(p);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  void* ptrs[] = {p->g.kinfo, p->g.ent_g, p->g.ent_sz, p->g.tile_ptr, p->g.stick_pos,
                  p->g.col_of_i1, p->g.stick_at, p->g.flat, p->g.kin, p->vplan64, p->vplan32, p->beta64, p->beta_lp,
                  p->dmat, p->drange, p->tw_z, p->tw_x, p->sbuf, p->proj_part, p->proj_q};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

static void build_plan(qm_hpsi_plan* p, const double cell[9], const int32_t grid[3],
                       const qm_kset* ks, int32_t nbnd_max, int32_t nproj, const double* vloc_r,
                       const void* beta, const double* dmat, qm_prec prec, hipStream_t s) {
  QM_REQUIRE(cell && grid && ks, QM_E_ARG, "cell, grid and ks must be non-NULL");
  QM_REQUIRE(ks->nk >= 1 && ks->k_cart && ks->npw && ks->miller, QM_E_ARG,
             "kset needs nk >= 1 and non-NULL k_cart, npw, miller");
  QM_REQUIRE(nbnd_max >= 1 && nproj >= 0, QM_E_ARG, "nbnd_max >= 1 and nproj >= 0 required");
  QM_REQUIRE(vloc_r, QM_E_ARG, "vloc_r must be non-NULL");
  QM_REQUIRE(nproj == 0 || (beta && dmat), QM_E_ARG, "beta and dmat required when nproj > 0");
  QM_REQUIRE(prec == QM_PREC_FP64 || prec == QM_PREC_FP32 || prec == QM_PREC_MIXED, QM_E_ARG,
             "unknown precision");
  p->N1 = grid[0];
  p->N2 = grid[1];
  p->N3 = grid[2];
  QM_REQUIRE(p->N1 == p->N2, QM_E_SHAPE, "grid needs N1 == N2");
  QM_REQUIRE(fft_len_supported(p->N1) && fft_len_supported(p->N3), QM_E_SHAPE,
             "grid length not supported");
  p->nk = ks->nk;
  p->nbnd_max = nbnd_max;
  p->nproj = nproj;
  p->prec = prec;
  p->zts = kTileSticks;
  if (const char* xm = std::getenv("QM_XY_MODE")) p->xy_forced = std::atoi(xm);
  if (const char* tm = std::getenv("QM_TRIDIAG_MODE")) p->trd_forced = std::atoi(tm);
  if (const char* tf = std::getenv("QM_TRD_FINISH_MIN")) p->trd_fin_min = std::max(2, std::atoi(tf));
  if (const char* cm = std::getenv("QM_CHOL_MODE")) p->chol_forced = std::atoi(cm);
  if (const char* om = std::getenv("QM_OVERLAP")) p->overlap_forced = std::atoi(om) != 0;
  std::memcpy(p->cell, cell, sizeof(p->cell));
  // reciprocal rows b_i = 2 pi (A^-1)^T
  const double* a = cell;
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  QM_REQUIRE(std::fabs(det) > 1e-12, QM_E_ARG, "cell is singular");
  const double tp = 2.0 * 3.14159265358979323846 / det;
  // b1 = 2pi (a2 x a3)/det etc.
  const double b[9] = {tp * (a[4] * a[8] - a[5] * a[7]), tp * (a[5] * a[6] - a[3] * a[8]),
                       tp * (a[3] * a[7] - a[4] * a[6]), tp * (a[7] * a[2] - a[8] * a[1]),
                       tp * (a[8] * a[0] - a[6] * a[2]), tp * (a[6] * a[1] - a[7] * a[0]),
                       tp * (a[1] * a[5] - a[2] * a[4]), tp * (a[2] * a[3] - a[0] * a[5]),
                       tp * (a[0] * a[4] - a[1] * a[3])};
  std::memcpy(p->recip, b, sizeof(b));

  const int N1 = p->N1, N2 = p->N2, N3 = p->N3;
  std::vector<int32_t> ent_g, ent_sz, tile_ptr, stick_pos, col_of_i1(size_t(p->nk) * N1, -1), flat;
  std::vector<double> kin;
  p->kinfo.resize(p->nk);
  int64_t g_off = 0, stick_off = 0, tile_off = 0;
  std::vector<int32_t> stick_of(size_t(N1) * N2);
  std::vector<std::vector<int32_t>> sat_k(p->nk);   // per k: [N2][nax] stick index or -1
  // zero middle band of the xy transforms: x and y indices [R1 F, 2 R1 F) must hold no stick
  const int zf = zero_mid_f(fft_split_r2(N1)), zlo = fft_split_r1(N1) * zf, zhi = 2 * zlo;
  bool zmid = zf > 0 && N1 == N2;
  for (int k = 0; k < p->nk; ++k) {
    const int npw = ks->npw[k];
    QM_REQUIRE(npw >= 1, QM_E_ARG, "every k needs npw >= 1");
    const int32_t* m = ks->miller + 3 * g_off;
    std::vector<int64_t> keys(npw);
    std::vector<int32_t> ii(3 * size_t(npw));
    const int Ns[3] = {N1, N2, N3};
    for (int g = 0; g < npw; ++g) {
      for (int d = 0; d < 3; ++d) {
        const int v = m[3 * g + d];
        QM_REQUIRE(2 * std::abs(int64_t(v)) < Ns[d], QM_E_ARG,
                   "Miller index outside the FFT grid (need 2|m_i| < N_i)");
        ii[3 * g + d] = ((v % Ns[d]) + Ns[d]) % Ns[d];
      }
      keys[g] = (int64_t(ii[3 * g]) * N2 + ii[3 * g + 1]) * N3 + ii[3 * g + 2];
      flat.push_back(int32_t(keys[g]));
    }
    {
      std::vector<int64_t> sk(keys);
      std::sort(sk.begin(), sk.end());
      QM_REQUIRE(std::adjacent_find(sk.begin(), sk.end()) == sk.end(), QM_E_ARG,
                 "duplicate G vector in a sphere");
    }
    // sticks (i1, i2) sorted by (i2, i1)
    std::vector<char> present(size_t(N1) * N2, 0);
    for (int g = 0; g < npw; ++g) present[size_t(ii[3 * g + 1]) * N1 + ii[3 * g]] = 1;
    std::fill(stick_of.begin(), stick_of.end(), -1);
    int nstick = 0;
    std::vector<int32_t> st_i1, st_i2;
    for (int i2 = 0; i2 < N2; ++i2)
      for (int i1 = 0; i1 < N1; ++i1)
        if (present[size_t(i2) * N1 + i1]) {
          stick_of[size_t(i2) * N1 + i1] = nstick++;
          st_i1.push_back(i1);
          st_i2.push_back(i2);
        }
    std::vector<int> ia_of(N1, -1);
    for (int s2 = 0; s2 < nstick; ++s2) ia_of[st_i1[s2]] = 1;
    int nax = 0;
    for (int i1 = 0; i1 < N1; ++i1)
      if (ia_of[i1] > 0) ia_of[i1] = nax++;
      else ia_of[i1] = -1;
    for (int i1 = 0; i1 < N1; ++i1) col_of_i1[size_t(k) * N1 + i1] = ia_of[i1];
    sat_k[k].assign(size_t(N2) * nax, -1);
    for (int i2 = 0; i2 < N2; ++i2)
      for (int i1 = 0; i1 < N1; ++i1)
        if (ia_of[i1] >= 0) sat_k[k][size_t(i2) * nax + ia_of[i1]] = stick_of[size_t(i2) * N1 + i1];
    for (int s2 = 0; s2 < nstick; ++s2) stick_pos.push_back(st_i2[s2] | (ia_of[st_i1[s2]] << 16));
    for (int s2 = 0; s2 < nstick; ++s2)
      if ((st_i1[s2] >= zlo && st_i1[s2] < zhi) || (st_i2[s2] >= zlo && st_i2[s2] < zhi)) zmid = false;
    // entries grouped by stick tile; inside a tile ordered by (i3, stick) so consecutive
    // threads of the z kernels touch neighbouring x-columns of one plane (adjacent in the
    // usual G orders)
    std::vector<int32_t> order(npw);
    std::vector<int64_t> ekey(npw), skey(npw);
    for (int g = 0; g < npw; ++g) {
      const int st = stick_of[size_t(ii[3 * g + 1]) * N1 + ii[3 * g]];
      const int z = ii[3 * g + 2];
      ekey[g] = int64_t(st) * N3 + z;
      skey[g] = (int64_t(st / kTileSticks) * N3 + z) * kTileSticks + (st % kTileSticks);
      order[g] = g;
    }
    std::sort(order.begin(), order.end(), [&](int x, int y) { return skey[x] < skey[y]; });
    const int ntile = (nstick + kTileSticks - 1) / kTileSticks;
    int t = 0;
    for (int e = 0; e < npw; ++e) {
      const int g = order[e];
      ent_g.push_back(g);
      ent_sz.push_back(int32_t(ekey[g]));
      const int st = int(ekey[g] / N3);
      while (t <= st / kTileSticks) {
        tile_ptr.push_back(e);
        ++t;
      }
    }
    while (t <= ntile) {
      tile_ptr.push_back(npw);
      ++t;
    }
    // kinetic 1/2 |k + G|^2
    const double* kc = ks->k_cart + 3 * k;
    for (int g = 0; g < npw; ++g) {
      double q[3];
      for (int d = 0; d < 3; ++d)
        q[d] = kc[d] + m[3 * g] * b[d] + m[3 * g + 1] * b[3 + d] + m[3 * g + 2] * b[6 + d];
      kin.push_back(0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
    }
    KInfo& ki = p->kinfo[k];
    ki.npw = npw;
    ki.nstick = nstick;
    ki.ntile = ntile;
    ki.nax = nax;
    ki.g_off = g_off;
    ki.stick_off = stick_off;
    ki.tile_off = tile_off;
    ki.sbuf_off = int64_t(nbnd_max) * N3 * stick_off;
    ki.beta_off = int64_t(nproj) * g_off;
    p->nax_max = std::max(p->nax_max, nax);
    p->npw_max = std::max(p->npw_max, npw);
    g_off += npw;
    stick_off += nstick;
    tile_off += ntile + 1;
  }
  p->npw_total = g_off;
  p->zero_mid = zmid ? 1 : 0;
  if (const char* zm = std::getenv("QM_ZERO_MID")) p->zero_mid = p->zero_mid && std::atoi(zm) != 0;
  QM_REQUIRE(N1 <= 65535 && p->nax_max <= 32767, QM_E_SHAPE, "grid too large for stick tables");

  p->g.kinfo = upload(p->kinfo, s);
  p->g.ent_g = upload(ent_g, s);
  p->g.ent_sz = upload(ent_sz, s);
  p->g.tile_ptr = upload(tile_ptr, s);
  p->g.stick_pos = upload(stick_pos, s);
  p->g.col_of_i1 = upload(col_of_i1, s);
  {
    std::vector<int32_t> stick_at(size_t(p->nk) * N2 * p->nax_max, -1);
    for (int k = 0; k < p->nk; ++k) {
      const int nax = p->kinfo[k].nax;
      for (int i2 = 0; i2 < N2; ++i2)
        for (int ia = 0; ia < nax; ++ia)
          stick_at[(size_t(k) * N2 + i2) * p->nax_max + ia] = sat_k[k][size_t(i2) * nax + ia];
    }
    p->g.stick_at = upload(stick_at, s);
  }
  p->g.flat = upload(flat, s);
  p->g.kin = upload(kin, s);
  // twiddles exp(+2 pi i m / N), exact octant reduction
  auto roots = [](int n) {
    std::vector<double2> w(n);
    for (int mm = 0; mm < n; ++mm) {
      double c = 0, sn = 0;
      ct::sincos_frac(mm, n, c, sn);
      w[mm] = make_double2(c, sn);
    }
    return w;
  };
  p->tw_z = upload(roots(N3), s);
  p->tw_x = upload(roots(N1), s);
  // V(r)
  const int64_t nr = int64_t(N1) * N2 * N3;
  QM_HIP(hipMalloc(&p->vplan64, nr * sizeof(double)));
  QM_HIP(hipMalloc(&p->vplan32, nr * sizeof(float)));
  launch_vplan(p, vloc_r, s);
  // beta (c128 copy; lower-precision copies made on demand)
  if (nproj > 0) {
    const size_t bb = size_t(nproj) * size_t(p->npw_total) * 16;
    QM_HIP(hipMalloc(&p->beta64, bb));
    QM_HIP(hipMemcpyAsync(p->beta64, beta, bb, hipMemcpyDeviceToDevice, s));
    // D: real symmetric
    double dmax = 0;
    for (int64_t i = 0; i < int64_t(nproj) * nproj; ++i) dmax = std::max(dmax, std::fabs(dmat[i]));
    std::vector<int32_t> dr(2 * size_t(nproj));
    for (int i = 0; i < nproj; ++i) {
      int lo = nproj, hi = 0;
      for (int j = 0; j < nproj; ++j) {
        QM_REQUIRE(std::isfinite(dmat[size_t(i) * nproj + j]), QM_E_ARG, "D has a non-finite entry");
        QM_REQUIRE(std::fabs(dmat[size_t(i) * nproj + j] - dmat[size_t(j) * nproj + i]) <= 1e-12 * dmax,
                   QM_E_ARG, "D must be symmetric");
        if (dmat[size_t(i) * nproj + j] != 0.0) {
          lo = std::min(lo, j);
          hi = std::max(hi, j + 1);
        }
      }
      if (lo >= hi) lo = hi = 0;
      dr[2 * i] = lo;
      dr[2 * i + 1] = hi;
    }
    p->dmat = upload(std::vector<double>(dmat, dmat + size_t(nproj) * nproj), s);
    p->drange = upload(dr, s);
    // P and Q for every k at nbnd_max
    QM_HIP(hipMalloc(&p->proj_q, size_t(2) * p->nk * nproj * nbnd_max * 16));
    std::vector<GemmCN> cn;
    for (int k = 0; k < p->nk; ++k)
      cn.push_back(GemmCN{nullptr, nullptr, nullptr, nproj, nbnd_max, p->kinfo[k].npw, 0, 0, 0});
    // room for up to 16 K splits of every k (the autotuner tries 1 .. 16)
    int64_t mn = 0;
    for (const GemmCN& g : cn) mn += int64_t(g.M) * g.N;
    p->proj_part_bytes = std::max<int64_t>(zgemm_cn_work_bytes(cn), 16 * mn * 16);
    QM_HIP(hipMalloc(&p->proj_part, p->proj_part_bytes));
  }
  if (prec != QM_PREC_FP64) convert_beta(p, prec, s);
  p->sbuf_elems = int64_t(nbnd_max) * N3 * stick_off;
  QM_HIP(hipMalloc(&p->sbuf, size_t(p->sbuf_elems) * 16));
  QM_HIP(hipStreamSynchronize(s));
}

static qm_status fail(qm_hpsi_plan* p, const qm::Error& e) {
  if (p) p->err = e.what();
  return e.code;
}

// Replay a captured launch sequence for (k, nbnd, psi, hpsi, prec), capturing it on the
// plan's own stream the first time (the caller's stream may be the null stream, which cannot
// be captured).  Graphs hold kernel nodes only.
void apply_graph(qm_hpsi_plan* p, int k, const void* psi, void* hpsi, int nbnd, hipStream_t s) {
  const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? p->nk : k + 1;
  for (auto& g : p->graphs)
    if (g.k == k && g.nbnd == nbnd && g.prec == int(p->prec) && g.psi == psi && g.hpsi == hpsi) {
      g.last_use = ++p->graph_clock;
      QM_HIP(hipGraphLaunch(g.exec, s));
      return;
    }
  if (!p->capture_stream) QM_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
  convert_beta(p, p->prec, s);                     // any one-time conversion happens eagerly
  if (side_stream_wanted(p, p->prec)) ensure_side_stream(p);   // created outside the capture
  QM_HIP(hipStreamSynchronize(s));
  hipGraph_t graph = nullptr;
  QM_HIP(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
  try {
    apply_h_slices(p, contiguous_slices(p, k0, k1, nbnd), psi, hpsi, p->capture_stream, p->prec);
  } catch (...) {
    (void)hipStreamEndCapture(p->capture_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  QM_HIP(hipStreamEndCapture(p->capture_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  QM_HIP(ie);
  if (p->graphs.size() >= 8) {   // evict the least recently used entry
    size_t lru = 0;
    for (size_t i = 1; i < p->graphs.size(); ++i)
      if (p->graphs[i].last_use < p->graphs[lru].last_use) lru = i;
    (void)hipGraphExecDestroy(p->graphs[lru].exec);
    p->graphs.erase(p->graphs.begin() + lru);
  }
  p->graphs.push_back({k, nbnd, int(p->prec), psi, hpsi, exec, ++p->graph_clock});
  QM_HIP(hipGraphLaunch(exec, s));
}

}  // namespace qm

using namespace qm;

#define QM_API_GUARD(plan, ...)                                             \
  try {                                                                     \
    __VA_ARGS__;                                                                   \
    return QM_OK;                                                           \
  } catch (const qm::Error& e) {                                            \
    return qm::fail(plan, e);                                               \
  } catch (const std::bad_alloc&) {                                         \
    if (plan) plan->err = "host allocation failed";                         \
    return QM_E_NOMEM;                                                      \
  } catch (const std::exception& e) {                                       \
    if (plan) plan->err = e.what();                                         \
    return QM_E_STATE;                                                      \
  }

extern "C" {

qm_status qm_hpsi_plan_create(const double cell[9], const int32_t grid[3], const qm_kset* ks,
                              int32_t nbnd_max, int32_t nproj, const double* vloc_r,
                              const void* beta, const double* dmat, qm_prec prec, void* stream,
                              qm_hpsi_plan** out) {
  if (!out) {
    g_create_err = "out must be non-NULL";
    return QM_E_ARG;
  }
  *out = nullptr;
  qm_hpsi_plan* p = nullptr;
  try {
    p = new qm_hpsi_plan();
    build_plan(p, cell, grid, ks, nbnd_max, nproj, vloc_r, beta, dmat, prec,
               reinterpret_cast<hipStream_t>(stream));
    *out = p;
    g_create_err.clear();
    return QM_OK;
  } catch (const qm::Error& e) {
    g_create_err = e.what();
    plan_free(p);
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_err = "host allocation failed";
    plan_free(p);
    return QM_E_NOMEM;
  } catch (const std::exception& e) {
    g_create_err = e.what();
    plan_free(p);
    return QM_E_STATE;
  }
}

void qm_hpsi_plan_destroy(qm_hpsi_plan* plan) { plan_free(plan); }

const char* qm_last_error(const qm_hpsi_plan* plan) {
  return plan ? plan->err.c_str() : g_create_err.c_str();
}

qm_status qm_hpsi_plan_set_precision(qm_hpsi_plan* plan, qm_prec prec, void* stream) {
  if (!plan) return QM_E_ARG;
  QM_API_GUARD(plan, {
    QM_REQUIRE(prec == QM_PREC_FP64 || prec == QM_PREC_FP32 || prec == QM_PREC_MIXED, QM_E_ARG,
               "unknown precision");
    plan->prec = prec;
    convert_beta(plan, prec, reinterpret_cast<hipStream_t>(stream));
    QM_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  })
}

qm_status qm_apply_h(qm_hpsi_plan* plan, int32_t k, const void* psi, void* hpsi, int32_t nbnd,
                     void* stream) {
  if (!plan) return QM_E_ARG;
  QM_API_GUARD(plan, {
    QM_REQUIRE(psi && hpsi, QM_E_ARG, "psi and hpsi must be non-NULL");
    QM_REQUIRE(psi != hpsi, QM_E_ARG, "hpsi must not alias psi");
    QM_REQUIRE(nbnd >= 1 && nbnd <= plan->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
    QM_REQUIRE(k >= -1 && k < plan->nk, QM_E_ARG, "k out of range");
    const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? plan->nk : k + 1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (plan->use_graphs && k1 - k0 <= kMaxSlices)
      apply_graph(plan, k, psi, hpsi, nbnd, s);
    else
      apply_h_slices(plan, contiguous_slices(plan, k0, k1, nbnd), psi, hpsi, s, plan->prec);
  })
}

qm_status qm_hpsi_plan_set_graphs(qm_hpsi_plan* plan, int32_t enable) {
  if (!plan) return QM_E_ARG;
  plan->use_graphs = enable ? 1 : 0;
  for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
  plan->graphs.clear();
  return QM_OK;
}

qm_status qm_apply_h_timed(qm_hpsi_plan* plan, int32_t k, const void* psi, void* hpsi,
                           int32_t nbnd, double* times_ms, void* stream) {
  if (!plan) return QM_E_ARG;
  StageEvents ev{};
  struct Release {   // the events are destroyed on every return path
    StageEvents& e;
    ~Release() {
      for (hipEvent_t& x : e.ev)
        if (x) (void)hipEventDestroy(x);
    }
  } release{ev};
  QM_API_GUARD(plan, {
    QM_REQUIRE(times_ms, QM_E_ARG, "times_ms must be non-NULL");
    QM_REQUIRE(psi && hpsi && psi != hpsi, QM_E_ARG, "psi and hpsi must be distinct and non-NULL");
    QM_REQUIRE(nbnd >= 1 && nbnd <= plan->nbnd_max, QM_E_ARG, "need 1 <= nbnd <= nbnd_max");
    QM_REQUIRE(k >= -1 && k < plan->nk, QM_E_ARG, "k out of range");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ev.s = s;
    for (int i = 0; i <= QM_NSTAGES; ++i) QM_HIP(hipEventCreate(&ev.ev[i]));
    for (int i = 0; i < QM_NSTAGES; ++i) ev.used[i] = false;
    const int k0 = k < 0 ? 0 : k, k1 = k < 0 ? plan->nk : k + 1;
    QM_REQUIRE(k1 - k0 <= kMaxSlices, QM_E_ARG, "timed application handles at most 32 k-points");
    QM_HIP(hipEventRecord(ev.ev[0], s));
    apply_h_slices(plan, contiguous_slices(plan, k0, k1, nbnd), psi, hpsi, s, plan->prec, &ev);
    QM_HIP(hipStreamSynchronize(s));
    int last = 0;
    for (int i = 0; i < QM_NSTAGES; ++i) {
      times_ms[i] = 0.0;
      if (ev.used[i]) {
        float ms = 0.f;
        QM_HIP(hipEventElapsedTime(&ms, ev.ev[last], ev.ev[i + 1]));
        times_ms[i] = ms;
        last = i + 1;
      }
    }
  })
}

}  // extern "C"
