// Internal declarations of the gfx950 H|psi> / Davidson library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/qm_hpsi.h"

namespace qm {

struct Error : std::runtime_error {
  qm_status code;
  Error(qm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define QM_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError(); /* do not leave the error for the next check */         \
      throw ::qm::Error(e_ == hipErrorOutOfMemory ? QM_E_NOMEM : QM_E_HIP,             \
                        std::string(#call) + ": " + hipGetErrorString(e_));            \
    }                                                                                  \
  } while (0)

// allow a kernel the whole 160 KiB LDS of a gfx950 CU for dynamic shared memory, minus its
// static shared memory
inline hipError_t allow_full_lds(const void* f) {
  hipFuncAttributes at{};
  hipError_t e = hipFuncGetAttributes(&at, f);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(160 * 1024 - at.sharedSizeBytes));
}

#define QM_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw ::qm::Error(code, msg); \
  } while (0)

// Per-k description used by every kernel; lives in device memory.
struct KInfo {
  int32_t npw;      // sphere size
  int32_t nstick;   // z-sticks holding at least one G
  int32_t ntile;    // stick tiles of the z kernels
  int32_t nax;      // active x-columns (distinct i1 over the sticks)
  int64_t g_off;    // prefix sum of npw over earlier k
  int64_t stick_off;// prefix sum of nstick
  int64_t tile_off; // prefix sum of (ntile + 1)
  int64_t sbuf_off; // offset of this k's stick buffer (band 0), in complex-double elements
  int64_t beta_off; // element offset of beta_k (= nproj * g_off)
};

// Device-resident G-space tables of one plan.
struct GTables {
  KInfo* kinfo = nullptr;        // [nk]
  int32_t* ent_g = nullptr;      // [sum npw] caller index of the G, entries sorted by (stick, i3)
  int32_t* ent_sz = nullptr;     // [sum npw] stick_local_in_k * N3 + i3
  int32_t* tile_ptr = nullptr;   // [sum (ntile+1)] entry offset (within k) of each tile
  int32_t* stick_pos = nullptr;  // [sum nstick] i2 | (ia << 16)
  int32_t* col_of_i1 = nullptr;  // [nk][N1] active-column index of i1, or -1
  int32_t* stick_at = nullptr;   // [nk][N2][nax_max] stick index of (i2, active column), or -1
  int32_t* flat = nullptr;       // [sum npw] C-order grid index of each G, caller order
  double* kin = nullptr;         // [sum npw] 1/2|k+G|^2 in caller order
};

struct DavState;  // Davidson workspace (davidson.hip)
struct TdWork;    // real-time propagation workspace (tddft.hip)

// One k-point's band block in a batched H application: nb rows of npw_k
// coefficients starting at element offsets psi_off / hpsi_off of the call's
// base pointers, consecutive rows npw_k apart.
constexpr int kMaxSlices = 32;
struct KSlice {
  int32_t k, nb;
  int64_t psi_off, hpsi_off;
};

// Optional per-stage event recorder: mark(i) records event i+1 after stage i.
struct StageEvents {
  hipEvent_t ev[QM_NSTAGES + 1];
  bool used[QM_NSTAGES];
  hipStream_t s;
  void mark(int i) {
    if (hipEventRecord(ev[i + 1], s) == hipSuccess) used[i] = true;
  }
};

}  // namespace qm

struct qm_hpsi_plan {
  int32_t N1 = 0, N2 = 0, N3 = 0;
  int32_t nk = 0, nbnd_max = 0, nproj = 0;
  qm_prec prec = QM_PREC_FP64;
  int32_t zts = 32;               // sticks per z-kernel tile
  int32_t nax_max = 0;
  int32_t zero_mid = 0;           // LocalArgs::zero_mid, for every k of the plan
  int64_t npw_total = 0;
  int32_t npw_max = 0;
  double cell[9] = {0}, recip[9] = {0};
  std::vector<qm::KInfo> kinfo;   // host copy
  qm::GTables g;
  void* vplan64 = nullptr;        // float64 [N3 slot][N2][N1], scaled by 1/N_r
  void* vplan32 = nullptr;        // float32, same layout
  void* beta64 = nullptr;         // c128 copy of beta
  void* beta_lp = nullptr;        // c64 (FP32) or bf16 pairs (MIXED) copy, per prec
  int32_t beta_lp_kind = -1;      // which representation beta_lp holds (qm_prec) or -1
  double* dmat = nullptr;         // [nproj][nproj]
  int32_t* drange = nullptr;      // [nproj][2] nonzero column range per row of D
  double2* tw_z = nullptr;        // exp(+2 pi i m / N3), m < N3
  double2* tw_x = nullptr;        // exp(+2 pi i m / N1), m < N1
  void* sbuf = nullptr;           // stick buffer, sized for float64 (reused by float32)
  int64_t sbuf_elems = 0;
  void* proj_part = nullptr;      // split-K partial projections
  int64_t proj_part_bytes = 0;
  void* proj_q = nullptr;         // Q = D P, c128 [nk][nproj][nbnd_max] or float in lower precisions
  int32_t proj_splits = 1;
  int32_t tuned_splits[3] = {0, 0, 0};  // projector split-K chosen by the autotuner, per precision
  std::string err;
  qm::DavState* dav = nullptr;
  // concurrent Davidson lanes of qm_davidson_solve (disjoint k ranges), their streams
  std::vector<qm::DavState*> dav_lanes;
  std::vector<hipStream_t> lane_streams;
  // captured qm_apply_h launch sequences (kernel nodes only), replayed on the caller's stream
  struct GraphEntry {
    int32_t k, nbnd, prec;
    const void* psi;
    void* hpsi;
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t capture_stream = nullptr;
  int32_t use_graphs = 1;
  // The projection beta^H psi and D of an H application run on a side stream while the
  // local part runs on the caller's stream (fork and join through two events), so the
  // MFMA-bound GEMM shares the chip with the VALU-bound FFT kernels; the expansion then
  // runs on the caller's stream.  Per precision (0 float64, 1 float32, 2 mixed) the
  // autotuner keeps it or turns it off, whichever is faster; overlap_forced (environment
  // QM_OVERLAP = 0 or 1) overrides that.
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int32_t overlap_tuned[3] = {1, 1, 1};
  int32_t overlap_forced = -1;
  // xy-plane kernel per real type of the local part (0 float64, 1 float32): 1 the two-pass
  // kernel with a row scratch, 2 the lane-group kernel (grids 20, 40, 72), 3 the two-pass
  // kernel with the x-row exchanges in the rows' own slots, 0 the built-in choice; set by the
  // autotuner.  xy_forced (environment QM_XY_MODE = 1, 2 or 3) overrides both.
  int32_t xy_variant[2] = {0, 0};
  int32_t xy_forced = 0;
  // Davidson tridiagonalisation: 1 one workgroup per k-point, 2 many workgroups per k-point
  // (one launch per step), 0 chosen by basis size (environment QM_TRIDIAG_MODE).
  int32_t trd_forced = 0;
  // Householder steps with at least this many tile slots per row (nt + 1) have each row block's
  // slots added by the tile that completes the block, so the step's last workgroup reads A v
  // per row instead of every slot (environment QM_TRD_FINISH_MIN)
  int32_t trd_fin_min = 16;
  // CholQR Cholesky + inverse: 1 one workgroup per k-point, 2 blocked on many workgroups,
  // 0 blocked up to 576 bands (environment QM_CHOL_MODE).
  int32_t chol_forced = 0;
  // density / Hartree workspace (density.hip), allocated on first use
  double* rho_part = nullptr;     // per band-group partial densities [G][slot][i2][i1]
  int64_t rho_part_bytes = 0;
  double* dens_wf = nullptr;      // per (k, band) pair weight w_k f_kn / Omega
  int64_t dens_wf_n = 0;
  void* grid_c = nullptr;         // complex float64 grid [N1][N2][N3] of the Poisson solve
  double* grid_sum = nullptr;     // [2] reduction results
  qm::TdWork* td = nullptr;       // propagation work buffers (tddft.hip), allocated on first use
};

namespace qm {
// Working memory of one H application given by the caller instead of the plan's buffers
// (the allocation-free entry point): one k-point slice per launch sequence, its stick block
// at sbuf, its projections P and D-applied block Q at P and Q ([nproj][nb] c128 each), the
// projector GEMM's split-K partial sums in part.  nullptr everywhere below means the plan's
// own buffers (stick block of k at kinfo[k].sbuf_off, P/Q blocks of k at k nproj nbnd_max).
struct HpsiWork {
  void* sbuf = nullptr;
  double2* P = nullptr;
  double2* Q = nullptr;
  void* part = nullptr;
  int64_t part_bytes = 0;
};
// launchers (fft.hip / gemm.hip); k0..k1 is the k range, psi/hpsi point at k0's first band
void launch_hpsi_local(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                       hipStream_t s, bool fp32, StageEvents* ev = nullptr,
                       const HpsiWork* wk = nullptr);
void launch_vplan(qm_hpsi_plan* p, const double* vloc_r, hipStream_t s);
// scatter + float64 inverse z transform of the slices into the plan's stick buffer
void launch_zinv_f64(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, hipStream_t s);
// Split-K scratch of the projector GEMM.  Calls that may run at the same time on different
// streams (Davidson lanes, which own disjoint k-points) each pass their own.
struct ProjScratch {
  void* part = nullptr;
  int64_t bytes = 0;
};
// parts: kNlAll the whole non-local term, kNlProject P = beta^H psi and Q = D P only,
// kNlExpand H psi += beta Q only (Q from an earlier kNlProject call)
enum { kNlAll = 0, kNlProject = 1, kNlExpand = 2 };
void launch_nonlocal(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                     hipStream_t s, qm_prec prec, StageEvents* ev = nullptr,
                     const ProjScratch* ps = nullptr, const HpsiWork* wk = nullptr,
                     int parts = kNlAll);
// H applied to every slice (local + non-local), in chunks of kMaxSlices.  At most one slice
// per k-point per call (stick buffer, P and Q are addressed per k).
// side_ok = false keeps the projection on s (callers that run several streams of their own).
void apply_h_slices(qm_hpsi_plan* p, const std::vector<KSlice>& sl, const void* psi, void* hpsi,
                    hipStream_t s, qm_prec prec, StageEvents* ev = nullptr,
                    const ProjScratch* ps = nullptr, const HpsiWork* wk = nullptr,
                    bool side_ok = true);
std::vector<KSlice> contiguous_slices(const qm_hpsi_plan* p, int k0, int k1, int nbnd);
// whether H applications in precision prec run the projection on the side stream, and the
// side stream's creation on first use
bool side_stream_wanted(const qm_hpsi_plan* p, qm_prec prec);
void ensure_side_stream(qm_hpsi_plan* p);
// qm_apply_h's graph path: replay (capturing on first use) the launch sequence of k (-1: all)
// at nbnd bands for these buffers in the plan's precision
void apply_graph(qm_hpsi_plan* p, int k, const void* psi, void* hpsi, int nbnd, hipStream_t s);
int xy_group_lanes(int nx);                       // lanes per line of the lane-group kernel, 0: none
// 1 two-pass with row scratch, 2 lane-group, 3 two-pass with the exchanges in the rows' slots
int xy_pick(const qm_hpsi_plan* p, int real_type);
// row stride (complex elements) of the two-pass xy-plane kernel's LDS plane for an N1 = n grid,
// and the kernel's LDS bytes (own: exchanges in the rows' own slots)
int xy_row_stride(int n, int nax_max, bool own);
size_t xy_lds_bytes(int n, int ns, size_t real_bytes, bool own);
void convert_beta(qm_hpsi_plan* p, qm_prec prec, hipStream_t s);
bool fft_len_supported(int n);
int fft_split_r1(int n);
int fft_split_r2(int n);

// complex GEMMs (c128 data, float64 arithmetic) used by the Davidson and the non-local term
// C[b](i,j) = alpha * sum_g conj(A[b](i,g)) B[b](j,g) + beta_c * C   (row-major, K = g contiguous)
struct GemmCN {
  const void* A; const void* B; void* C;
  int32_t M, N, K;
  int64_t lda, ldb, ldc;
};
// Y[b](j,g) = alpha * sum_i W[b](i,j) A[b](i,g) + beta_y * Y
struct GemmEX {
  const void* W; const void* A; void* Y;
  int32_t M, N, K;        // M = rows of Y (j), N = cols of Y (g), K = i
  int64_t ldw, lda, ldy;
  // optional [M] device list: row j of the product is W's column rows[j] and goes to Y's row
  // rows[j] (float64 operands only, lp = 0)
  const int32_t* rows = nullptr;
};
void zgemm_cn_batched(const std::vector<GemmCN>& probs, double alpha, double beta_c,
                      void* work, int64_t work_bytes, hipStream_t s, StageEvents* ev = nullptr,
                      int stage0 = 0, int lp = 0, int force_split = 0);
int64_t zgemm_cn_work_bytes(const std::vector<GemmCN>& probs);
void zgemm_ex_batched(const std::vector<GemmEX>& probs, double alpha, double beta_y,
                      hipStream_t s, int lp = 0);
// lp: 0 float64 operands, 1 float32 (A of CN / A of EX stored float32), 2 bfloat16 (same
// operands stored bfloat16); B of CN and W of EX are always c128 and converted on load.
// lp 3: every operand c128, rounded to float32 on load, float32 MFMA arithmetic, float64
// output (the subspace products of the reduced-precision phase of the Davidson ladder)
void convert_beta_lp(const void* beta64, void* out, int64_t n, int kind, hipStream_t s);

void plan_upload_davidson(qm_hpsi_plan* p);
void davidson_free(qm_hpsi_plan* p);
void density_free(qm_hpsi_plan* p);
void td_free(qm_hpsi_plan* p);
// unnormalised 3-D transform (sign +1: sum e^{+iG.r}; -1: e^{-iG.r}) of nbatch complex
// float64 grids [N1][N2][N3], consecutive in memory, in place
void fft3_batched(qm_hpsi_plan* p, double2* c, int64_t nbatch, int sign, hipStream_t s);
// y = x + z over the plan's grid (float64), on stream s
void grid_add(qm_hpsi_plan* p, const double* x, const double* z, double* y, hipStream_t s);
}  // namespace qm
