/*
 * qm_hpsi.h - C ABI of the MI355X (gfx950) plane-wave Kohn-Sham H|psi> and
 * block-Davidson library.
 *
 * Physics (Hartree atomic units; bohr, Ha).  At a k-point the Hamiltonian acts
 * on plane-wave coefficients c(G) of the G-sphere S_k as
 *
 *   (H c)(G) = 1/2 |k+G|^2 c(G)                                  kinetic, Sec. 4.3
 *            + sum_{G'} V(G-G') c(G')                             local, eq. KSHamMat
 *            + sum_ij beta_i(k+G) D_ij sum_{G'} conj(beta_j(k+G')) c(G')
 *                                                                 Kleinman-Bylander, Sec. 2.3
 *
 * with V(dG) = (1/N_r) sum_r V(r) e^{-i dG.r} the grid Fourier coefficient of
 * the local potential sampled on the FFT grid (dG modulo the grid).  The
 * library evaluates the local term as the paper's Sec. 4.3 describes (inverse
 * FFT of the sphere, multiply by V(r), forward FFT, keep the sphere), with
 * the stick-pruned 3-D transform of Sec. 4.3 ("Optimizing FFT operations for
 * G-Space"), and the non-local term as two complex GEMMs.  The eigensolver is
 * a block Davidson on H(k) (Sec. 5, 'dft' module: Davidson with H as a
 * Hermitian black box applied to trial blocks).
 *
 * Conventions shared by every entry point
 *  - Status codes only: no exception or abort crosses this ABI.  After a
 *    failure qm_last_error() returns a message; outputs are unspecified but
 *    the plan stays usable.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary memory.  The caller owns every buffer it passes.
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.
 *    qm_apply_h is asynchronous on it; the Davidson calls synchronise it once
 *    per iteration to read the convergence numbers.
 *  - Complex numbers are interleaved (re, im) float64 pairs ("c128").
 *  - Band blocks are [nk][nbnd][npw_k], k-blocks concatenated in k order,
 *    G in the caller's order given by the Miller list.
 *  - A plan is not thread-safe; use one plan per stream.
 */
#ifndef QM_HPSI_H
#define QM_HPSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QM_OK = 0,
  QM_E_ARG = 1,            /* invalid argument (shape, range, duplicate G, non-Hermitian D ...) */
  QM_E_SHAPE = 2,          /* grid or size not supported by the kernels */
  QM_E_HIP = 3,            /* a HIP runtime call failed */
  QM_E_NOMEM = 4,          /* device allocation failed */
  QM_E_NOT_SPD = 5,        /* Cholesky of a Gram matrix failed (linearly dependent block) */
  QM_E_NOT_CONVERGED = 6,  /* Davidson reached max_iter; eig/resnorm/stats are still filled */
  QM_E_NAN = 7,            /* NaN or Inf met in a residual norm or Rayleigh quotient */
  QM_E_STATE = 8           /* call not valid in the plan's current state */
} qm_status;

typedef enum {
  QM_PREC_FP64 = 0,   /* FFT, pointwise and projector GEMMs in float64 */
  QM_PREC_FP32 = 1,   /* FFT and pointwise in float32, projector GEMMs float32 (MFMA) */
  QM_PREC_MIXED = 2   /* FFT float32, projector GEMMs bfloat16 inputs with float32 accumulation */
} qm_prec;

typedef enum {
  QM_PRECOND_TETER = 0,  /* Teter-Payne-Allan K(x), x = (1/2|k+G|^2)/<X_n|T|X_n> */
  QM_PRECOND_MLP = 1     /* learned per-(G, band) gain network, Teter as fallback */
} qm_precond;

typedef struct qm_hpsi_plan qm_hpsi_plan;

/* k-point set and G-spheres (host memory, read during plan creation only).
 *  k_cart [nk][3]     k in cartesian bohr^-1.
 *  npw    [nk]        sphere size per k (>= 1).
 *  miller [sum npw][3] integer triples m, G = m1 b1 + m2 b2 + m3 b3, k blocks
 *                     concatenated; any order, no duplicates, 2|m_i| < N_i. */
typedef struct {
  int32_t nk;
  const double *k_cart;
  const int32_t *npw;
  const int32_t *miller;
} qm_kset;

/* Davidson options (host).  Zero-initialise and set what you need; zero
 * fields take the defaults in brackets. */
typedef struct {
  double tol;             /* convergence: max_n ||H x_n - theta_n x_n||_2 <= tol, Ha [1e-8] */
  int32_t max_iter;       /* iteration limit [200] */
  int32_t max_basis;      /* basis columns per k before a restart [4*nbnd] */
  int32_t precond;        /* qm_precond [QM_PRECOND_TETER] */
  int32_t restart;        /* qm_davidson_step: 1 = discard state and start from psi [0] */
  double switch_resid;    /* precision ladder: while max residual > switch_resid the
                             corrections are applied with the plan's reduced-precision
                             H (float32 FFTs; float32 or bfloat16 projector GEMMs with
                             float32 accumulation); below it, and for every reported
                             residual, float64.  It also switches when the max residual
                             has not fallen by 20% over four iterations.  Residual
                             norms, Rayleigh-Ritz, Cholesky orthonormalisation and the
                             projected eigenproblem stay float64 unless subspace_fp32.
                             0 = float64 throughout [0] */
  const void *mlp_weights;/* device float32 weights of the learned preconditioner
                             (layout in qm_mlp_*), required for QM_PRECOND_MLP */
  int32_t lanes;          /* qm_davidson_solve with k = -1: split the k-points into this
                             many contiguous groups and solve them at the same time, each
                             on its own stream and host thread (k-points are independent
                             problems, so results equal the one-group solve up to
                             rounding; the precision ladder switches per group).  0 or 1:
                             one group [0] */
  int32_t extra_bands;    /* buffer bands: the block holds nbnd + extra_bands Ritz vectors
                             (the extra ones start from a fixed pseudo-random block), all
                             of them corrected while unconverged, but only the nbnd lowest
                             decide convergence and are returned.  Keeps a degenerate level
                             cut by the band count from stalling the highest wanted bands.
                             Needs nbnd + extra_bands <= the plan's nbnd_max [0] */
  int32_t subspace_fp32;  /* 1: while the ladder runs H in reduced precision, the subspace
                             products (block Gram-Schmidt, CholQR Gram matrices and their
                             application, V^H (H V), Ritz vectors) round the float64 basis
                             to float32 and multiply in float32 MFMAs with float64 output.
                             0: they stay float64 [0] */
} qm_dav_opts;

/* Davidson statistics (host), filled by qm_davidson_solve. */
typedef struct {
  int32_t iterations;     /* Davidson iterations of the slowest k */
  int32_t converged;      /* 1 if every requested k converged */
  int64_t n_hpsi_bands;   /* band-applications of H (all precisions) */
  int64_t n_hpsi_bands_lowp; /* of which in reduced precision */
  double max_resnorm;     /* final max residual, Ha */
  double t_hpsi_ms;       /* device time in H application (HIP events) */
  double t_subspace_ms;   /* device time in orthonormalisation, V^H (H V) and Ritz vectors
                             with residuals (HIP events) */
  double t_eig_ms;        /* device time in the projected eigenproblem (HIP events); with
                             lanes, each of the three is the largest over the lanes */
  double t_total_ms;      /* wall time of the call */
  int64_t n_gs;           /* Gram-Schmidt orthogonalisations of a k-point's corrections */
  int64_t n_gs_second;    /* of which needed a second pass (some column kept less than
                             1/sqrt 2 of its norm in the first) */
} qm_dav_stats;

/* ------------------------------------------------------------------ plan */

/* Create an H(k) plan (Sec. 2.2 basis, Sec. 2.3 projectors, Sec. 4.3 grid).
 *  cell     host [9]  rows a_1, a_2, a_3 (bohr).
 *  grid     host [3]  FFT grid N1, N2, N3.  Supported: N1 == N2, and N1, N3 in
 *                     {12,16,18,20,24,27,28,30,32,36,40,45,48,54,56,60,64,72,80,
 *                      81,90,96,100,108,120,128,144}; else QM_E_SHAPE.
 *  ks       k-points and spheres (see qm_kset).
 *  nbnd_max largest band count any later call will pass (sizes the workspace).
 *  nproj    number of projectors (>= 0).
 *  vloc_r   device float64 [N1][N2][N3], C order; grid point j at sum_i (j_i/N_i) a_i; Ha.
 *  beta     device c128 [nk][nproj][npw_k], <k+G|beta_i> in the caller's G order.
 *  dmat     host float64 [nproj][nproj], real symmetric, Ha (D_ij of Sec. 2.3).
 *  prec     qm_prec used by qm_apply_h.
 *  stream   hipStream_t for the set-up copies.
 *  out      receives the plan.
 * The plan copies V, beta and D (in its working precisions) and owns its
 * workspace, so inputs may be freed after the call returns.  Environment:
 * QM_XY_MODE=1 forces the two-pass xy-plane kernel with a row scratch, QM_XY_MODE=2 the
 * lane-group kernel (grids of 20, 40 and 72 points along x), QM_XY_MODE=3 the two-pass kernel
 * with the x-row exchanges in the plane rows' own LDS slots (same transform, for
 * comparisons); otherwise qm_hpsi_plan_autotune picks one per precision.  For the Davidson calls on the plan
 * (same results up to the order of float64 additions, for comparisons):
 * QM_TRIDIAG_MODE=1 reduces the projected matrix in one workgroup per k-point, =2 with one
 * launch per Householder step on many workgroups (default: from a basis of 192 columns);
 * QM_CHOL_MODE=1 factors the CholQR Gram matrices in one workgroup per k-point, =2 blocked
 * on many workgroups (default: blocked up to 576 bands, the largest it supports). */
qm_status qm_hpsi_plan_create(const double cell[9], const int32_t grid[3], const qm_kset *ks,
                              int32_t nbnd_max, int32_t nproj, const double *vloc_r,
                              const void *beta, const double *dmat, qm_prec prec, void *stream,
                              qm_hpsi_plan **out);

void qm_hpsi_plan_destroy(qm_hpsi_plan *plan);

/* Message of the last failure on this plan (or of the last failed create
 * when plan is NULL); "" if none.  Valid until the next call on the plan. */
const char *qm_last_error(const qm_hpsi_plan *plan);

/* Change the precision qm_apply_h uses (reconverts beta; synchronous). */
qm_status qm_hpsi_plan_set_precision(qm_hpsi_plan *plan, qm_prec prec, void *stream);

/* Launch mode of qm_apply_h: enable = 1 (default) replays a hipGraph captured once per
 * (k, nbnd, psi, hpsi, precision) - up to 8 are cached per plan, least recently used
 * evicted - so repeated applications cost one graph launch; enable = 0 launches the
 * kernels one by one.  Changing the mode drops the cached graphs. */
qm_status qm_hpsi_plan_set_graphs(qm_hpsi_plan *plan, int32_t enable);

/* Autotune for nbnd bands, timing the candidates with HIP events on stream: the split-K
 * count of the projector GEMM in every precision, the xy-plane FFT kernel (two-pass or
 * lane-group, where the grid has both) of the float64 and float32 local parts, and, per
 * precision, whether qm_apply_h runs the projection beta^H psi and D on a side stream of
 * the plan, concurrently with the local part (the default before tuning; the environment
 * variable QM_OVERLAP=0 or 1 fixes it at plan creation).  The choices are kept in the plan.  If the environment variable QM_AUTOTUNE_CACHE names a
 * file, choices are read from and written to it (one JSON object keyed by problem shape).
 * Synchronous. */
qm_status qm_hpsi_plan_autotune(qm_hpsi_plan *plan, int32_t nbnd, void *stream);

/* ------------------------------------------------------------------ H|psi> */

/* hpsi = H(k) psi for a block of bands (eq. KSHamMat + KB term).
 *  k      k index, or -1 for every k of the plan in one batched launch sequence.
 *  psi    device c128, [nbnd][npw_k] for one k, [nk][nbnd][npw_k] for k = -1.
 *  hpsi   device c128, same layout; must not alias psi.
 *  nbnd   1 <= nbnd <= nbnd_max.
 * Precision per qm_hpsi_plan_create/set_precision; psi and hpsi are c128
 * whatever the precision. */
qm_status qm_apply_h(qm_hpsi_plan *plan, int32_t k, const void *psi, void *hpsi, int32_t nbnd,
                     void *stream);

/* qm_apply_h with HIP events recorded on stream between its kernels; synchronises
 * the stream and writes the duration of each stage in milliseconds to times_ms
 * (host float64 [QM_NSTAGES]): 0 scatter + z inverse, 1 xy planes (y/x transforms
 * and V), 2 z forward + gather + kinetic, 3 projection GEMM, 4 split-K reduction,
 * 5 D application, 6 expansion GEMM.  Stages that do not run report 0. */
#define QM_NSTAGES 7
qm_status qm_apply_h_timed(qm_hpsi_plan *plan, int32_t k, const void *psi, void *hpsi,
                           int32_t nbnd, double *times_ms, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc.  The same H|psi> as qm_apply_h (same arguments,
 * layouts, precision and results to rounding), launched kernel by kernel on stream, with no
 * device or pinned allocation and no graph of its own.  Its working memory (stick buffer,
 * projections, split-K partial sums) is one static device array of QM_NOALLOC_SCRATCH_MIB
 * MiB, of which each GPU the library runs on holds its own copy until the process ends, in
 * place of the plan's own buffers; k-points are applied one after the other, their bands in
 * chunks that fit in the array.  Every call on one GPU shares that GPU's array: calls whose
 * work may overlap in time on one GPU (different streams, or different host threads) race
 * and give wrong results - serialise them.  Errors: QM_E_ARG as for qm_apply_h, and when one
 * band of a k-point needs more working memory than the array holds (sizes below); QM_E_STATE
 * when the plan's precision needs the reduced-precision copy of beta and it has
 * not been built (call qm_hpsi_plan_set_precision, which builds it, before capturing).
 * Per band of k the array must hold nstick_k * N3 * (16 in float64, 8 otherwise) bytes of
 * sticks plus 3 * nproj * 16 bytes: the 216-atom cell at 108^3 needs 3.9 MB per band in
 * float64, so 64 MiB processes 17 bands at a time. */
#define QM_NOALLOC_SCRATCH_MIB 64
qm_status qm_apply_h_noalloc(qm_hpsi_plan *plan, int32_t k, const void *psi, void *hpsi,
                             int32_t nbnd, void *stream);

/* ------------------------------------------------------------------ Davidson */

/* One block-Davidson iteration (Sec. 5, 'dft' module: the Davidson "with overlap" that
 * only needs H applied to blocks of trial vectors; the algorithm's details are not given
 * there, this is the block Davidson of Davidson 1975 and Liu 1978 with an explicitly
 * orthonormalised basis) on k (or all k with k = -1), state kept in the plan.
 * First call (or opts->restart = 1): orthonormalise psi, apply H, Rayleigh-Ritz.
 * Later calls: corrections for unconverged bands, restart if the basis is full,
 * orthonormalise, apply H, Rayleigh-Ritz.  Every call writes the current Ritz
 * vectors to psi (device c128, layout as qm_apply_h), Ritz values to eig and
 * residual norms to resnorm (host float64 [nk_sel][nbnd], ascending per k),
 * and the number of unconverged (k, band) pairs to *n_unconverged (host). */
qm_status qm_davidson_step(qm_hpsi_plan *plan, int32_t k, void *psi, double *eig,
                           double *resnorm, int32_t nbnd, const qm_dav_opts *opts,
                           int32_t *n_unconverged, void *stream);

/* Iterate qm_davidson_step (same passage) from the start block psi until every
 * residual norm is <= opts->tol or max_iter is reached (then QM_E_NOT_CONVERGED with
 * all outputs filled).  psi receives the Ritz vectors; stats may be NULL.  Unlike a
 * sequence of qm_davidson_step calls, the iterations in between form Ritz vectors and
 * residuals only for the bands being corrected (as the Quantum ESPRESSO Davidson forms
 * residuals only for its unconverged bands); every band's vector and residual is formed
 * from the final Ritz pairs before a convergence verdict and before the return.
 * Errors: QM_E_NOT_SPD when a block to be orthonormalised is linearly dependent (for
 * example two equal start vectors), QM_E_NAN when a residual norm is not finite; in both
 * cases the Davidson state is dropped and the plan stays usable for qm_apply_h. */
qm_status qm_davidson_solve(qm_hpsi_plan *plan, int32_t k, void *psi, double *eig,
                            double *resnorm, int32_t nbnd, const qm_dav_opts *opts,
                            qm_dav_stats *stats, void *stream);

/* ------------------------------------------------------------------ learned preconditioner */

/* Per-(G, band) network with shared weights (an extension of the paper's
 * Davidson; not in the paper).  Inputs f = [x, log(1 + x), (theta_n - T_n)/T_n,
 * |r_n(G)| sqrt(npw_k)/||r_n||, T(G)] with T(G) = 1/2|k+G|^2 (Ha), T_n the
 * band kinetic energy <x_n|T|x_n> and x = T(G)/T_n; hidden layer 128 with SiLU;
 * two outputs o; complex gain g = K(x) [exp(2 tanh o_0) + 0.5 i tanh o_1] with
 * K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4) (Teter,
 * Payne and Allan); correction t_n(G) = g r_n(G).  A zero output layer gives
 * the Teter preconditioner exactly; the real factor stays within [e^-2, e^2].
 * Weights: one device float32 buffer of QM_MLP_NPARAM numbers laid out
 * W1[128][5], b1[128], W2[2][128], b2[2]. */
#define QM_MLP_NIN 5
#define QM_MLP_NHID 128
#define QM_MLP_NPARAM (128 * 5 + 128 + 2 * 128 + 2)

/* Gains for n feature rows: feat device float32 [n][5] -> gain device float32 [n][2]. */
qm_status qm_mlp_forward(const float *weights, const float *feat, float *gain, int64_t n,
                         void *stream);

/* Loss and gradient of the per-band cosine loss
 *   L = (1/nbands) sum_b [1 - |<t_b, d_b>|^2 / (||t_b||^2 ||d_b||^2)],  t = g r,
 * rows of band b are [band_ptr[b], band_ptr[b+1]).  feat [n][5], resid [n][2] (r),
 * target [n][2] (d), band_ptr int32 [nbands+1] and grad [QM_MLP_NPARAM] are device
 * arrays; *loss is written on the host.  Synchronises the stream. */
qm_status qm_mlp_loss_grad(const float *weights, const float *feat, const float *resid,
                           const float *target, const int32_t *band_ptr, int32_t nbands,
                           float *grad, double *loss, void *stream);

/* One Adam step (Kingma and Ba) on the weights with moment buffers m, v (device
 * float32 [QM_MLP_NPARAM]); t is the 1-based step count. */
qm_status qm_mlp_adam(float *weights, const float *grad, float *m, float *v, int32_t t,
                      float lr, float beta1, float beta2, float eps, void *stream);

/* Training rows from the current Davidson state of the plan (after a
 * qm_davidson_step without buffer bands, else QM_E_STATE): for every unconverged
 * (k, band) of that state, npw_k rows
 * of features (as above), residual r_n(G) and target d_n(G) = P x_n/||P x_n|| - x_n,
 * with P the projector onto the converged eigenvectors x_star (device c128,
 * layout as psi) whose eigenvalues eig_star (host [nk_sel][nbnd]) lie within
 * cluster_tol (Ha; 0 = 1e-6) of eig_star[n].  Outputs are device arrays with
 * capacity cap_rows rows / cap_bands bands; *nrows and *nbands (host) receive
 * the counts and band_ptr (device int32 [nbands+1]) the row offsets. */
qm_status qm_dav_training_pairs(qm_hpsi_plan *plan, const void *x_star, const double *eig_star,
                                double cluster_tol, float *feat, float *resid, float *target,
                                int32_t *band_ptr, int64_t cap_rows, int32_t cap_bands,
                                int64_t *nrows, int32_t *nbands, void *stream);

/* ------------------------------------------------------------------ density, Hartree, SCF */

/* Electron density (Sec. 2.1: n(r) = sum_i f_i |psi_i(r)|^2 over the occupied states) of
 * the band block psi on the plan's FFT grid:
 *   rho(r) = sum_k weights[k] sum_n occ[k][n] |psi_kn(r)|^2,
 *   psi_kn(r) = Omega^-1/2 sum_G c_kn(G) e^{i(k+G).r},
 * so unit-norm bands integrate to one over the cell and rho integrates to
 * sum_k weights[k] sum_n occ[k][n] (occ = 2 for a doubly occupied band, weights summing to 1).
 *  k        k index, or -1 for every k of the plan (at most 32).
 *  psi      device c128 [nk_sel][nbnd][npw_k] (as qm_apply_h).
 *  weights  host float64 [nk_sel] k-point weights; occ host float64 [nk_sel][nbnd].
 *  rho      device float64 [N1][N2][N3], C order, grid point j at sum_i (j_i/N_i) a_i; e/bohr^3.
 * Float64 whatever the plan's precision; deterministic (groups of bands are summed in a
 * fixed order).  Uses the plan's stick buffer: not concurrent with other calls on the plan. */
qm_status qm_density(qm_hpsi_plan *plan, int32_t k, const void *psi, int32_t nbnd,
                     const double *weights, const double *occ, double *rho, void *stream);

/* Hartree potential (Sec. 2.1, the Hartree term of V_aux: the classical potential of the
 * charge density), the periodic solution of Poisson's equation in Hartree units:
 *   V_H(G) = 4 pi n(G) / |G|^2 for G != 0, V_H(G = 0) = 0,
 *   n(G) = (1/N_r) sum_r rho(r) e^{-iG.r}, G = m.B with m in the centred range of the grid.
 *  rho, vh    device float64 [N1][N2][N3] (layout as qm_density); vh must not alias rho.
 *  e_hartree  host, may be NULL: 1/2 integral V_H rho = 1/2 (Omega/N_r) sum_r V_H rho (Ha).
 * Synchronises the stream when e_hartree is requested. */
qm_status qm_hartree(qm_hpsi_plan *plan, const double *rho, double *vh, double *e_hartree,
                     void *stream);

/* Replace the plan's local potential V(r) (device float64 [N1][N2][N3], Ha, layout as in
 * qm_hpsi_plan_create); later H applications (and captured graphs) use the new values. */
qm_status qm_hpsi_plan_set_vloc(qm_hpsi_plan *plan, const double *vloc_r, void *stream);

/* Hartree-only SCF options (host); zero fields take the defaults in brackets. */
typedef struct {
  double alpha;           /* linear mixing n <- n + alpha (n_out - n) [0.7] */
  double tol;             /* stop when ||n_out - n||_2 over the cell <= tol (electrons/bohr^1.5) [1e-9] */
  int32_t max_iter;       /* SCF iterations [100] */
  int32_t pad;
  qm_dav_opts dav;        /* options of the Davidson solve of every iteration [tol 1e-10] */
} qm_scf_opts;

typedef struct {
  int32_t iterations;     /* SCF iterations done */
  int32_t converged;      /* 1 if the density residual reached tol */
  int64_t dav_iterations; /* Davidson iterations summed over the SCF iterations */
  int64_t n_hpsi_bands;   /* band-applications of H summed over the SCF iterations */
  double residual;        /* final ||n_out - n||_2 */
  double e_hartree;       /* Hartree energy of the final density, Ha */
  double t_total_ms;      /* wall time */
} qm_scf_stats;

/* Hartree-only self-consistent field (Sec. 2.1, the cycle n -> V -> {psi} -> n_out, mixed until
 * n_out = n; exchange-correlation left out): starting from the uniform density, every
 * iteration sets V = vext + V_H[n] (qm_hartree, qm_hpsi_plan_set_vloc), solves the Davidson
 * for nbnd bands of every k from the previous iteration's vectors (qm_davidson_solve), forms
 * n_out from the nocc lowest bands of every k doubly occupied with the k weights (qm_density)
 * and mixes linearly (the paper's code uses Broyden mixing; linear mixing here).
 *  vext      device float64 [N1][N2][N3] external (ionic) potential, Ha.
 *  kweights  host float64 [nk]; the electron count is 2 nocc sum_k kweights[k].
 *  psi       device c128 [nk][nbnd][npw_k]: in, start vectors; out, the last Davidson vectors.
 *  eig       host float64 [nk][nbnd]: last Ritz values.  rho, vh: device float64 grids, out:
 *            the final density and its Hartree potential.
 * The plan keeps the last iteration's V.  QM_E_NOT_CONVERGED (outputs filled) when max_iter is
 * reached; Davidson errors are passed on. */
qm_status qm_scf_hartree(qm_hpsi_plan *plan, const double *vext_r, const double *kweights,
                         int32_t nocc, void *psi, int32_t nbnd, const qm_scf_opts *opts,
                         double *eig, double *rho, double *vh, qm_scf_stats *stats, void *stream);

/* ------------------------------------------------------------------ real-time propagation */

/* psi_out = sum_{r=0}^{order} (-i dt)^r / r! H^r psi_in (Sec. 5, 'tddft' module: the Taylor
 * expansion of exp(-i dt H) truncated at order k), with the plan's H and precision; the
 * series is built term by term, t_r = (-i dt / r) H t_{r-1}.
 *  k             k index or -1 for every k (layouts as qm_apply_h); psi_in may equal psi_out.
 *  dt            time step in Hartree atomic units (hbar / Ha); 1 <= order <= 64.
 * Work buffers (4 band blocks of nbnd_max bands over every k, 3 grids) are allocated in the
 * plan on first use. */
qm_status qm_expm_taylor(qm_hpsi_plan *plan, int32_t k, const void *psi_in, void *psi_out,
                         int32_t nbnd, double dt, int32_t order, void *stream);

/* nsteps steps of the enforced-time-reversal-symmetry propagator (Sec. 5, 'tddft' module, prop;
 * the time-dependent Kohn-Sham equations of Sec. 2.4) for the Hartree-only model
 * H[psi] = T + V_ext + V_H[n(psi)] + V_NL, n(psi) = sum_k kweights[k] sum_n occ[k][n] |psi_kn|^2:
 *   psi_bar   = exp(-i dt H[psi_n]) psi_n,
 *   psi_{n+1} = exp(-i dt H[psi_bar] / 2) exp(-i dt H[psi_n] / 2) psi_n,
 * each exponential by qm_expm_taylor with the given order.  psi (device c128 [nk][nbnd][npw_k])
 * is advanced in place; the plan's V is left at V_ext + V_H[n(psi_bar)] of the last step. */
qm_status qm_td_etrs(qm_hpsi_plan *plan, const double *vext_r, const double *kweights,
                     const double *occ, void *psi, int32_t nbnd, double dt, int32_t order,
                     int32_t nsteps, void *stream);

/* ------------------------------------------------------------------ GW matrix elements */

/* Plane-wave matrix elements of the GW polarizability (Sec. 5, 'gw' module, Epsilon matrix
 * elements):  M[n][n'][g] = <n k+q| e^{i(q+G_g).r} |n' k> = sum_G' conj(c_{n,kq}(G_g + G'))
 * c_{n',k}(G'), computed as the paper describes: both band sets to real space (inverse FFT),
 * the product conj(u_{n,k+q}(r)) u_{n',k}(r), its inverse FFT (with 1/N_r) read at G_g.
 *  kq, k     plan k-point indices of k+q and of k (their spheres hold the coefficients).
 *  psi_kq    device c128 [nb1][npw_kq]; psi_k device c128 [nb2][npw_k].
 *  miller_g  host int32 [ng][3], 2|m_i| < N_i; mtx device c128 [nb1][nb2][ng].
 * The grid must hold the products without aliasing (components up to the sum of the two
 * spheres' radii).  Float64; allocates (nb1 + 2 nb2) full complex grids for the call;
 * synchronises the stream. */
qm_status qm_mtxel(qm_hpsi_plan *plan, int32_t kq, const void *psi_kq, int32_t nb1, int32_t k,
                   const void *psi_k, int32_t nb2, const int32_t *miller_g, int32_t ng, void *mtx,
                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QM_HPSI_H */
