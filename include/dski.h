/*
 * dski.h -- C ABI of the MI355X (gfx950) D-SKI library: GP regression with
 * derivative observations under structured kernel interpolation.
 *
 * The operator (Sec. 3.1, "D-SKI"):  for n points x_i in R^d with values and
 * gradients observed, the N x N matrix, N = n(d+1),
 *
 *     K~ = [W; dW_1; ...; dW_d] K_UU [W; dW_1; ...; dW_d]^T + D,
 *
 * where W holds convolution interpolation weights onto a uniform grid U
 * (Keys' cubic kernel, a = -1/2, or the quintic kernel of Meijering et al.,
 * Sec. 3.1), dW_p their derivatives along axis p, K_UU the kernel on the grid
 * (SE, App. A: a Kronecker product of symmetric Toeplitz factors applied by
 * FFT over circulant embeddings, Sec. 2; or the thin-plate spline kernel of
 * App. A: a multi-level Toeplitz matrix applied by a d-dimensional circulant
 * embedding), and D = diag(sigma_f^2 1_n, sigma_g^2 1_{nd}) the value /
 * gradient noise.
 * On top of it: truncated pivoted Cholesky preconditioning (Sec. 3.3),
 * preconditioned CG, stochastic Lanczos quadrature for log det (Sec. 2), and
 * the log marginal likelihood eq. (1) with its hyper-parameter gradient.
 *
 * Conventions, for every call:
 *  - Pointers are DEVICE pointers unless the name ends in _host.
 *  - Ownership: the caller allocates and frees every buffer it passes.  The
 *    library owns only what sits behind the opaque handles (plan, precond)
 *    and releases it in the matching *_destroy.  No call keeps a caller
 *    pointer after it returns (X is copied into the plan).
 *  - Errors: every call returns a dski_status.  0 = success; > 0 = finished
 *    with a warning, outputs valid; < 0 = error, outputs unspecified but no
 *    memory is leaked.  dski_last_error() returns the message of the last
 *    failure on the calling thread.  No exception or abort crosses the ABI.
 *  - Streams: device work is enqueued on `stream` (0 = the null stream).
 *    Calls with *_host outputs synchronise `stream` before returning.  A plan
 *    (and its preconditioners) must not be used by two calls at once.
 *  - Layout of an N-vector: block-major [f(x_1..x_n); d_1 f(x_1..x_n); ...;
 *    d_d f(x_1..x_n)] (the block form of Sec. 3.1), points in USER order.
 *    A block of R vectors is column-major with leading dimension ld >= N.
 *  - Hyper-parameters are natural logs: log ell_1..log ell_d, log s,
 *    log sigma_f, log sigma_g (this order wherever a gradient is returned).
 *  - Arithmetic: N-vectors are stored in FP32; interpolation, K_UU, dot
 *    products and all scalars are computed in FP64.  Every call that takes
 *    N-vectors has an *_f64 twin with FP64 storage (same semantics), for
 *    problems whose conditioning needs it.
 */
#ifndef DSKI_H
#define DSKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSKI_OK = 0,
  DSKI_NOT_CONVERGED = 1,      /* PCG hit max_iter; last iterate returned          */
  DSKI_RANK_TRUNCATED = 2,     /* pivoted Cholesky stopped before rank k           */
  DSKI_EINVAL = -1,            /* bad argument, shape, or non-finite input         */
  DSKI_ENOMEM = -2,            /* device allocation failed                         */
  DSKI_EHIP = -3,              /* a HIP runtime call failed                        */
  DSKI_EBREAKDOWN = -4,        /* p^T K~ p <= 0 or r^T M^{-1} r < 0 in PCG         */
  DSKI_ENOTSUP = -5            /* configuration the library does not support       */
} dski_status;

typedef struct dski_plan_s* dski_plan;       /* points, grid, tile order, spectra  */
typedef struct dski_precond_s* dski_precond; /* pivots, factor, log det M          */
typedef void* dski_stream;                   /* a hipStream_t                      */

/* Message of the last error on this thread ("" if none). */
const char* dski_last_error(void);

/* Build version string (library build identifier). */
const char* dski_version(void);

/* Interpolation kernels of the D-SKI weights (Sec. 3.1). */
#define DSKI_INTERP_CUBIC 0    /* Keys' cubic convolution (a = -1/2), 4 nodes per axis      */
#define DSKI_INTERP_QUINTIC 1  /* the quintic convolution kernel of Meijering et al. (1999):
                                * 6 nodes per axis, C^2, reproduces quartics               */

/* Create a D-SKI plan for n points in d = 1..3 dimensions (Sec. 3.1).
 *   X        : n x d row-major FP64 point coordinates (device).
 *   grid_m   : d grid sizes m_p >= S (host), S = 4 (cubic) or 6 (quintic)
 *              stencil nodes per axis.
 *   lo, hi   : data box per axis (host, FP64).  The grid is h_p =
 *              (hi_p - lo_p)/(m_p - S + 1), first node lo_p - (S/2 - 1) h_p,
 *              so every point of the box has its S-node stencil inside the
 *              grid.  NULL for both = the bounding box of X.
 *   interp   : DSKI_INTERP_CUBIC or DSKI_INTERP_QUINTIC.
 * Setup (per data set, independent of the hyper-parameters): cell index and
 * offsets of every point, points sorted by cell ("tile order"), per-axis FFT
 * sizes.  Points outside the box give DSKI_EINVAL.  Hyper-parameters start at
 * log ell = log s = 0, log sigma = log 0.1; call dski_set_hypers. */
dski_status dski_plan_create(dski_plan* out, int n, int d, const double* X,
                             const int* grid_m_host, const double* lo_host,
                             const double* hi_host, int interp, dski_stream stream);
dski_status dski_plan_destroy(dski_plan plan);

/* D-SKIP operator (Sec. 3.2) for higher d: the kernel matrix of the product SE
 * kernel with derivatives as the Hadamard product over axes of the 1-D D-SKI
 * factors Khat_p (grid of m_1d nodes on [lo_p, hi_p]; the (a, b) block uses
 * derivative weights on the side whose block is the derivative along p), each
 * compressed by rank_r Lanczos steps with full re-orthogonalisation from the
 * normalised Rademacher column `node` of `seed` (leaves 0..d-1), combined by a
 * binary tree (pairs (0,1), (2,3), ..., internal nodes recompressed by rank_r
 * Lanczos steps and numbered on from d; the root is the exact Hadamard product of
 * its two children), applied by the SKIP reduction (A o B) v = rowsum((Qa Ta) o
 * ((Qb Tb) C^T)), C = Qa^T diag(v) Qb.
 * X: device, n x d row-major FP64 (copied); 2 <= d <= 64; m_1d >= 4;
 * 1 <= rank_r <= 64; lo_host/hi_host: d entries each, or both NULL for the
 * bounding box; log_ell_host: d length scales (the factors depend on them; the
 * build runs here and again in dski_set_hypers when a length scale changes).
 * The plan works with every solver call (pivchol_build, pcg_solve, slq_logdet,
 * dski_mvm*); dski_mvm_dtheta supports s and the noise levels; mll_and_grad and
 * dski_mvm_stage return DSKI_ENOTSUP.  Tile order is the identity.
 * Errors: DSKI_EINVAL on bad arguments or points outside the box. */
dski_status dskip_plan_create(dski_plan* out, int n, int d, const double* X, int m_1d,
                              int rank_r, uint64_t seed, const double* lo_host,
                              const double* hi_host, const double* log_ell_host,
                              dski_stream stream);

/* D-SKIP plan facts: grid size, requested rank, and the number of Lanczos
 * vectors kept in the two root factors (< rank_r after an early breakdown). */
dski_status dskip_plan_info(dski_plan plan, int* m_1d, int* rank_r, int* k_a, int* k_b);

/* Plan geometry: n, d, N, total grid nodes, and per axis (d entries each)
 * the grid size, circulant FFT length, grid spacing and first node. */
dski_status dski_plan_info(dski_plan plan, int* n, int* d, int* N, long long* grid_nodes,
                           int* m_host, int* fft_len_host, double* h_host, double* lo_host);

/* Set hyper-parameters (natural logs; log_ell has d entries).  Recomputes the
 * circulant eigenvalues of every Toeplitz factor of K_UU on the device. */
dski_status dski_set_hypers(dski_plan plan, const double* log_ell_host, double log_s,
                            double log_sigma_f, double log_sigma_g, dski_stream stream);

/* Y = K~ V for R vectors (user order).  V and Y must not overlap. */
dski_status dski_mvm(dski_plan plan, int R, const float* V, int ldv, float* Y, int ldy,
                     dski_stream stream);
dski_status dski_mvm_f64(dski_plan plan, int R, const double* V, int ldv, double* Y, int ldy,
                         dski_stream stream);

/* Y = (d K~ / d theta_which) V, which = 0..d+2 in hyper-parameter order
 * (derivative of the approximate kernel, Sec. 3: weights fixed). */
dski_status dski_mvm_dtheta(dski_plan plan, int which, int R, const float* V, int ldv,
                            float* Y, int ldy, dski_stream stream);
dski_status dski_mvm_dtheta_f64(dski_plan plan, int which, int R, const double* V, int ldv,
                                double* Y, int ldy, dski_stream stream);

/* Posterior mean at test points (Sec. 1: O(1) prediction per test point).  With
 * alpha = K~^{-1} y (from pcg_solve_f64 or pcg_solve), the posterior mean of
 * the test observations [f(x*); grad f(x*)] is K_{*X} alpha, which under D-SKI
 * (Sec. 3.1) is S_* K_UU S^T alpha.
 * dski_predict_grid forms the grid vector g = K_UU S^T alpha once: alpha is an
 *   N-vector in user order (device, FP64, block-major as every N-vector), g
 *   receives M = prod m_p doubles (device, grid in C order).
 * dski_predict interpolates g at n_test points X_test (device, n_test x d
 *   row-major, FP64; each inside the interpolation box of the plan) on their
 *   cubic stencils: out (device, n_test x (d + 1) row-major) receives per
 *   point [mean f, mean df/dx_1, ..., mean df/dx_d].  It synchronizes `stream`;
 *   DSKI_EINVAL if a test point lies outside the box (out then holds the
 *   clamped points' values).  D-SKI plans only (DSKI_ENOTSUP for D-SKIP). */
dski_status dski_predict_grid(dski_plan plan, const double* alpha, double* g, dski_stream stream);
dski_status dski_predict(dski_plan plan, const double* g, int n_test, const double* X_test, double* out,
                         dski_stream stream);

/* Predictive variance of f at test points (Sec. 4.4, first approach): the
 * pivoted-Cholesky preconditioner M = D + L L^T stands in for K~,
 *   v^(x) = k(x, x) - K_{xX} M^{-1} K_{Xx},
 * with k(x, x) = w_x^T K_UU w_x and K_{Xx} = S K_UU w_x those of the D-SKI
 * kernel (w_x the value stencil of x).  Since L L^T <= K, v^ <= v (equality
 * at full rank).  pc must be built on `plan` (dski_precond_build).  X_test:
 * device, n_test x d row-major FP64, inside the interpolation box; out:
 * device, n_test FP64.  Points go through in batches of up to 128 (one grid
 * column each); the call uses the plan's scratch buffers and synchronizes
 * `stream`.  DSKI_EINVAL for a point outside the box, DSKI_ENOTSUP for D-SKIP. */
dski_status dski_predict_var(dski_plan plan, dski_precond pc, int n_test, const double* X_test,
                             double* out, dski_stream stream);

/* Randomized predictive variance of f at test points (Sec. 4.4, second
 * approach): the pivoted-Cholesky estimate v^ of dski_predict_var as control
 * variate for a diagonal estimator over the test points,
 *   v = v^ - (1/R) sum_r z_r .* (K_{X'X} (K~^{-1} - M^{-1}) K_{XX'} z_r),
 * unbiased for v when E[z z^T] = I (Rademacher or Gaussian probes; the n_test
 * probes sqrt(n_test) e_j give the exact variance).  Per chunk of up to 32
 * probes: test stencils weighted by z scattered onto the grid, K_UU, gather
 * (K_{XX'} z), block PCG with pc to relative residual tol (FP64 vectors) and
 * M^{-1}, scatter of the difference, K_UU, stencil reads at the test points.
 * Zp: device, R x n_test row-major FP64 (row r = probe r).  X_test, out as for
 * dski_predict_var.  Allocates a work buffer of 3 N min(R, 32) + n_test doubles per call and
 * synchronizes `stream`.  DSKI_NOT_CONVERGED if a solve reached max_iter (out
 * then uses its last iterate), DSKI_EINVAL for a point outside the box,
 * DSKI_ENOTSUP for D-SKIP.  The probe scatter adds overlapping stencils with
 * atomics, so repeated calls can differ in the last bits. */
dski_status dski_predict_var_probes(dski_plan plan, dski_precond pc, int n_test, const double* X_test,
                                    int R, const double* Zp, double tol, int max_iter, double* out,
                                    dski_stream stream);

/* Active-subspace dimension reduction (Sec. 3.4).  C = (1/n) sum_i g_i g_i^T
 * over n gradient samples g_i in R^D; P holds its d dominant eigenvectors, and
 * a GP on the reduced points u_i = P^T x_i with gradients P^T g_i uses the
 * kernel k(P^T x, P^T x').
 * dski_active_subspace: G device FP64, component p of sample i at
 *   G[p*ldg + i] (the derivative blocks of an N-vector, ldg >= n); 1 <= d <=
 *   D <= 64.  P_host (D x d row-major) receives the eigenvectors as columns,
 *   each signed so that its entry of largest magnitude is positive; eig_host
 *   (D) all eigenvalues of C in decreasing order.  C is formed on the GPU
 *   (per-block partials summed on the host in block order), then a cyclic
 *   Jacobi eigen-decomposition runs on the host.  Synchronizes `stream`;
 *   DSKI_ENOTSUP for D > 64.
 * dski_active_project: X device n x D row-major, P device D x d row-major;
 *   U (device, n x d row-major) receives P^T x_i; if G is given (layout as
 *   above), Gu (device, d blocks of n) receives P^T g_i, so that the values
 *   followed by Gu form the reduced N-vector.  G and Gu are both NULL or both
 *   set.  Asynchronous on `stream`. */
dski_status dski_active_subspace(int n, int D, const double* G, int ldg, int d, double* P_host,
                                 double* eig_host, dski_stream stream);
dski_status dski_active_project(int n, int D, int d, const double* X, const double* G, int ldg,
                                const double* P, double* U, double* Gu, dski_stream stream);

/* Expected-improvement acquisition over n_cand candidates (Sec. 4.4, Alg. 1),
 * for minimisation: EI = E[max(f_best - xi - Y, 0)] with Y ~ N(mu, sigma^2),
 * sigma = sqrt(max(var, 0)) (a negative variance estimate counts as zero).
 * mu: device, mean of candidate j at mu[j*mu_stride] (mu_stride = d + 1 reads
 * the value column of dski_predict's output); var: device, n_cand; xi >= 0 an
 * exploration margin; ei: device, n_cand (may be NULL) receives every EI.
 * best_idx_host / best_ei_host receive the largest EI and its candidate (the
 * first on a tie; candidates whose EI is not finite are never chosen).
 * Synchronizes `stream`; DSKI_EINVAL if no EI is finite. */
dski_status dski_expected_improvement(int n_cand, const double* mu, int mu_stride, const double* var,
                                      double f_best, double xi, double* ei, int* best_idx_host,
                                      double* best_ei_host, dski_stream stream);

/* Tile order: the internal point order (sorted by interpolation cell) that the
 * solvers use.  dir = +1: user -> tile, dir = -1: tile -> user.  perm_host (n
 * ints, may be NULL) receives, for tile position k, the user index. */
dski_status dski_permute(dski_plan plan, int dir, int R, const float* in, int ldi, float* out,
                         int ldo, dski_stream stream);
dski_status dski_permute_f64(dski_plan plan, int dir, int R, const double* in, int ldi,
                             double* out, int ldo, dski_stream stream);
dski_status dski_tile_order(dski_plan plan, int* perm_host);

/* Y = K~ V on tile-ordered vectors (the product the PCG iterations run). */
dski_status dski_mvm_tiled(dski_plan plan, int R, const float* V, int ldv, float* Y, int ldy,
                           dski_stream stream);
dski_status dski_mvm_tiled_f64(dski_plan plan, int R, const double* V, int ldv, double* Y,
                               int ldy, dski_stream stream);

/* dski_mvm_tiled for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the grid workspace (M x R doubles, M = grid
 * nodes) in a fixed 16 MiB device array of the library instead of the plan's
 * growable buffer.  No call allocates or frees device memory.  Limits:
 * M * R <= 2,097,152 (e.g. R <= 52 on a 200 x 200 grid, R <= 18 on 48^3);
 * beyond that DSKI_EINVAL; D-SKIP plans DSKI_ENOTSUP.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (two streams, two host threads) race and must be ordered
 * by the caller.  The array is held on each GPU until the process ends. */
dski_status dski_mvm_tiled_noalloc(dski_plan plan, int R, const float* V, int ldv, float* Y,
                                   int ldy, dski_stream stream);

/* One stage of dski_mvm_tiled, for profiling and custom pipelines: stage 0 =
 * scatter G = S^T V into the plan's FP64 grid workspace (M x R), stage 1 =
 * G <- K_UU G in place (FFT, one launch per axis), stage 2 = gather
 * Y = S G + D V.  Stages 1 and 2 use the grid left by the last stage 0 of at
 * least R columns on this plan; any other call may overwrite it. */
dski_status dski_mvm_stage(dski_plan plan, int stage, int R, const float* V, int ldv, float* Y,
                           int ldy, dski_stream stream);

/* Times the interchangeable kernel variants for R right-hand sides on this
 * plan's shape (scatter: LDS node tiles with the base number of columns per
 * work-group / direct one column per thread / direct two columns per thread /
 * LDS node tiles with 1.5, 2 and 5 times the base columns / in 3-D, node tiles
 * whose work is split into (node, first-axis cell) items ordered by length;
 * gather: 2 / 1 / 4 columns per thread; K_UU factor of each axis: circulant
 * FFT / dense Toeplitz product on the FP64 matrix cores) and keeps the fastest
 * of each.  Scatter variants 0-5 give bitwise-identical results, and so do the
 * gather variants; scatter variant 6 agrees with them up to the grouping of
 * its additions (outside 3-D it runs variant 3's kernel and is not timed); the
 * K_UU variants agree up to rounding.  times_host (16 entries, may be NULL)
 * receives the measured microseconds: scatter (7; -1 for variant 6 outside
 * 3-D), gather (3), then FFT and dense for axes 0, 1, 2 (all 0 for a D-SKIP
 * plan; dense is -1 on an axis longer than 448 nodes, which has no dense
 * form).  The scatter forms are
 * timed once more with FP64 column values (their column chunks differ); that
 * choice, not reported, serves the FP64 MVMs and solvers.  1 <= R <= 32. */
dski_status dski_autotune(dski_plan plan, int R, double* times_host, dski_stream stream);

/* dski_autotune with a per-shape cache: cache_path (host string) names a text
 * file of tuned shapes, one line each, keyed by the device architecture, plan
 * kind, d, stencil width, n, grid sizes and R.  A matching line sets the
 * variants without timing anything (*hit_host = 1, times_host filled with -1);
 * otherwise the tuner runs and appends its choice (*hit_host = 0).  hit_host and
 * times_host may be NULL.  Calls in one process are serialised; the file is
 * not locked against other processes.  DSKI_EINVAL when the path is empty or
 * cannot be appended to. */
dski_status dski_autotune_cached(dski_plan plan, int R, const char* cache_path, int* hit_host,
                                 double* times_host, dski_stream stream);

/* Select the scatter (0..6, for FP32 and FP64 column values alike) and gather
 * (0..2) variants directly. */
dski_status dski_set_variants(dski_plan plan, int scatter_variant, int gather_variant);

/* K_UU factor of one axis: 0 circulant FFT, 1 dense Toeplitz product on the
 * matrix cores (grid size <= 448 on that axis; larger axes keep the FFT). */
dski_status dski_set_kuu_variant(dski_plan plan, int axis, int variant);

/* PCG launch mode: 1 (default) replays bursts of 8 iterations from a HIP graph
 * captured once per solve on a side stream (ordered with the caller's stream
 * by events); 0 launches every kernel directly.  Results are bitwise equal. */
dski_status dski_set_graph(dski_plan plan, int on);

/* Kernels of K_UU (App. A). */
#define DSKI_KERNEL_SE 0      /* squared exponential, ARD length scales (default)          */
#define DSKI_KERNEL_SPLINE 1  /* thin-plate spline s^2 (r^3 + a r^2 + b) (d odd) or
                               * s^2 (r^2 log r + a r^2 + b) (d even)                      */

/* Select the kernel of a D-SKI plan.  The spline kernel (App. A; the implicit
 * surface of Sec. 4.3) is not a product kernel: K_UU is a symmetric multi-level
 * Toeplitz matrix, applied by its d-dimensional circulant embedding (FFT along
 * every axis, lengths L_p >= 2 m_p - 1).  Its a and b (not given in the paper)
 * are those of the Williams-Fitzgibbon thin-plate covariances with domain size R
 * = twice the grid diameter: d odd a = -3R/2, b = R^3/2; d even
 * a = -(1 + 2 log R)/2, b = R^2/2, which makes K_UU positive definite on the
 * grid.  Hyper-parameters: s and the noise levels; the length scales passed to
 * dski_set_hypers are ignored and their gradient entries are zero.  Every
 * solver call works on such a plan; dski_mvm_tiled_noalloc and the dense K_UU
 * variant do not apply.  Computes the spectrum once (on `stream`).
 * DSKI_ENOTSUP for D-SKIP plans. */
dski_status dski_set_kernel(dski_plan plan, int kernel, dski_stream stream);

/* Storage precision (32 or 64 bits) of the N-vectors that slq_logdet creates
 * internally (probes, Krylov vectors).  Default 32. */
dski_status dski_plan_set_precision(dski_plan plan, int bits);

/* Truncated pivoted Cholesky of the noise-free K (Sec. 3.3; greedy largest
 * residual diagonal, lowest index among exact ties) and the preconditioner
 * M = D + L L^T, kept as G = D^{-1/2} L = U S V^T (U FP64, orthonormal
 * columns): M^{-1} = D^{-1/2}(I - U diag(s^2/(1+s^2)) U^T) D^{-1/2}.  rank_host
 * receives the rank reached
 * (< k when the largest residual diagonal fell below 1e-12 x the largest
 * initial one: DSKI_RANK_TRUNCATED).  piv_host (k ints, user-order indices
 * into the N-vector, may be NULL) receives the pivots. */
dski_status pivchol_build(dski_plan plan, int k, dski_precond* out, int* rank_host,
                          int* piv_host, dski_stream stream);

/* The same factorisation with the pivot of step j dictated by
 * forced_piv_host[j] (k user-order N-indices, host memory) instead of the
 * largest residual diagonal: it lets a caller reproduce another
 * implementation's pivot sequence, which the near-constant D-SKI diagonal
 * leaves to rounding at near-ties (Sec. 3.3).  The stop test still looks at
 * the largest residual diagonal; a forced pivot whose residual diagonal is not
 * positive (e.g. one chosen before) ends the factorisation there
 * (DSKI_RANK_TRUNCATED).  DSKI_EINVAL if an index is outside 0..N-1. */
dski_status pivchol_build_forced(dski_plan plan, int k, const int* forced_piv_host,
                                 dski_precond* out, int* rank_host, int* piv_host,
                                 dski_stream stream);
dski_status dski_precond_destroy(dski_precond pc);

/* Z = M^{-1} R for R vectors (user order); the Woodbury identity of Sec. 3.3
 * with two noise levels (one projection onto U, one correction). */
dski_status dski_precond_apply(dski_precond pc, int R, const float* Rm, int ld, float* Z,
                               int ldz, dski_stream stream);
dski_status dski_precond_apply_f64(dski_precond pc, int R, const double* Rm, int ld, double* Z,
                                   int ldz, dski_stream stream);

/* log det M (host FP64). */
dski_status dski_precond_logdet(dski_precond pc, double* out_host);

/* Copy the rank-r factor L (N x r, column-major, user order, FP64) to the
 * device buffer Lout (ld >= N). */
dski_status dski_precond_factor(dski_precond pc, double* Lout, int ld, dski_stream stream);

/* Preconditioned CG on the R columns of B independently (they share every
 * MVM, not their Krylov spaces), x_0 = 0 (Sec. 2, Sec. 3.3).  Column c stops
 * when ||r||_2 <= tol_host[c] ||b_c||_2 (recurrence residual).  The iterate is
 * accumulated and returned in FP64 (X, N x R, ld >= N): at the conditioning of
 * these systems an FP32-rounded solution alone would carry a true residual
 * well above 1e-4.
 *   pc        : NULL = no preconditioner.
 *   iters_host, relres_host : R entries each (may be NULL).
 *   alpha_beta: NULL or a device FP64 buffer of 2*max_iter*R entries that
 *               receives alpha_j (column c at [c*max_iter + j]) and beta_j (at
 *               [R*max_iter + c*max_iter + j]) for the Lanczos tridiagonal.
 * Returns DSKI_NOT_CONVERGED if a column reached max_iter. */
dski_status pcg_solve(dski_plan plan, dski_precond pc, int R, const float* B, int ldb,
                      double* X, int ldx, const double* tol_host, int max_iter,
                      int* iters_host, double* relres_host, double* alpha_beta,
                      dski_stream stream);
dski_status pcg_solve_f64(dski_plan plan, dski_precond pc, int R, const double* B, int ldb,
                          double* X, int ldx, const double* tol_host, int max_iter,
                          int* iters_host, double* relres_host, double* alpha_beta,
                          dski_stream stream);

/* Stochastic Lanczos quadrature estimate of log det K~ (Sec. 2).  Probe i is
 * z_i = C w_i with w_i the Rademacher column i of the SplitMix64 stream
 * `seed` (see dski_rademacher) and C C^T = M (plain w_i when pc is NULL).
 * lanczos_steps = 0: T_i from the CG coefficients of the block PCG on the
 *   probes, run to tol (storage precision: dski_plan_set_precision).
 * lanczos_steps > 0: that many steps of the explicit Lanczos process of the
 *   preconditioned operator (M-inner product) per probe, with full
 *   re-orthogonalisation, FP64 vectors; a probe whose Krylov space is exhausted
 *   earlier stops there.  (The same tridiagonal as CG's in exact arithmetic;
 *   a short run without re-orthogonalisation is ill-conditioned.)
 * logdet = log det M + (1/t) sum_i (z_i^T M^{-1} z_i) e_1^T log(T_i) e_1. */
dski_status slq_logdet(dski_plan plan, dski_precond pc, int num_probes, int lanczos_steps,
                       double tol, int max_iter, uint64_t seed, double* logdet_host,
                       double* stderr_host, dski_stream stream);

/* Log marginal likelihood eq. (1) and its gradient (d+3 entries, hyper-
 * parameter order) at the plan's current hyper-parameters.  One PCG on
 * [y, z_1..z_t]; log det by SLQ from the same run; the trace terms
 * tr(K~^{-1} dK~) by E[(K~^{-1} z)^T dK~ (M^{-1} z)].  pc NULL: build rank k.
 * y is an N-vector in user order.  num_probes = 0 gives the data-fit part only
 * (-y^T alpha / 2 - N log(2 pi) / 2 and its gradient, log det reported as 0),
 * which a caller combines with its own log det model. */
dski_status mll_and_grad(dski_plan plan, dski_precond pc, int k, const float* y,
                         int num_probes, uint64_t seed, double tol, int max_iter,
                         double* mll_host, double* grad_host, double* logdet_host,
                         int* iters_host, dski_stream stream);
dski_status mll_and_grad_f64(dski_plan plan, dski_precond pc, int k, const double* y,
                             int num_probes, uint64_t seed, double tol, int max_iter,
                             double* mll_host, double* grad_host, double* logdet_host,
                             int* iters_host, dski_stream stream);

/* mll_and_grad with a warm start for the data solve (hyper-parameter searches
 * move theta a little between evaluations, so the last alpha is a good start):
 * x0 (N doubles, device, user order, or NULL for x_0 = 0) starts alpha; the
 * solve of K~ dx = y - K~ x0 stops when ||y - K~ alpha|| <= tol ||y||, alpha =
 * x0 + dx.  The probe columns still start at zero (their Lanczos runs define
 * the quadrature).  alpha_out (N doubles, device, user order, or NULL)
 * receives alpha in FP64.  Otherwise as mll_and_grad (FP32 vectors). */
dski_status mll_and_grad_warm(dski_plan plan, dski_precond pc, int k, const float* y, int num_probes,
                              uint64_t seed, double tol, int max_iter, const double* x0, double* alpha_out,
                              double* mll_host, double* grad_host, double* logdet_host, int* iters_host,
                              dski_stream stream);

/* out[c*ld + i] = +-1 (FP32): Rademacher column col0+c of the counter-based
 * SplitMix64 stream `seed` (Steele et al. 2014): entry i of column c is -1
 * iff bit 63 of mix64(seed + (c*N + i + 1) * 0x9E3779B97F4A7C15) is set. */
dski_status dski_rademacher(uint64_t seed, int col0, int ncols, int N, float* out, int ld,
                            dski_stream stream);

/* Host utility: e_1^T log(T) e_1 for the Lanczos tridiagonal of J CG steps with
 * coefficients alpha, beta (host arrays, as returned by pcg_solve):
 * T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j
 * (Gauss quadrature of Sec. 2's Lanczos connection).  Up to J = 64 by the
 * symmetric tridiagonal QR algorithm on the first row of the eigenvectors;
 * longer tridiagonals by the trapezoidal rule on the integral representation of
 * log(T) in log t, O(J * nodes) with about 250 nodes instead of O(J^2).  *ok = 0
 * if T is not positive definite or the iteration fails. */
double dski_lanczos_quad_log(const double* alpha_host, const double* beta_host, int J, int* ok);

/* ---------------------------------------------------------------------------------
 * Learned log-determinant surrogate (a network of this project, not of the paper):
 * y = w3 . gelu(W2 gelu(W1 x + b1) + b2) + b3 with the exact GELU, FP32, F inputs,
 * H units per hidden layer (H <= 128, F <= 16), and forward-mode tangents along
 * the first J inputs (J <= min(F, 8)).  Parameters are packed row-major:
 * W1 (H x F), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1); H F + H^2 + 3 H + 1 floats.
 * X is a device B x F row-major batch; y (B), dy (B x J) are device outputs.
 * Training loss: (1/B) sum_b [(y_b - t_b)^2 + lam sum_j (dy_bj - g_bj)^2]. */
typedef struct dski_mlp_s* dski_mlp;

/* params_host: the packed parameters (copied).  Errors: DSKI_EINVAL. */
dski_status mlp_create(dski_mlp* out, int F, int H, int J, const float* params_host, dski_stream stream);
dski_status mlp_destroy(dski_mlp net);
dski_status mlp_num_params(dski_mlp net, int* n);
/* Copies the current parameters and/or the gradient of the last mlp_backward (host, may be NULL). */
dski_status mlp_get_params(dski_mlp net, float* params_host, float* grad_host);
/* y = network(X). */
dski_status mlp_forward(dski_mlp net, int B, const float* X, float* y, dski_stream stream);
/* y and dy[b, j] = d y_b / d x_bj for j < J (tangent propagation). */
dski_status mlp_jvp(dski_mlp net, int B, const float* X, float* y, float* dy, dski_stream stream);
/* Gradient of the training loss with respect to every parameter (kept in the
 * network for mlp_step); t (B) and g (B x J) are device targets; loss_host may
 * be NULL.  Deterministic: batch sums in FP64 in a fixed order. */
dski_status mlp_backward(dski_mlp net, int B, const float* X, const float* t, const float* g, float lam,
                         double* loss_host, dski_stream stream);
/* One Adam step (Kingma & Ba 2015) with the gradient of the last mlp_backward. */
dski_status mlp_step(dski_mlp net, float lr, float beta1, float beta2, float eps, dski_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* DSKI_H */
