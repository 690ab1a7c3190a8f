// Internal declarations of the D-SKI library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dski.h"

#define DSKI_MAXD 3     // D-SKI grid dimensions
#define DSKIP_MAXD 64   // D-SKIP input dimensions

namespace dski {

// p[i] when ok, else zero, without a branch: the load is issued from index i
// or from the valid index `safe`, and the value selected afterwards, so that
// neighbouring loads stay in flight together (a load under a branch is waited
// for inside the branch).
template <typename T>
__device__ __forceinline__ T ld_or0(const T* __restrict__ p, size_t i, size_t safe, bool ok) {
  const T v = p[ok ? i : safe];
  return ok ? v : (T)0;
}

void set_error(const char* fmt, ...);

struct HipError {
  hipError_t e;
};

#define DSKI_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess) {                                                             \
      ::dski::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                      \
      return DSKI_EHIP;                                                                 \
    }                                                                                   \
  } while (0)

#define DSKI_TRY(call)                 \
  do {                                 \
    dski_status _s = (call);           \
    if (_s < 0) return _s;             \
  } while (0)

// Device buffer that grows on demand (contents not preserved on growth).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  dski_status reserve(size_t want);
  void release();
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Radix plan of the length-2^lg FFT along a grid axis: passes of radix 8
// while three or more factors of two remain, then one pass of radix 4 or 2.
// The inverse transform runs the same radices in reverse order.  Pass s of a
// direction has stride Ns = product of the radices before it; its twiddles
// e^{-+2 pi i r k / (radix Ns)} (r = 1..radix-1, k < Ns) are stored at
// fft_tw_offset + (r - 1) Ns + k, forward passes first, then the inverse ones
// (already conjugated).
__host__ __device__ constexpr int fft_npass(int lg) { return lg / 3 + (lg % 3 != 0 ? 1 : 0); }
__host__ __device__ constexpr int fft_radix_dir(int lg, int s, int dir) {
  const int t = dir > 0 ? s : fft_npass(lg) - 1 - s;
  return t < lg / 3 ? 8 : (lg % 3 == 2 ? 4 : 2);
}
__host__ __device__ constexpr int fft_ns(int lg, int s, int dir) {
  int ns = 1;
  for (int t = 0; t < s; ++t) ns *= fft_radix_dir(lg, t, dir);
  return ns;
}
__host__ __device__ constexpr int fft_tw_offset(int lg, int s, int dir) {
  int off = 0;
  if (dir < 0)
    for (int t = 0; t < fft_npass(lg); ++t) off += (fft_radix_dir(lg, t, +1) - 1) * fft_ns(lg, t, +1);
  for (int t = 0; t < s; ++t) off += (fft_radix_dir(lg, t, dir) - 1) * fft_ns(lg, t, dir);
  return off;
}
__host__ __device__ constexpr int fft_tw_size(int lg) { return fft_tw_offset(lg, fft_npass(lg), -1); }
constexpr int kFftMaxLog2 = 11;  // L <= 2048, m <= 1024 per axis
constexpr int kKernelSE = 0;
constexpr int kKernelSpline = 1;
constexpr int kDenseMaxM = 448;  // largest axis for the dense matrix-core Toeplitz product

// Per-axis geometry of the grid and its circulant embedding.
struct Axis {
  int m = 0;          // grid nodes
  int ncell = 0;      // interpolation cells = m - S + 1 (S stencil nodes per axis)
  int L = 0;          // circulant length (power of two >= 2m - 1)
  double lo = 0, h = 0;
  double* twiddle = nullptr;  // fft_tw_size(log2 L) complex pass twiddles (device, interleaved re, im)
  double* spec = nullptr;     // L circulant eigenvalues of T_p, scaled (device)
  double* dspec = nullptr;    // L eigenvalues of dT_p / dlog ell_p, scaled (device)
  double* col = nullptr;      // m first column of T_p (device)
};

struct DskipData;  // D-SKIP factors (dskip.hip)

// State of the device-side pivoted Cholesky.
struct PivState {
  int piv;        // chosen tile-order N-index
  int stop;       // 1 once the factorisation has stopped
  int rank;       // columns produced
  double dpiv;    // residual diagonal at the pivot
  double dmax0;   // largest initial diagonal
};

}  // namespace dski

struct dski_plan_s {
  int kind = 0;                // 0 D-SKI (grid), 1 D-SKIP (Hadamard of 1-D factors)
  dski::DskipData* ds = nullptr;
  int n = 0, d = 0, N = 0;
  int S = 4;                   // stencil nodes per axis: 4 cubic (Keys), 6 quintic
  int kernel = 0;              // kKernelSE (separable Toeplitz factors) or kKernelSpline
  double spline_R = 0;         // spline kernel: domain size R (twice the grid diameter)
  double* bttb_spec = nullptr; // spline kernel: spectrum of the embedded K_UU / prod L (device)
  dski::DevBuf bttb_work;      // spline kernel: complex embedded columns
  long long M = 0;             // grid nodes
  int ncells = 0;              // total interpolation cells
  dski::Axis ax[DSKI_MAXD];
  // hyper-parameters
  double ell[DSKI_MAXD] = {1, 1, 1};
  double s = 1, sf = 0.1, sg = 0.1;
  // point data in tile order (device)
  int* perm = nullptr;         // tile position -> user index
  int* cell = nullptr;         // linear cell id per tile position (per axis: first stencil node)
  double* toff = nullptr;      // d x n offsets in [0, 1] (SoA, FP64); the weights follow from them
  int* cell_start = nullptr;   // ncells + 1
  // scatter region tables (per node tile: its region's points, see mvm.hip)
  int* tile_off = nullptr;     // tiles + 1 slot offsets
  int* tile_lcs = nullptr;     // tiles x (region cells + 1) local point ranges
  int* tile_pts = nullptr;     // slots: point (tile order)
  int* tile_cl = nullptr;      // slots: last-axis anchor node of the point
  long long tile_slots = 0;
  // 3-D grouped scatter (see mvm.hip): per staged chunk of every tile, its
  // (node, first-axis cell) items ordered by their work
  unsigned short* grp_items = nullptr;  // node * 8 + group
  int* grp_chunk_off = nullptr;         // chunks + 1 item offsets
  int* grp_tile_chunk = nullptr;        // tiles + 1 first chunk of each tile
  // workspaces
  dski::DevBuf grid;           // grid buffer, M * Rmax values (FP32 or FP64)
  dski::DevBuf vin, vout;      // tile-ordered FP32 vectors
  dski::DevBuf partial;        // FP64 block partials
  dski::DevBuf scal;           // FP64 small scalars
  int precision = 32;          // storage of N-vectors inside slq_logdet (32 or 64)
  // kernel variants chosen by dski_autotune (defaults: the LDS-tiled kernels)
  int scatter_variant = 0;     // 0 LDS node tiles, 1 direct 1 column/thread, 2 direct 2 columns/thread,
                               // 3 / 4 / 5 LDS node tiles with 1.5 / 2 / 5 times the columns per work-group
  int scatter_variant64 = 0;   // the same choice for FP64 column values (tuned separately)
  int gather_variant = 0;      // columns per gather thread: 0 -> 2, 1 -> 1, 2 -> 4 (3-D: always 1)
  int use_graph = 1;           // PCG bursts replayed from a captured HIP graph
  int kuu_variant[DSKI_MAXD] = {0, 0, 0};  // per axis: 0 FFT, 1 dense matrix-core product
};

struct dski_precond_s {
  dski_plan plan = nullptr;
  int k = 0;                   // rank
  double logdet = 0;
  int* piv_tile = nullptr;     // device, k pivots (tile-order N-index)
  double* L = nullptr;         // device, N x k FP64 (tile order, column-major)
  double* U = nullptr;         // device, N x k FP64 left singular vectors of D^{-1/2} L (column-major)
  double* Ur = nullptr;        // device, the same N x k row-major (row e at Ur + e k)
  double* w = nullptr;         // device, k: sigma_i^2 / (1 + sigma_i^2)
  double* rootc = nullptr;     // device, k: sqrt(1 + sigma_i^2) - 1
  dski::DevBuf work;
};

namespace dski {

constexpr int kBlock = 256;

// --- plan / grid ------------------------------------------------------------------
// T is the storage type of N-vectors (float or double), GT that of the grid
// (instantiated for FP64 grids: <float, double>, <double, double>); sums and
// transforms run in FP64.
template <typename GT>
dski_status apply_kuu(dski_plan p, int R, GT* G, hipStream_t st, int dwhich = -1);
template <typename GT>
dski_status kuu_axis(dski_plan p, int R, GT* G, hipStream_t st, int dwhich, int a, int variant);
template <typename T, typename GT>
dski_status scatter(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st);
dski_status scatter_tables(dski_plan p, hipStream_t st);  // build the region tables (plan set-up)
dski_status bttb_build_spectrum(dski_plan p, hipStream_t st);  // spline kernel: spectrum of K_UU
template <typename T, typename GT>
dski_status gather(dski_plan p, int R, const GT* G, const T* V, int ldv, T* Y, int ldy,
                   double nv, double ng, double* pq_partial, hipStream_t st);
template <typename T>
dski_status mvm_dtheta(dski_plan p, int which, int R, const T* V, int ldv, T* Y, int ldy,
                       hipStream_t st);
int gather_blocks(dski_plan p);
template <typename T>
dski_status mvm_tiled(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double* pq_partial,
                      hipStream_t st);
dski_status permute(dski_plan p, int dir, int R, const float* in, int ldi, float* out, int ldo,
                    hipStream_t st);
dski_status permute(dski_plan p, int dir, int R, const double* in, int ldi, double* out, int ldo,
                    hipStream_t st);

// --- preconditioner -----------------------------------------------------------------
// Z = M^{-1} Rm (tile order).  rz_partial (optional): block partials of sum Rm*Z per column.
template <typename T>
dski_status precond_apply_tiled(dski_precond pc, int R, const T* Rm, int ld, T* Z, int ldz,
                                double* rz_partial, int* nblk_out, hipStream_t st);
// Z = C W with C C^T = M (tile order).
template <typename T>
dski_status precond_factor_apply_tiled(dski_precond pc, int R, const T* W, int ld, T* Z, int ldz,
                                       hipStream_t st);
// Low-rank part of r^T M^{-1} r for R <= kFinalMaxR FP64 columns (tile order):
// with M^{-1} = D^{-1/2}(I - U diag(w) U^T)D^{-1/2} and t = U^T D^{-1/2} r,
// kq[c] = sum_i w_i t_i^2, so that r^T M^{-1} r = ||D^{-1/2} r||^2 - kq[c]
// (the projection and reduction of one application, without its final pass).
dski_status precond_lowrank_quad(dski_precond pc, int R, const double* Rm, int ld, double* kq, hipStream_t st);
int vec_blocks(int N);

// --- PCG core (tile order) -----------------------------------------------------------
struct PcgResult {
  std::vector<int> iters;
  std::vector<double> relres;
  std::vector<double> rz0;     // r_0^T M^{-1} r_0 per column
  bool breakdown = false;
};
// X (storage type, may be NULL) and/or X64 (FP64, may be NULL) receive the iterate.
// verify_mask (host, R flags, may be NULL): columns whose convergence is confirmed
// with the true residual b - K~ x (and resumed if needed; their CG history then
// no longer describes a single Krylov run).
template <typename T>
dski_status pcg_tiled(dski_plan p, dski_precond pc, int R, const T* B, int ldb, T* X, int ldx,
                      const double* tol_host, int max_iter, int fixed_iters, double* alpha_beta,
                      PcgResult& res, hipStream_t st, double* X64 = nullptr,
                      const int* verify_mask = nullptr);

// --- D-SKIP ----------------------------------------------------------------------------
// Y = ks K V + diag(nv on value rows, ng on gradient rows) V (D-SKIP, identity tile order)
template <typename T>
dski_status dskip_apply(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double ks, double nv, double ng,
                        double* pq_partial, hipStream_t st);
template <typename T>
dski_status dskip_mvm(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double* pq_partial,
                      hipStream_t st);
dski_status dskip_set_hypers(dski_plan p, const double* log_ell, hipStream_t st);
dski_status dskip_diag(dski_plan p, double* diag, hipStream_t st);
// one pivoted-Cholesky step j (after the arg-max partials pv/pi of nblk blocks)
dski_status dskip_pc_step(dski_plan p, int j, const double* pv, const int* pi, int nblk, double rel_tol,
                          PivState* ps, int* piv_list, double* L, double* lrow, double* dres, const int* forced,
                          hipStream_t st);
void dskip_destroy(dski_plan p);

// --- host numerics ---------------------------------------------------------------------
double gauss_quad_log(const double* alpha, const double* beta, int J, int* ok);
double gauss_quad_log_tri(const double* diag, const double* off, int J, int* ok);
int sym_eig_jacobi(int k, double* A, double* V, double* w);

// --- rng ---------------------------------------------------------------------------------
template <typename T>
dski_status rademacher(uint64_t seed, int col0, int ncols, int N, T* out, int ld, hipStream_t st);

// deterministic reductions
dski_status reduce_partials(const double* partial, int nblk, int ncol, double* out,
                            hipStream_t st);

}  // namespace dski
