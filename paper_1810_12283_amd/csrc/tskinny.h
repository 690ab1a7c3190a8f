// Tall-skinny products with the N x k preconditioner factor U (FP64, column-
// major), shared by the preconditioner and the fused PCG iteration (device
// helpers and kernels that each translation unit instantiates for itself).
//
//   projection  t = U^T (pre .* X)   one wavefront per 64 rows on the FP64
//                                matrix cores (v_mfma_f64_16x16x4f64): U is the
//                                A operand, read straight from its row-major
//                                copy (4 rows x 16 consecutive columns per
//                                load), the
//                                64 x R block of X, staged unscaled in LDS, the
//                                B operand with the row scale applied in
//                                registers; one partial per wavefront,
//                                output-major, reduced in a fixed order.
//   correction  z = post .* (pre .* X - U coef)   one wavefront per 64 rows on
//                                the FP64 matrix cores (A = U, B = coef), the
//                                result transposed through LDS so that X and Z
//                                move one row per lane.
#pragma once

#include <algorithm>

#include "internal.h"

namespace dski {

constexpr int kFinalMaxR = 32;  // columns per tall-skinny launch
constexpr int kProjRows = 64;   // rows per projection wavefront

typedef double dski_pdbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Fixed-order sum of the nblk partials of one output (output-major layout),
// by one wavefront: lane l adds blocks l, l + 64, ..., then a shuffle tree.
__device__ __forceinline__ double wave_out_sum(const double* __restrict__ part, int nblk, int o) {
  const int lane = threadIdx.x & 63;
  double a = 0.0;
  const double* p = part + (size_t)o * nblk;
  for (int b = lane; b < nblk; b += 64) a += p[b];
  return wave_sum64(a);
}

inline int pad4(int x) { return (x + 3) & ~3; }
__host__ __device__ inline int proj_waves(int N) { return (N + kProjRows - 1) / kProjRows; }

// Row stride (elements) of a wavefront's 64-row block of X in LDS: odd, so
// that the four rows of one matrix-core step fall on different banks.
template <int CB>
struct ProjLds {
  static constexpr int XP = 16 * CB + 1;
  static constexpr int per_wave = kProjRows * XP;
  template <typename S>
  static constexpr size_t bytes() { return 4 * sizeof(S) * (size_t)per_wave; }  // four wavefronts
};

// Partials of t = U^T (scale .* X) over rows e0 .. e0 + 63 (rows >= N count as
// zero): sx holds this wavefront's X rows (row stride XP, columns >= R zero),
// the row scale is pre_v below row n and pre_g from n on.  Writes
// partial[(i R + c) nw + w] for i < k, c < R.  CB = column blocks of 16.
template <int CB, typename S>
__device__ __forceinline__ void wave_project(const double* __restrict__ Ur, int N, int n, int k, int R, int e0,
                                             const S* __restrict__ sx, double pre_v, double pre_g,
                                             double* __restrict__ partial, int nw, int w) {
  constexpr int XP = ProjLds<CB>::XP;
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  // the B operands of all 16 steps (rows 4 s + kq), scaled, for every column block
  double bop[16][CB];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int row = 4 * s + kq, e = e0 + row;
    const double sc = e < n ? pre_v : pre_g;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) bop[s][cb] = sc * (double)sx[row * XP + 16 * cb + r16];
  }
  for (int i0 = 0; i0 < k; i0 += 64) {  // groups of four 16-column blocks of U
    dski_pdbl4 acc[4][CB];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[b][cb] = dski_pdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two halves of 8 steps: 32 loads in flight
      double aop[8][4];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int e = e0 + 4 * (8 * h + s) + kq;
#pragma unroll
        for (int b = 0; b < 4; ++b) {  // row-major U: 16 consecutive columns of 4 rows per load
          const int i = i0 + 16 * b + r16;
          aop[s][b] = ld_or0(Ur, (size_t)e * k + i, 0, i < k && e < N);
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[b][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[s][b], bop[8 * h + s][cb], acc[b][cb], 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 16 * b + kq + 4 * r, c = 16 * cb + r16;
          if (i < k && c < R) partial[((size_t)i * R + c) * nw + w] = acc[b][cb][r];
        }
  }
}

// Sets the dynamic LDS limit of a kernel once (above 64 KiB it must be raised).
template <typename K>
static inline dski_status lds_limit(K* kern, size_t bytes, bool& done) {
  if (!done && bytes > 65536) {
    DSKI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes));
  }
  done = true;
  return DSKI_OK;
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Standalone projection: partials of t = U^T (pre .* X), one per wavefront.
template <typename T, int CB>
static __global__ __launch_bounds__(256) void k_ts_proj(const T* __restrict__ X, int ld, int N, int n, int R,
                                                        double pre_v, double pre_g, const double* __restrict__ Ur,
                                                        int k, double* __restrict__ partial) {
  extern __shared__ __align__(16) char smem[];
  constexpr int XP = ProjLds<CB>::XP;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + wv, nw = proj_waves(N);
  if (w >= nw) return;
  T* sx = reinterpret_cast<T*>(smem) + (size_t)wv * ProjLds<CB>::per_wave;
  const int e0 = w * kProjRows, e = e0 + lane;
#pragma unroll
  for (int c = 0; c < 16 * CB; ++c) sx[lane * XP + c] = ld_or0(X, (size_t)c * ld + e, 0, c < R && e < N);
  wave_lds_fence();
  wave_project<CB>(Ur, N, n, k, R, e0, sx, pre_v, pre_g, partial, nw, w);
}

template <typename T>
static inline dski_status launch_proj(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                      const double* Ur, int k, double* partial, hipStream_t st) {
  const int nb = (proj_waves(N) + 3) / 4;
  if (R <= 16) {
    constexpr size_t sh = ProjLds<1>::bytes<T>();
    static bool done = false;
    DSKI_TRY(lds_limit(&k_ts_proj<T, 1>, sh, done));
    k_ts_proj<T, 1><<<nb, 256, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, Ur, k, partial);
  } else {
    constexpr size_t sh = ProjLds<2>::bytes<T>();
    static bool done = false;
    DSKI_TRY(lds_limit(&k_ts_proj<T, 2>, sh, done));
    k_ts_proj<T, 2><<<nb, 256, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, Ur, k, partial);
  }
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// Reduction of per-tile partials in up to two jobs (blockIdx.y), one wavefront
// per output:  out[o] = sum_b partial[o, b];  optional t_out = out, and
//   coef[o] = sgn * c[o / R] * (out[o] + t_prev[o]).
struct RedJob {
  const double* partial;   // output-major: nout x nblk
  int nblk, nout, R;
  double* out;             // may be NULL
  const double* c;         // may be NULL (no coefficients)
  const double* t_prev;    // may be NULL
  double sgn;
  double* coef;            // may be NULL
  const int* mask;         // optional: only write out[o] when mask[o % R] (per-column flag)
};

static __global__ void k_ts_reduce(RedJob j0, RedJob j1) {
  const RedJob& J = blockIdx.y == 0 ? j0 : j1;
  int o = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (o >= J.nout) return;
  double t = wave_out_sum(J.partial, J.nblk, o);
  if ((threadIdx.x & 63) == 0) {
    bool write = !J.mask || J.mask[o % J.R];
    if (J.out && write) J.out[o] = t;
    if (J.coef) J.coef[o] = J.sgn * J.c[o / J.R] * (t + (J.t_prev ? J.t_prev[o] : 0.0));
  }
}

static inline dski_status launch_reduce(const RedJob& a, const RedJob* b, hipStream_t st) {
  int nout = std::max(a.nout, b ? b->nout : 0);
  dim3 grid((nout + 3) / 4, b ? 2 : 1);
  RedJob bb = b ? *b : a;
  k_ts_reduce<<<grid, 256, 0, st>>>(a, bb);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// The same reduction for block-major partials (partial[b nout + o], written
// coalesced by one work-group each): a work-group takes 16 consecutive outputs;
// its 256 threads split the blocks into 16 contiguous parts (thread = output +
// 16 part), each part added in order, the parts combined in a fixed order.
static __global__ __launch_bounds__(256) void k_ts_reduce_bm(RedJob j0, RedJob j1) {
  const RedJob& J = blockIdx.y == 0 ? j0 : j1;
  __shared__ double q[16][17];
  const int ol = threadIdx.x & 15, part = threadIdx.x >> 4;
  const int o = blockIdx.x * 16 + ol;
  if (blockIdx.x * 16 >= J.nout) return;
  const int per = (J.nblk + 15) / 16, b0 = part * per, b1 = min(J.nblk, b0 + per);
  double a = 0.0;
  if (o < J.nout) {
    for (int b = b0; b < b1; b += 16) {  // sixteen loads in flight (zeros past b1), added in order
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = ld_or0(J.partial, (size_t)(b + u) * J.nout + o, 0, b + u < b1);
#pragma unroll
      for (int u = 0; u < 16; ++u) a += v[u];
    }
  }
  q[part][ol] = a;
  __syncthreads();
  if (part == 0 && o < J.nout) {
    double t = 0.0;
#pragma unroll
    for (int pp = 0; pp < 16; ++pp) t += q[pp][ol];
    const bool write = !J.mask || J.mask[o % J.R];
    if (J.out && write) J.out[o] = t;
    if (J.coef) J.coef[o] = J.sgn * J.c[o / J.R] * (t + (J.t_prev ? J.t_prev[o] : 0.0));
  }
}

static inline dski_status launch_reduce_bm(const RedJob& a, const RedJob* b, hipStream_t st) {
  const int nout = std::max(a.nout, b ? b->nout : 0);
  dim3 grid((nout + 15) / 16, b ? 2 : 1);
  RedJob bb = b ? *b : a;
  k_ts_reduce_bm<<<grid, 256, 0, st>>>(a, bb);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// z[e, c] = post_e * (pre_e * X[e, c] - sum_i U[e, i] coef[i, c]), one wavefront
// per 32 rows, eight per work-group (256 rows, so that the partials are per
// vec_blocks block).  The product U coef runs on the FP64 matrix cores (A = U,
// 16 rows x 4 of its columns per operand; B = coef, 4 x 16) for CB blocks of 16
// columns, and on the vector ALU for VC further columns (17 - 20 columns: one
// block plus up to four, instead of two blocks).  Per chunk of 64 columns of U
// the work-group stages that chunk of coef in LDS (its loads issued first, so
// that waiting for them does not wait for U), and every wavefront issues all
// of its U operands before the first product; steps past k are skipped.  The
// result goes through LDS, and each lane then takes one row and half of the
// columns for X, Z and the partials of X.z (fixed order), stored output-major
// (dot_partial[c * blocks + block]).
constexpr int kFinalRows = 32;
constexpr int kFinalWaves = 8;
static_assert(kFinalRows * kFinalWaves == kBlock, "dot partials are counted per vec_blocks block");
template <typename T, int CB, int VC>
static __global__ __launch_bounds__(512) void k_ts_final(const T* __restrict__ X, int ld, int N, int n, int R,
                                                         double pre_v, double pre_g, double post_v, double post_g,
                                                         const double* __restrict__ U, int k,
                                                         const double* __restrict__ coef, T* __restrict__ Z,
                                                         int ldz, double* __restrict__ dot_partial) {
  constexpr int FR = kFinalRows, EB = FR / 16, CW = 16 * CB + VC, XP = CW + 1, HC = (CW + 1) / 2;
  constexpr int NT = 64 * kFinalWaves, CF = (64 * CW + NT - 1) / NT;  // coef entries per thread and chunk
  static_assert(CW <= 32, "columns per launch");
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[kFinalWaves][CW];
  __shared__ double s_coef[64 * XP];  // one chunk: row i - i0, column c
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int e0 = (blockIdx.x * kFinalWaves + wv) * FR;
  double* sz = reinterpret_cast<double*>(smem) + (size_t)wv * FR * XP;
  // this lane's row (rl) and half of the columns (hh) of X (clamped indices,
  // masked at use)
  const int rl = lane & (FR - 1), hh = lane / FR;
  const int e = e0 + rl;
  const bool in = e < N;
  T xr[HC];
  dski_pdbl4 acc[EB][CB];
  double vacc[EB][VC > 0 ? VC : 1];
#pragma unroll
  for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[eb][cb] = dski_pdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < VC; ++v) vacc[eb][v] = 0.0;
  }
  // U indices are clamped instead of masked: a column i >= k meets a zero
  // coefficient, a row past N is never stored
  const size_t nk_last = (size_t)N * (size_t)(k > 0 ? k : 1) - 1;
  for (int i0 = 0; i0 < k; i0 += 64) {
    double cf[CF];
#pragma unroll
    for (int u = 0; u < CF; ++u) {
      const int f = threadIdx.x + NT * u, il = f / CW, c = f - il * CW;
      cf[u] = ld_or0(coef, (size_t)(i0 + il) * R + c, 0, f < 64 * CW && i0 + il < k && c < R);
    }
    if (i0 == 0) {
#pragma unroll
      for (int j = 0; j < HC; ++j) {
        const int c = hh * HC + j;
        xr[j] = X[(size_t)(c < R ? c : R - 1) * ld + (in ? e : 0)];
      }
    }
    double av[16][EB];
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int i = i0 + 4 * st + kq;
#pragma unroll
      for (int eb = 0; eb < EB; ++eb) {
        const size_t o = (size_t)i * N + (size_t)(e0 + 16 * eb + r16);
        av[st][eb] = U[o < nk_last ? o : nk_last];
      }
    }
    if (i0 > 0) __syncthreads();  // every wavefront is done with the previous chunk
#pragma unroll
    for (int u = 0; u < CF; ++u) {
      const int f = threadIdx.x + NT * u, il = f / CW, c = f - il * CW;
      if (f < 64 * CW) s_coef[il * XP + c] = cf[u];
    }
    __syncthreads();
    const int steps = min(16, (k - i0 + 3) / 4);  // steps holding a column i < k
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      if (st < steps) {
        const double* crow = s_coef + (4 * st + kq) * XP;
        double bv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) bv[cb] = crow[16 * cb + r16];
#pragma unroll
        for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[eb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st][eb], bv[cb], acc[eb][cb], 0, 0, 0);
#pragma unroll
          for (int v = 0; v < VC; ++v) vacc[eb][v] += av[st][eb] * crow[16 * CB + v];
        }
      }
    }
  }
  if (k <= 0) {  // no product: X alone
#pragma unroll
    for (int j = 0; j < HC; ++j) {
      const int c = hh * HC + j;
      xr[j] = X[(size_t)(c < R ? c : R - 1) * ld + (in ? e : 0)];
    }
  }
  // D register r of lane l: row 16 eb + l / 16 + 4 r, column 16 cb + l % 16;
  // the vector columns summed over the four lanes that share a row
#pragma unroll
  for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) sz[(16 * eb + kq + 4 * r) * XP + 16 * cb + r16] = acc[eb][cb][r];
#pragma unroll
    for (int v = 0; v < VC; ++v) {
      double x = vacc[eb][v];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (kq == 0) sz[(16 * eb + r16) * XP + 16 * CB + v] = x;
    }
  }
  wave_lds_fence();
  const double pre = e < n ? pre_v : pre_g, post = e < n ? post_v : post_g;
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;  // at most CW: inside the LDS row of XP = CW + 1
    double dot = 0.0;
    if (in && c < R) {
      const double xv = (double)xr[j];
      const T z = (T)(post * (pre * xv - sz[rl * XP + c]));
      Z[(size_t)c * ldz + e] = z;
      dot = xv * (double)z;
    }
    sz[rl * XP + c] = dot;
  }
  if (!dot_partial) return;
  wave_lds_fence();
  {  // column sums over the wavefront's 32 rows: lane c + 32 h sums rows 16 h ..
    const int c = lane & 31, h = lane >> 5;
    double a = 0.0;
    if (c < CW) {
#pragma unroll
      for (int j = 0; j < 16; ++j) a += sz[(16 * h + j) * XP + c];
    }
    a += __shfl_xor(a, 32, 64);
    if (h == 0 && c < CW) red[wv][c] = a;
  }
  __syncthreads();
  if (threadIdx.x < R) {
    const int c = threadIdx.x;
    dot_partial[(size_t)c * gridDim.x + blockIdx.x] =
        ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) + ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c]));
  }
}

template <typename T, int CB, int VC>
static inline dski_status launch_final_cw(int nb, const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                          double post_v, double post_g, const double* U, int k, const double* coef,
                                          T* Z, int ldz, double* dot_partial, hipStream_t st) {
  constexpr size_t sh = sizeof(double) * kFinalWaves * kFinalRows * (16 * CB + VC + 1);
  static bool done = false;
  DSKI_TRY(lds_limit(&k_ts_final<T, CB, VC>, sh, done));
  k_ts_final<T, CB, VC><<<nb, 64 * kFinalWaves, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef,
                                                          Z, ldz, dot_partial);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

template <typename T>
static inline dski_status launch_final(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                       double post_v, double post_g, const double* U, int k,
                                       const double* coef, T* Z, int ldz, double* dot_partial, hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  if (R > kFinalMaxR) {
    set_error("at most %d columns per tall-skinny launch", kFinalMaxR);
    return DSKI_ENOTSUP;
  }
  constexpr int rows = kFinalRows * kFinalWaves;
  const int nb = (N + rows - 1) / rows;  // = vec_blocks(N): 256 rows per work-group
  if (R <= 16)
    return launch_final_cw<T, 1, 0>(nb, X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef, Z, ldz,
                                    dot_partial, st);
  if (R <= 20)
    return launch_final_cw<T, 1, 4>(nb, X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef, Z, ldz,
                                    dot_partial, st);
  return launch_final_cw<T, 2, 0>(nb, X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef, Z, ldz,
                                  dot_partial, st);
}

}  // namespace dski
