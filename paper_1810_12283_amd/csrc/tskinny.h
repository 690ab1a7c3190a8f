// Tall-skinny products with the N x k preconditioner factor U (FP64, column-
// major), shared by the preconditioner and the fused PCG iteration (device
// helpers and kernels that each translation unit instantiates for itself).
//
//   projection  t = U^T (pre .* X)   one wavefront per 64 rows on the FP64
//                                matrix cores (v_mfma_f64_16x16x4f64): U is the
//                                A operand, read straight from memory (16
//                                columns x 4 consecutive rows per load), the
//                                64 x R block of X, staged unscaled in LDS, the
//                                B operand with the row scale applied in
//                                registers; one partial per wavefront,
//                                output-major, reduced in a fixed order.
//   correction  z = post .* (pre .* X - U coef)   one thread per row, all columns
//                                in registers (padded to a multiple of 4), coef
//                                in LDS, U loads issued 16 at a time with the
//                                next 16 in flight.
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
__device__ __forceinline__ void wave_project(const double* __restrict__ U, int N, int n, int k, int R, int e0,
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
    const double* ub[4];
    bool ok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + 16 * b + r16;
      ok[b] = i < k;
      ub[b] = U + (size_t)(ok[b] ? i : 0) * N;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two halves of 8 steps: 32 loads in flight
      double aop[8][4];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int e = e0 + 4 * (8 * h + s) + kq;
#pragma unroll
        for (int b = 0; b < 4; ++b) aop[s][b] = ld_or0(ub[b], (size_t)e, 0, ok[b] && e < N);
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
                                                        double pre_v, double pre_g, const double* __restrict__ U,
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
  wave_project<CB>(U, N, n, k, R, e0, sx, pre_v, pre_g, partial, nw, w);
}

template <typename T>
static inline dski_status launch_proj(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                      const double* U, int k, double* partial, hipStream_t st) {
  const int nb = (proj_waves(N) + 3) / 4;
  if (R <= 16) {
    constexpr size_t sh = ProjLds<1>::bytes<T>();
    static bool done = false;
    DSKI_TRY(lds_limit(&k_ts_proj<T, 1>, sh, done));
    k_ts_proj<T, 1><<<nb, 256, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, partial);
  } else {
    constexpr size_t sh = ProjLds<2>::bytes<T>();
    static bool done = false;
    DSKI_TRY(lds_limit(&k_ts_proj<T, 2>, sh, done));
    k_ts_proj<T, 2><<<nb, 256, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, partial);
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

// z[e, c] = post_e * (pre_e * X[e, c] - sum_i U[e, i] coef[i, c]), one thread per
// row with all RB (>= R, multiple of 4) columns in registers; coef (k x R) is
// staged in LDS as chunks of kc x RB with zero padding; per-block partials of X.z stored
// output-major (dot_partial[c * blocks + block]).
template <typename T, int RB>
static __global__ __launch_bounds__(256) void k_ts_final(const T* __restrict__ X, int ld, int N, int n, int R,
                                                         double pre_v, double pre_g, double post_v, double post_g,
                                                         const double* __restrict__ U, int k,
                                                         const double* __restrict__ coef, int kc, T* __restrict__ Z,
                                                         int ldz, double* __restrict__ dot_partial) {
  extern __shared__ __align__(16) char smem[];
  double* sco = reinterpret_cast<double*>(smem);  // kc x RB
  __shared__ double red[4][RB];
  const int e = blockIdx.x * 256 + threadIdx.x;
  const bool in = e < N;
  const int ec = in ? e : N - 1;
  double acc[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) acc[c] = 0.0;
  // X first: its loads overlap the U stream below
  double xv[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) xv[c] = (double)ld_or0(X, (size_t)c * ld + e, 0, in && c < R);
  for (int i0 = 0; i0 < k; i0 += kc) {
    const int kn = min(kc, k - i0);
    if (i0 > 0) __syncthreads();
    for (int f = threadIdx.x; f < kn * RB; f += 256) {
      const int i = f / RB, c = f % RB;
      sco[f] = c < R ? coef[(i0 + i) * R + c] : 0.0;
    }
    __syncthreads();
    // U rows in blocks of 16, the next block loaded while the current one is used
    constexpr int KB = 16;
    double u[KB], un[KB];
    int i = 0;
    if (kn >= KB) {
#pragma unroll
      for (int j = 0; j < KB; ++j) u[j] = U[(size_t)(i0 + j) * N + ec];
    }
    for (; i + KB <= kn; i += KB) {
      const bool more = i + 2 * KB <= kn;
      if (more) {
#pragma unroll
        for (int j = 0; j < KB; ++j) un[j] = U[(size_t)(i0 + i + KB + j) * N + ec];
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        const double* cr = sco + (i + j) * RB;
#pragma unroll
        for (int c = 0; c < RB; c += 2) {
          const double2 cc = *reinterpret_cast<const double2*>(cr + c);
          acc[c] += u[j] * cc.x;
          acc[c + 1] += u[j] * cc.y;
        }
      }
      if (more) {
#pragma unroll
        for (int j = 0; j < KB; ++j) u[j] = un[j];
      }
    }
    // the remaining rows (fewer than KB): loads issued together, then used
    if (i < kn) {
#pragma unroll
      for (int j = 0; j < KB; ++j) u[j] = i + j < kn ? U[(size_t)(i0 + i + j) * N + ec] : 0.0;
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        if (i + j < kn) {
          const double* cr = sco + (i + j) * RB;
#pragma unroll
          for (int c = 0; c < RB; c += 2) {
            const double2 cc = *reinterpret_cast<const double2*>(cr + c);
            acc[c] += u[j] * cc.x;
            acc[c + 1] += u[j] * cc.y;
          }
        }
      }
    }
  }
  const double pre = e < n ? pre_v : pre_g, post = e < n ? post_v : post_g;
#pragma unroll
  for (int c = 0; c < RB; ++c) {
    double dot = 0.0;
    if (in && c < R) {
      const T z = (T)(post * (pre * xv[c] - acc[c]));
      Z[(size_t)c * ldz + e] = z;
      dot = xv[c] * (double)z;
    }
    acc[c] = dot;
  }
  if (dot_partial) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < RB; ++c) {
      if (c < R) {
        const double v = wave_sum64(acc[c]);
        if (lane == 0) red[wv][c] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < R) {
      const int c = threadIdx.x;
      dot_partial[(size_t)c * gridDim.x + blockIdx.x] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    }
  }
}

template <typename T>
static inline dski_status launch_final(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                       double post_v, double post_g, const double* U, int k,
                                       const double* coef, T* Z, int ldz, double* dot_partial, hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  const int nb = (N + 255) / 256;
  const int RB = pad4(R);
  const int kc = std::max(1, std::min(std::max(k, 1), 6144 / RB));  // coef rows per LDS chunk (<= 48 KiB)
  const size_t sh = sizeof(double) * (size_t)kc * RB;
#define DSKI_FINAL_CASE(V)                                                                                   \
  case V:                                                                                                    \
    k_ts_final<T, V><<<nb, 256, sh, st>>>(X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef, kc, Z, \
                                          ldz, dot_partial);                                                    \
    break;
  switch (RB) {
    DSKI_FINAL_CASE(4)
    DSKI_FINAL_CASE(8)
    DSKI_FINAL_CASE(12)
    DSKI_FINAL_CASE(16)
    DSKI_FINAL_CASE(20)
    DSKI_FINAL_CASE(24)
    DSKI_FINAL_CASE(28)
    DSKI_FINAL_CASE(32)
    default:
      set_error("at most %d columns per tall-skinny launch", kFinalMaxR);
      return DSKI_ENOTSUP;
  }
#undef DSKI_FINAL_CASE
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

}  // namespace dski
