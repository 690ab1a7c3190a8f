// Tall-skinny products with the N x k preconditioner factor U, shared by the
// preconditioner and the fused PCG iteration (device helpers and kernels that
// each translation unit instantiates for itself).
#pragma once

#include "internal.h"

namespace dski {

constexpr int kFinalMaxR = 32;  // columns per tall-skinny launch

template <typename T>
inline const T* u_of(dski_precond pc);
template <>
inline const float* u_of<float>(dski_precond pc) { return pc->U; }
template <>
inline const double* u_of<double>(dski_precond pc) { return pc->Ud; }

// LDS plan of a projection tile: U tile (RT x (k+1), T), v tile (RT x R, FP64),
// coefficients (k x R, FP64), two row-split partial sums (2 x k x R, FP64); at
// most 48 KiB so that several work-groups share a CU.
struct ProjLds {
  int RT = 128;
  size_t oU = 0, ox = 0, ocoef = 0, ored = 0, bytes = 0;
};

inline ProjLds proj_lds(int k, int R, size_t tsize) {
  ProjLds L;
  for (L.RT = 128; L.RT >= 8; L.RT /= 2) {
    size_t u = ((size_t)L.RT * (k + 1) * tsize + 15) / 16 * 16;
    L.oU = 0;
    L.ox = u;
    L.ocoef = L.ox + sizeof(double) * (size_t)L.RT * R;
    L.ored = L.ocoef + sizeof(double) * (size_t)k * R;
    L.bytes = L.ored + sizeof(double) * 2 * (size_t)k * R;
    if (L.bytes <= 49152) break;
  }
  return L;
}

template <typename T>
__device__ __forceinline__ void tile_load_u(const T* __restrict__ U, int N, int k, int e0, int rn, int RT,
                                            T* __restrict__ sU) {
  for (int f = threadIdx.x; f < k * RT; f += blockDim.x) {
    int i = f / RT, r = f % RT;
    sU[r * (k + 1) + i] = r < rn ? U[(size_t)i * N + e0 + r] : (T)0;
  }
}

// partial[i, c] of sum over the tile rows of sU[r, i] * sx[r, c]; 2 x 4 outputs per
// task, rows split in two halves whose sums are added in a fixed order.
template <typename T>
__device__ __forceinline__ void tile_proj(const T* __restrict__ sU, const double* __restrict__ sx,
                                          int rn, int RT, int k, int R, double* __restrict__ sred,
                                          double* __restrict__ partial) {
  const int ni = (k + 1) / 2, nc = (R + 3) / 4;
  const int ntask = ni * nc * 2;
  const int half = RT / 2;
  for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
    int rs = task & 1, rest = task >> 1;
    int cb = rest % nc, ib = rest / nc;
    int i0 = 2 * ib, c0 = 4 * cb;
    double acc[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    int rb = rs * half, re = min(rn, rb + half);
    for (int r = rb; r < re; ++r) {
      const T* ur = sU + r * (k + 1);
      double u0 = (double)ur[i0];
      double u1 = i0 + 1 < k ? (double)ur[i0 + 1] : 0.0;
      const double* xr = sx + r * R;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double x = c0 + j < R ? xr[c0 + j] : 0.0;
        acc[0][j] += u0 * x;
        acc[1][j] += u1 * x;
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + a < k && c0 + j < R) sred[((size_t)rs * k + i0 + a) * R + c0 + j] = acc[a][j];
  }
  __syncthreads();
  // output-major partials: partial[f * blocks + block]
  for (int f = threadIdx.x; f < k * R; f += blockDim.x)
    partial[(size_t)f * gridDim.x + blockIdx.x] = sred[f] + sred[(size_t)k * R + f];
}

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

// z[e, c] = post_e * (pre_e * X[e, c] - sum_i U[e, i] coef[i, c]) for a group of
// `cg` columns per blockIdx.y (one thread per row, the group's columns in
// registers, U loads issued 8 at a time); per-block partials of X.z stored
// output-major (dot_partial[c * blocks + block]).  coef[i, c] is the same for all
// threads of a group (scalar loads).
constexpr int kFinalGroup = 8;

template <typename T>
static __global__ __launch_bounds__(256) void k_ts_final(const T* __restrict__ X, int ld, int N, int n, int R,
                                                         double pre_v, double pre_g, double post_v, double post_g,
                                                         const T* __restrict__ U, int k,
                                                         const double* __restrict__ coef, T* __restrict__ Z,
                                                         int ldz, double* __restrict__ dot_partial, int cgs) {
  __shared__ double red[4][kFinalGroup];
  const int c0 = blockIdx.y * cgs;
  const int cg = min(cgs, R - c0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[kFinalGroup];
#pragma unroll
  for (int c = 0; c < kFinalGroup; ++c) acc[c] = 0.0;
  if (e < N) {
    int i = 0;
    for (; i + 8 <= k; i += 8) {
      double u[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) u[j] = (double)U[(size_t)(i + j) * N + e];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double* cr = coef + (i + j) * R + c0;
#pragma unroll
        for (int c = 0; c < kFinalGroup; ++c)
          if (c < cg) acc[c] += u[j] * cr[c];
      }
    }
    for (; i < k; ++i) {
      double u = (double)U[(size_t)i * N + e];
      const double* cr = coef + i * R + c0;
#pragma unroll
      for (int c = 0; c < kFinalGroup; ++c)
        if (c < cg) acc[c] += u * cr[c];
    }
  }
  const double pre = e < n ? pre_v : pre_g, post = e < n ? post_v : post_g;
#pragma unroll
  for (int c = 0; c < kFinalGroup; ++c) {
    if (c < cg) {
      double dot = 0.0;
      if (e < N) {
        double x = (double)X[(size_t)(c0 + c) * ld + e];
        T z = (T)(post * (pre * x - acc[c]));
        Z[(size_t)(c0 + c) * ldz + e] = z;
        dot = x * (double)z;
      }
      acc[c] = dot;
    }
  }
  if (dot_partial) {
#pragma unroll
    for (int c = 0; c < kFinalGroup; ++c) {
      if (c < cg) {
        double v = wave_sum64(acc[c]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < cg) {
      int c = threadIdx.x;
      dot_partial[(size_t)(c0 + c) * gridDim.x + blockIdx.x] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    }
  }
}

// launch helper: balanced column groups of at most kFinalGroup columns
template <typename T>
static inline void launch_final(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                double post_v, double post_g, const T* U, int k, const double* coef, T* Z,
                                int ldz, double* dot_partial, hipStream_t st) {
  const int ng = (R + kFinalGroup - 1) / kFinalGroup;
  const int cgs = (R + ng - 1) / ng;
  dim3 grid((N + 255) / 256, ng);
  k_ts_final<T><<<grid, 256, 0, st>>>(X, ld, N, n, R, pre_v, pre_g, post_v, post_g, U, k, coef, Z, ldz,
                                      dot_partial, cgs);
}

// partial t over a row tile of  v = pre .* X - U coef  (coef may be NULL)
template <typename T>
static __global__ __launch_bounds__(256) void k_ts_proj(const T* __restrict__ X, int ld, int N, int n, int R,
                                                 double pre_v, double pre_g, const T* __restrict__ U, int k,
                                                 const double* __restrict__ coef, int RT, ProjLds L,
                                                 double* __restrict__ partial) {
  extern __shared__ __align__(16) char smem[];
  T* sU = reinterpret_cast<T*>(smem + L.oU);
  double* sx = reinterpret_cast<double*>(smem + L.ox);
  double* sred = reinterpret_cast<double*>(smem + L.ored);
  const int e0 = blockIdx.x * RT;
  const int rn = min(RT, N - e0);
  tile_load_u<T>(U, N, k, e0, rn, RT, sU);
  for (int f = threadIdx.x; f < RT * R; f += blockDim.x) {
    int r = f % RT, c = f / RT;
    int e = e0 + r;
    sx[r * R + c] = r < rn ? (e < n ? pre_v : pre_g) * (double)X[(size_t)c * ld + e] : 0.0;
  }
  if (coef) {
    double* sco = reinterpret_cast<double*>(smem + L.ocoef);
    for (int f = threadIdx.x; f < k * R; f += blockDim.x) sco[f] = coef[f];
  }
  __syncthreads();
  if (coef) {
    // sx[r, c] -= sum_i sU[r, i] coef[i, c]: 4 threads per row, each a quarter of
    // the columns in registers; U and coef read from LDS
    double* sco = reinterpret_cast<double*>(smem + L.ocoef);
    const int cq = (R + 3) / 4;
    for (int task = threadIdx.x; task < rn * 4; task += blockDim.x) {
      const int r = task >> 2, c0 = (task & 3) * cq;
      const int cn = min(cq, R - c0);
      double acc[kFinalMaxR / 4];
#pragma unroll
      for (int c = 0; c < kFinalMaxR / 4; ++c) acc[c] = 0.0;
      const T* ur = sU + r * (k + 1);
      for (int i = 0; i < k; ++i) {
        double u = (double)ur[i];
        const double* cr = sco + i * R + c0;
#pragma unroll
        for (int c = 0; c < kFinalMaxR / 4; ++c)
          if (c < cn) acc[c] += u * cr[c];
      }
#pragma unroll
      for (int c = 0; c < kFinalMaxR / 4; ++c)
        if (c < cn) sx[r * R + c0 + c] -= acc[c];
    }
    __syncthreads();
  }
  tile_proj<T>(sU, sx, rn, RT, k, R, sred, partial);
}

// Wavefront-shuffle variant of the projection: grid (row blocks of 256, column
// groups of `cgs`); each thread owns one row and its group's columns,
//   v = pre .* X - U coef   (coef may be NULL),
// and every output (i, c) is a wavefront shuffle-tree sum over the block's rows,
// combined over the 4 wavefronts in a fixed order.  No LDS tiles, many blocks.
constexpr int kShflGroup = 4;
constexpr int kShflChunk = 32;

template <typename T>
__device__ __forceinline__ void shfl_project(const T* __restrict__ U, int N, int e, int k, int R, int c0,
                                             int cg, const double v[kShflGroup],
                                             double (*red)[kShflChunk][kShflGroup],
                                             double* __restrict__ partial) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = 0; i0 < k; i0 += kShflChunk) {
    const int ni = min(kShflChunk, k - i0);
    for (int ii = 0; ii < ni; ++ii) {
      double u = e < N ? (double)U[(size_t)(i0 + ii) * N + e] : 0.0;
#pragma unroll
      for (int c = 0; c < kShflGroup; ++c) {
        if (c < cg) {
          double sm = wave_sum64(u * v[c]);
          if (lane == 0) red[wv][ii][c] = sm;
        }
      }
    }
    __syncthreads();
    for (int f = threadIdx.x; f < ni * cg; f += blockDim.x) {
      int ii = f / cg, c = f % cg;
      double t = red[0][ii][c] + red[1][ii][c] + red[2][ii][c] + red[3][ii][c];
      partial[((size_t)(i0 + ii) * R + c0 + c) * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

template <typename T>
static __global__ __launch_bounds__(256) void k_ts_proj_shfl(const T* __restrict__ X, int ld, int N, int n, int R,
                                                             double pre_v, double pre_g, const T* __restrict__ U,
                                                             int k, const double* __restrict__ coef, int cgs,
                                                             double* __restrict__ partial) {
  __shared__ double red[4][kShflChunk][kShflGroup];
  const int c0 = blockIdx.y * cgs;
  const int cg = min(cgs, R - c0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double v[kShflGroup];
#pragma unroll
  for (int c = 0; c < kShflGroup; ++c) v[c] = 0.0;
  if (e < N) {
    const double pre = e < n ? pre_v : pre_g;
#pragma unroll
    for (int c = 0; c < kShflGroup; ++c)
      if (c < cg) v[c] = pre * (double)X[(size_t)(c0 + c) * ld + e];
    if (coef) {
      for (int i = 0; i < k; ++i) {
        double u = (double)U[(size_t)i * N + e];
        const double* cr = coef + i * R + c0;
#pragma unroll
        for (int c = 0; c < kShflGroup; ++c)
          if (c < cg) v[c] -= u * cr[c];
      }
    }
  }
  shfl_project<T>(U, N, e, k, R, c0, cg, v, red, partial);
}

template <typename T>
static inline void launch_proj_shfl(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                    const T* U, int k, const double* coef, double* partial, int* nblk,
                                    hipStream_t st) {
  const int ng = (R + kShflGroup - 1) / kShflGroup;
  const int cgs = (R + ng - 1) / ng;
  dim3 grid((N + 255) / 256, ng);
  *nblk = grid.x;
  k_ts_proj_shfl<T><<<grid, 256, 0, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, coef, cgs, partial);
}

}  // namespace dski
