// Tall-skinny products with the N x k preconditioner factor U (FP64, column-
// major), shared by the preconditioner and the fused PCG iteration (device
// helpers and kernels that each translation unit instantiates for itself).
//
//   projection  t = U^T v        v = pre .* X staged in LDS (row tile of RT rows,
//                                columns padded to a multiple of 4 with zeros),
//                                U staged in sub-tiles of SUBR rows; every thread
//                                owns 2 x 4 outputs per task and streams the rows
//                                of the sub-tile from LDS (no branches in the row
//                                loop); per-tile partials are written
//                                output-major and reduced in a fixed order.
//   correction  z = post .* (pre .* X - U coef)   one thread per row, all columns
//                                in registers (padded to a multiple of 4), coef
//                                in LDS, U loads issued 8 at a time.
// Global loads into LDS are issued in batches of four per thread so that
// several are in flight before the first wait.  With R = 17 these products do
// about 6 flops per byte, below the vector-ALU ridge: they stay on the vector
// units.
#pragma once

#include <algorithm>

#include "internal.h"

namespace dski {

constexpr int kFinalMaxR = 32;  // columns per tall-skinny launch

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
inline int pad2(int x) { return (x + 1) & ~1; }

// Launch plan of a projection: row tile RT, padded widths, U sub-tile rows,
// task split and the LDS layout  [sx: RT x RP][sU: SUBR x KP][sred: 2 x KP x RP].
struct ProjPlan {
  int RT = 128;    // rows per work-group
  int RP = 4;      // columns, padded to 4
  int KP = 2;      // rank, padded to 2
  int SUBR = 64;   // U rows per LDS sub-tile
  int S = 1;       // row splits of a sub-tile (1 or 2)
  int tasks = 0;   // (KP/2) (RP/4) S
  int tpt = 1;     // tasks per thread: 1, 2, 4 or 8
  size_t oU = 0, ored = 0, bytes = 0;
  int nblk(int N) const { return (N + RT - 1) / RT; }
};

inline ProjPlan proj_plan(int k, int R, int RT) {
  ProjPlan P;
  P.RT = RT;
  P.RP = pad4(std::max(R, 1));
  P.KP = pad2(std::max(k, 1));
  P.SUBR = 64;
  while (P.SUBR > 16 && (size_t)P.SUBR * P.KP * sizeof(double) > 32768) P.SUBR /= 2;
  const int t1 = (P.KP / 2) * (P.RP / 4);
  P.S = t1 <= 128 ? 2 : 1;
  P.tasks = t1 * P.S;
  P.tpt = 1;
  while (P.tpt * 256 < P.tasks) P.tpt *= 2;
  for (;;) {  // at most 64 KiB of LDS per work-group
    P.oU = sizeof(double) * (size_t)P.RT * P.RP;
    P.ored = P.oU + sizeof(double) * (size_t)P.SUBR * P.KP;
    P.bytes = P.ored + (P.S == 2 ? sizeof(double) * 2 * (size_t)P.KP * P.RP : 0);
    if (P.bytes <= 65536 || P.RT <= 64) break;
    P.RT /= 2;
  }
  return P;
}

// t-partials of one row tile: sx (RT x RP, FP64, zero-padded) is in LDS; U rows
// e0 .. e0 + rn - 1 are staged through sU.  Writes partial[(i R + c) nblk + blk]
// for i < k, c < R.  Called by all 256 threads (contains barriers).
template <int TPT>
__device__ __forceinline__ void tile_project(const double* __restrict__ U, int N, int k, int R, int e0, int rn,
                                             const ProjPlan& L, const double* __restrict__ sx,
                                             double* __restrict__ sU, double* __restrict__ sred,
                                             double* __restrict__ partial) {
  const int KP = L.KP, RP = L.RP, SUBR = L.SUBR, S = L.S;
  const int ni = KP / 2, nc = RP / 4;
  const int half = SUBR / S;
  int ib[TPT], cb[TPT], hs[TPT];
  double acc[TPT][2][4];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    int task = threadIdx.x + 256 * q;
    if (task >= L.tasks) task = L.tasks - 1;  // idle duplicate, never written
    hs[q] = task % S;
    int rest = task / S;
    cb[q] = rest % nc;
    ib[q] = rest / nc;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[q][a][j] = 0.0;
  }
  // U sub-tiles: each thread holds its share (<= 16 values, SUBR KP <= 4096) of
  // the next sub-tile in registers while the current one is used from LDS
  const int tot = SUBR * KP;
  double cur[16], nxt[16];
  auto load_sub = [&](int s0, double (&v)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int f = threadIdx.x + 256 * u;
      const int i = f / SUBR, r = f % SUBR;
      v[u] = (f < tot && i < k && s0 + r < rn) ? U[(size_t)i * N + e0 + s0 + r] : 0.0;
    }
  };
  load_sub(0, cur);
  for (int s0 = 0; s0 < rn; s0 += SUBR) {
    __syncthreads();  // previous sub-tile consumed
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int f = threadIdx.x + 256 * u;
      if (f < tot) sU[(f % SUBR) * KP + f / SUBR] = cur[u];
    }
    const bool more = s0 + SUBR < rn;
    if (more) load_sub(s0 + SUBR, nxt);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const double* up = sU + (size_t)hs[q] * half * KP + 2 * ib[q];
      const double* xp = sx + (size_t)(s0 + hs[q] * half) * RP + 4 * cb[q];
      for (int r0 = 0; r0 < half; r0 += 4) {  // half is a multiple of 4
        double2 u[4], x01[4], x23[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // all reads of 4 rows before the first use
          u[j] = *reinterpret_cast<const double2*>(up + (size_t)(r0 + j) * KP);
          x01[j] = *reinterpret_cast<const double2*>(xp + (size_t)(r0 + j) * RP);
          x23[j] = *reinterpret_cast<const double2*>(xp + (size_t)(r0 + j) * RP + 2);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[q][0][0] += u[j].x * x01[j].x;
          acc[q][0][1] += u[j].x * x01[j].y;
          acc[q][0][2] += u[j].x * x23[j].x;
          acc[q][0][3] += u[j].x * x23[j].y;
          acc[q][1][0] += u[j].y * x01[j].x;
          acc[q][1][1] += u[j].y * x01[j].y;
          acc[q][1][2] += u[j].y * x23[j].x;
          acc[q][1][3] += u[j].y * x23[j].y;
        }
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
    }
  }
  const int nblk = gridDim.x;
  if (S == 1) {
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      if (threadIdx.x + 256 * q >= L.tasks) continue;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = 2 * ib[q] + a, c = 4 * cb[q] + j;
          if (i < k && c < R) partial[((size_t)i * R + c) * nblk + blockIdx.x] = acc[q][a][j];
        }
    }
    return;
  }
  // S == 2: add the two row halves in a fixed order
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    if (threadIdx.x + 256 * q >= L.tasks) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        sred[((size_t)hs[q] * KP + 2 * ib[q] + a) * RP + 4 * cb[q] + j] = acc[q][a][j];
  }
  __syncthreads();
  for (int f = threadIdx.x; f < k * R; f += 256) {
    const int i = f / R, c = f % R;
    partial[(size_t)f * nblk + blockIdx.x] = sred[(size_t)i * RP + c] + sred[((size_t)KP + i) * RP + c];
  }
}

// Standalone projection: partials of t = U^T (pre .* X) over row tiles of L.RT rows.
template <typename T, int TPT>
static __global__ __launch_bounds__(256) void k_ts_proj(const T* __restrict__ X, int ld, int N, int n, int R,
                                                        double pre_v, double pre_g, const double* __restrict__ U,
                                                        int k, ProjPlan L, double* __restrict__ partial) {
  extern __shared__ __align__(16) char smem[];
  double* sx = reinterpret_cast<double*>(smem);
  double* sU = reinterpret_cast<double*>(smem + L.oU);
  double* sred = reinterpret_cast<double*>(smem + L.ored);
  const int RT = L.RT, RP = L.RP;
  const int e0 = blockIdx.x * RT;
  const int rn = min(RT, N - e0);
  const int tot = RT * RP;
  for (int f0 = threadIdx.x; f0 < tot; f0 += 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + 256 * u;
      const int c = f / RT, r = f % RT;
      const int e = e0 + r;
      v[u] = (f < tot && c < R && r < rn) ? (e < n ? pre_v : pre_g) * (double)X[(size_t)c * ld + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + 256 * u;
      if (f < tot) sx[(f % RT) * RP + f / RT] = v[u];
    }
  }
  tile_project<TPT>(U, N, k, R, e0, rn, L, sx, sU, sred, partial);
}

template <typename T>
static inline dski_status launch_proj(const T* X, int ld, int N, int n, int R, double pre_v, double pre_g,
                                      const double* U, int k, const ProjPlan& L, double* partial,
                                      hipStream_t st) {
  const int nb = L.nblk(N);
  switch (L.tpt) {
    case 1: k_ts_proj<T, 1><<<nb, 256, L.bytes, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, L, partial); break;
    case 2: k_ts_proj<T, 2><<<nb, 256, L.bytes, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, L, partial); break;
    case 4: k_ts_proj<T, 4><<<nb, 256, L.bytes, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, L, partial); break;
    default: k_ts_proj<T, 8><<<nb, 256, L.bytes, st>>>(X, ld, N, n, R, pre_v, pre_g, U, k, L, partial); break;
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
  for (int c = 0; c < RB; ++c) xv[c] = (in && c < R) ? (double)X[(size_t)c * ld + e] : 0.0;
  for (int i0 = 0; i0 < k; i0 += kc) {
    const int kn = min(kc, k - i0);
    if (i0 > 0) __syncthreads();
    for (int f = threadIdx.x; f < kn * RB; f += 256) {
      const int i = f / RB, c = f % RB;
      sco[f] = c < R ? coef[(i0 + i) * R + c] : 0.0;
    }
    __syncthreads();
    // U rows in blocks of 8, the next block loaded while the current one is used
    double u[8], un[8];
    int i = 0;
    if (kn >= 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) u[j] = U[(size_t)(i0 + j) * N + ec];
    }
    for (; i + 8 <= kn; i += 8) {
      const bool more = i + 16 <= kn;
      if (more) {
#pragma unroll
        for (int j = 0; j < 8; ++j) un[j] = U[(size_t)(i0 + i + 8 + j) * N + ec];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
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
        for (int j = 0; j < 8; ++j) u[j] = un[j];
      }
    }
    for (; i < kn; ++i) {
      const double uu = U[(size_t)(i0 + i) * N + ec];
      const double* cr = sco + i * RB;
#pragma unroll
      for (int c = 0; c < RB; c += 2) {
        const double2 cc = *reinterpret_cast<const double2*>(cr + c);
        acc[c] += uu * cc.x;
        acc[c + 1] += uu * cc.y;
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
