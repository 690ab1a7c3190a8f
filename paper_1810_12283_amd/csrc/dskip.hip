// D-SKIP: the value-and-gradient kernel matrix of a product kernel as a
// Hadamard product of one-dimensional D-SKI factors (Sec. 3.2).
//
// For axis p the factor is the full N x N matrix (N = n(d+1), block-major)
//   Khat_p[(a,i),(b,j)] = [W_p^{(a)} T_p W_p^{(b)T}]_{ij},
// where W_p^{(a)} holds the 1-D Keys derivative weights when block a is the
// derivative along p and the value weights otherwise (eq. (skip) for d = 2).
// So Khat_p = S_p G_p S_p^T with G_p the 2n x 2n 1-D D-SKI matrix of
// coordinate p and S_p: 2n -> N the block selection.  G_p is applied with a
// one-dimensional D-SKI plan (scatter, circulant FFT, gather).
//
// Each factor is compressed by r Lanczos steps with full re-orthogonalisation
// (classical Gram-Schmidt applied twice), started from the normalised
// Rademacher column `node` of the SplitMix64 stream (leaves are nodes 0..d-1).
// For d > 2 the factors are combined by a binary tree, pairs (0,1), (2,3), ...
// level by level, an odd factor moving up unchanged; every internal node except
// the root is recompressed by r Lanczos steps on the Hadamard product of its
// children (internal nodes are numbered on from d in creation order); the root
// is the exact Hadamard product of its two rank-r children:
//   K = s^2 (Qa Ta Qa^T) o (Qb Tb Qb^T),    K~ = K + D.
//
// Root MVM (the SKIP reduction), per column v:
//   C = Qa^T diag(v) Qb                                   (r x r, a reduction over N rows)
//   y_i = sum_k (Qa Ta)_{ik} sum_l (Qb Tb)_{il} C_{kl}     (independent rows)
// 2 N r^2 FMAs per phase and column.  Factors are stored column-major N x RP,
// RP in {32, 64} (zero-padded), in FP64, with FP32 copies for the solvers' FP32
// MVM.  The FP64 MVM accumulates in FP64 on the vector ALU; the FP32 MVM runs
// both phases on the FP32 matrix cores, FP64 across wavefronts and chunks.
#include <cmath>
#include <cstring>
#include <functional>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "pivot.h"
#include "tskinny.h"

namespace dski {

struct DskipFactor {
  int k = 0;              // Lanczos vectors kept
  double* Q = nullptr;    // N x RP, column-major, zero beyond k
  double* A = nullptr;    // Q T
};

struct DskipData {
  int m1 = 0, r = 0, RP = 0;
  uint64_t seed = 0;
  std::vector<double> ell;
  bool built = false;
  std::vector<dski_plan> sub;     // 1-D D-SKI plans, one per axis (2n-vectors)
  std::vector<int*> iperm;        // user index -> tile position of each sub-plan (device)
  DskipFactor fa, fb;             // root factors (FP64)
  float* Qa32 = nullptr;          // FP32 copies of the root factors
  float* Aa32 = nullptr;
  float* Qb32 = nullptr;
  float* Ab32 = nullptr;
  DevBuf work;                    // Lanczos work vectors
  DevBuf gram;                    // Hadamard partials and Gram matrices
  DevBuf rows;                    // pivot rows of the root factors (pivoted Cholesky)
};

// Scratch buffer released when it goes out of scope (error paths included).
struct TmpBuf : DevBuf {
  ~TmpBuf() { release(); }
};

// ---------------------------------------------------------------- elementwise kernels
__global__ void k_extract_col(const double* __restrict__ X, int n, int d, int p, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[(size_t)i * d + p];
}

__global__ void k_inverse_perm(const int* __restrict__ perm, int n, int* __restrict__ iperm) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) iperm[perm[k]] = k;
}

// u = S_p^T q in the sub-plan's tile order: value part sums the blocks a != p+1.
__global__ void k_compress(const double* __restrict__ q, int n, int d, int p, const int* __restrict__ perm,
                           double* __restrict__ u) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int i = perm[k];
  double val = 0.0;
  for (int a = 0; a <= d; ++a)
    if (a != p + 1) val += q[(size_t)a * n + i];
  u[k] = val;
  u[n + k] = q[(size_t)(p + 1) * n + i];
}

// w = S_p y (y in the sub-plan's tile order).
__global__ void k_expand(const double* __restrict__ y, int n, int d, int p, const int* __restrict__ iperm,
                         double* __restrict__ w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = iperm[i];
  double val = y[k], der = y[n + k];
  for (int a = 0; a <= d; ++a) w[(size_t)a * n + i] = (a == p + 1) ? der : val;
}

__global__ void k_scale_copy(const double* __restrict__ x, int N, double s, double* __restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = s * x[i];
}

// Per-block partial dots of the first ncol columns of Q with w, output-major:
// part[c * gridDim.x + b].  Grid (nb, ncol).
__global__ void k_cols_dot(const double* __restrict__ Q, int N, const double* __restrict__ w,
                           double* __restrict__ part) {
  const int c = blockIdx.y;
  double a = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    a += Q[(size_t)c * N + i] * w[i];
  a = wave_sum64(a);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)c * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w -= Q[:, :ncol] h  (fixed order over the columns).
__global__ void k_cols_sub(const double* __restrict__ Q, int N, int ncol, const double* __restrict__ h,
                           double* __restrict__ w) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc = w[i];
  for (int c = 0; c < ncol; ++c) acc -= Q[(size_t)c * N + i] * h[c];
  w[i] = acc;
}

// A = Q T for the first k columns (T k x k dense, row-major, in device memory).
__global__ void k_q_times_t(const double* __restrict__ Q, int N, int k, const double* __restrict__ T,
                            double* __restrict__ A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (i >= N) return;
  double acc = 0.0;
  for (int l = 0; l < k; ++l) acc += Q[(size_t)l * N + i] * T[l * k + c];
  A[(size_t)c * N + i] = acc;
}

__global__ void k_to_f32(const double* __restrict__ x, size_t len, float* __restrict__ y) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// FP32 row-major copy of a column-major N x RP factor: y[i RP + c] = x[c N + i].
__global__ void k_to_f32_rows(const double* __restrict__ x, int N, int RP, float* __restrict__ y) {
  const size_t len = (size_t)N * RP;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < len; o += (size_t)gridDim.x * blockDim.x)
    y[o] = (float)x[(o % RP) * N + o / RP];
}

// ---------------------------------------------------------------- Hadamard MVM, FP64 vector ALU
// (the FP64 MVM and the Lanczos products of the build)
// Phase 1: per-chunk partials of C_c = Qa^T diag(v_c) Qb for a group of CG
// columns.  Thread t owns the output row k = t / (RP/4) and the column quad
// l0 = 4 (t mod RP/4) (RP = 64: four such (k, quad) pairs).  Rows are staged in
// LDS tiles of 64 (column-major, padded); partials are written block-major,
// part[b * (R RP RP) + (c RP + k) RP + l], four consecutive l per thread.
template <int RP, int CG, typename TF, typename T>
__global__ __launch_bounds__(256) void k_had_gram(const TF* __restrict__ Qa, const TF* __restrict__ Qb, int N,
                                                  const T* __restrict__ V, int ldv, int R, int rows,
                                                  double* __restrict__ part) {
  constexpr int RT = 64;
  constexpr int NQ = RP * RP / 1024;
  __shared__ double sA[RP][RT + 1];
  __shared__ double sB[RP][RT + 1];
  __shared__ double sV[CG][RT + 1];
  const int c0 = blockIdx.y * CG;
  const int e0 = blockIdx.x * rows;
  const int e1 = min(N, e0 + rows);
  int kq[NQ], lq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    int o = threadIdx.x + 256 * q;
    kq[q] = o / (RP / 4);
    lq[q] = 4 * (o % (RP / 4));
  }
  double acc[NQ][4][CG];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < CG; ++c) acc[q][j][c] = 0.0;
  for (int r0 = e0; r0 < e1; r0 += RT) {
    const int rn = min(RT, e1 - r0);
    __syncthreads();
    for (int f = threadIdx.x; f < RP * RT; f += 256) {
      int k = f / RT, i = f % RT;
      bool in = i < rn;
      sA[k][i] = in ? (double)Qa[(size_t)k * N + r0 + i] : 0.0;
      sB[k][i] = in ? (double)Qb[(size_t)k * N + r0 + i] : 0.0;
    }
    for (int f = threadIdx.x; f < CG * RT; f += 256) {
      int c = f / RT, i = f % RT;
      sV[c][i] = (i < rn && c0 + c < R) ? (double)V[(size_t)(c0 + c) * ldv + r0 + i] : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < rn; ++i) {
      double vv[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) vv[c] = sV[c][i];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double a = sA[kq[q]][i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double ab = a * sB[lq[q] + j][i];
#pragma unroll
          for (int c = 0; c < CG; ++c) acc[q][j][c] += ab * vv[c];
        }
      }
    }
  }
  const size_t nout = (size_t)R * RP * RP;
  double* pb = part + (size_t)blockIdx.x * nout;
#pragma unroll
  for (int c = 0; c < CG; ++c) {
    if (c0 + c >= R) break;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double* o = pb + ((size_t)(c0 + c) * RP + kq[q]) * RP + lq[q];
      reinterpret_cast<double2*>(o)[0] = make_double2(acc[q][0][c], acc[q][1][c]);
      reinterpret_cast<double2*>(o)[1] = make_double2(acc[q][2][c], acc[q][3][c]);
    }
  }
}

// C[f] = sum over chunks b of part[b * nout + f], in the order b = s, s + 4, ...
// for the four slices s, then slices 0 + 1 + 2 + 3.  64 outputs per block.
// Sum over chunks b = s, s + 4, ... of the slice s (four loads in flight, added
// in order), then slices 0 + 1 + 2 + 3.
__device__ __forceinline__ double had_slice_sum(const double* __restrict__ part, int nchunk, size_t nout, size_t f,
                                                int s) {
  double a = 0.0;
  int b = s;
  for (; b + 12 < nchunk; b += 16) {
    const double x0 = part[(size_t)b * nout + f], x1 = part[(size_t)(b + 4) * nout + f];
    const double x2 = part[(size_t)(b + 8) * nout + f], x3 = part[(size_t)(b + 12) * nout + f];
    a += x0;
    a += x1;
    a += x2;
    a += x3;
  }
  for (; b < nchunk; b += 4) a += part[(size_t)b * nout + f];
  return a;
}

__global__ void k_had_reduce(const double* __restrict__ part, int nchunk, int nout, double* __restrict__ C) {
  __shared__ double red[4][64];
  const int fl = threadIdx.x & 63, s = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + fl;
  red[s][fl] = f < nout ? had_slice_sum(part, nchunk, nout, f, s) : 0.0;
  __syncthreads();
  if (s == 0 && f < nout) C[f] = ((red[0][fl] + red[1][fl]) + red[2][fl]) + red[3][fl];
}

// The same sums, written in FP32 as the matrix-core fragments of phase 2:
// C_c[16g + m][4s + kk] goes to Cf[(((c H + g) 4 + kk) 16 + m) S + s]
// (H = RP/16, S = RP/4), so that lane l = 16 kk + m of a wavefront finds its S
// operands of (c, g) contiguous and the lanes follow one another.
template <int RP>
__global__ void k_had_reduce_frag(const double* __restrict__ part, int nchunk, int R, float* __restrict__ Cf) {
  constexpr int H = RP / 16, S = RP / 4;
  __shared__ double red[4][64];
  const int nout = R * RP * RP;
  const int fl = threadIdx.x & 63, s = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + fl;
  red[s][fl] = f < nout ? had_slice_sum(part, nchunk, nout, f, s) : 0.0;
  __syncthreads();
  if (s == 0 && f < nout) {
    const int c = f / (RP * RP), k = (f / RP) % RP, l = f % RP;
    const int g = k / 16, m = k % 16, kk = l % 4, st = l / 4;
    Cf[(((c * H + g) * 4 + kk) * 16 + m) * S + st] = (float)(((red[0][fl] + red[1][fl]) + red[2][fl]) + red[3][fl]);
  }
}

// Phase 2: Y_c = ks * rowsum(Aa o (Ab C_c^T)) + D V_c, one thread per row,
// CG2 columns per block with their C_c in LDS; optional per-block partials of
// V_c . Y_c, output-major pq[c * gridDim.x + b].
template <int RP, int CG2, typename TF, typename T>
__global__ __launch_bounds__(256) void k_had_apply(const TF* __restrict__ Aa, const TF* __restrict__ Ab, int N,
                                                   int n, const double* __restrict__ C, int R,
                                                   const T* __restrict__ V, int ldv, T* __restrict__ Y, int ldy,
                                                   double ks, double nv, double ng, double* __restrict__ pq) {
  __shared__ double sC[CG2][RP][RP];
  __shared__ double red[4];
  const int c0 = blockIdx.y * CG2;
  for (int f = threadIdx.x; f < CG2 * RP * RP; f += 256) {
    int c = f / (RP * RP);
    (&sC[0][0][0])[f] = c0 + c < R ? C[(size_t)c0 * RP * RP + f] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  double acc[CG2];
#pragma unroll
  for (int c = 0; c < CG2; ++c) acc[c] = 0.0;
  if (i < N) {
    double b[RP];
#pragma unroll
    for (int l = 0; l < RP; ++l) b[l] = (double)Ab[(size_t)l * N + i];
    for (int k = 0; k < RP; ++k) {
      const double a = (double)Aa[(size_t)k * N + i];
#pragma unroll
      for (int c = 0; c < CG2; ++c) {
        const double* cr = &sC[c][k][0];
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < RP; ++l) s += b[l] * cr[l];
        acc[c] += a * s;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CG2; ++c) {
    if (c0 + c >= R) break;
    double dot = 0.0;
    if (i < N) {
      double v = (double)V[(size_t)(c0 + c) * ldv + i];
      T out = (T)(ks * acc[c] + (i < n ? nv : ng) * v);
      Y[(size_t)(c0 + c) * ldy + i] = out;
      dot = v * (double)out;
    }
    if (pq) {
      dot = wave_sum64(dot);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
      __syncthreads();
      if (threadIdx.x == 0)
        pq[(size_t)(c0 + c) * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
  }
}

// ---------------------------------------------------------------- Hadamard MVM, matrix cores
// The FP32 root MVM of the solvers runs both phases on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, D += A B with A 16 x 4 and B 4 x 16: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; register r of lane l holds D[4(l/16) + r][l%16]).
// The FP32 matrix cores of this GPU deliver about three times the FP64 ones.
// A wavefront accumulates at most a few hundred rows in FP32; wavefronts,
// work-groups and the row sums of phase 2 are added in FP64 (relative error a
// few 1e-7, against 1e-5 required for FP32 MVMs).
// Qa and Qb have FP32 row-major copies (N x RP) for the Gram phase, Qa Ta and
// Qb Tb stay column-major: in both phases a wavefront's operand loads are runs
// of 16 consecutive floats.  Each wavefront loads the operands of its next step
// while the matrix cores work on the current one.
typedef float had_flt4 __attribute__((ext_vector_type(4)));

// Phase 1: per-chunk partials of C_c = Qa^T diag(v_c) Qb, contracting over the
// rows four at a time: A[m][kk] = Qa[i0 + kk][16h + m] v_c[i0 + kk] and
// B[kk][j] = Qb[i0 + kk][16g + j], so lane l loads entry 16h + l%16 of row
// i0 + l/16 of each row-major copy.  The 8 wavefronts of a work-group take
// interleaved 4-row steps of the chunk; their tiles are added in FP64 through
// LDS one 16-row band of one column at a time (wave order fixed), and written
// block-major, part[b * (R RP RP) + (c RP + k) RP + l].
template <int RP, int CG>
struct GramStep {
  float qa[RP / 16], qb[RP / 16], v[CG];
  bool ok;  // the row belongs to this chunk: applied to v at use, so that the
            // prefetch never waits for its loads
};

template <int RP, int CG>
__device__ __forceinline__ void gram_load(GramStep<RP, CG>& o, const float* __restrict__ Qar,
                                          const float* __restrict__ Qbr, const float* __restrict__ V, int ldv,
                                          int R, int c0, int i, bool ok, int lc) {
  const size_t row = ok ? (size_t)i : 0;  // row 0 stands in for rows outside the chunk
#pragma unroll
  for (int h = 0; h < RP / 16; ++h) {
    o.qa[h] = Qar[row * RP + 16 * h + lc];
    o.qb[h] = Qbr[row * RP + 16 * h + lc];
  }
#pragma unroll
  for (int c = 0; c < CG; ++c) o.v[c] = V[(size_t)min(c0 + c, R - 1) * ldv + row];
  o.ok = ok;
}

template <int RP, int CG>
__global__ __launch_bounds__(512) void k_had_gram_mfma(const float* __restrict__ Qar, const float* __restrict__ Qbr,
                                                       int N, const float* __restrict__ V, int ldv, int R, int rows,
                                                       double* __restrict__ part) {
  constexpr int H = RP / 16;
  constexpr int NW = 8;
  __shared__ double red[NW - 1][16 * RP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int c0 = blockIdx.y * CG;
  const int e0 = blockIdx.x * rows;
  const int e1 = min(N, e0 + rows);
  had_flt4 acc[CG][H][H];
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int g = 0; g < H; ++g) acc[c][h][g] = had_flt4{0.f, 0.f, 0.f, 0.f};
  // macro-steps of MS 4-row steps; the operands of the next macro-step are
  // loaded while the current one runs
  constexpr int MS = RP == 32 ? 4 : 2;
  GramStep<RP, CG> cur[MS];
  int i0 = e0 + 4 * wv;
#pragma unroll
  for (int q = 0; q < MS; ++q) {
    const int i = i0 + 4 * NW * q + lr;
    gram_load<RP, CG>(cur[q], Qar, Qbr, V, ldv, R, c0, i, i < e1, lc);
  }
  for (; i0 < e1; i0 += 4 * NW * MS) {
    GramStep<RP, CG> nxt[MS];
#pragma unroll
    for (int q = 0; q < MS; ++q) {
      const int i = i0 + 4 * NW * (MS + q) + lr;
      gram_load<RP, CG>(nxt[q], Qar, Qbr, V, ldv, R, c0, i, i < e1, lc);
    }
    // keep the prefetch ahead of the products (the scheduler would otherwise
    // sink the loads next to their first use at the end of the macro-step)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < MS; ++q) {
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        // rows outside the chunk and columns beyond R contribute zero
        const float vv = cur[q].ok && c0 + c < R ? cur[q].v[c] : 0.f;
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const float a = cur[q].qa[h] * vv;
#pragma unroll
          for (int g = 0; g < H; ++g)
            acc[c][h][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, cur[q].qb[g], acc[c][h][g], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < MS; ++q) cur[q] = nxt[q];
  }
  const size_t nout = (size_t)R * RP * RP;
  double* pb = part + (size_t)blockIdx.x * nout;
#pragma unroll
  for (int c = 0; c < CG; ++c) {
    if (c0 + c >= R) break;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      if (wv > 0) {
#pragma unroll
        for (int g = 0; g < H; ++g)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wv - 1][(4 * lr + r) * RP + 16 * g + lc] = (double)acc[c][h][g][r];
      }
      __syncthreads();
      if (wv == 0) {
#pragma unroll
        for (int g = 0; g < H; ++g)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = (4 * lr + r) * RP + 16 * g + lc;
            double t = (double)acc[c][h][g][r];
#pragma unroll
            for (int w = 0; w < NW - 1; ++w) t += red[w][o];
            pb[((size_t)(c0 + c) * RP + 16 * h + 4 * lr + r) * RP + 16 * g + lc] = t;
          }
      }
      __syncthreads();
    }
  }
}

// Phase 2: Y_c = ks * rowsum(Aa o (Ab C_c^T)) + D V_c, per 16-row tile as the
// transposed product P^T = C_c Ab^T contracting over l four at a time:
// A[m][kk] = C_c[16g + m][4s + kk] (rounded to FP32, in registers for the
// wavefront's CG2 columns) and B[kk][j] = Ab[i0 + j][4s + kk].  Register r of
// lane l then holds P[i0 + l%16][16g + 4(l/16) + r]: each lane multiplies its
// entries by the matching ones of Aa and adds them in FP64, and the four lanes
// of a row (l, l + 16, l + 32, l + 48) add theirs; lanes 0..15 write rows
// i0..i0+15.  A wavefront covers 64 rows (4 tiles), a work-group 256 rows;
// per-block partials of V_c . Y_c are output-major, pq[c * gridDim.x + b].
template <int RP>
struct ApplyTile {
  float ab[RP / 4], aa[RP / 16][4];
};

template <int RP>
__device__ __forceinline__ void apply_load(ApplyTile<RP>& o, const float* __restrict__ Aa,
                                           const float* __restrict__ Ab, int N, int i0, int lr, int lc) {
  const bool ok = i0 + lc < N;
  const size_t i = ok ? (size_t)(i0 + lc) : 0;
#pragma unroll
  for (int s = 0; s < RP / 4; ++s) o.ab[s] = ld_or0(Ab, (size_t)(4 * s + lr) * N + i, (size_t)(4 * s + lr) * N, ok);
#pragma unroll
  for (int g = 0; g < RP / 16; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      o.aa[g][r] = ld_or0(Aa, (size_t)(16 * g + 4 * lr + r) * N + i, (size_t)(16 * g + 4 * lr + r) * N, ok);
}

template <int RP, int CG2>
__global__ __launch_bounds__(256) void k_had_apply_mfma(const float* __restrict__ Aa, const float* __restrict__ Ab,
                                                        int N, int n, const float* __restrict__ Cf, int R,
                                                        const float* __restrict__ V, int ldv, float* __restrict__ Y,
                                                        int ldy, double ks, double nv, double ng,
                                                        double* __restrict__ pq) {
  constexpr int H = RP / 16;
  constexpr int S = RP / 4;
  constexpr int FR = H * 64 * S;  // fragment floats per column
  __shared__ double red[CG2][4];
  __shared__ float4 sC[CG2 * FR / 4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int c0 = blockIdx.y * CG2;
  const int base = blockIdx.x * 256 + wv * 64;
  // every operand of the wavefront's 4 tiles is requested before the first product
  ApplyTile<RP> tile[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) apply_load<RP>(tile[t], Aa, Ab, N, base + 16 * t, lr, lc);
  float xv[4][CG2];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < CG2; ++c) {
      const int row = base + 16 * t + lc;
      const size_t vo = (size_t)min(c0 + c, R - 1) * ldv;
      xv[t][c] = ld_or0(V, vo + row, vo, lr == 0 && row < N && c0 + c < R);
    }
  // the fragments of this work-group's columns (zero beyond R) through LDS
  {
    const int nc = min(CG2, R - c0);
    const float4* src = reinterpret_cast<const float4*>(Cf + (size_t)c0 * FR);
    for (int e = threadIdx.x; e < CG2 * FR / 4; e += 256)
      sC[e] = e < nc * FR / 4 ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  float cf[CG2][H][S];
#pragma unroll
  for (int c = 0; c < CG2; ++c)
#pragma unroll
    for (int g = 0; g < H; ++g)
#pragma unroll
      for (int q = 0; q < S / 4; ++q) {
        const float4 w = sC[(((c * H + g) * 64 + lane) * S) / 4 + q];
        cf[c][g][4 * q] = w.x;
        cf[c][g][4 * q + 1] = w.y;
        cf[c][g][4 * q + 2] = w.z;
        cf[c][g][4 * q + 3] = w.w;
      }
  double dot[CG2];
#pragma unroll
  for (int c = 0; c < CG2; ++c) dot[c] = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i0 = base + 16 * t;
    if (i0 >= N) break;  // uniform over the wavefront
    had_flt4 acc[CG2][H];
#pragma unroll
    for (int c = 0; c < CG2; ++c)
#pragma unroll
      for (int g = 0; g < H; ++g) acc[c][g] = had_flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int c = 0; c < CG2; ++c)
#pragma unroll
        for (int g = 0; g < H; ++g)
          acc[c][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(cf[c][g][s], tile[t].ab[s], acc[c][g], 0, 0, 0);
    const int row = i0 + lc;
#pragma unroll
    for (int c = 0; c < CG2; ++c) {
      if (c0 + c >= R) break;
      double v = 0.0;
#pragma unroll
      for (int g = 0; g < H; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) v += (double)tile[t].aa[g][r] * (double)acc[c][g][r];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      const bool wr = lr == 0 && row < N;
      const double x = (double)xv[t][c];
      const float out = (float)(ks * v + (row < n ? nv : ng) * x);
      if (wr) Y[(size_t)(c0 + c) * ldy + row] = out;
      dot[c] += wr ? x * (double)out : 0.0;
    }
  }
  if (pq) {
#pragma unroll
    for (int c = 0; c < CG2; ++c) {
      if (c0 + c >= R) break;
      const double w = wave_sum64(dot[c]);
      if (lane == 0) red[c][wv] = w;
    }
    __syncthreads();
    if (threadIdx.x < CG2 && c0 + (int)threadIdx.x < R) {
      const int c = threadIdx.x;
      pq[(size_t)(c0 + c) * gridDim.x + blockIdx.x] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
    }
  }
}

// Row chunks of the Gram phase: enough work-groups to fill the CUs, at least 64
// rows each; for wide blocks the partial volume (chunks x R RP^2) caps the count.
static int had_chunks(int N, int R) {
  int cap = R == 1 ? 256 : 64;
  return std::max(1, std::min(cap, (N + 63) / 64));
}

// Y = ks (A o B) V + D V with A = Qa Ta Qa^T, B = Qb Tb Qb^T given as (Q, Q T).
template <int RP, typename TF, typename T>
static dski_status had_apply_rp(DevBuf& gram, const TF* Qa, const TF* Aa, const TF* Qb, const TF* Ab, int N,
                                int n, int R, const T* V, int ldv, T* Y, int ldy, double ks, double nv,
                                double ng, double* pq, hipStream_t st) {
  if constexpr (std::is_same<TF, float>::value && std::is_same<T, float>::value) {
    // matrix-core form (FP32 factors in the layouts the kernels expect)
    // 6 columns per wavefront at rank 32 (a 17-column block is 3 near-equal
    // groups), 2 at rank 64; about one Gram work-group per CU
    constexpr int MG = RP == 32 ? 6 : 2;
    const int ng1 = (R + MG - 1) / MG;
    const int nchunk = std::max(1, std::min((N + 255) / 256, 255 / ng1));
    const int rows = (N + nchunk - 1) / nchunk;
    const size_t nout = (size_t)R * RP * RP;
    DSKI_TRY(gram.reserve(sizeof(double) * (nout * (size_t)nchunk + nout) + 256));
    double* part = gram.as<double>();
    float* Cf = reinterpret_cast<float*>(part + nout * (size_t)nchunk);
    k_had_gram_mfma<RP, MG><<<dim3(nchunk, ng1), 512, 0, st>>>(Qa, Qb, N, V, ldv, R, rows, part);
    DSKI_HIP(hipGetLastError());
    k_had_reduce_frag<RP><<<(unsigned)((nout + 63) / 64), 256, 0, st>>>(part, nchunk, R, Cf);
    DSKI_HIP(hipGetLastError());
    constexpr int AG = RP == 32 ? 3 : 1;  // columns per apply wavefront: two wavefronts per SIMD
    k_had_apply_mfma<RP, AG><<<dim3((N + 255) / 256, (R + AG - 1) / AG), 256, 0, st>>>(Aa, Ab, N, n, Cf, R, V, ldv,
                                                                                      Y, ldy, ks, nv, ng, pq);
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  } else {
    constexpr int CG = RP == 32 ? 4 : 2;
    constexpr int CG2 = RP == 32 ? 4 : 1;
    const bool one = R == 1;
    const int ngroups = one ? 1 : (R + CG - 1) / CG;
    const int nchunk = had_chunks(N, R);
    const int rows = (N + nchunk - 1) / nchunk;
    const size_t nout = (size_t)R * RP * RP;
    DSKI_TRY(gram.reserve(sizeof(double) * (nout * (size_t)nchunk + nout) + 256));
    double* part = gram.as<double>();
    double* C = part + nout * (size_t)nchunk;
    if (one)
      k_had_gram<RP, 1, TF, T><<<dim3(nchunk, 1), 256, 0, st>>>(Qa, Qb, N, V, ldv, R, rows, part);
    else
      k_had_gram<RP, CG, TF, T><<<dim3(nchunk, ngroups), 256, 0, st>>>(Qa, Qb, N, V, ldv, R, rows, part);
    DSKI_HIP(hipGetLastError());
    k_had_reduce<<<(unsigned)((nout + 63) / 64), 256, 0, st>>>(part, nchunk, (int)nout, C);
    DSKI_HIP(hipGetLastError());
    const int nb = (N + 255) / 256;
    if (one)
      k_had_apply<RP, 1, TF, T><<<dim3(nb, 1), 256, 0, st>>>(Aa, Ab, N, n, C, R, V, ldv, Y, ldy, ks, nv, ng, pq);
    else
      k_had_apply<RP, CG2, TF, T><<<dim3(nb, (R + CG2 - 1) / CG2), 256, 0, st>>>(Aa, Ab, N, n, C, R, V, ldv, Y,
                                                                                ldy, ks, nv, ng, pq);
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  }
}

template <typename TF, typename T>
static dski_status had_apply(DskipData* D, DevBuf& gram, const TF* Qa, const TF* Aa, const TF* Qb, const TF* Ab, int N, int n,
                             int R, const T* V, int ldv, T* Y, int ldy, double ks, double nv, double ng, double* pq,
                             hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  if (D->RP == 32)
    return had_apply_rp<32, TF, T>(gram, Qa, Aa, Qb, Ab, N, n, R, V, ldv, Y, ldy, ks, nv, ng, pq, st);
  return had_apply_rp<64, TF, T>(gram, Qa, Aa, Qb, Ab, N, n, R, V, ldv, Y, ldy, ks, nv, ng, pq, st);
}

// ---------------------------------------------------------------- Lanczos
// r steps on a symmetric operator (FP64, N-vectors) with full
// re-orthogonalisation; apply(x, y, stream) writes y = F x.  The factor
// receives Q (N x RP, zero beyond the steps kept) and A = Q T.  The runs of one
// tree level are independent: each has its own stream and buffers, their
// steps are issued in turn and the host waits once per step for all of them
// (a run's step count depends on its own breakdown test only, so every factor
// is the one a run by itself would give).
struct LanczosJob {
  int node = 0;
  std::function<dski_status(const double*, double*, hipStream_t)> apply;
  DskipFactor* out = nullptr;
  hipStream_t st = nullptr;
  DevBuf work;                  // w, partials, h, h2, |w|^2, T
  DevBuf tmp;                   // operator scratch (1-D D-SKI vectors or Hadamard partials)
  std::vector<double> alpha, beta;
  bool done = false;
};

static void free_factor(DskipFactor& f) {
  (void)hipFree(f.Q);
  (void)hipFree(f.A);
  f = DskipFactor{};
}

static dski_status lanczos_batch(DskipData* D, int N, std::vector<LanczosJob>& jobs, double* hpin) {
  const int RP = D->RP, r = D->r;
  const int nb = std::min(256, std::max(1, (N + 1023) / 1024));
  const int vb = (N + kBlock - 1) / kBlock;
  const size_t wlen = (size_t)N + 2 * (size_t)RP * nb + 4 * (size_t)RP + (size_t)RP * RP + 64;
  auto bufs = [&](LanczosJob& J, double** w, double** part, double** h, double** h2, double** nn, double** Tdev) {
    *w = J.work.as<double>();
    *part = *w + N;
    *h = *part + 2 * (size_t)RP * nb;
    *h2 = *h + RP;
    *nn = *h2 + RP;
    *Tdev = *nn + 2 * RP;
  };
  for (auto& J : jobs) {
    DSKI_TRY(J.work.reserve(sizeof(double) * wlen));
    DskipFactor& out = *J.out;
    if (!out.Q) DSKI_HIP(hipMalloc(&out.Q, sizeof(double) * (size_t)N * RP));
    if (!out.A) DSKI_HIP(hipMalloc(&out.A, sizeof(double) * (size_t)N * RP));
    DSKI_HIP(hipMemsetAsync(out.Q, 0, sizeof(double) * (size_t)N * RP, J.st));
    DSKI_HIP(hipMemsetAsync(out.A, 0, sizeof(double) * (size_t)N * RP, J.st));
    // q_0 = z / ||z|| with z the Rademacher column `node` (||z|| = sqrt(N))
    DSKI_TRY(rademacher<double>(D->seed, J.node, 1, N, out.Q, N, J.st));
    k_scale_copy<<<vb, kBlock, 0, J.st>>>(out.Q, N, 1.0 / std::sqrt((double)N), out.Q);
    J.alpha.clear();
    J.beta.clear();
    J.done = false;
  }
  for (int j = 0; j < r; ++j) {
    bool any = false;
    for (size_t i = 0; i < jobs.size(); ++i) {
      LanczosJob& J = jobs[i];
      if (J.done) continue;
      any = true;
      double *w, *part, *h, *h2, *nn, *Tdev;
      bufs(J, &w, &part, &h, &h2, &nn, &Tdev);
      const double* Q = J.out->Q;
      DSKI_TRY(J.apply(Q + (size_t)j * N, w, J.st));
      // pass 1: h = Q^T w (alpha = h_j = q_j . w), w -= Q h; pass 2 the same
      for (int pass = 0; pass < 2; ++pass) {
        double* hh = pass == 0 ? h : h2;
        k_cols_dot<<<dim3(nb, j + 1), kBlock, 0, J.st>>>(Q, N, w, part);
        RedJob jr{part, nb, j + 1, 1, hh, nullptr, nullptr, 1.0, nullptr, nullptr};
        DSKI_TRY(launch_reduce(jr, nullptr, J.st));
        k_cols_sub<<<vb, kBlock, 0, J.st>>>(Q, N, j + 1, hh, w);
      }
      k_cols_dot<<<dim3(nb, 1), kBlock, 0, J.st>>>(w, N, w, part);
      RedJob jn{part, nb, 1, 1, nn, nullptr, nullptr, 1.0, nullptr, nullptr};
      DSKI_TRY(launch_reduce(jn, nullptr, J.st));
      DSKI_HIP(hipGetLastError());
      DSKI_HIP(hipMemcpyAsync(hpin + 2 * i, h + j, sizeof(double), hipMemcpyDeviceToHost, J.st));
      DSKI_HIP(hipMemcpyAsync(hpin + 2 * i + 1, nn, sizeof(double), hipMemcpyDeviceToHost, J.st));
    }
    if (!any) break;
    for (size_t i = 0; i < jobs.size(); ++i) {
      LanczosJob& J = jobs[i];
      if (J.done) continue;
      DSKI_HIP(hipStreamSynchronize(J.st));
      const double ha = hpin[2 * i], hn = hpin[2 * i + 1];
      const double b = std::sqrt(std::max(hn, 0.0));
      J.alpha.push_back(ha);
      if (j == r - 1 || b <= 1e-12 * std::max(std::fabs(ha), 1.0)) {
        J.done = true;
        continue;
      }
      J.beta.push_back(b);
      double *w, *part, *h, *h2, *nn, *Tdev;
      bufs(J, &w, &part, &h, &h2, &nn, &Tdev);
      k_scale_copy<<<vb, kBlock, 0, J.st>>>(w, N, 1.0 / b, J.out->Q + (size_t)(j + 1) * N);
    }
  }
  for (auto& J : jobs) {
    const int k = (int)J.alpha.size();
    std::vector<double> T((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
      T[(size_t)j * k + j] = J.alpha[j];
      if (j + 1 < k) T[(size_t)j * k + j + 1] = T[(size_t)(j + 1) * k + j] = J.beta[j];
    }
    double *w, *part, *h, *h2, *nn, *Tdev;
    bufs(J, &w, &part, &h, &h2, &nn, &Tdev);
    DSKI_HIP(hipMemcpyAsync(Tdev, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, J.st));
    k_q_times_t<<<dim3(vb, k), kBlock, 0, J.st>>>(J.out->Q, N, k, Tdev, J.out->A);
    DSKI_HIP(hipGetLastError());
    DSKI_HIP(hipStreamSynchronize(J.st));  // T lives on the host stack
    J.out->k = k;
  }
  return DSKI_OK;
}

// Streams for the independent Lanczos runs of the build (default priority),
// ordered after the caller's stream at creation and drained before the build
// continues on the caller's stream.
struct BuildStreams {
  std::vector<hipStream_t> st;
  hipEvent_t ev = nullptr;
  double* hpin = nullptr;
  ~BuildStreams() {
    for (auto s : st) (void)hipStreamDestroy(s);
    if (ev) (void)hipEventDestroy(ev);
    if (hpin) (void)hipHostFree(hpin);
  }
  dski_status init(int n, hipStream_t caller) {
    DSKI_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    DSKI_HIP(hipEventRecord(ev, caller));
    for (int i = 0; i < n; ++i) {
      hipStream_t s = nullptr;
      DSKI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      st.push_back(s);
      DSKI_HIP(hipStreamWaitEvent(s, ev, 0));
    }
    DSKI_HIP(hipHostMalloc(&hpin, sizeof(double) * 2 * (size_t)std::max(n, 1), hipHostMallocDefault));
    return DSKI_OK;
  }
  // every stream drained (the caller's stream then follows on the host side)
  dski_status join() {
    for (auto s : st) DSKI_HIP(hipStreamSynchronize(s));
    return DSKI_OK;
  }
};

static dski_status dskip_build(dski_plan p, hipStream_t st) {
  DskipData* D = p->ds;
  const int n = p->n, d = p->d, N = p->N;
  const int pb = (n + kBlock - 1) / kBlock;
  for (int a = 0; a < d; ++a) {
    double le = std::log(D->ell[a]);
    DSKI_TRY(dski_set_hypers(D->sub[a], &le, 0.0, 0.0, 0.0, st));
    D->sub[a]->sf = 0.0;  // G_p is the noise-free 1-D D-SKI matrix
    D->sub[a]->sg = 0.0;
  }
  free_factor(D->fa);
  free_factor(D->fb);
  BuildStreams bs;
  DSKI_TRY(bs.init(d, st));
  std::vector<DskipFactor> level(d);
  dski_status rc = DSKI_OK;
  {
    // leaves: the 1-D factor of every axis
    std::vector<LanczosJob> jobs(d);
    for (int a = 0; a < d && rc >= 0; ++a) {
      LanczosJob& J = jobs[a];
      J.node = a;
      J.out = &level[a];
      J.st = bs.st[a];
      rc = J.tmp.reserve(sizeof(double) * 4 * (size_t)std::max(n, 1));
      dski_plan sp = D->sub[a];
      int* iperm = D->iperm[a];
      double* u = J.tmp.as<double>();
      double* y = u + 2 * (size_t)n;
      J.apply = [=](const double* q, double* w, hipStream_t s) -> dski_status {
        k_compress<<<pb, kBlock, 0, s>>>(q, n, d, a, sp->perm, u);
        DSKI_TRY(mvm_tiled<double>(sp, 1, u, 2 * n, y, 2 * n, nullptr, s));
        k_expand<<<pb, kBlock, 0, s>>>(y, n, d, a, iperm, w);
        DSKI_HIP(hipGetLastError());
        return DSKI_OK;
      };
    }
    if (rc >= 0) rc = lanczos_batch(D, N, jobs, bs.hpin);
    if (rc < 0) (void)bs.join();  // nothing in flight before buffers are freed
  }
  // binary tree: pairs (0,1), (2,3), ... recompressed level by level; an odd
  // factor moves up unchanged; internal nodes numbered on from d
  int node = d;
  while (rc >= 0 && level.size() > 2) {
    const size_t np = level.size() / 2;
    std::vector<DskipFactor> nxt(np);
    std::vector<LanczosJob> jobs(np);
    for (size_t i = 0; i < np; ++i) {
      LanczosJob& J = jobs[i];
      J.node = node++;
      J.out = &nxt[i];
      J.st = bs.st[i];
      DskipFactor* fa = &level[2 * i];
      DskipFactor* fb = &level[2 * i + 1];
      DevBuf* gram = &J.tmp;
      J.apply = [=](const double* q, double* w, hipStream_t s) -> dski_status {
        return had_apply<double, double>(D, *gram, fa->Q, fa->A, fb->Q, fb->A, N, n, 1, q, N, w, N, 1.0, 0.0, 0.0,
                                         nullptr, s);
      };
    }
    rc = lanczos_batch(D, N, jobs, bs.hpin);
    if (rc < 0) (void)bs.join();
    if (level.size() % 2) nxt.push_back(level.back());
    for (size_t i = 0; i < np; ++i) {
      free_factor(level[2 * i]);
      free_factor(level[2 * i + 1]);
    }
    if (rc < 0)
      for (auto& f : nxt) free_factor(f);
    level.swap(nxt);
  }
  DSKI_TRY(bs.join());
  if (rc < 0) {
    for (auto& f : level) free_factor(f);
    return rc;
  }
  D->fa = level[0];
  D->fb = level[1];
  size_t len = (size_t)N * D->RP;
  const int cb = (int)std::min<size_t>((len + kBlock - 1) / kBlock, 4096);
  k_to_f32_rows<<<cb, kBlock, 0, st>>>(D->fa.Q, N, D->RP, D->Qa32);
  k_to_f32<<<cb, kBlock, 0, st>>>(D->fa.A, len, D->Aa32);
  k_to_f32_rows<<<cb, kBlock, 0, st>>>(D->fb.Q, N, D->RP, D->Qb32);
  k_to_f32<<<cb, kBlock, 0, st>>>(D->fb.A, len, D->Ab32);
  DSKI_HIP(hipGetLastError());
  D->built = true;
  return DSKI_OK;
}

// ---------------------------------------------------------------- solver hooks
template <typename T>
struct FactorsOf;
template <>
struct FactorsOf<float> {
  static void get(DskipData* D, const float** q, const float** a, const float** qb, const float** ab) {
    *q = D->Qa32;
    *a = D->Aa32;
    *qb = D->Qb32;
    *ab = D->Ab32;
  }
};
template <>
struct FactorsOf<double> {
  static void get(DskipData* D, const double** q, const double** a, const double** qb, const double** ab) {
    *q = D->fa.Q;
    *a = D->fa.A;
    *qb = D->fb.Q;
    *ab = D->fb.A;
  }
};

template <typename T>
dski_status dskip_apply(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double ks, double nv, double ng,
                        double* pq_partial, hipStream_t st) {
  DskipData* D = p->ds;
  if (!D || !D->built) {
    set_error("D-SKIP factors not built");
    return DSKI_EINVAL;
  }
  const T *Qa, *Aa, *Qb, *Ab;
  FactorsOf<T>::get(D, &Qa, &Aa, &Qb, &Ab);
  return had_apply<T, T>(D, D->gram, Qa, Aa, Qb, Ab, p->N, p->n, R, V, ldv, Y, ldy, ks, nv, ng, pq_partial, st);
}

template <typename T>
dski_status dskip_mvm(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double* pq_partial, hipStream_t st) {
  return dskip_apply<T>(p, R, V, ldv, Y, ldy, p->s * p->s, p->sf * p->sf, p->sg * p->sg, pq_partial, st);
}
template dski_status dskip_mvm<float>(dski_plan, int, const float*, int, float*, int, double*, hipStream_t);
template dski_status dskip_mvm<double>(dski_plan, int, const double*, int, double*, int, double*, hipStream_t);
template dski_status dskip_apply<float>(dski_plan, int, const float*, int, float*, int, double, double, double,
                                        double*, hipStream_t);
template dski_status dskip_apply<double>(dski_plan, int, const double*, int, double*, int, double, double, double,
                                         double*, hipStream_t);

dski_status dskip_set_hypers(dski_plan p, const double* log_ell, hipStream_t st) {
  DskipData* D = p->ds;
  bool same = D->built;
  for (int a = 0; a < p->d; ++a) {
    double e = std::exp(log_ell[a]);
    if (e != D->ell[a]) same = false;
    D->ell[a] = e;
  }
  if (same) return DSKI_OK;
  return dskip_build(p, st);
}

// diag K[e] = s^2 (sum_k Aa[e,k] Qa[e,k]) (sum_l Ab[e,l] Qb[e,l])
__global__ void k_dskip_diag(const double* __restrict__ Qa, const double* __restrict__ Aa,
                             const double* __restrict__ Qb, const double* __restrict__ Ab, int N, int RP, double s2,
                             double* __restrict__ diag) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double x = 0.0, y = 0.0;
  for (int k = 0; k < RP; ++k) {
    x += Aa[(size_t)k * N + e] * Qa[(size_t)k * N + e];
    y += Ab[(size_t)k * N + e] * Qb[(size_t)k * N + e];
  }
  diag[e] = s2 * x * y;
}

dski_status dskip_diag(dski_plan p, double* diag, hipStream_t st) {
  DskipData* D = p->ds;
  if (!D->built) {
    set_error("D-SKIP factors not built");
    return DSKI_EINVAL;
  }
  k_dskip_diag<<<(p->N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D->fa.Q, D->fa.A, D->fb.Q, D->fb.A, p->N, D->RP,
                                                                 p->s * p->s, diag);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// Pivot selection plus the pivot's rows of Qa, Qb and of L.
__global__ void k_dskip_pivot(const double* __restrict__ pv, const int* __restrict__ pi, int nblk, int j,
                              double rel_tol, PivState* __restrict__ ps, int* __restrict__ piv_list,
                              const double* __restrict__ Qa, const double* __restrict__ Qb, int N, int RP,
                              double* __restrict__ prow, const double* __restrict__ L, double* __restrict__ lrow,
                              const int* __restrict__ forced, const double* __restrict__ dres) {
  const int e = pivot_select_block(pv, pi, nblk, j, rel_tol, ps, piv_list, forced, dres);
  if (e < 0) return;
  for (int k = threadIdx.x; k < RP; k += blockDim.x) {
    prow[k] = Qa[(size_t)k * N + e];
    prow[RP + k] = Qb[(size_t)k * N + e];
  }
  for (int l = threadIdx.x; l < j; l += blockDim.x) lrow[l] = L[(size_t)l * N + e];
}

// Column j of L: K[e, piv] = s^2 (Aa[e,:] . Qa[piv,:]) (Ab[e,:] . Qb[piv,:]).
__global__ void k_dskip_column(int j, const PivState* __restrict__ ps, const double* __restrict__ Aa,
                               const double* __restrict__ Ab, int N, int RP, double s2,
                               const double* __restrict__ prow, const double* __restrict__ lrow,
                               double* __restrict__ L, double* __restrict__ dres) {
  if (ps->stop) return;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double x = 0.0, y = 0.0;
  for (int k = 0; k < RP; ++k) {
    x += Aa[(size_t)k * N + e] * prow[k];
    y += Ab[(size_t)k * N + e] * prow[RP + k];
  }
  double acc = s2 * x * y;
  for (int l = 0; l < j; ++l) acc -= L[(size_t)l * N + e] * lrow[l];
  double lj = acc / sqrt(ps->dpiv);
  L[(size_t)j * N + e] = lj;
  double dn = dres[e] - lj * lj;
  if (e == ps->piv) dn = -INFINITY;
  dres[e] = dn;
}

dski_status dskip_pc_step(dski_plan p, int j, const double* pv, const int* pi, int nblk, double rel_tol,
                          PivState* ps, int* piv_list, double* L, double* lrow, double* dres, const int* forced,
                          hipStream_t st) {
  DskipData* D = p->ds;
  DSKI_TRY(D->rows.reserve(sizeof(double) * 2 * D->RP));
  double* prow = D->rows.as<double>();
  k_dskip_pivot<<<1, kBlock, 0, st>>>(pv, pi, nblk, j, rel_tol, ps, piv_list, D->fa.Q, D->fb.Q, p->N, D->RP, prow,
                                      L, lrow, forced, dres);
  k_dskip_column<<<(p->N + kBlock - 1) / kBlock, kBlock, 0, st>>>(j, ps, D->fa.A, D->fb.A, p->N, D->RP,
                                                                  p->s * p->s, prow, lrow, L, dres);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

void dskip_destroy(dski_plan p) {
  DskipData* D = p->ds;
  if (!D) return;
  for (auto sp : D->sub) dski_plan_destroy(sp);
  for (auto ip : D->iperm) (void)hipFree(ip);
  free_factor(D->fa);
  free_factor(D->fb);
  (void)hipFree(D->Qa32);
  (void)hipFree(D->Aa32);
  (void)hipFree(D->Qb32);
  (void)hipFree(D->Ab32);
  D->work.release();
  D->gram.release();
  D->rows.release();
  delete D;
  p->ds = nullptr;
}

__global__ void k_iota(int* __restrict__ x, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = i;
}

static dski_status dskip_create_impl(dski_plan p, const double* X, const double* lo, const double* hi,
                                     const double* log_ell, hipStream_t st) {
  DskipData* D = p->ds;
  const int n = p->n, d = p->d, N = p->N;
  DSKI_HIP(hipMalloc(&p->perm, sizeof(int) * (size_t)std::max(n, 1)));
  k_iota<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(p->perm, n);
  DSKI_HIP(hipGetLastError());
  TmpBuf col;
  DSKI_TRY(col.reserve(sizeof(double) * (size_t)n));
  for (int a = 0; a < d; ++a) {
    k_extract_col<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(X, n, d, a, col.as<double>());
    DSKI_HIP(hipGetLastError());
    dski_plan sp = nullptr;
    int m = D->m1;
    DSKI_TRY(dski_plan_create(&sp, n, 1, col.as<double>(), &m, lo ? lo + a : nullptr, hi ? hi + a : nullptr,
                              DSKI_INTERP_CUBIC, st));
    D->sub.push_back(sp);
    int* ip = nullptr;
    DSKI_HIP(hipMalloc(&ip, sizeof(int) * (size_t)n));
    D->iperm.push_back(ip);
    k_inverse_perm<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(sp->perm, n, ip);
    DSKI_HIP(hipGetLastError());
  }
  DSKI_HIP(hipStreamSynchronize(st));
  col.release();
  size_t len = (size_t)N * D->RP;
  DSKI_HIP(hipMalloc(&D->Qa32, sizeof(float) * len));
  DSKI_HIP(hipMalloc(&D->Aa32, sizeof(float) * len));
  DSKI_HIP(hipMalloc(&D->Qb32, sizeof(float) * len));
  DSKI_HIP(hipMalloc(&D->Ab32, sizeof(float) * len));
  D->ell.assign(d, 0.0);
  for (int a = 0; a < d; ++a) D->ell[a] = std::exp(log_ell[a]);
  return dskip_build(p, st);
}

}  // namespace dski

using namespace dski;

extern "C" dski_status dskip_plan_create(dski_plan* out, int n, int d, const double* X, int m_1d, int rank_r,
                                         uint64_t seed, const double* lo_host, const double* hi_host,
                                         const double* log_ell_host, dski_stream stream) {
  if (!out) {
    set_error("out is NULL");
    return DSKI_EINVAL;
  }
  *out = nullptr;
  if (n < 1 || d < 2 || d > DSKIP_MAXD || !X || m_1d < 4 || rank_r < 1 || rank_r > 64 || !log_ell_host ||
      ((lo_host == nullptr) != (hi_host == nullptr))) {
    set_error("dskip_plan_create: bad arguments (n=%d >= 1, 2 <= d=%d <= %d, m_1d=%d >= 4, 1 <= rank_r=%d <= 64, "
              "log_ell required)",
              n, d, DSKIP_MAXD, m_1d, rank_r);
    return DSKI_EINVAL;
  }
  for (int a = 0; a < d; ++a)
    if (!std::isfinite(log_ell_host[a])) {
      set_error("non-finite log length scale");
      return DSKI_EINVAL;
    }
  if ((long long)n * (d + 1) > (1ll << 31) - 1) {
    set_error("n too large");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  dski_plan p = new dski_plan_s();
  p->kind = 1;
  p->n = n;
  p->d = d;
  p->N = n * (d + 1);
  p->s = 1.0;
  p->sf = 0.1;
  p->sg = 0.1;
  p->ds = new DskipData();
  p->ds->m1 = m_1d;
  p->ds->r = std::min(rank_r, p->N);
  p->ds->RP = rank_r <= 32 ? 32 : 64;
  p->ds->seed = seed;
  dski_status rc = dskip_create_impl(p, X, lo_host, hi_host, log_ell_host, st);
  if (rc < 0) {
    dski_plan_destroy(p);
    return rc;
  }
  *out = p;
  return DSKI_OK;
}

extern "C" dski_status dskip_plan_info(dski_plan p, int* m_1d, int* rank_r, int* k_a, int* k_b) {
  if (!p || p->kind != 1) {
    set_error("dskip_plan_info: not a D-SKIP plan");
    return DSKI_EINVAL;
  }
  if (m_1d) *m_1d = p->ds->m1;
  if (rank_r) *rank_r = p->ds->r;
  if (k_a) *k_a = p->ds->fa.k;
  if (k_b) *k_b = p->ds->fb.k;
  return DSKI_OK;
}
