// Learned log-determinant surrogate: a two-hidden-layer GELU network in FP32
// with forward-mode tangents for its input derivative and the weight gradient
// of a value-and-gradient-matching loss (training on the device).
//
//   a1 = W1 x + b1, h1 = gelu(a1); a2 = W2 h1 + b2, h2 = gelu(a2); y = w3 . h2 + b3
//   tangents along the first J inputs:  da1_j = W1 e_j, dh1_j = gelu'(a1) da1_j,
//   da2_j = W2 dh1_j, dh2_j = gelu'(a2) da2_j, dy_j = w3 . dh2_j
//   loss = (1/B) sum_b [(y_b - t_b)^2 + lam sum_j (dy_bj - g_bj)^2]
//
// The batch is laid out as K = (1 + J) B rows of H values: the value rows of
// the B samples, then their tangent rows along input 0, 1, .., J - 1.  Layer 1
// and the GELU factors are elementwise kernels; the three products with the
// H x H matrix W2 run on the FP32 matrix cores (v_mfma_f32_16x16x4f32): the
// layer-2 pre-activations of all K rows (rows x W2^T), the layer-1 deltas of
// all K rows (rows x W2), and the weight gradient D2^T S1 contracted over the
// K rows in chunks.  Per-sample reductions over the hidden units (y, dy_j) use
// one work-group per sample.  The chunks of every batch contraction are added
// in FP64 in a fixed order: deterministic.  Adam (Kingma & Ba) updates the
// packed parameters in place.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

struct dski_mlp_s {
  int F = 8, H = 128, J = 5, maxB = 0;
  int np = 0;                 // packed parameters
  float* params = nullptr;    // W1 (H x F), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1), row-major
  float* grad = nullptr;      // packed gradient of the last mlp_backward
  float* m = nullptr;         // Adam moments
  float* v = nullptr;
  int t = 0;                  // Adam step count
  dski::DevBuf work;          // per-sample activations, deltas and partials
  dski::DevBuf scal;          // loss partials
};

namespace dski {

struct MlpOff {
  int W1, b1, W2, b2, w3, b3, n;
};
static MlpOff mlp_off(int F, int H) {
  MlpOff o;
  o.W1 = 0;
  o.b1 = o.W1 + H * F;
  o.W2 = o.b1 + H;
  o.b2 = o.W2 + H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.n = o.b3 + 1;
  return o;
}

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d1f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}
__device__ __forceinline__ float gelu_d2f(float a) {
  return 0.39894228040143268f * expf(-0.5f * a * a) * (2.0f - a * a);
}

constexpr int kMlpMaxH = 128;
constexpr int kMlpMaxF = 16;
constexpr int kMlpMaxJ = 8;

// Block sum over H <= 128 threads (two wavefronts), result to all threads.
__device__ __forceinline__ float block_sum128(float v, float* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = red[0];
  if (blockDim.x > 64) s += red[1];
  return s;
}

// Saved rows (each H floats), row index of (j, b) = j * B + b, (1 + J) B rows:
//   S1 = [h1; dh1_1..J], C = layer-2 pre-activations (then the layer-1 deltas),
//   D2 = [da2; dda2_1..J], D1 = [da1; dda1_1..J];
// per sample (B rows): A1 = a1, P3 = the w3-gradient terms; E = [ey; eg_1..J]
// ((1 + J) B scalars).
struct MlpWork {
  float *S1, *C, *D2, *P3, *D1, *A1, *E;
  double* part;
  size_t rows;  // (1 + J) B
};

typedef float mlp_flt4 __attribute__((ext_vector_type(4)));

// Layer 1, one thread per (sample b, unit i): a1 = W1 x + b1, h1 = gelu(a1),
// tangent rows dh1_j = gelu'(a1) W1[i][j] (j < J).
__global__ void k_mlp_l1(const float* __restrict__ P, int F, int H, int J, MlpOff o, int B,
                         const float* __restrict__ X, MlpWork w) {
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (long long)B * H) return;
  const int b = (int)(f / H), i = (int)(f % H);
  float a1 = P[o.b1 + i];
  for (int j = 0; j < F; ++j) a1 += P[o.W1 + i * F + j] * X[(size_t)b * F + j];
  w.A1[f] = a1;
  w.S1[f] = gelu_f(a1);
  const float g1 = gelu_d1f(a1);
  for (int j = 0; j < J; ++j) w.S1[((size_t)(j + 1) * B + b) * H + i] = g1 * P[o.W1 + i * F + j];
}

// C (M x H) = A (M x H) times Bv (H x H), Bv[k][c] = W[c][k] (TB) or W[k][c], on the
// FP32 matrix cores (D += A B, A 16 x 4 and B 4 x 16: lane l holds A[l%16][l/16]
// and B[l/16][l%16], register q of lane l holds D[4(l/16) + q][l%16]).  A
// work-group stages Bv (zero-padded to 128 x 128) in LDS; each wavefront takes
// 16 rows, loads its 16 x 128 operand block into registers at once and runs
// 32 k-steps over the 8 column blocks.  Accumulation in FP32 over the H terms
// of each dot product, as in a vector-ALU loop.
template <bool TB>
__global__ __launch_bounds__(256) void k_mlp_mm(const float* __restrict__ A, long long M, const float* __restrict__ W,
                                                int H, float* __restrict__ C) {
  __shared__ float sB[128 * 128];
  for (int f = threadIdx.x; f < 128 * 128; f += 256) {
    const int k = f >> 7, c = f & 127;
    sB[f] = k < H && c < H ? (TB ? W[c * H + k] : W[k * H + c]) : 0.f;
  }
  const int lane = threadIdx.x & 63;
  const long long r0 = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const long long row = r0 + (lane & 15);
  const int kq = lane >> 4;
  float aop[32];
#pragma unroll
  for (int s4 = 0; s4 < 32; ++s4) {
    const int k = 4 * s4 + kq;
    aop[s4] = row < M && k < H ? A[row * H + k] : 0.f;
  }
  __syncthreads();
  mlp_flt4 acc[8];
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) acc[cb] = mlp_flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s4 = 0; s4 < 32; ++s4) {
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[s4], sB[(4 * s4 + kq) * 128 + 16 * cb + (lane & 15)],
                                                     acc[cb], 0, 0, 0);
  }
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) {
    const int c = 16 * cb + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long r = r0 + 4 * kq + q;
      if (r < M && c < H) C[r * H + c] = acc[cb][q];
    }
  }
}

// Per sample (one work-group of 128 threads, thread = layer-2 unit): a2 = C + b2,
// h2 = gelu(a2), tangents dh2_j = gelu'(a2) C_j, y = w3 . h2 + b3, dy_j = w3 .
// dh2_j; mode 1 also the loss deltas, the layer-2 deltas
// da2 = ey w3 gelu'(a2) + sum_j eg_j w3 gelu''(a2) da2_j, dda2_j = eg_j w3 gelu'(a2),
// and the sample's share of the w3 gradient, ey h2 + sum_j eg_j dh2_j (row b of P3).
__global__ __launch_bounds__(128) void k_mlp_l2(const float* __restrict__ P, int H, int J, MlpOff o, int B,
                                                const float* __restrict__ tv, const float* __restrict__ tg,
                                                float lam, int mode, float* __restrict__ y_out,
                                                float* __restrict__ dy_out, MlpWork w,
                                                double* __restrict__ loss_part) {
  __shared__ float red[2];
  const int b = blockIdx.x;
  const int i = threadIdx.x;
  const bool u = i < H;
  float a2 = 0.f, g2 = 0.f, g2d = 0.f, h2 = 0.f;
  float ta2[kMlpMaxJ], th2[kMlpMaxJ];
#pragma unroll
  for (int j = 0; j < kMlpMaxJ; ++j) ta2[j] = 0.f;
  if (u) {
    a2 = w.C[(size_t)b * H + i] + P[o.b2 + i];
#pragma unroll
    for (int j = 0; j < kMlpMaxJ; ++j)
      if (j < J) ta2[j] = w.C[((size_t)(j + 1) * B + b) * H + i];
    g2 = gelu_d1f(a2);
    g2d = gelu_d2f(a2);
    h2 = gelu_f(a2);
  }
#pragma unroll
  for (int j = 0; j < kMlpMaxJ; ++j) th2[j] = g2 * ta2[j];
  const float w3i = u ? P[o.w3 + i] : 0.f;
  float y = block_sum128(w3i * h2, red) + P[o.b3];
  float dy[kMlpMaxJ];
#pragma unroll
  for (int j = 0; j < kMlpMaxJ; ++j) dy[j] = j < J ? block_sum128(w3i * th2[j], red) : 0.f;
  if (i == 0) {
    if (y_out) y_out[b] = y;
    if (dy_out)
      for (int j = 0; j < J; ++j) dy_out[(size_t)b * J + j] = dy[j];
  }
  if (mode == 0) return;
  const float ey = 2.0f * (y - tv[b]) / (float)B;
  float eg[kMlpMaxJ];
  double lpart = (double)(y - tv[b]) * (double)(y - tv[b]);
#pragma unroll
  for (int j = 0; j < kMlpMaxJ; ++j) {
    eg[j] = 0.f;
    if (j < J) {
      const float dd = dy[j] - tg[(size_t)b * J + j];
      eg[j] = 2.0f * lam * dd / (float)B;
      lpart += (double)lam * (double)dd * (double)dd;
    }
  }
  if (i == 0) {
    loss_part[b] = lpart;
    w.E[b] = ey;
    for (int j = 0; j < J; ++j) w.E[(size_t)(j + 1) * B + b] = eg[j];
  }
  if (u) {
    float p3 = ey * h2;
    float da2 = ey * w3i * g2;
    for (int j = 0; j < J; ++j) {
      const float ddh2 = eg[j] * w3i;
      da2 += ddh2 * g2d * ta2[j];
      p3 += eg[j] * th2[j];
      w.D2[((size_t)(j + 1) * B + b) * H + i] = ddh2 * g2;
    }
    w.D2[(size_t)b * H + i] = da2;
    w.P3[(size_t)b * H + i] = p3;
  }
}

// Layer-1 deltas from the products C = D2 W2 (one thread per (sample, unit)):
// da1 = dh1 gelu'(a1) + sum_j ddh1_j gelu''(a1) W1[l][j], dda1_j = ddh1_j gelu'(a1).
__global__ void k_mlp_d1(const float* __restrict__ P, int F, int H, int J, MlpOff o, int B, MlpWork w) {
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= (long long)B * H) return;
  const int b = (int)(f / H), l = (int)(f % H);
  const float a1 = w.A1[f];
  const float g1 = gelu_d1f(a1), g1d = gelu_d2f(a1);
  float da1 = w.C[f] * g1;
  for (int j = 0; j < J; ++j) {
    const size_t r = ((size_t)(j + 1) * B + b) * H + l;
    const float ddh1 = w.C[r];
    da1 += ddh1 * g1d * P[o.W1 + l * F + j];
    w.D1[r] = ddh1 * g1;
  }
  w.D1[f] = da1;
}

// Chunk partials of dW2 = D2^T S1 (H x H, contracting over the K rows) on the
// FP32 matrix cores: work-group c takes rows [c chunk, (c + 1) chunk) four at a
// time; its four wavefronts take the four 64 x 64 quadrants of the product
// (A[m][kk] = D2[r + kk][16 h + m], B[kk][n] = S1[r + kk][16 g + n]).  Each
// chunk's tile is written in FP64: part[(c H + i) H + l].
__global__ __launch_bounds__(256) void k_mlp_gram(const float* __restrict__ D2, const float* __restrict__ S1,
                                                  long long K, int H, long long chunk, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h0 = (wv >> 1) * 4, g0 = (wv & 1) * 4;
  const long long k0 = (long long)blockIdx.x * chunk, k1 = k0 + chunk < K ? k0 + chunk : K;
  const int kq = lane >> 4, m = lane & 15;
  mlp_flt4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = mlp_flt4{0.f, 0.f, 0.f, 0.f};
  for (long long r = k0; r < k1; r += 4) {
    const long long rr = r + kq;
    const bool ok = rr < k1;
    float av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int ci = 16 * (h0 + a) + m, cl = 16 * (g0 + a) + m;
      av[a] = ok && ci < H ? D2[rr * H + ci] : 0.f;
      bv[a] = ok && cl < H ? S1[rr * H + cl] : 0.f;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[c], acc[a][c], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * (h0 + a) + 4 * kq + q, l = 16 * (g0 + c) + m;
        if (i < H && l < H) part[((size_t)blockIdx.x * H + i) * H + l] = (double)acc[a][c][q];
      }
}

// Chunk partials of dW1's value part, part[c][i][l] = sum over the rows b of chunk
// c of D1[b][i] X[b][l] (FP64): threads over the (i, l) entries, one work-group
// per chunk of rows.
__global__ void k_mlp_tn_chunks(const float* __restrict__ A, int na, const float* __restrict__ Bm, int nb,
                                long long K, long long chunk, double* __restrict__ part) {
  const long long k0 = (long long)blockIdx.x * chunk, k1 = k0 + chunk < K ? k0 + chunk : K;
  for (int f = threadIdx.x; f < na * nb; f += blockDim.x) {
    const int i = f / nb, l = f % nb;
    double acc = 0.0;
    for (long long r = k0; r < k1; ++r) acc += (double)A[r * na + i] * (double)Bm[r * nb + l];
    part[(size_t)blockIdx.x * na * nb + f] = acc;
  }
}

// Chunk partials of column sums over B rows of H values, for G sources at once:
// source g (blockIdx.y) starts at src + offs[g] rows; out[(g nchunk + c) H + i] (FP64).
struct MlpColSrc {
  const float* p[kMlpMaxJ + 3];
};
__global__ void k_mlp_colsums(MlpColSrc src, int B, int H, long long chunk, double* __restrict__ out) {
  const int g = blockIdx.y, c = blockIdx.x, nchunk = gridDim.x;
  const long long k0 = (long long)c * chunk, k1 = k0 + chunk < B ? k0 + chunk : B;
  const float* A = src.p[g];
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    double acc = 0.0;
    for (long long r = k0; r < k1; ++r) acc += (double)A[r * H + i];
    out[((size_t)g * nchunk + c) * H + i] = acc;
  }
}

// out[f] (FP32) = sum over chunks of part[c][f], plus (optionally) add[f]
__global__ void k_mlp_sum_chunks(const double* __restrict__ part, int nchunk, int nout, float* __restrict__ out,
                                 const double* __restrict__ add) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nout) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * nout + f];
  if (add) s += add[f];
  out[f] = (float)s;
}

// The small gradients from chunk partials added in a fixed order (FP64), one
// thread per entry: W1 = the value rows' D1^T X plus the tangent column sums
// (dW1[i][j] += sum_b dda1_j[b][i], j < J), then w3 (column sums of P3), b1 and b2
// (column sums of the value rows of D1 and D2).  cs holds nchunk x H partials of
// each column-sum source: D1 row groups 0..J, then D2's value rows (cs2), then P3
// (pw3).
__global__ void k_mlp_small_grads(const double* __restrict__ pW1, const double* __restrict__ pw3,
                                  const double* __restrict__ cs, const double* __restrict__ cs2, int nchunk, int H,
                                  int F, int J, MlpOff o, float* __restrict__ grad) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  auto csum = [&](int g, int i) {  // column sum of D1 row group g, unit i
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += cs[((size_t)g * nchunk + c) * H + i];
    return v;
  };
  if (f < H * F) {
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += pW1[(size_t)c * H * F + f];
    const int i = f / F, j = f % F;
    if (j < J) v += csum(j + 1, i);
    grad[o.W1 + f] = (float)v;
  } else if (f < H * F + H) {
    const int i = f - H * F;
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += pw3[(size_t)c * H + i];
    grad[o.w3 + i] = (float)v;
  } else if (f < H * F + 2 * H) {
    const int i = f - H * F - H;
    grad[o.b1 + i] = (float)csum(0, i);
  } else if (f < H * F + 3 * H) {
    const int i = f - H * F - 2 * H;
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += cs2[(size_t)c * H + i];
    grad[o.b2 + i] = (float)v;
  }
}

// b3 = sum_b ey_b (FP64, one work-group).
__global__ __launch_bounds__(256) void k_mlp_b3(const float* __restrict__ E, int B, float* __restrict__ out) {
  __shared__ double red[256];
  double e = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) e += (double)E[b];
  red[threadIdx.x] = e;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)red[0];
}

__global__ void k_mlp_loss(const double* __restrict__ lp, int B, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) s += lp[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)B;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const float g = G[f];
  const float mm = b1 * m[f] + (1.0f - b1) * g;
  const float vv = b2 * v[f] + (1.0f - b2) * g * g;
  m[f] = mm;
  v[f] = vv;
  P[f] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

constexpr int kMlpChunks = 64;      // chunks of the small batch contractions (dW1, dw3, column sums)
constexpr int kMlpGramChunks = 64;  // chunks of dW2 = D2^T S1

static dski_status mlp_reserve(dski_mlp net, int B, MlpWork& w) {
  const int H = net->H, J = net->J;
  const size_t rows = (size_t)(1 + J) * B;
  const size_t fl = 4 * rows * H + 2 * (size_t)B * H + rows + 64;
  const size_t parts = (size_t)kMlpGramChunks * H * H +
                       (size_t)kMlpChunks * ((size_t)H * net->F + (size_t)(J + 3) * H) + B + 64;
  DSKI_TRY(net->work.reserve(sizeof(float) * fl + sizeof(double) * parts + 256));
  float* base = net->work.as<float>();
  w.S1 = base;
  w.C = w.S1 + rows * H;
  w.D2 = w.C + rows * H;
  w.D1 = w.D2 + rows * H;
  w.P3 = w.D1 + rows * H;
  w.A1 = w.P3 + (size_t)B * H;
  w.E = w.A1 + (size_t)B * H;
  size_t off = ((sizeof(float) * fl) + 63) / 64 * 64;
  w.part = reinterpret_cast<double*>(net->work.as<char>() + off);
  w.rows = rows;
  return DSKI_OK;
}

}  // namespace dski

using namespace dski;

extern "C" {

dski_status mlp_create(dski_mlp* out, int F, int H, int J, const float* params_host, dski_stream stream) {
  if (!out || F < 1 || F > kMlpMaxF || H < 1 || H > kMlpMaxH || J < 0 || J > kMlpMaxJ || J > F || !params_host) {
    set_error("mlp_create: bad arguments (F <= %d, H <= %d, J <= min(F, %d), params required)", kMlpMaxF, kMlpMaxH,
              kMlpMaxJ);
    return DSKI_EINVAL;
  }
  *out = nullptr;
  dski_mlp net = new dski_mlp_s();
  net->F = F;
  net->H = H;
  net->J = J;
  MlpOff o = mlp_off(F, H);
  net->np = o.n;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto fail = [&](const char* what) {
    set_error("mlp_create: %s", what);
    (void)hipFree(net->params);
    (void)hipFree(net->grad);
    (void)hipFree(net->m);
    (void)hipFree(net->v);
    delete net;
    return DSKI_EHIP;
  };
  if (hipMalloc(&net->params, sizeof(float) * o.n) != hipSuccess ||
      hipMalloc(&net->grad, sizeof(float) * o.n) != hipSuccess ||
      hipMalloc(&net->m, sizeof(float) * o.n) != hipSuccess || hipMalloc(&net->v, sizeof(float) * o.n) != hipSuccess)
    return fail("allocation failed");
  if (hipMemcpyAsync(net->params, params_host, sizeof(float) * o.n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(net->m, 0, sizeof(float) * o.n, st) != hipSuccess ||
      hipMemsetAsync(net->v, 0, sizeof(float) * o.n, st) != hipSuccess ||
      hipMemsetAsync(net->grad, 0, sizeof(float) * o.n, st) != hipSuccess)
    return fail("upload failed");
  if (hipStreamSynchronize(st) != hipSuccess) return fail("upload failed");
  *out = net;
  return DSKI_OK;
}

dski_status mlp_destroy(dski_mlp net) {
  if (!net) return DSKI_OK;
  (void)hipFree(net->params);
  (void)hipFree(net->grad);
  (void)hipFree(net->m);
  (void)hipFree(net->v);
  net->work.release();
  net->scal.release();
  delete net;
  return DSKI_OK;
}

dski_status mlp_num_params(dski_mlp net, int* n) {
  if (!net || !n) {
    set_error("mlp_num_params: NULL argument");
    return DSKI_EINVAL;
  }
  *n = net->np;
  return DSKI_OK;
}

dski_status mlp_get_params(dski_mlp net, float* params_host, float* grad_host) {
  if (!net) {
    set_error("mlp_get_params: NULL network");
    return DSKI_EINVAL;
  }
  if (params_host) DSKI_HIP(hipMemcpy(params_host, net->params, sizeof(float) * net->np, hipMemcpyDeviceToHost));
  if (grad_host) DSKI_HIP(hipMemcpy(grad_host, net->grad, sizeof(float) * net->np, hipMemcpyDeviceToHost));
  return DSKI_OK;
}

static dski_status mlp_eval(dski_mlp net, int B, const float* X, float* y, float* dy, hipStream_t st) {
  if (!net || B < 0 || (B > 0 && (!X || !y))) {
    set_error("mlp_forward: bad arguments");
    return DSKI_EINVAL;
  }
  if (B == 0) return DSKI_OK;
  const int F = net->F, H = net->H, J = dy ? net->J : 0;
  MlpOff o = mlp_off(F, H);
  MlpWork w;
  DSKI_TRY(mlp_reserve(net, B, w));
  w.rows = (size_t)(1 + J) * B;
  const long long BH = (long long)B * H;
  k_mlp_l1<<<(unsigned)((BH + 255) / 256), 256, 0, st>>>(net->params, F, H, J, o, B, X, w);
  k_mlp_mm<true><<<(unsigned)((w.rows + 63) / 64), 256, 0, st>>>(w.S1, (long long)w.rows, net->params + o.W2, H,
                                                                 w.C);
  k_mlp_l2<<<B, 128, 0, st>>>(net->params, H, J, o, B, nullptr, nullptr, 0.f, 0, y, dy, w, nullptr);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

dski_status mlp_forward(dski_mlp net, int B, const float* X, float* y, dski_stream stream) {
  return mlp_eval(net, B, X, y, nullptr, static_cast<hipStream_t>(stream));
}

dski_status mlp_jvp(dski_mlp net, int B, const float* X, float* y, float* dy, dski_stream stream) {
  if (!dy) {
    set_error("mlp_jvp: dy is NULL");
    return DSKI_EINVAL;
  }
  return mlp_eval(net, B, X, y, dy, static_cast<hipStream_t>(stream));
}

dski_status mlp_backward(dski_mlp net, int B, const float* X, const float* t, const float* g, float lam,
                         double* loss_host, dski_stream stream) {
  if (!net || B <= 0 || !X || !t || (net->J > 0 && !g)) {
    set_error("mlp_backward: bad arguments");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int F = net->F, H = net->H, J = net->J;
  MlpOff o = mlp_off(F, H);
  MlpWork w;
  DSKI_TRY(mlp_reserve(net, B, w));
  const int nchunk = kMlpChunks;
  double* pW2 = w.part;                                // kMlpGramChunks x H x H
  double* pW1 = pW2 + (size_t)kMlpGramChunks * H * H;  // nchunk x H x F
  double* cs = pW1 + (size_t)nchunk * H * F;           // column sums of D1 row groups: (J+1) x nchunk x H
  double* cs2 = cs + (size_t)(J + 1) * nchunk * H;     // column sums of D2 rows 0..B-1: nchunk x H
  double* pw3 = cs2 + (size_t)nchunk * H;              // column sums of P3: nchunk x H
  double* lp = pw3 + (size_t)nchunk * H;               // B loss partials
  double* lsum = lp + B;
  const size_t K = (size_t)(1 + J) * B;
  const long long BH = (long long)B * H;
  const unsigned mmb = (unsigned)((K + 63) / 64);
  // forward: layer 1, layer-2 pre-activations of all K rows (matrix cores), layer 2,
  // loss and layer-2 deltas
  k_mlp_l1<<<(unsigned)((BH + 255) / 256), 256, 0, st>>>(net->params, F, H, J, o, B, X, w);
  k_mlp_mm<true><<<mmb, 256, 0, st>>>(w.S1, (long long)K, net->params + o.W2, H, w.C);
  k_mlp_l2<<<B, 128, 0, st>>>(net->params, H, J, o, B, t, g, lam, 1, nullptr, nullptr, w, lp);
  // layer-1 deltas: C = D2 W2 (matrix cores), then the GELU factors
  k_mlp_mm<false><<<mmb, 256, 0, st>>>(w.D2, (long long)K, net->params + o.W2, H, w.C);
  k_mlp_d1<<<(unsigned)((BH + 255) / 256), 256, 0, st>>>(net->params, F, H, J, o, B, w);
  DSKI_HIP(hipGetLastError());
  // dW2 = D2^T S1 (matrix cores, FP64 chunk partials)
  const long long gch = (((long long)K + kMlpGramChunks - 1) / kMlpGramChunks + 3) / 4 * 4;
  k_mlp_gram<<<kMlpGramChunks, 256, 0, st>>>(w.D2, w.S1, (long long)K, H, gch, pW2);
  // the small contractions in row chunks: dW1 = D1^T X (value rows), and in one
  // launch the column sums of each D1 row group, of the D2 value rows and of P3
  const long long chB = ((long long)B + nchunk - 1) / nchunk;
  k_mlp_tn_chunks<<<nchunk, std::min(1024, H * F), 0, st>>>(w.D1, H, X, F, (long long)B, chB, pW1);
  MlpColSrc src{};
  for (int gi = 0; gi <= J; ++gi) src.p[gi] = w.D1 + (size_t)gi * B * H;
  src.p[J + 1] = w.D2;
  src.p[J + 2] = w.P3;
  k_mlp_colsums<<<dim3(nchunk, J + 3), H, 0, st>>>(src, B, H, chB, cs);
  k_mlp_loss<<<1, 256, 0, st>>>(lp, B, lsum);
  k_mlp_sum_chunks<<<(H * H + 255) / 256, 256, 0, st>>>(pW2, kMlpGramChunks, H * H, net->grad + o.W2, nullptr);
  const int nsmall = H * F + 3 * H;
  k_mlp_small_grads<<<(nsmall + 255) / 256, 256, 0, st>>>(pW1, pw3, cs, cs2, nchunk, H, F, J, o, net->grad);
  k_mlp_b3<<<1, 256, 0, st>>>(w.E, B, net->grad + o.b3);
  DSKI_HIP(hipGetLastError());
  double hloss = 0.0;
  DSKI_HIP(hipMemcpyAsync(&hloss, lsum, sizeof(double), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  if (loss_host) *loss_host = hloss;
  return DSKI_OK;
}

dski_status mlp_step(dski_mlp net, float lr, float beta1, float beta2, float eps, dski_stream stream) {
  if (!net || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
    set_error("mlp_step: bad arguments");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  net->t += 1;
  const float c1 = 1.0f - powf(beta1, (float)net->t), c2 = 1.0f - powf(beta2, (float)net->t);
  k_adam<<<(net->np + 255) / 256, 256, 0, st>>>(net->params, net->grad, net->m, net->v, net->np, lr, beta1, beta2, eps,
                                               c1, c2);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

}  // extern "C"
