// Learned log-determinant surrogate: a two-hidden-layer GELU network in FP32
// with forward-mode tangents for its input derivative and the weight gradient
// of a value-and-gradient-matching loss (training on the device).
//
//   a1 = W1 x + b1, h1 = gelu(a1); a2 = W2 h1 + b2, h2 = gelu(a2); y = w3 . h2 + b3
//   tangents along the first J inputs:  da1_j = W1 e_j, dh1_j = gelu'(a1) da1_j,
//   da2_j = W2 dh1_j, dh2_j = gelu'(a2) da2_j, dy_j = w3 . dh2_j
//   loss = (1/B) sum_b [(y_b - t_b)^2 + lam sum_j (dy_bj - g_bj)^2]
//
// Per-sample kernel: one work-group of H threads per sample (thread = hidden
// unit), activations and tangents in LDS, W2 read column-major for W2 v and
// row-major for W2^T v (both copies kept) so that every load is coalesced.
// Weight gradients are products over the batch (K = (1 + J) B rows), split over
// K chunks with FP64 partials summed in a fixed order: deterministic.
// Adam (Kingma & Ba) updates the packed parameters in place.
#include <cmath>
#include <vector>

#include "internal.h"

struct dski_mlp_s {
  int F = 8, H = 128, J = 5, maxB = 0;
  int np = 0;                 // packed parameters
  float* params = nullptr;    // W1 (H x F), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1), row-major
  float* W2c = nullptr;       // W2 column-major copy
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

// Per-sample layout of the saved rows (each row H floats), (1 + J) B rows per group:
//   S1 = [h1; dh1_1..J], D2 = [da2; dda2_1..J], S2 = [h2; dh2_1..J], D1 = [da1; dda1_1..J]
// row index of (j, b) = j * B + b.  E = [ey; eg_1..J] ((1 + J) B scalars).
struct MlpWork {
  float *S1, *D2, *S2, *D1, *E;
  double* part;
  size_t rows;  // (1 + J) B
};

// mode 0: y (and dy if dy != NULL); mode 1: also the deltas of the loss.
__global__ __launch_bounds__(128) void k_mlp_sample(const float* __restrict__ P, const float* __restrict__ W2c,
                                                    int F, int H, int J, MlpOff o, int B,
                                                    const float* __restrict__ X, const float* __restrict__ tv,
                                                    const float* __restrict__ tg, float lam, int mode,
                                                    float* __restrict__ y_out, float* __restrict__ dy_out,
                                                    MlpWork w, double* __restrict__ loss_part) {
  __shared__ float sx[kMlpMaxF];
  __shared__ float sh1[kMlpMaxJ + 1][kMlpMaxH];
  __shared__ float sd2[kMlpMaxJ + 1][kMlpMaxH];
  __shared__ float red[2];
  const int b = blockIdx.x;
  const int i = threadIdx.x;
  if (i < F) sx[i] = X[(size_t)b * F + i];
  __syncthreads();
  const bool u = i < H;
  // layer 1 (thread i = unit i)
  float a1 = 0.f, g1 = 0.f, g1d = 0.f;
  float ta1[kMlpMaxJ];
  if (u) {
    a1 = P[o.b1 + i];
    for (int j = 0; j < F; ++j) a1 += P[o.W1 + i * F + j] * sx[j];
    g1 = gelu_d1f(a1);
    g1d = gelu_d2f(a1);
    sh1[0][i] = gelu_f(a1);
#pragma unroll
    for (int j = 0; j < kMlpMaxJ; ++j) {
      ta1[j] = j < J ? P[o.W1 + i * F + j] : 0.f;
      if (j < J) sh1[j + 1][i] = g1 * ta1[j];
    }
  }
  __syncthreads();
  // layer 2: a2_i = sum_l W2[i, l] h1_l (column-major copy: coalesced over i)
  float a2 = 0.f, g2 = 0.f, g2d = 0.f, h2 = 0.f;
  float ta2[kMlpMaxJ], th2[kMlpMaxJ];
#pragma unroll
  for (int j = 0; j < kMlpMaxJ; ++j) ta2[j] = 0.f;
  if (u) {
    a2 = P[o.b2 + i];
    for (int l = 0; l < H; ++l) {
      const float wv = W2c[l * H + i];
      a2 += wv * sh1[0][l];
#pragma unroll
      for (int j = 0; j < kMlpMaxJ; ++j)
        if (j < J) ta2[j] += wv * sh1[j + 1][l];
    }
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
  // loss deltas
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
  const size_t rows = w.rows;
  if (i == 0) {
    loss_part[b] = lpart;
    w.E[b] = ey;
    for (int j = 0; j < J; ++j) w.E[(size_t)(j + 1) * B + b] = eg[j];
  }
  if (u) {
    w.S1[(size_t)b * H + i] = sh1[0][i];
    w.S2[(size_t)b * H + i] = h2;
    float da2 = ey * w3i * g2;
    for (int j = 0; j < J; ++j) {
      const float ddh2 = eg[j] * w3i;
      da2 += ddh2 * g2d * ta2[j];
      const float dda2 = ddh2 * g2;
      sd2[j + 1][i] = dda2;
      w.S1[((size_t)(j + 1) * B + b) * H + i] = sh1[j + 1][i];
      w.S2[((size_t)(j + 1) * B + b) * H + i] = th2[j];
      w.D2[((size_t)(j + 1) * B + b) * H + i] = dda2;
    }
    sd2[0][i] = da2;
    w.D2[(size_t)b * H + i] = da2;
  }
  __syncthreads();
  // layer 1 deltas: dh1_l = sum_i W2[i, l] da2_i (row-major: coalesced over l)
  if (u) {
    const int l = i;
    float dh1 = 0.f;
    float ddh1[kMlpMaxJ];
#pragma unroll
    for (int j = 0; j < kMlpMaxJ; ++j) ddh1[j] = 0.f;
    for (int r = 0; r < H; ++r) {
      const float wv = P[o.W2 + r * H + l];
      dh1 += wv * sd2[0][r];
#pragma unroll
      for (int j = 0; j < kMlpMaxJ; ++j)
        if (j < J) ddh1[j] += wv * sd2[j + 1][r];
    }
    float da1 = dh1 * g1;
    for (int j = 0; j < J; ++j) {
      da1 += ddh1[j] * g1d * ta1[j];
      w.D1[((size_t)(j + 1) * B + b) * H + l] = ddh1[j] * g1;
    }
    w.D1[(size_t)b * H + l] = da1;
  }
  (void)rows;
}

// partial[c][i][l] = sum over k in chunk c of A[k][i] * Bm[k][l]  (FP64), rows k of
// A have lda floats, rows of Bm ldb floats; grid (M, nchunk), block ncols threads.
__global__ void k_mlp_gemm_tn(const float* __restrict__ A, int lda, const float* __restrict__ Bm, int ldb,
                              size_t K, int M, int ncols, size_t chunk, double* __restrict__ part) {
  const int i = blockIdx.x, c = blockIdx.y, l = threadIdx.x;
  if (l >= ncols) return;
  const size_t k0 = (size_t)c * chunk, k1 = k0 + chunk < K ? k0 + chunk : K;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  size_t k = k0;
  for (; k + 4 <= k1; k += 4) {
    acc0 += (double)A[k * lda + i] * (double)Bm[k * ldb + l];
    acc1 += (double)A[(k + 1) * lda + i] * (double)Bm[(k + 1) * ldb + l];
    acc2 += (double)A[(k + 2) * lda + i] * (double)Bm[(k + 2) * ldb + l];
    acc3 += (double)A[(k + 3) * lda + i] * (double)Bm[(k + 3) * ldb + l];
  }
  for (; k < k1; ++k) acc0 += (double)A[k * lda + i] * (double)Bm[k * ldb + l];
  part[((size_t)c * M + i) * ncols + l] = (acc0 + acc1) + (acc2 + acc3);
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

// column sums over row ranges: out[j][l] = sum_{b < B} M[(j * B + b) * H + l], j < nj (FP64).
// One work-group per j of S * H threads: slice s adds rows s, s + S, ... in
// order (eight loads in flight), then the S slices are added in order.
__global__ __launch_bounds__(1024) void k_mlp_colsum(const float* __restrict__ Mx, int B, int H,
                                                     double* __restrict__ out) {
  __shared__ double red[1024];
  const int j = blockIdx.x;
  const int S = blockDim.x / H;
  const int l = threadIdx.x % H, sl = threadIdx.x / H;
  double acc = 0.0;
  const float* col = Mx + (size_t)j * B * H + l;
#pragma unroll 8
  for (int b = sl; b < B; b += S) acc += (double)col[(size_t)b * H];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < H) {
    double t = 0.0;
    for (int q = 0; q < S; ++q) t += red[q * H + threadIdx.x];
    out[(size_t)j * H + threadIdx.x] = t;
  }
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

__global__ void k_mlp_transpose(const float* __restrict__ W, int H, float* __restrict__ Wc) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= H * H) return;
  const int r = f / H, c = f % H;
  Wc[c * H + r] = W[f];
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

static dski_status mlp_reserve(dski_mlp net, int B, MlpWork& w) {
  const int H = net->H, J = net->J;
  const size_t rows = (size_t)(1 + J) * B;
  const size_t fl = 4 * rows * H + rows + 64;
  const int nchunk = 16;
  const size_t parts = (size_t)nchunk * ((size_t)H * H + (size_t)H * net->F + H) + (size_t)(J + 2) * H +
                       (size_t)H * net->F + B + 64;
  DSKI_TRY(net->work.reserve(sizeof(float) * fl + sizeof(double) * parts + 256));
  float* base = net->work.as<float>();
  w.S1 = base;
  w.D2 = w.S1 + rows * H;
  w.S2 = w.D2 + rows * H;
  w.D1 = w.S2 + rows * H;
  w.E = w.D1 + rows * H;
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
    (void)hipFree(net->W2c);
    (void)hipFree(net->grad);
    (void)hipFree(net->m);
    (void)hipFree(net->v);
    delete net;
    return DSKI_EHIP;
  };
  if (hipMalloc(&net->params, sizeof(float) * o.n) != hipSuccess ||
      hipMalloc(&net->W2c, sizeof(float) * H * H) != hipSuccess ||
      hipMalloc(&net->grad, sizeof(float) * o.n) != hipSuccess ||
      hipMalloc(&net->m, sizeof(float) * o.n) != hipSuccess || hipMalloc(&net->v, sizeof(float) * o.n) != hipSuccess)
    return fail("allocation failed");
  if (hipMemcpyAsync(net->params, params_host, sizeof(float) * o.n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(net->m, 0, sizeof(float) * o.n, st) != hipSuccess ||
      hipMemsetAsync(net->v, 0, sizeof(float) * o.n, st) != hipSuccess ||
      hipMemsetAsync(net->grad, 0, sizeof(float) * o.n, st) != hipSuccess)
    return fail("upload failed");
  k_mlp_transpose<<<(H * H + 255) / 256, 256, 0, st>>>(net->params + o.W2, H, net->W2c);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return fail("transpose failed");
  *out = net;
  return DSKI_OK;
}

dski_status mlp_destroy(dski_mlp net) {
  if (!net) return DSKI_OK;
  (void)hipFree(net->params);
  (void)hipFree(net->W2c);
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
  MlpOff o = mlp_off(net->F, net->H);
  MlpWork w{};
  k_mlp_sample<<<B, 128, 0, st>>>(net->params, net->W2c, net->F, net->H, dy ? net->J : 0, o, B, X, nullptr,
                                  nullptr, 0.f, 0, y, dy, w, nullptr);
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
  const int nchunk = 16;
  double* pW2 = w.part;                                // nchunk x H x H
  double* pW1 = pW2 + (size_t)nchunk * H * H;          // nchunk x H x F
  double* pw3 = pW1 + (size_t)nchunk * H * F;          // nchunk x 1 x H
  double* cs = pw3 + (size_t)nchunk * H;               // column sums of D1 row groups: (J+1) x H
  double* cs2 = cs + (size_t)(J + 1) * H;              // column sums of D2 rows 0..B-1: H
  double* dadd = cs2 + H;                              // tangent columns of dW1: H x F
  double* lp = dadd + (size_t)H * F;                   // B loss partials
  double* lsum = lp + B;
  k_mlp_sample<<<B, 128, 0, st>>>(net->params, net->W2c, F, H, J, o, B, X, t, g, lam, 1, nullptr, nullptr, w, lp);
  DSKI_HIP(hipGetLastError());
  const size_t K = (size_t)(1 + J) * B;
  const size_t ch = (K + nchunk - 1) / nchunk;
  // dW2 = D2^T S1
  k_mlp_gemm_tn<<<dim3(H, nchunk), 128, 0, st>>>(w.D2, H, w.S1, H, K, H, H, ch, pW2);
  // dw3 = E^T S2
  k_mlp_gemm_tn<<<dim3(1, nchunk), 128, 0, st>>>(w.E, 1, w.S2, H, K, 1, H, ch, pw3);
  // dW1 = D1[0:B]^T X  (value rows only); tangent rows add their column sums below
  const size_t chB = ((size_t)B + nchunk - 1) / nchunk;
  k_mlp_gemm_tn<<<dim3(H, nchunk), 128, 0, st>>>(w.D1, H, X, F, (size_t)B, H, F, chB, pW1);
  const int cst = (1024 / H) * H;
  k_mlp_colsum<<<J + 1, cst, 0, st>>>(w.D1, B, H, cs);
  k_mlp_colsum<<<1, cst, 0, st>>>(w.D2, B, H, cs2);
  k_mlp_loss<<<1, 256, 0, st>>>(lp, B, lsum);
  DSKI_HIP(hipGetLastError());
  // assemble the packed gradient (FP32)
  std::vector<double> hcs((size_t)(J + 1) * H), hcs2(H);
  DSKI_HIP(hipMemcpyAsync(hcs.data(), cs, sizeof(double) * hcs.size(), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hcs2.data(), cs2, sizeof(double) * H, hipMemcpyDeviceToHost, st));
  double hloss = 0.0;
  DSKI_HIP(hipMemcpyAsync(&hloss, lsum, sizeof(double), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  // W1 tangent columns: dW1[i][j] += sum_b dda1_j[b][i]  (j < J); b1 = column sums of da1
  std::vector<double> addW1((size_t)H * F, 0.0);
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < J; ++j) addW1[(size_t)i * F + j] = hcs[(size_t)(j + 1) * H + i];
  DSKI_HIP(hipMemcpyAsync(dadd, addW1.data(), sizeof(double) * H * F, hipMemcpyHostToDevice, st));
  k_mlp_sum_chunks<<<(H * F + 255) / 256, 256, 0, st>>>(pW1, nchunk, H * F, net->grad + o.W1, dadd);
  k_mlp_sum_chunks<<<(H * H + 255) / 256, 256, 0, st>>>(pW2, nchunk, H * H, net->grad + o.W2, nullptr);
  k_mlp_sum_chunks<<<(H + 255) / 256, 256, 0, st>>>(pw3, nchunk, H, net->grad + o.w3, nullptr);
  std::vector<float> hb((size_t)2 * H + 1);
  for (int i = 0; i < H; ++i) {
    hb[i] = (float)hcs[i];        // b1
    hb[H + i] = (float)hcs2[i];   // b2
  }
  // db3 = sum_b ey_b = (2 / B) sum_b (y_b - t_b): from E row 0
  std::vector<float> hey(B);
  DSKI_HIP(hipMemcpyAsync(hey.data(), w.E, sizeof(float) * B, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  double db3 = 0.0;
  for (int b = 0; b < B; ++b) db3 += hey[b];
  DSKI_HIP(hipMemcpyAsync(net->grad + o.b1, hb.data(), sizeof(float) * H, hipMemcpyHostToDevice, st));
  DSKI_HIP(hipMemcpyAsync(net->grad + o.b2, hb.data() + H, sizeof(float) * H, hipMemcpyHostToDevice, st));
  float fb3 = (float)db3;
  DSKI_HIP(hipMemcpyAsync(net->grad + o.b3, &fb3, sizeof(float), hipMemcpyHostToDevice, st));
  DSKI_HIP(hipGetLastError());
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
  MlpOff o = mlp_off(net->F, net->H);
  k_mlp_transpose<<<(net->H * net->H + 255) / 256, 256, 0, st>>>(net->params + o.W2, net->H, net->W2c);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

}  // extern "C"
