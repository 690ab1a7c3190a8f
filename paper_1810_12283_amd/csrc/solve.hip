// Stochastic Lanczos quadrature for log det K~ and the log marginal likelihood
// eq. (1) with its hyper-parameter gradient.
//
// One block PCG carries the data solve alpha = K~^{-1} y and the probe solves
// u_i = K~^{-1} z_i, z_i = C w_i (C C^T = M, w_i Rademacher).  From the same run:
//   log det K~ ~ log det M + (1/t) sum_i (z_i^T M^{-1} z_i) e_1^T log(T_i) e_1,
// with T_i the Lanczos tridiagonal of probe i from its CG coefficients (Sec. 2);
//   d mll / d theta = 1/2 alpha^T K' alpha - 1/2 (1/t) sum_i u_i^T K' v_i,  v_i = M^{-1} z_i,
// where K' = dK~/dtheta is the derivative of the approximate kernel (Sec. 3):
// for ell_p and s it is S K_UU' S^T with K_UU' the Kronecker-Toeplitz matrix with
// the derivative spectrum on axis p (or 2 K_UU), so the products reduce to dot
// products of scattered grids; for the noise levels it is diagonal.
#include <algorithm>
#include <cmath>
#include <thread>

#include "internal.h"

namespace dski {

// partial[b, q] = sum over a chunk of a[pa[q]] . b[pb[q]] (columns of length len, offset lo)
template <typename T>
__global__ void k_pair_dots(const T* __restrict__ A, long long lda, const T* __restrict__ Bm,
                            long long ldb, const int* __restrict__ pairs, int npairs, long long lo,
                            long long len, double* __restrict__ partial) {
  int q = blockIdx.y;
  int ca = pairs[2 * q], cb = pairs[2 * q + 1];
  const T* a = A + (size_t)ca * lda + lo;
  const T* b = Bm + (size_t)cb * ldb + lo;
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    acc += (double)a[e] * (double)b[e];
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * npairs + q] = red[0] + red[1] + red[2] + red[3];
}

struct DotCtx {
  DevBuf buf;  // pairs (int) + partials + results
};

template <typename T>
static dski_status pair_dots(const T* A, long long lda, const T* B, long long ldb,
                             const std::vector<int>& pairs, long long lo, long long len,
                             std::vector<double>& out, DevBuf& buf, hipStream_t st) {
  int np = (int)pairs.size() / 2;
  out.assign(np, 0.0);
  if (np == 0 || len <= 0) return DSKI_OK;
  int nblk = (int)std::min<long long>(256, (len + kBlock - 1) / kBlock);
  size_t bytes = sizeof(int) * pairs.size() + 64 + sizeof(double) * ((size_t)nblk * np + np);
  DSKI_TRY(buf.reserve(bytes));
  int* dp = buf.as<int>();
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(dp) + ((sizeof(int) * pairs.size() + 63) / 64) * 64);
  double* res = part + (size_t)nblk * np;
  DSKI_HIP(hipMemcpyAsync(dp, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice, st));
  k_pair_dots<T><<<dim3(nblk, np), kBlock, 0, st>>>(A, lda, B, ldb, dp, np, lo, len, part);
  DSKI_HIP(hipGetLastError());
  DSKI_TRY(reduce_partials(part, nblk, np, res, st));
  DSKI_HIP(hipMemcpyAsync(out.data(), res, sizeof(double) * np, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  return DSKI_OK;
}

__global__ void k_copy_cols_d(const double* __restrict__ src, double* __restrict__ dst, long long M,
                              const int* __restrict__ cols, int nc) {
  int c = blockIdx.y;
  const double* s = src + (size_t)cols[c] * M;
  double* d = dst + (size_t)c * M;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < M;
       e += (long long)gridDim.x * blockDim.x)
    d[e] = s[e];
}

static const std::vector<int>& p00_pair() {
  static const std::vector<int> v = {0, 0};
  return v;
}

template <typename T>
__global__ void k_swap_cols(T* __restrict__ a, T* __restrict__ b, int N) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
    const T v = a[e];
    a[e] = b[e];
    b[e] = v;
  }
}

template <typename T>
static dski_status swap_first_column(T* a, T* b, int N, hipStream_t st) {
  k_swap_cols<T><<<std::max(1, std::min(1024, (N + kBlock - 1) / kBlock)), kBlock, 0, st>>>(a, b, N);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

struct ProbeRun {
  std::vector<double> quad, weight;
  double logdet = 0, stderr_ = 0;
  bool ok = true;
};

static void slq_combine(const std::vector<double>& ab, int max_iter, int R, int col0, int t,
                        const PcgResult& res, double logdetM, ProbeRun& out) {
  out.quad.assign(t, 0.0);
  out.weight.assign(t, 0.0);
  std::vector<double> vals(t);
  std::vector<int> okv(t, 1);
  // one Gauss quadrature per probe: probes spread over host threads
  auto work = [&](int i) {
    const int c = col0 + i;
    const int J = std::min(res.iters[c], max_iter);
    int ok = 0;
    const double q = gauss_quad_log(ab.data() + (size_t)c * max_iter,
                                    ab.data() + (size_t)R * max_iter + (size_t)c * max_iter, J, &ok);
    okv[i] = ok;
    out.quad[i] = q;
    out.weight[i] = res.rz0[c];
    vals[i] = q * res.rz0[c];
  };
  const int nth = std::max(1, std::min(t, (int)std::thread::hardware_concurrency()));
  if (nth <= 1) {
    for (int i = 0; i < t; ++i) work(i);
  } else {
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
      pool.emplace_back([&, w]() {
        for (int i = w; i < t; i += nth) work(i);
      });
    for (auto& th : pool) th.join();
  }
  double mean = 0.0;
  for (int i = 0; i < t; ++i) {
    if (!okv[i]) out.ok = false;
    mean += vals[i];
  }
  mean /= std::max(t, 1);
  double var = 0.0;
  for (int i = 0; i < t; ++i) var += (vals[i] - mean) * (vals[i] - mean);
  out.logdet = logdetM + mean;
  out.stderr_ = t > 1 ? std::sqrt(var / (t - 1) / t) : NAN;
}

}  // namespace dski

using namespace dski;

// ---------------------------------------------------------------- fixed-step Lanczos
// part[b, i t + c] = sum over a row chunk of A[i t + c] . Bv[c] (column stride N),
// for the first J vector slots i of each of the t columns.
__global__ void k_lz_dots(const double* __restrict__ A, const double* __restrict__ Bv, int N, int t, int J,
                          double* __restrict__ part) {
  const int q = blockIdx.y, c = q % t;
  const double* a = A + (size_t)q * N;
  const double* b = Bv + (size_t)c * N;
  double acc = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x)
    acc += a[e] * b[e];
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * ((size_t)J * t) + q] = (red[0] + red[1]) + (red[2] + red[3]);
}

// W[c] -= sum_{i < J} h[i t + c] Q[i t + c]   (Q column stride N)
__global__ void k_lz_sub(const double* __restrict__ Q, const double* __restrict__ h, int N, int t, int J,
                         double* __restrict__ W) {
  const int c = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
    double v = W[(size_t)c * N + e];
    for (int i = 0; i < J; ++i) v -= h[(size_t)i * t + c] * Q[((size_t)i * t + c) * N + e];
    W[(size_t)c * N + e] = v;
  }
}

// Out[c] = In[c] * f[c]
__global__ void k_lz_scale(const double* __restrict__ In, const double* __restrict__ f, int N,
                           double* __restrict__ Out) {
  const int c = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x)
    Out[(size_t)c * N + e] = In[(size_t)c * N + e] * f[c];
}

// Fixed-step SLQ (lanczos_steps > 0): for every probe z = C w the explicit
// Lanczos process of the preconditioned operator in the M-inner product (the
// process CG runs implicitly, Sec. 2), with full re-orthogonalisation:
// residual-space vectors q_j and z_j = M^{-1} q_j,
//   w = K~ z_j,  a_j = z_j . w,  w -= a_j q_j + b_{j-1} q_{j-1},
//   then twice  w -= sum_{i <= j} (z_i . w) q_i   (classical Gram-Schmidt),
//   b_j = sqrt(w . M^{-1} w),  q_{j+1} = w / b_j.
// The quadrature weight is ||z||^2_{M^{-1}}.  A short run without
// re-orthogonalisation is ill-conditioned (rounding-level changes of K~ or
// M^{-1} move its value by ~1e-3); this one is not.  All vectors FP64.
static dski_status slq_fixed_lanczos(dski_plan p, dski_precond pc, int t, int steps, uint64_t seed,
                                     double* logdet_host, double* stderr_host, hipStream_t st) {
  const int N = p->N;
  const size_t nr = (size_t)N * t;
  const int nb = std::max(1, std::min(256, (N + kBlock - 1) / kBlock));
  const int vb = std::max(1, std::min(1024, (N + kBlock - 1) / kBlock));
  DevBuf tmp;
  // Qs, Zs (steps + 1 slots of t columns each), W, ZW, X; partials and small scalars
  const size_t vec_doubles = 2 * (size_t)(steps + 1) * nr + 3 * nr;
  const size_t small = (size_t)nb * (steps + 1) * t + 2 * (size_t)(steps + 1) * t + 64;
  DSKI_TRY(tmp.reserve(sizeof(double) * (vec_doubles + small)));
  double* Qs = tmp.as<double>();
  double* Zs = Qs + (size_t)(steps + 1) * nr;
  double* W = Zs + (size_t)(steps + 1) * nr;
  double* ZW = W + nr;
  double* X = ZW + nr;
  double* part = X + nr;
  double* hdev = part + (size_t)nb * (steps + 1) * t;
  double* rdev = hdev + (size_t)(steps + 1) * t;
  auto dots = [&](const double* A, const double* Bv, int J, std::vector<double>& out) -> dski_status {
    k_lz_dots<<<dim3(nb, J * t), kBlock, 0, st>>>(A, Bv, N, t, J, part);
    DSKI_HIP(hipGetLastError());
    DSKI_TRY(reduce_partials(part, nb, J * t, rdev, st));
    out.assign((size_t)J * t, 0.0);
    DSKI_HIP(hipMemcpyAsync(out.data(), rdev, sizeof(double) * out.size(), hipMemcpyDeviceToHost, st));
    DSKI_HIP(hipStreamSynchronize(st));
    return DSKI_OK;
  };
  auto sub = [&](const std::vector<double>& h, int J) -> dski_status {
    DSKI_HIP(hipMemcpyAsync(hdev, h.data(), sizeof(double) * (size_t)J * t, hipMemcpyHostToDevice, st));
    k_lz_sub<<<dim3(vb, t), kBlock, 0, st>>>(Qs, hdev, N, t, J, W);
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  };
  auto scale = [&](const double* In, const std::vector<double>& f, double* Out) -> dski_status {
    DSKI_HIP(hipMemcpyAsync(hdev, f.data(), sizeof(double) * t, hipMemcpyHostToDevice, st));
    k_lz_scale<<<dim3(vb, t), kBlock, 0, st>>>(In, hdev, N, Out);
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  };
  auto msolve = [&](const double* In, double* Out) -> dski_status {
    if (pc) return precond_apply_tiled<double>(pc, t, In, N, Out, N, nullptr, nullptr, st);
    DSKI_HIP(hipMemcpyAsync(Out, In, sizeof(double) * nr, hipMemcpyDeviceToDevice, st));
    return DSKI_OK;
  };
  dski_status rc = DSKI_OK;
  do {
    // probes in user order -> tile order -> r_0 = z = C w
    rc = rademacher<double>(seed, 0, t, N, X, N, st);
    if (rc < 0) break;
    rc = permute(p, +1, t, X, N, ZW, N, st);
    if (rc < 0) break;
    if (pc) {
      rc = precond_factor_apply_tiled<double>(pc, t, ZW, N, W, N, st);
    } else {
      rc = hipMemcpyAsync(W, ZW, sizeof(double) * nr, hipMemcpyDeviceToDevice, st) == hipSuccess ? DSKI_OK
                                                                                                 : DSKI_EHIP;
    }
    if (rc < 0) break;
    rc = msolve(W, ZW);
    if (rc < 0) break;
    std::vector<double> nrm2;
    rc = dots(ZW, W, 1, nrm2);  // z . M^{-1} z  (slot 0 of ZW pairs with column c of W)
    if (rc < 0) break;
    std::vector<double> f(t);
    for (int c = 0; c < t; ++c) f[c] = nrm2[c] > 0.0 ? 1.0 / std::sqrt(nrm2[c]) : 0.0;
    rc = scale(W, f, Qs);
    if (rc < 0) break;
    rc = scale(ZW, f, Zs);
    if (rc < 0) break;
    std::vector<std::vector<double>> diag(t), off(t);
    std::vector<int> done(t, 0);
    std::vector<double> bprev(t, 0.0);
    for (int j = 0; j < steps && rc >= 0; ++j) {
      const double* Qj = Qs + (size_t)j * nr;
      const double* Zj = Zs + (size_t)j * nr;
      rc = mvm_tiled<double>(p, t, Zj, N, W, N, nullptr, st);
      if (rc < 0) break;
      std::vector<double> a;
      rc = dots(Zj, W, 1, a);
      if (rc < 0) break;
      // three-term step: coefficients a_j on slot j and b_{j-1} on slot j-1
      std::vector<double> h((size_t)(j + 1) * t, 0.0);
      for (int c = 0; c < t; ++c) {
        if (!done[c]) diag[c].push_back(a[c]);
        h[(size_t)j * t + c] = a[c];
        if (j > 0) h[(size_t)(j - 1) * t + c] = bprev[c];
      }
      rc = sub(h, j + 1);
      if (rc < 0) break;
      for (int pass = 0; pass < 2 && rc >= 0; ++pass) {  // full re-orthogonalisation
        std::vector<double> hh;
        rc = dots(Zs, W, j + 1, hh);
        if (rc < 0) break;
        rc = sub(hh, j + 1);
      }
      if (rc < 0) break;
      rc = msolve(W, ZW);
      if (rc < 0) break;
      std::vector<double> bb;
      rc = dots(ZW, W, 1, bb);
      if (rc < 0) break;
      if (j == steps - 1) break;
      for (int c = 0; c < t; ++c) {
        const double b = std::sqrt(std::fmax(bb[c], 0.0));
        // a vanishing b ends the column's process (Krylov space exhausted); its
        // later slots only carry zeros
        if (done[c] || !(b > 1e-14 * std::fabs(diag[c].back()))) {
          done[c] = 1;
          f[c] = 0.0;
          bprev[c] = 0.0;
        } else {
          off[c].push_back(b);
          f[c] = 1.0 / b;
          bprev[c] = b;
        }
      }
      rc = scale(W, f, Qs + (size_t)(j + 1) * nr);
      if (rc < 0) break;
      rc = scale(ZW, f, Zs + (size_t)(j + 1) * nr);
    }
    if (rc < 0) break;
    std::vector<double> vals(t);
    bool ok_all = true;
    for (int c = 0; c < t; ++c) {
      int ok = 0;
      const double q = gauss_quad_log_tri(diag[c].data(), off[c].data(), (int)diag[c].size(), &ok);
      if (!ok) ok_all = false;
      vals[c] = nrm2[c] * q;
    }
    if (!ok_all) {
      set_error("SLQ: non-positive Ritz value or quadrature failure");
      rc = DSKI_EBREAKDOWN;
      break;
    }
    double mean = 0.0;
    for (double v : vals) mean += v;
    mean /= t;
    double var = 0.0;
    for (double v : vals) var += (v - mean) * (v - mean);
    *logdet_host = (pc ? pc->logdet : 0.0) + mean;
    if (stderr_host) *stderr_host = t > 1 ? std::sqrt(var / (t - 1) / t) : NAN;
  } while (0);
  (void)hipStreamSynchronize(st);
  tmp.release();
  return rc;
}

template <typename T>
static dski_status slq_impl(dski_plan p, dski_precond pc, int t, int lanczos_steps, double tol, int max_iter,
                            uint64_t seed, double* logdet_host, double* stderr_host, hipStream_t st) {
  int N = p->N;
  int steps = lanczos_steps > 0 ? lanczos_steps : max_iter;
  size_t nr = (size_t)N * t;
  DevBuf tmp;
  DSKI_TRY(tmp.reserve(sizeof(T) * nr * 3 + sizeof(double) * 2 * (size_t)steps * t + 1024));
  T* W = tmp.as<T>();
  T* Z = W + nr;
  T* X = Z + nr;
  double* ab = reinterpret_cast<double*>(tmp.as<char>() + ((sizeof(T) * nr * 3 + 63) / 64) * 64);
  dski_status rc = DSKI_OK;
  do {
    // probes in user order -> tile order -> z = C w
    rc = rademacher<T>(seed, 0, t, N, X, N, st);
    if (rc < 0) break;
    rc = permute(p, +1, t, X, N, W, N, st);
    if (rc < 0) break;
    if (pc)
      rc = precond_factor_apply_tiled<T>(pc, t, W, N, Z, N, st);
    else
      rc = hipMemcpyAsync(Z, W, sizeof(T) * nr, hipMemcpyDeviceToDevice, st) == hipSuccess ? DSKI_OK
                                                                                             : DSKI_EHIP;
    if (rc < 0) break;
    std::vector<double> tols(t, lanczos_steps > 0 ? 0.0 : tol);
    PcgResult res;
    rc = pcg_tiled<T>(p, pc, t, Z, N, X, N, tols.data(), steps, lanczos_steps, ab, res, st);
    if (rc < 0) break;
    std::vector<double> hab(2 * (size_t)steps * t);
    if (hipMemcpyAsync(hab.data(), ab, sizeof(double) * hab.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("SLQ copy failed");
      rc = DSKI_EHIP;
      break;
    }
    ProbeRun pr;
    slq_combine(hab, steps, t, 0, t, res, pc ? pc->logdet : 0.0, pr);
    if (!pr.ok) {
      set_error("SLQ: non-positive Ritz value or quadrature failure");
      rc = DSKI_EBREAKDOWN;
      break;
    }
    *logdet_host = pr.logdet;
    if (stderr_host) *stderr_host = pr.stderr_;
  } while (0);
  tmp.release();
  return rc;
}

// Warm start of the data column: r0 = y - K~ x0 (FP64 in, storage T out).
template <typename T>
__global__ void k_warm_residual(const T* __restrict__ y, const double* __restrict__ kx0, int N, T* __restrict__ r0) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x)
    r0[e] = (T)((double)y[e] - kx0[e]);
}

// alpha = x0 + dx (FP64) into the storage-type data column and an FP64 copy.
template <typename T>
__global__ void k_warm_alpha(const double* __restrict__ x0, const double* __restrict__ dx, int N, T* __restrict__ a,
                             double* __restrict__ a64) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
    const double v = x0[e] + dx[e];
    a[e] = (T)v;
    a64[e] = v;
  }
}

template <typename T>
static dski_status mll_impl(dski_plan p, dski_precond pc, const T* y, int t, uint64_t seed, double tol,
                            int max_iter, double* mll_host, double* grad_host, double* logdet_host,
                            int* iters_host, hipStream_t st, const double* x0 = nullptr,
                            double* alpha_out = nullptr) {
  int N = p->N, n = p->n, d = p->d;
  long long M = p->M;
  dski_status rc = DSKI_OK;
  int R = 1 + t;
  size_t nr = (size_t)N * R;
  DevBuf tmp, dotbuf;
  int* dcols = nullptr;
  do {
    // buffers: B (R cols), X (R cols), Vv (t cols), W (t cols), CG history
    size_t fl = nr * 2 + (size_t)N * t * 2;
    rc = tmp.reserve(sizeof(T) * fl + sizeof(double) * 2 * (size_t)max_iter * R + 1024);
    if (rc < 0) break;
    T* B = tmp.as<T>();
    T* X = B + nr;
    T* Vv = X + nr;
    T* W = Vv + (size_t)N * t;
    double* ab = reinterpret_cast<double*>(tmp.as<char>() + ((sizeof(T) * fl + 63) / 64) * 64);
    rc = permute(p, +1, 1, y, N, B, N, st);
    if (rc < 0) break;
    rc = rademacher<T>(seed, 0, t, N, Vv, N, st);
    if (rc < 0) break;
    rc = permute(p, +1, t, Vv, N, W, N, st);
    if (rc < 0) break;
    rc = precond_factor_apply_tiled<T>(pc, t, W, N, B + N, N, st);
    if (rc < 0) break;
    std::vector<double> tols(R, tol);
    PcgResult res;
    std::vector<int> verify(R, 0);
    verify[0] = 1;  // the data solve alpha; probe columns keep a single Krylov run for SLQ
    // warm start of the data column (x0 in user order): solve K~ dx = y - K~ x0 to
    // the tolerance of ||y - K~ alpha|| <= tol ||y||, then alpha = x0 + dx
    DevBuf warm;
    double* x0t = nullptr;
    double* X64 = nullptr;
    T* ysave = nullptr;
    const int wb = std::max(1, std::min(1024, (N + kBlock - 1) / kBlock));
    if (x0 || alpha_out) {
      rc = warm.reserve(sizeof(double) * ((size_t)N * 2 + nr) + sizeof(T) * (size_t)N + 256);
      if (rc < 0) break;
      x0t = warm.as<double>();
      double* kx0 = x0t + N;
      X64 = kx0 + N;
      ysave = reinterpret_cast<T*>(X64 + nr);
      if (x0) {
        rc = permute(p, +1, 1, x0, N, x0t, N, st);
        if (rc < 0) break;
        rc = mvm_tiled<double>(p, 1, x0t, N, kx0, N, nullptr, st);
        if (rc < 0) break;
        std::vector<double> yy, rr;
        rc = pair_dots<T>(B, N, B, N, p00_pair(), 0, N, yy, dotbuf, st);
        if (rc < 0) break;
        k_warm_residual<T><<<wb, kBlock, 0, st>>>(B, kx0, N, ysave);
        if (hipGetLastError() != hipSuccess) {
          set_error("mll_and_grad: warm-start launch failed");
          rc = DSKI_EHIP;
          break;
        }
        // B[:, 0] <- r0; y waits in ysave until the solve is done
        rc = swap_first_column<T>(B, ysave, N, st);
        if (rc < 0) break;
        rc = pair_dots<T>(B, N, B, N, p00_pair(), 0, N, rr, dotbuf, st);
        if (rc < 0) break;
        if (rr[0] > 0.0) tols[0] = tol * std::sqrt(yy[0] / rr[0]);
      } else if (hipMemsetAsync(x0t, 0, sizeof(double) * N, st) != hipSuccess) {
        set_error("mll_and_grad: clearing the start failed");
        rc = DSKI_EHIP;
        break;
      }
    }
    rc = pcg_tiled<T>(p, pc, R, B, N, X, N, tols.data(), max_iter, 0, ab, res, st, X64, verify.data());
    if (rc < 0) break;
    dski_status pcg_rc = rc;
    if (x0 || alpha_out) {
      // alpha = x0 + dx in the data column (storage type) and in FP64; y back in B[:, 0]
      k_warm_alpha<T><<<wb, kBlock, 0, st>>>(x0t, X64, N, X, X64);
      if (hipGetLastError() != hipSuccess) {
        set_error("mll_and_grad: warm-start launch failed");
        rc = DSKI_EHIP;
        break;
      }
      if (x0) {
        rc = swap_first_column<T>(B, ysave, N, st);
        if (rc < 0) break;
      }
      if (alpha_out) {
        rc = permute(p, -1, 1, X64, N, alpha_out, N, st);
        if (rc < 0) break;
      }
    }
    // v_i = M^{-1} z_i
    rc = precond_apply_tiled<T>(pc, t, B + N, N, Vv, N, nullptr, nullptr, st);
    if (rc < 0) break;
    // log det by SLQ from the same run
    std::vector<double> hab(2 * (size_t)max_iter * R);
    if (hipMemcpyAsync(hab.data(), ab, sizeof(double) * hab.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("mll_and_grad: copy failed");
      rc = DSKI_EHIP;
      break;
    }
    ProbeRun pr;
    if (t > 0) {
      slq_combine(hab, max_iter, R, 1, t, res, pc->logdet, pr);
      if (!pr.ok) {
        set_error("mll_and_grad: SLQ quadrature failed");
        rc = DSKI_EBREAKDOWN;
        break;
      }
    } else {  // data-fit part only: no log det term
      pr.ok = true;
      pr.logdet = 0.0;
    }
    // data fit y^T alpha; alpha^T alpha and u_i^T v_i on value rows and on gradient rows
    std::vector<double> yal, aa_v, aa_g, uv_v, uv_g;
    std::vector<int> p00 = {0, 0};
    rc = pair_dots<T>(B, N, X, N, p00, 0, N, yal, dotbuf, st);
    if (rc < 0) break;
    rc = pair_dots<T>(X, N, X, N, p00, 0, n, aa_v, dotbuf, st);
    if (rc < 0) break;
    rc = pair_dots<T>(X, N, X, N, p00, n, N - n, aa_g, dotbuf, st);
    if (rc < 0) break;
    std::vector<int> puv;
    for (int i = 0; i < t; ++i) {
      puv.push_back(1 + i);
      puv.push_back(i);
    }
    rc = pair_dots<T>(X, N, Vv, N, puv, 0, n, uv_v, dotbuf, st);
    if (rc < 0) break;
    rc = pair_dots<T>(X, N, Vv, N, puv, n, N - n, uv_g, dotbuf, st);
    if (rc < 0) break;
    // grids G = [S^T alpha, S^T u_1..u_t, S^T v_1..v_t]; H = K' [S^T alpha, S^T v_i]
    int Rg = 1 + 2 * t;
    rc = p->grid.reserve(sizeof(double) * (size_t)M * (Rg + 1 + t));
    if (rc < 0) break;
    double* G = p->grid.as<double>();
    double* H = G + (size_t)M * Rg;
    rc = scatter<T, double>(p, R, X, N, G, st);
    if (rc < 0) break;
    rc = scatter<T, double>(p, t, Vv, N, G + (size_t)M * R, st);
    if (rc < 0) break;
    std::vector<int> cols;
    cols.push_back(0);
    for (int i = 0; i < t; ++i) cols.push_back(R + i);
    std::vector<int> gp = {0, 0};  // (H col, G col) pairs
    for (int i = 0; i < t; ++i) {
      gp.push_back(1 + i);
      gp.push_back(1 + i);
    }
    if (hipMalloc(&dcols, sizeof(int) * cols.size()) != hipSuccess) {
      dcols = nullptr;
      set_error("allocation failed");
      rc = DSKI_ENOMEM;
      break;
    }
    if (hipMemcpyAsync(dcols, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
      set_error("copy failed");
      rc = DSKI_EHIP;
      break;
    }
    std::vector<double> g(d + 3, 0.0);
    for (int which = 0; which <= d && rc >= 0; ++which) {
      int nb = (int)std::min<long long>(1024, (M + kBlock - 1) / kBlock);
      k_copy_cols_d<<<dim3(nb, 1 + t), kBlock, 0, st>>>(G, H, M, dcols, 1 + t);
      rc = apply_kuu<double>(p, 1 + t, H, st, which < d ? which : -1);
      if (rc < 0) break;
      std::vector<double> dots;
      rc = pair_dots<double>(H, M, G, M, gp, 0, M, dots, dotbuf, st);
      if (rc < 0) break;
      double scale = which < d ? 1.0 : 2.0;  // d K_UU / d log s = 2 K_UU
      double tr = 0.0;
      for (int i = 0; i < t; ++i) tr += dots[1 + i];
      if (t > 0) tr /= t;
      g[which] = scale * (0.5 * dots[0] - 0.5 * tr);
    }
    if (rc < 0) break;
    double sf2 = p->sf * p->sf, sg2 = p->sg * p->sg;
    double trv = 0.0, trg = 0.0;
    for (int i = 0; i < t; ++i) {
      trv += uv_v[i];
      trg += uv_g[i];
    }
    // dK~/dlog sigma = 2 sigma^2 on the value (gradient) rows
    g[d + 1] = sf2 * (aa_v[0] - (t > 0 ? trv / t : 0.0));
    g[d + 2] = sg2 * (aa_g[0] - (t > 0 ? trg / t : 0.0));
    const double log2pi = 1.8378770664093453;
    double mll = -0.5 * (yal[0] + pr.logdet + (double)N * log2pi);
    if (mll_host) *mll_host = mll;
    if (grad_host)
      for (int j = 0; j < d + 3; ++j) grad_host[j] = g[j];
    if (logdet_host) *logdet_host = pr.logdet;
    if (iters_host)
      for (int r = 0; r < R; ++r) iters_host[r] = res.iters[r];
    rc = pcg_rc;
  } while (0);
  if (dcols) (void)hipFree(dcols);
  tmp.release();
  dotbuf.release();
  return rc;
}

template <typename T>
static dski_status mll_user(dski_plan p, dski_precond pc_in, int k, const T* y, int t, uint64_t seed,
                            double tol, int max_iter, double* mll_host, double* grad_host,
                            double* logdet_host, int* iters_host, hipStream_t st, const double* x0 = nullptr,
                            double* alpha_out = nullptr) {
  if (!p || !y || t < 0 || tol <= 0 || max_iter <= 0 || (!pc_in && k < 0) ||
      (pc_in && pc_in->plan != p) || p->N == 0) {
    set_error("mll_and_grad: bad arguments");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("mll_and_grad: the length-scale gradient needs a D-SKI plan (D-SKIP factors are not "
              "differentiated)");
    return DSKI_ENOTSUP;
  }
  dski_precond pc = pc_in;
  if (!pc) {
    int rank = 0;
    dski_status rc = pivchol_build(p, k, &pc, &rank, nullptr, st);
    if (rc < 0) return rc;
  }
  dski_status rc = mll_impl<T>(p, pc, y, t, seed, tol, max_iter, mll_host, grad_host, logdet_host,
                               iters_host, st, x0, alpha_out);
  if (!pc_in) dski_precond_destroy(pc);
  return rc;
}

extern "C" {

dski_status slq_logdet(dski_plan p, dski_precond pc, int t, int lanczos_steps, double tol, int max_iter,
                       uint64_t seed, double* logdet_host, double* stderr_host, dski_stream stream) {
  if (!p || t <= 0 || lanczos_steps < 0 || (lanczos_steps == 0 && (tol <= 0 || max_iter <= 0)) ||
      (pc && pc->plan != p) || !logdet_host || p->N == 0) {
    set_error("slq_logdet: bad arguments");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (lanczos_steps > 0) return slq_fixed_lanczos(p, pc, t, lanczos_steps, seed, logdet_host, stderr_host, st);
  if (p->precision == 64)
    return slq_impl<double>(p, pc, t, lanczos_steps, tol, max_iter, seed, logdet_host, stderr_host, st);
  return slq_impl<float>(p, pc, t, lanczos_steps, tol, max_iter, seed, logdet_host, stderr_host, st);
}

dski_status mll_and_grad(dski_plan p, dski_precond pc, int k, const float* y, int t, uint64_t seed,
                         double tol, int max_iter, double* mll_host, double* grad_host,
                         double* logdet_host, int* iters_host, dski_stream stream) {
  return mll_user<float>(p, pc, k, y, t, seed, tol, max_iter, mll_host, grad_host, logdet_host,
                         iters_host, static_cast<hipStream_t>(stream));
}

dski_status mll_and_grad_warm(dski_plan p, dski_precond pc, int k, const float* y, int t, uint64_t seed,
                              double tol, int max_iter, const double* x0, double* alpha_out, double* mll_host,
                              double* grad_host, double* logdet_host, int* iters_host, dski_stream stream) {
  return mll_user<float>(p, pc, k, y, t, seed, tol, max_iter, mll_host, grad_host, logdet_host, iters_host,
                         static_cast<hipStream_t>(stream), x0, alpha_out);
}

dski_status mll_and_grad_f64(dski_plan p, dski_precond pc, int k, const double* y, int t, uint64_t seed,
                             double tol, int max_iter, double* mll_host, double* grad_host,
                             double* logdet_host, int* iters_host, dski_stream stream) {
  return mll_user<double>(p, pc, k, y, t, seed, tol, max_iter, mll_host, grad_host, logdet_host,
                          iters_host, static_cast<hipStream_t>(stream));
}

}  // extern "C"
