// Active-subspace dimension reduction (Sec. 3.4).  The active subspace of
// f: R^D -> R is spanned by the dominant eigenvectors of C = int grad f grad f^T,
// estimated by Monte Carlo as the mean of g_i g_i^T over the n gradient samples;
// with P (D x d, orthonormal columns) the GP uses k(P^T x, P^T x'), i.e. the
// reduced points u_i = P^T x_i with gradients P^T g_i.
//
// C is an n-long reduction of D x D products: one pass over the gradients on the
// GPU (per-block partials of the upper triangle, rows staged through LDS), the
// partials summed on the host in block order (deterministic), and a cyclic
// Jacobi eigen-decomposition of the small symmetric matrix on the host.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace dski {

constexpr int kActMaxD = 64;                                     // ambient dimension limit
constexpr int kActPairs = kActMaxD * (kActMaxD + 1) / 2;         // upper-triangle entries
constexpr int kActRows = 32;                                     // gradient rows per LDS tile
constexpr int kActPerThread = (kActPairs + 255) / 256;

// Block b sums g_i[p] g_i[q] (p <= q) over the rows [b*chunk, (b+1)*chunk);
// gradient component p of sample i is at G[p*ldg + i].  Pair t + 256 s of the
// upper triangle (row-major order) belongs to thread t.
__global__ __launch_bounds__(256) void k_grad_cov_part(const double* __restrict__ G, int ldg, int n, int D,
                                                       int chunk, double* __restrict__ part) {
  __shared__ double T[kActRows][kActMaxD + 1];
  __shared__ unsigned short pp[kActPairs];
  const int npairs = D * (D + 1) / 2;
  for (int q = threadIdx.x; q < npairs; q += 256) {
    int p = 0, rem = q;
    while (rem >= D - p) {
      rem -= D - p;
      ++p;
    }
    pp[q] = (unsigned short)(p | ((p + rem) << 8));
  }
  double acc[kActPerThread];
#pragma unroll
  for (int s = 0; s < kActPerThread; ++s) acc[s] = 0.0;
  const int i_lo = blockIdx.x * chunk, i_hi = min(n, i_lo + chunk);
  for (int i0 = i_lo; i0 < i_hi; i0 += kActRows) {
    __syncthreads();
    for (int e = threadIdx.x; e < kActRows * D; e += 256) {
      const int p = e / kActRows, r = e % kActRows, i = i0 + r;
      T[r][p] = i < i_hi ? G[(size_t)p * ldg + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kActPerThread; ++s) {
      const int q = threadIdx.x + 256 * s;
      if (q < npairs) {
        const int p1 = pp[q] & 0xff, p2 = pp[q] >> 8;
        double a = 0.0;
#pragma unroll 8
        for (int r = 0; r < kActRows; ++r) a += T[r][p1] * T[r][p2];
        acc[s] += a;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kActPerThread; ++s) {
    const int q = threadIdx.x + 256 * s;
    if (q < npairs) part[(size_t)blockIdx.x * npairs + q] = acc[s];
  }
}

// One thread per sample: U[i, :] = x_i^T P (row-major n x d) and
// Gu[j*n + i] = g_i^T P[:, j] (d blocks of n, as the derivative blocks of an
// N-vector).
__global__ __launch_bounds__(256) void k_active_project(int n, int D, int d, const double* __restrict__ X,
                                                        const double* __restrict__ G, int ldg,
                                                        const double* __restrict__ P, double* __restrict__ U,
                                                        double* __restrict__ Gu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < d; ++j) {
    double u = 0.0, g = 0.0;
    for (int p = 0; p < D; ++p) {
      const double w = P[(size_t)p * d + j];
      u += X[(size_t)i * D + p] * w;
      if (G) g += G[(size_t)p * ldg + i] * w;
    }
    U[(size_t)i * d + j] = u;
    if (Gu) Gu[(size_t)j * n + i] = g;
  }
}

// Cyclic Jacobi eigen-decomposition of the symmetric D x D matrix A (row-major,
// overwritten): rotations zero each off-diagonal entry in turn until the
// off-diagonal mass is below 1e-30 of the total.  V receives the eigenvectors
// as columns, lam the eigenvalues (unsorted).
static void jacobi_eig(int D, std::vector<double>& A, std::vector<double>& V, std::vector<double>& lam) {
  V.assign((size_t)D * D, 0.0);
  for (int i = 0; i < D; ++i) V[(size_t)i * D + i] = 1.0;
  double tot = 0.0;
  for (double a : A) tot += a * a;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) off += 2.0 * A[(size_t)p * D + q] * A[(size_t)p * D + q];
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) {
        const double apq = A[(size_t)p * D + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * D + p], aqq = A[(size_t)q * D + q];
        // rotation angle from tan(2 theta) = 2 apq / (aqq - app), smaller root
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < D; ++k) {  // columns p, q
          const double akp = A[(size_t)k * D + p], akq = A[(size_t)k * D + q];
          A[(size_t)k * D + p] = c * akp - s * akq;
          A[(size_t)k * D + q] = s * akp + c * akq;
        }
        for (int k = 0; k < D; ++k) {  // rows p, q
          const double apk = A[(size_t)p * D + k], aqk = A[(size_t)q * D + k];
          A[(size_t)p * D + k] = c * apk - s * aqk;
          A[(size_t)q * D + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < D; ++k) {
          const double vkp = V[(size_t)k * D + p], vkq = V[(size_t)k * D + q];
          V[(size_t)k * D + p] = c * vkp - s * vkq;
          V[(size_t)k * D + q] = s * vkp + c * vkq;
        }
      }
  }
  lam.resize(D);
  for (int i = 0; i < D; ++i) lam[i] = A[(size_t)i * D + i];
}

}  // namespace dski

using namespace dski;

extern "C" dski_status dski_active_subspace(int n, int D, const double* G, int ldg, int d, double* P_host,
                                            double* eig_host, dski_stream stream) {
  if (n < 1 || D < 1 || d < 1 || d > D || !G || ldg < n || !P_host || !eig_host) {
    set_error("dski_active_subspace: bad arguments");
    return DSKI_EINVAL;
  }
  if (D > kActMaxD) {
    set_error("dski_active_subspace: D=%d above the limit %d", D, kActMaxD);
    return DSKI_ENOTSUP;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int npairs = D * (D + 1) / 2;
  const int nb = std::max(1, std::min(512, (n + 255) / 256));
  const int chunk = ((n + nb - 1) / nb + kActRows - 1) / kActRows * kActRows;
  const int nblk = (n + chunk - 1) / chunk;
  DevBuf part;
  dski_status rc = part.reserve(sizeof(double) * (size_t)nblk * npairs);
  if (rc != DSKI_OK) return rc;
  std::vector<double> hp((size_t)nblk * npairs);
  k_grad_cov_part<<<nblk, 256, 0, st>>>(G, ldg, n, D, chunk, part.as<double>());
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part.p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  part.release();
  if (e != hipSuccess) {
    set_error("dski_active_subspace: %s", hipGetErrorString(e));
    return DSKI_EHIP;
  }
  std::vector<double> A((size_t)D * D, 0.0);
  for (int q = 0, p1 = 0, p2 = 0; q < npairs; ++q) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += hp[(size_t)b * npairs + q];
    s /= n;
    A[(size_t)p1 * D + p2] = s;
    A[(size_t)p2 * D + p1] = s;
    if (++p2 == D) p2 = ++p1;
  }
  std::vector<double> V, lam;
  jacobi_eig(D, A, V, lam);
  std::vector<int> order(D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
  for (int j = 0; j < D; ++j) eig_host[j] = lam[order[j]];
  for (int j = 0; j < d; ++j) {
    const int c = order[j];
    // sign: the entry of largest magnitude positive (lowest index on a tie)
    int im = 0;
    for (int p = 1; p < D; ++p)
      if (std::fabs(V[(size_t)p * D + c]) > std::fabs(V[(size_t)im * D + c])) im = p;
    const double sg = V[(size_t)im * D + c] < 0 ? -1.0 : 1.0;
    for (int p = 0; p < D; ++p) P_host[(size_t)p * d + j] = sg * V[(size_t)p * D + c];
  }
  return DSKI_OK;
}

extern "C" dski_status dski_active_project(int n, int D, int d, const double* X, const double* G, int ldg,
                                           const double* P, double* U, double* Gu, dski_stream stream) {
  if (n < 0 || D < 1 || d < 1 || d > D || (n > 0 && (!X || !P || !U)) || (G && ldg < n) || (!G != !Gu)) {
    set_error("dski_active_project: bad arguments");
    return DSKI_EINVAL;
  }
  if (n == 0) return DSKI_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  k_active_project<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, D, d, X, G, ldg, P, U, Gu);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}
