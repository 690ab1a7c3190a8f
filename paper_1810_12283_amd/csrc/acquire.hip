// Expected-improvement acquisition over a candidate set (Sec. 4.4, Alg. 1: the
// next sample maximises EI built from the posterior mean and variance).  The
// test functions are minimised: with Y ~ N(mu, sigma^2) the posterior of f at a
// candidate, EI = E[max(f_best - xi - Y, 0)]
//    = (f_best - xi - mu) Phi(z) + sigma phi(z),  z = (f_best - xi - mu) / sigma,
// and max(f_best - xi - mu, 0) where sigma = sqrt(max(v, 0)) is zero.  One pass
// computes EI per candidate and per-block (value, index) maxima; the host picks
// the largest over the blocks, the first index on a tie.
#include <cmath>
#include <vector>

#include "internal.h"

namespace dski {

__device__ inline double ei_value(double mu, double v, double f_best, double xi) {
  const double s = sqrt(fmax(v, 0.0));
  const double imp = f_best - xi - mu;
  if (s == 0.0) return fmax(imp, 0.0);
  const double z = imp / s;
  const double Phi = 0.5 * erfc(-z * 0.70710678118654752440);     // 1/sqrt(2)
  const double phi = exp(-0.5 * z * z) * 0.39894228040143267794;   // 1/sqrt(2 pi)
  return imp * Phi + s * phi;
}

__global__ __launch_bounds__(256) void k_ei(int nc, const double* __restrict__ mu, int mu_stride,
                                            const double* __restrict__ var, double f_best, double xi,
                                            double* __restrict__ ei, double* __restrict__ bval,
                                            int* __restrict__ bidx) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int j = blockIdx.x * 256 + threadIdx.x;
  double e = -1.0;  // below any EI (EI >= 0)
  if (j < nc) {
    e = ei_value(mu[(size_t)j * mu_stride], var[j], f_best, xi);
    if (ei) ei[j] = e;
    // a NaN would absorb every partner it meets in the tree below and an
    // infinite EI would win it: neither may be chosen
    if (!isfinite(e)) e = -1.0;
  }
  sv[threadIdx.x] = e;
  si[threadIdx.x] = j;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + h];
      // larger value wins; on equal values the lower index
      if (b > a || (b == a && si[threadIdx.x + h] < si[threadIdx.x])) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = si[threadIdx.x + h];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bval[blockIdx.x] = sv[0];
    bidx[blockIdx.x] = si[0];
  }
}

}  // namespace dski

using namespace dski;

extern "C" dski_status dski_expected_improvement(int n_cand, const double* mu, int mu_stride, const double* var,
                                                 double f_best, double xi, double* ei, int* best_idx_host,
                                                 double* best_ei_host, dski_stream stream) {
  if (n_cand < 1 || !mu || !var || mu_stride < 1 || !best_idx_host || !best_ei_host || !std::isfinite(f_best) ||
      !(xi >= 0.0)) {
    set_error("dski_expected_improvement: bad arguments");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb = (n_cand + 255) / 256;
  DevBuf blk;
  DSKI_TRY(blk.reserve((sizeof(double) + sizeof(int)) * (size_t)nb + 64));
  double* bval = blk.as<double>();
  int* bidx = reinterpret_cast<int*>(bval + nb);
  k_ei<<<nb, 256, 0, st>>>(n_cand, mu, mu_stride, var, f_best, xi, ei, bval, bidx);
  std::vector<double> hv(nb);
  std::vector<int> hi(nb);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hv.data(), bval, sizeof(double) * nb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hi.data(), bidx, sizeof(int) * nb, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  blk.release();
  if (e != hipSuccess) {
    set_error("dski_expected_improvement: %s", hipGetErrorString(e));
    return DSKI_EHIP;
  }
  int b = 0;
  for (int k = 1; k < nb; ++k)
    if (hv[k] > hv[b]) b = k;
  if (!(hv[b] >= 0.0)) {
    set_error("dski_expected_improvement: no candidate has a finite mean and variance");
    return DSKI_EINVAL;
  }
  *best_idx_host = hi[b];
  *best_ei_host = hv[b];
  return DSKI_OK;
}
