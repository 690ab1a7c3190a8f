// Posterior mean at test points (Sec. 1: O(1) prediction per test point).
// With alpha = K~^{-1} y the posterior mean of the test observations
// [f(x*); grad f(x*)] is K_{*X} alpha, and under D-SKI (Sec. 3.1)
// K_{*X} = S_* K_UU S^T: the grid vector g = K_UU S^T alpha is formed once (one
// scatter and the K_UU factors, as in the MVM) and every test point then
// interpolates g on its cubic stencil, value and d derivative weights, with
// 4^d grid reads whatever the number of training points.
#include "internal.h"

namespace dski {

struct PredGeo {
  int m[DSKI_MAXD];
  double lo[DSKI_MAXD], h[DSKI_MAXD], ih[DSKI_MAXD];
};

// One thread per test point: cell and offset as for the training points (a
// point outside the interpolation box sets err), then the stencil sums in
// FP64; out row u = [mean f, mean d f / d x_1 .. d x_D].
template <int D>
__global__ __launch_bounds__(256) void k_predict(const double* __restrict__ g, PredGeo geo, int ns,
                                                 const double* __restrict__ Xs, double* __restrict__ out,
                                                 int* __restrict__ err) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= ns) return;
  double w[D][4], dw[D][4];
  long long c0[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s = (Xs[(size_t)u * D + a] - geo.lo[a]) / geo.h[a];
    if (!(s >= 1.0 - 1e-9 && s <= (double)(geo.m[a] - 2) + 1e-9)) {
      atomicOr(err, 1);
      s = fmin(fmax(s, 1.0), (double)(geo.m[a] - 2));
    }
    int i = (int)floor(s);
    i = i < 1 ? 1 : (i > geo.m[a] - 3 ? geo.m[a] - 3 : i);
    const double t = fmin(fmax(s - (double)i, 0.0), 1.0);
    keys_weights(t, geo.ih[a], w[a], dw[a]);
    c0[a] = i - 1;
  }
  double acc[D + 1];
#pragma unroll
  for (int q = 0; q <= D; ++q) acc[q] = 0.0;
  constexpr int NS = D == 1 ? 4 : (D == 2 ? 16 : 64);
  for (int e = 0; e < NS; ++e) {
    int o[D];
    int rem = e;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      o[a] = rem & 3;
      rem >>= 2;
    }
    long long node = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) node = node * geo.m[a] + c0[a] + o[a];
    const double gv = g[node];
    double wp = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) wp *= w[a][o[a]];
    acc[0] += wp * gv;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      double dq = dw[q][o[q]];
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (a != q) dq *= w[a][o[a]];
      acc[1 + q] += dq * gv;
    }
  }
#pragma unroll
  for (int q = 0; q <= D; ++q) out[(size_t)u * (D + 1) + q] = acc[q];
}

}  // namespace dski

using namespace dski;

extern "C" dski_status dski_predict_grid(dski_plan p, const double* alpha, double* g, dski_stream stream) {
  if (!p || !alpha || !g) {
    set_error("dski_predict_grid: bad arguments");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("dski_predict_grid: D-SKI plans only");
    return DSKI_ENOTSUP;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = p->N;
  // alpha into tile order (the plan's point order), then g = K_UU S^T alpha
  DSKI_TRY(p->vout.reserve(sizeof(double) * (size_t)std::max(N, 1) + 64));
  double* at = p->vout.as<double>();
  DSKI_TRY(permute(p, +1, 1, alpha, N, at, N, st));
  DSKI_TRY(scatter<double>(p, 1, at, N, g, st));
  DSKI_TRY(apply_kuu(p, 1, g, st));
  return DSKI_OK;
}

extern "C" dski_status dski_predict(dski_plan p, const double* g, int n_test, const double* X_test, double* out,
                                    dski_stream stream) {
  if (!p || n_test < 0 || (n_test > 0 && (!g || !X_test || !out))) {
    set_error("dski_predict: bad arguments");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("dski_predict: D-SKI plans only");
    return DSKI_ENOTSUP;
  }
  if (n_test == 0) return DSKI_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  PredGeo geo{};
  for (int a = 0; a < p->d; ++a) {
    geo.m[a] = p->ax[a].m;
    geo.lo[a] = p->ax[a].lo;
    geo.h[a] = p->ax[a].h;
    geo.ih[a] = 1.0 / p->ax[a].h;
  }
  DSKI_TRY(p->vout.reserve(sizeof(int) + 64));  // the plan's scratch: the out-of-box flag
  int* err = p->vout.as<int>();
  DSKI_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
  const unsigned nb = (unsigned)((n_test + 255) / 256);
  switch (p->d) {
    case 1: k_predict<1><<<nb, 256, 0, st>>>(g, geo, n_test, X_test, out, err); break;
    case 2: k_predict<2><<<nb, 256, 0, st>>>(g, geo, n_test, X_test, out, err); break;
    case 3: k_predict<3><<<nb, 256, 0, st>>>(g, geo, n_test, X_test, out, err); break;
    default: set_error("d=%d not supported", p->d); return DSKI_ENOTSUP;
  }
  DSKI_HIP(hipGetLastError());
  int herr = 0;
  DSKI_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  if (herr) {
    set_error("dski_predict: a test point lies outside the interpolation box (or is not finite)");
    return DSKI_EINVAL;
  }
  return DSKI_OK;
}
