// Posterior mean at test points (Sec. 1: O(1) prediction per test point).
// With alpha = K~^{-1} y the posterior mean of the test observations
// [f(x*); grad f(x*)] is K_{*X} alpha, and under D-SKI (Sec. 3.1)
// K_{*X} = S_* K_UU S^T: the grid vector g = K_UU S^T alpha is formed once (one
// scatter and the K_UU factors, as in the MVM) and every test point then
// interpolates g on its cubic stencil, value and d derivative weights, with
// 4^d grid reads whatever the number of training points.
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "interp.h"
#include "tskinny.h"

namespace dski {

// Calls f(D, S) with the plan's dimension and stencil width as integral
// constants (d = 1..3 is checked by the callers' plans).
template <int V>
using IC = std::integral_constant<int, V>;
template <typename F>
static void with_ds(dski_plan p, F&& f) {
  const bool q = p->S == kInterpQuintic;
  switch (p->d) {
    case 1: q ? f(IC<1>{}, IC<kInterpQuintic>{}) : f(IC<1>{}, IC<kInterpCubic>{}); break;
    case 2: q ? f(IC<2>{}, IC<kInterpQuintic>{}) : f(IC<2>{}, IC<kInterpCubic>{}); break;
    default: q ? f(IC<3>{}, IC<kInterpQuintic>{}) : f(IC<3>{}, IC<kInterpCubic>{}); break;
  }
}

struct PredGeo {
  int m[DSKI_MAXD];
  double lo[DSKI_MAXD], h[DSKI_MAXD], ih[DSKI_MAXD];
};

// Stencil of test point u (S nodes per axis, H = S/2 - 1 below the anchor):
// value and derivative weights per axis and the first stencil node; a point
// outside the interpolation box (or not finite) sets err and is clamped into it.
template <int D, int S>
__device__ inline void pred_stencil(const double* __restrict__ Xs, int u, const PredGeo& geo,
                                    double (&w)[D][S], double (&dw)[D][S], long long (&c0)[D],
                                    int* __restrict__ err) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    constexpr int H = S / 2 - 1;
    const double smin = (double)H, smax = (double)(geo.m[a] - S + H + 1);
    double s = (Xs[(size_t)u * D + a] - geo.lo[a]) / geo.h[a];
    if (!(s >= smin - 1e-9 && s <= smax + 1e-9)) {
      atomicOr(err, 1);
      s = fmin(fmax(s, smin), smax);
    }
    int i = (int)floor(s);
    const int imax = geo.m[a] - S + H;
    i = i < H ? H : (i > imax ? imax : i);
    const double t = fmin(fmax(s - (double)i, 0.0), 1.0);
    interp_weights<S>(t, geo.ih[a], w[a], dw[a]);
    c0[a] = i - H;
  }
}

// Grid node and value weight of stencil entry e (axis offsets in base S, the
// last axis fastest).
template <int D, int S>
__device__ inline long long stencil_node(int e, const PredGeo& geo, const double (&w)[D][S],
                                         const long long (&c0)[D], int (&o)[D], double& wp) {
  int rem = e;
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    o[a] = rem % S;
    rem /= S;
  }
  long long node = 0;
  wp = 1.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    node = node * geo.m[a] + c0[a] + o[a];
    wp *= w[a][o[a]];
  }
  return node;
}

// One thread per test point: the stencil sums in FP64; out row u =
// [mean f, mean d f / d x_1 .. d x_D].
template <int D, int S>
__global__ __launch_bounds__(256) void k_predict(const double* __restrict__ g, PredGeo geo, int ns,
                                                 const double* __restrict__ Xs, double* __restrict__ out,
                                                 int* __restrict__ err) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= ns) return;
  double w[D][S], dw[D][S];
  long long c0[D];
  pred_stencil<D, S>(Xs, u, geo, w, dw, c0, err);
  double acc[D + 1];
#pragma unroll
  for (int q = 0; q <= D; ++q) acc[q] = 0.0;
  constexpr int NS = D == 1 ? S : (D == 2 ? S * S : S * S * S);
  for (int e = 0; e < NS; ++e) {
    int o[D];
    double wp;
    const long long node = stencil_node<D, S>(e, geo, w, c0, o, wp);
    const double gv = g[node];
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

// Predictive variance (Sec. 4.4, first approach) of f at a batch of test
// points, one grid column per point.  k_var_fill writes the value stencil w_x
// of point r0 + j into column j of G (zeroed before); k_var_kxx reads the same
// stencil against K_UU w_x to give k(x, x) = w_x^T K_UU w_x; k_var_sqnorm
// forms per-block partials of ||D^{-1/2} K_{Xx}||^2 (kVarSplit blocks per
// column); k_var_final subtracts K_{xX} M^{-1} K_{Xx} = that norm - kq, kq the
// preconditioner's low-rank term.
template <int D, int S>
__global__ __launch_bounds__(256) void k_var_fill(PredGeo geo, int r0, int nb_pts, const double* __restrict__ Xs,
                                                  double* __restrict__ G, long long M, int* __restrict__ err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb_pts) return;
  double w[D][S], dw[D][S];
  long long c0[D];
  pred_stencil<D, S>(Xs, r0 + j, geo, w, dw, c0, err);
  constexpr int NS = D == 1 ? S : (D == 2 ? S * S : S * S * S);
  for (int e = 0; e < NS; ++e) {
    int o[D];
    double wp;
    const long long node = stencil_node<D, S>(e, geo, w, c0, o, wp);
    G[(size_t)j * M + node] = wp;
  }
}

template <int D, int S>
__global__ __launch_bounds__(256) void k_var_kxx(PredGeo geo, int r0, int nb_pts, const double* __restrict__ Xs,
                                                 const double* __restrict__ G, long long M,
                                                 double* __restrict__ kxx, int* __restrict__ err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb_pts) return;
  double w[D][S], dw[D][S];
  long long c0[D];
  pred_stencil<D, S>(Xs, r0 + j, geo, w, dw, c0, err);
  constexpr int NS = D == 1 ? S : (D == 2 ? S * S : S * S * S);
  double acc = 0.0;
  for (int e = 0; e < NS; ++e) {
    int o[D];
    double wp;
    const long long node = stencil_node<D, S>(e, geo, w, c0, o, wp);
    acc += wp * G[(size_t)j * M + node];
  }
  kxx[j] = acc;
}

constexpr int kVarSplit = 8;

// grid (kVarSplit, columns): block (b, j) sums (D^{-1/2} Y)_e^2 over rows
// e = b*256 + t + s*kVarSplit*256 of column j (value rows e < n scaled by
// 1/sigma_f^2, gradient rows by 1/sigma_g^2).
__global__ __launch_bounds__(256) void k_var_sqnorm(const double* __restrict__ Y, int N, int n, double iv,
                                                    double ig, double* __restrict__ part) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const double* y = Y + (size_t)j * N;
  double s = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < N; e += kVarSplit * 256) {
    const double v = y[e];
    s += (e < n ? iv : ig) * v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)j * kVarSplit + blockIdx.x] = red[0];
}

// out[j] = k(x, x) - (||D^{-1/2} K_{Xx}||^2 - kq[j]); one thread per point.
__global__ __launch_bounds__(256) void k_var_final(const double* __restrict__ kxx, const double* __restrict__ part,
                                                   const double* __restrict__ kq, int b,
                                                   double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= b) return;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kVarSplit; ++q) s += part[(size_t)j * kVarSplit + q];
  out[j] = kxx[j] - (s - kq[j]);
}

// Randomized variance (Sec. 4.4, second approach), per chunk of probes.
// k_probe_scatter: grid column r receives sum_j z_{r0+r, j} w_{x_j} (test-point
// value stencils weighted by the probe; FP64 atomic adds, as stencils overlap).
template <int D, int S>
__global__ __launch_bounds__(256) void k_probe_scatter(PredGeo geo, int ns, const double* __restrict__ Xs,
                                                       const double* __restrict__ Zp, int r0,
                                                       double* __restrict__ G, long long M, int* __restrict__ err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (j >= ns) return;
  double w[D][S], dw[D][S];
  long long c0[D];
  pred_stencil<D, S>(Xs, j, geo, w, dw, c0, err);
  const double z = Zp[(size_t)(r0 + r) * ns + j];
  constexpr int NS = D == 1 ? S : (D == 2 ? S * S : S * S * S);
  for (int e = 0; e < NS; ++e) {
    int o[D];
    double wp;
    const long long node = stencil_node<D, S>(e, geo, w, c0, o, wp);
    atomicAdd(&G[(size_t)r * M + node], z * wp);
  }
}

// acc[j] += sum_r z_{r0+r, j} w_{x_j}^T G_r over the rc columns of the chunk.
template <int D, int S>
__global__ __launch_bounds__(256) void k_probe_read(PredGeo geo, int ns, const double* __restrict__ Xs,
                                                    const double* __restrict__ Zp, int r0, int rc,
                                                    const double* __restrict__ G, long long M,
                                                    double* __restrict__ acc, int* __restrict__ err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ns) return;
  double w[D][S], dw[D][S];
  long long c0[D];
  pred_stencil<D, S>(Xs, j, geo, w, dw, c0, err);
  constexpr int NS = D == 1 ? S : (D == 2 ? S * S : S * S * S);
  double a = acc[j];
  for (int r = 0; r < rc; ++r) {
    double e_r = 0.0;
    for (int e = 0; e < NS; ++e) {
      int o[D];
      double wp;
      const long long node = stencil_node<D, S>(e, geo, w, c0, o, wp);
      e_r += wp * G[(size_t)r * M + node];
    }
    a += Zp[(size_t)(r0 + r) * ns + j] * e_r;
  }
  acc[j] = a;
}

__global__ __launch_bounds__(256) void k_sub_inplace(double* __restrict__ a, const double* __restrict__ b,
                                                     size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    a[e] -= b[e];
}

__global__ __launch_bounds__(256) void k_probe_final(const double* __restrict__ acc, int ns, double inv_r,
                                                     double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < ns) out[j] -= inv_r * acc[j];
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
  DSKI_TRY((scatter<double, double>)(p, 1, at, N, g, st));
  DSKI_TRY(apply_kuu<double>(p, 1, g, st));
  return DSKI_OK;
}

static PredGeo pred_geo(dski_plan p) {
  PredGeo geo{};
  for (int a = 0; a < p->d; ++a) {
    geo.m[a] = p->ax[a].m;
    geo.lo[a] = p->ax[a].lo;
    geo.h[a] = p->ax[a].h;
    geo.ih[a] = 1.0 / p->ax[a].h;
  }
  return geo;
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
  const PredGeo geo = pred_geo(p);
  DSKI_TRY(p->vout.reserve(sizeof(int) + 64));  // the plan's scratch: the out-of-box flag
  int* err = p->vout.as<int>();
  DSKI_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
  const unsigned nb = (unsigned)((n_test + 255) / 256);
  with_ds(p, [&](auto Dc, auto Sc) {
    constexpr int D_ = decltype(Dc)::value, S_ = decltype(Sc)::value;
    k_predict<D_, S_><<<nb, 256, 0, st>>>(g, geo, n_test, X_test, out, err);
  });
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

extern "C" dski_status dski_predict_var(dski_plan p, dski_precond pc, int n_test, const double* X_test,
                                        double* out, dski_stream stream) {
  if (!p || !pc || pc->plan != p || n_test < 0 || (n_test > 0 && (!X_test || !out))) {
    set_error("dski_predict_var: bad arguments");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("dski_predict_var: D-SKI plans only");
    return DSKI_ENOTSUP;
  }
  if (n_test == 0) return DSKI_OK;
  if (p->d < 1 || p->d > 3) {
    set_error("d=%d not supported", p->d);
    return DSKI_ENOTSUP;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PredGeo geo = pred_geo(p);
  const long long M = p->M;
  const int N = p->N;
  // test points per batch: up to 128, with the grid columns and the two
  // N-vectors of a batch within 2 GiB
  const size_t per_pt = sizeof(double) * ((size_t)M + 2 * (size_t)N);
  const int B = (int)std::max<size_t>(1, std::min<size_t>({(size_t)128, (size_t)n_test, ((size_t)2 << 30) / per_pt}));
  DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)M * B));
  DSKI_TRY(p->vin.reserve(sizeof(double) * 2 * (size_t)N * B + 64));
  DSKI_TRY(p->vout.reserve(sizeof(double) * 2 * (size_t)B + 64));
  DSKI_TRY(p->partial.reserve(sizeof(double) * (size_t)kVarSplit * B + 64));
  DSKI_TRY(p->scal.reserve(sizeof(int) + 64));
  double* G = p->grid.as<double>();
  double* Y = p->vin.as<double>();          // K_{Xx}, N x B (tile order)
  double* Z = Y + (size_t)N * B;            // zeros: the gather's noise input (noise weights 0)
  double* kxx = p->vout.as<double>();
  double* kq = kxx + B;
  double* part = p->partial.as<double>();
  int* err = p->scal.as<int>();
  DSKI_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
  DSKI_HIP(hipMemsetAsync(Z, 0, sizeof(double) * (size_t)N * B, st));
  for (int r0 = 0; r0 < n_test; r0 += B) {
    const int b = std::min(B, n_test - r0);
    const unsigned gb = (unsigned)((b + 255) / 256);
    DSKI_HIP(hipMemsetAsync(G, 0, sizeof(double) * (size_t)M * b, st));
    with_ds(p, [&](auto Dc, auto Sc) {
      constexpr int D_ = decltype(Dc)::value, S_ = decltype(Sc)::value;
      k_var_fill<D_, S_><<<gb, 256, 0, st>>>(geo, r0, b, X_test, G, M, err);
    });
    DSKI_HIP(hipGetLastError());
    DSKI_TRY(apply_kuu<double>(p, b, G, st));  // G = K_UU w_x
    with_ds(p, [&](auto Dc, auto Sc) {
      constexpr int D_ = decltype(Dc)::value, S_ = decltype(Sc)::value;
      k_var_kxx<D_, S_><<<gb, 256, 0, st>>>(geo, r0, b, X_test, G, M, kxx, err);
    });
    DSKI_HIP(hipGetLastError());
    DSKI_TRY((gather<double, double>)(p, b, G, Z, N, Y, N, 0.0, 0.0, nullptr, st));  // Y = S K_UU w_x
    // K_{xX} M^{-1} K_{Xx} = ||D^{-1/2} K_{Xx}||^2 - kq: the norm here, kq from
    // the preconditioner's projection, one tall-skinny launch of columns at a time
    k_var_sqnorm<<<dim3(kVarSplit, (unsigned)b), 256, 0, st>>>(Y, N, p->n, 1.0 / (p->sf * p->sf),
                                                                1.0 / (p->sg * p->sg), part);
    DSKI_HIP(hipGetLastError());
    for (int c0 = 0; c0 < b; c0 += kFinalMaxR)
      DSKI_TRY(precond_lowrank_quad(pc, std::min(kFinalMaxR, b - c0), Y + (size_t)c0 * N, N, kq + c0, st));
    k_var_final<<<gb, 256, 0, st>>>(kxx, part, kq, b, out + r0);
    DSKI_HIP(hipGetLastError());
  }
  int herr = 0;
  DSKI_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  if (herr) {
    set_error("dski_predict_var: a test point lies outside the interpolation box (or is not finite)");
    return DSKI_EINVAL;
  }
  return DSKI_OK;
}

namespace {
struct ScopedBuf {
  dski::DevBuf b;
  ~ScopedBuf() { b.release(); }
};
}  // namespace

extern "C" dski_status dski_predict_var_probes(dski_plan p, dski_precond pc, int n_test, const double* X_test,
                                               int R, const double* Zp, double tol, int max_iter, double* out,
                                               dski_stream stream) {
  if (!p || !pc || pc->plan != p || n_test < 0 || R < 1 || !(tol > 0.0) || max_iter < 1 ||
      (n_test > 0 && (!X_test || !Zp || !out))) {
    set_error("dski_predict_var_probes: bad arguments");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("dski_predict_var_probes: D-SKI plans only");
    return DSKI_ENOTSUP;
  }
  if (n_test == 0) return DSKI_OK;
  // the control variate v^ (also rejects points outside the box)
  DSKI_TRY(dski_predict_var(p, pc, n_test, X_test, out, stream));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PredGeo geo = pred_geo(p);
  const long long M = p->M;
  const int N = p->N;
  const int C = std::min(R, kFinalMaxR);  // probes per chunk
  ScopedBuf wb;
  DSKI_TRY(wb.b.reserve(sizeof(double) * (3 * (size_t)N * C + (size_t)n_test) + 256));
  double* Y = wb.b.as<double>();         // K_{XX'} z, N x C (tile order)
  double* U1 = Y + (size_t)N * C;        // K~^{-1} K_{XX'} z, then minus M^{-1} K_{XX'} z
  double* U2 = U1 + (size_t)N * C;       // zeros (the gather's noise input), then M^{-1} K_{XX'} z
  double* acc = U2 + (size_t)N * C;
  int* err = reinterpret_cast<int*>(acc + n_test);
  DSKI_HIP(hipMemsetAsync(acc, 0, sizeof(double) * (size_t)n_test + sizeof(int), st));
  dski_status status = DSKI_OK;
  const unsigned gb = (unsigned)((n_test + 255) / 256);
  for (int r0 = 0; r0 < R; r0 += C) {
    const int rc = std::min(C, R - r0);
    DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)M * rc));
    double* G = p->grid.as<double>();
    DSKI_HIP(hipMemsetAsync(G, 0, sizeof(double) * (size_t)M * rc, st));
    DSKI_HIP(hipMemsetAsync(U2, 0, sizeof(double) * (size_t)N * rc, st));
    with_ds(p, [&](auto Dc, auto Sc) {
      constexpr int D_ = decltype(Dc)::value, S_ = decltype(Sc)::value;
      k_probe_scatter<D_, S_><<<dim3(gb, rc), 256, 0, st>>>(geo, n_test, X_test, Zp, r0, G, M, err);
    });
    DSKI_HIP(hipGetLastError());
    DSKI_TRY(apply_kuu<double>(p, rc, G, st));
    DSKI_TRY((gather<double, double>)(p, rc, G, U2, N, Y, N, 0.0, 0.0, nullptr, st));  // Y = K_{XX'} z
    PcgResult res;
    std::vector<double> tols(rc, tol);
    std::vector<int> verify(rc, 1);
    const dski_status pr = pcg_tiled<double>(p, pc, rc, Y, N, U1, N, tols.data(), max_iter, 0, nullptr, res, st,
                                             nullptr, verify.data());
    if (pr < 0) return pr;
    if (pr == DSKI_NOT_CONVERGED) status = DSKI_NOT_CONVERGED;
    DSKI_TRY(precond_apply_tiled<double>(pc, rc, Y, N, U2, N, nullptr, nullptr, st));
    k_sub_inplace<<<1024, 256, 0, st>>>(U1, U2, (size_t)N * rc);
    DSKI_HIP(hipGetLastError());
    DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)M * rc));  // the solver's products may have resized it
    G = p->grid.as<double>();
    DSKI_TRY((scatter<double, double>)(p, rc, U1, N, G, st));
    DSKI_TRY(apply_kuu<double>(p, rc, G, st));
    with_ds(p, [&](auto Dc, auto Sc) {
      constexpr int D_ = decltype(Dc)::value, S_ = decltype(Sc)::value;
      k_probe_read<D_, S_><<<gb, 256, 0, st>>>(geo, n_test, X_test, Zp, r0, rc, G, M, acc, err);
    });
    DSKI_HIP(hipGetLastError());
  }
  k_probe_final<<<gb, 256, 0, st>>>(acc, n_test, 1.0 / R, out);
  DSKI_HIP(hipGetLastError());
  DSKI_HIP(hipStreamSynchronize(st));
  return status;
}
