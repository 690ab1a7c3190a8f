// Truncated pivoted Cholesky of the noise-free D-SKI matrix and the
// preconditioner M = D + L L^T (Sec. 3.3).
//
// Diagonal and rows use the separable form of the D-SKI entries (the D-SKI
// matrix of a product kernel is a Hadamard product of 1-D SKI factors,
// Sec. 3.2):  K[(a,i),(b,j)] = s^2 prod_p  w_p^{(a)}(x_ip)^T T_p w_p^{(b)}(x_jp),
// where w_p^{(a)} are the S value weights (S = 4 cubic, 6 quintic), or
// derivative weights when block a is the derivative along axis p.  A row costs
// O(N d S + sum_p m_p), the diagonal O(N d S^2).
//
// Greedy pivoting on the largest residual diagonal entry, lowest index among
// exact ties; every step runs on the device (no host round trip per pivot).
//
// With G = D^{-1/2} L = U S V^T (Gram matrix of G and its eigen-decomposition),
//   M^{-1} = D^{-1/2} (I - U diag(s^2 / (1 + s^2)) U^T) D^{-1/2}   (Woodbury),
//   C = D^{1/2} (I + U diag(sqrt(1 + s^2) - 1) U^T),  C C^T = M,
//   log det M = sum log D_ii + sum log(1 + s_i^2);
// U is kept in FP64 so that the applied M^{-1} stays symmetric positive definite.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "interp.h"
#include "pivot.h"
#include "tskinny.h"

namespace dski {

struct GeoP {
  int d, n, N;
  int m[DSKI_MAXD];
  int nc[DSKI_MAXD];
  double invh[DSKI_MAXD];
  const double* col[DSKI_MAXD];  // first column of T_p (unscaled)
  double s2;
};

static GeoP geop_of(dski_plan p) {
  GeoP g{};
  g.d = p->d;
  g.n = p->n;
  g.N = p->N;
  for (int a = 0; a < p->d; ++a) {
    g.m[a] = p->ax[a].m;
    g.nc[a] = p->ax[a].ncell;
    g.invh[a] = 1.0 / p->ax[a].h;
    g.col[a] = p->ax[a].col;
  }
  g.s2 = p->s * p->s;
  return g;
}

// First stencil node of every axis of cell id cl.
__device__ __forceinline__ void cell_coords(int cl, const GeoP& g, int c[DSKI_MAXD]) {
  for (int a = g.d - 1; a >= 0; --a) {
    c[a] = cl % g.nc[a];
    cl /= g.nc[a];
  }
}

// diag[e] for e = blk * n + k (tile order)
template <int S>
__global__ void k_pc_diag(GeoP g, const int* __restrict__ cell, const double* __restrict__ toff,
                          double* __restrict__ diag) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.N) return;
  int blk = e / g.n, k = e % g.n;
  double v = g.s2;
  for (int a = 0; a < g.d; ++a) {
    double w[S];
    interp_weights_one<S>((double)toff[(size_t)a * g.n + k], g.invh[a], blk == a + 1, w);
    double q = 0.0;
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) q += w[i] * g.col[a][i > j ? i - j : j - i] * w[j];
    v *= q;
  }
  diag[e] = v;
}

// Block-wise arg-max of the residual diagonal (ties -> lowest index).
__global__ void k_argmax_partial(const double* __restrict__ dres, int N, double* __restrict__ pv,
                                 int* __restrict__ pi) {
  __shared__ double sv[kBlock];
  __shared__ int si[kBlock];
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
    double v = dres[e];
    if (v > best || (v == best && e < bi)) {
      best = v;
      bi = e;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double v = sv[threadIdx.x + off];
      int i = si[threadIdx.x + off];
      if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && i < si[threadIdx.x])) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = i;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

// Final arg-max, stop test, pivot bookkeeping, pivot-row factors a_p and the
// pivot's row of L.  One work-group.
template <int S>
__global__ void k_pivot_select(GeoP g, const double* __restrict__ pv, const int* __restrict__ pi,
                               int nblk, int j, double rel_tol, PivState* __restrict__ ps,
                               int* __restrict__ piv_list, const int* __restrict__ cell,
                               const double* __restrict__ toff, double* __restrict__ arow,
                               const double* __restrict__ L, double* __restrict__ lrow,
                               const int* __restrict__ forced, const double* __restrict__ dres) {
  const int e = pivot_select_block(pv, pi, nblk, j, rel_tol, ps, piv_list, forced, dres);
  if (e < 0) return;
  int blk = e / g.n, k = e % g.n;
  int c[DSKI_MAXD];
  cell_coords(cell[k], g, c);
  // a_p[u] = sum_o T_p[u, c_p + o] w_p^{(blk)}(x_kp)[o], u < m_p (c_p the first stencil node)
  int off = 0;
  for (int a = 0; a < g.d; ++a) {
    double w[S];
    interp_weights_one<S>((double)toff[(size_t)a * g.n + k], g.invh[a], blk == a + 1, w);
    for (int u = threadIdx.x; u < g.m[a]; u += blockDim.x) {
      double acc = 0.0;
      for (int o = 0; o < S; ++o) {
        int v = c[a] + o;
        acc += g.col[a][u > v ? u - v : v - u] * w[o];
      }
      arow[off + u] = acc;
    }
    off += g.m[a];
  }
  for (int l = threadIdx.x; l < j; l += blockDim.x) lrow[l] = L[(size_t)l * g.N + e];
}

// Column j of L and the residual-diagonal update.
template <int S>
__global__ void k_pc_column(GeoP g, int j, const PivState* __restrict__ ps,
                            const int* __restrict__ cell, const double* __restrict__ toff,
                            const double* __restrict__ arow, const double* __restrict__ lrow,
                            double* __restrict__ L, double* __restrict__ dres) {
  if (ps->stop) return;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.N) return;
  int blk = e / g.n, k = e % g.n;
  int c[DSKI_MAXD];
  cell_coords(cell[k], g, c);
  double row = g.s2;
  int off = 0;
  for (int a = 0; a < g.d; ++a) {
    double w[S];
    interp_weights_one<S>((double)toff[(size_t)a * g.n + k], g.invh[a], blk == a + 1, w);
    double q = 0.0;
    for (int o = 0; o < S; ++o) q += w[o] * arow[off + c[a] + o];
    row *= q;
    off += g.m[a];
  }
  double acc = row;
  for (int l = 0; l < j; ++l) acc -= L[(size_t)l * g.N + e] * lrow[l];
  double lj = acc / sqrt(ps->dpiv);
  L[(size_t)j * g.N + e] = lj;
  double dn = dres[e] - lj * lj;
  if (e == ps->piv) dn = -INFINITY;
  dres[e] = dn;
}

// ---------------------------------------------------------------- spline kernel
// The spline kernel is not separable, so its diagonal and rows come from the
// kernel itself.  Diagonal entry of row (block, point): with the tensor weights
// w_a = prod_p w_p[o_{a,p}] of the point's stencil, sum_{a,b} w_a w_b k(|u_a - u_b|)
// depends only on the node offsets Delta = o_a - o_b, so it is
//   s^2 sum_Delta prod_p ac_p[Delta_p] k(|Delta h|),  ac_p[D] = sum_o w_p[o] w_p[o - D]
// ((2S-1)^d terms).  A row is K e_piv = S K_UU S^T e_piv: the pivot's stencil
// written into a grid column, one K_UU product and one gather.
__device__ __forceinline__ double spline_prof(double r, int d, double R) {
  if (d & 1) return r * r * r - 1.5 * R * r * r + 0.5 * R * R * R;
  const double rl = r > 0.0 ? r * r * log(r) : 0.0;
  return rl - 0.5 * (1.0 + 2.0 * log(R)) * r * r + 0.5 * R * R;
}

struct GeoS {
  int d, n, N;
  int m[DSKI_MAXD], nc[DSKI_MAXD];
  double invh[DSKI_MAXD], h[DSKI_MAXD];
  double s2, R;
};

static GeoS geos_of(dski_plan p) {
  GeoS g{};
  g.d = p->d;
  g.n = p->n;
  g.N = p->N;
  for (int a = 0; a < p->d; ++a) {
    g.m[a] = p->ax[a].m;
    g.nc[a] = p->ax[a].ncell;
    g.invh[a] = 1.0 / p->ax[a].h;
    g.h[a] = p->ax[a].h;
  }
  g.s2 = p->s * p->s;
  g.R = p->spline_R;
  return g;
}

template <int S>
__global__ void k_pc_diag_spline(GeoS g, const double* __restrict__ toff, double* __restrict__ diag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.N) return;
  const int blk = e / g.n, k = e % g.n;
  constexpr int NA = 2 * S - 1;
  double ac[DSKI_MAXD][NA];
  for (int a = 0; a < g.d; ++a) {
    double w[S];
    interp_weights_one<S>(toff[(size_t)a * g.n + k], g.invh[a], blk == a + 1, w);
    for (int dd = 0; dd < NA; ++dd) {
      const int D = dd - (S - 1);
      double acc = 0.0;
      for (int o = 0; o < S; ++o)
        if (o - D >= 0 && o - D < S) acc += w[o] * w[o - D];
      ac[a][dd] = acc;
    }
  }
  int tot = 1;
  for (int a = 0; a < g.d; ++a) tot *= NA;
  double v = 0.0;
  for (int f = 0; f < tot; ++f) {
    int rem = f;
    double prod = 1.0, r2 = 0.0;
    for (int a = g.d - 1; a >= 0; --a) {
      const int dd = rem % NA;
      rem /= NA;
      prod *= ac[a][dd];
      const double x = (double)(dd - (S - 1)) * g.h[a];
      r2 += x * x;
    }
    v += prod * spline_prof(sqrt(r2), g.d, g.R);
  }
  diag[e] = g.s2 * v;
}

__global__ void k_fill_zero_d(double* __restrict__ x, long long len) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// Pivot selection, the pivot's row of L, and its stencil written into the
// (zeroed) grid column G: value weights, or derivative weights on the axis of
// its block.
template <int S>
__global__ void k_pivot_select_spline(GeoS g, const double* __restrict__ pv, const int* __restrict__ pi, int nblk,
                                      int j, double rel_tol, PivState* __restrict__ ps, int* __restrict__ piv_list,
                                      const int* __restrict__ cell, const double* __restrict__ toff,
                                      const double* __restrict__ L, double* __restrict__ lrow,
                                      const int* __restrict__ forced, const double* __restrict__ dres,
                                      double* __restrict__ G) {
  const int e = pivot_select_block(pv, pi, nblk, j, rel_tol, ps, piv_list, forced, dres);
  if (e < 0) return;
  const int blk = e / g.n, k = e % g.n;
  for (int l = threadIdx.x; l < j; l += blockDim.x) lrow[l] = L[(size_t)l * g.N + e];
  int c[DSKI_MAXD];
  int cl = cell[k];
  for (int a = g.d - 1; a >= 0; --a) {
    c[a] = cl % g.nc[a];
    cl /= g.nc[a];
  }
  double w[DSKI_MAXD][S];
  for (int a = 0; a < g.d; ++a)
    interp_weights_one<S>(toff[(size_t)a * g.n + k], g.invh[a], blk == a + 1, w[a]);
  int tot = 1;
  for (int a = 0; a < g.d; ++a) tot *= S;
  for (int f = threadIdx.x; f < tot; f += blockDim.x) {
    int rem = f;
    long long node = 0, stride = 1;
    double wp = 1.0;
    for (int a = g.d - 1; a >= 0; --a) {
      const int o = rem % S;
      rem /= S;
      node += (long long)(c[a] + o) * stride;
      stride *= g.m[a];
      wp *= w[a][o];
    }
    G[node] = wp;
  }
}

// Column j of L from the pivot's row (tile order) and the residual-diagonal update.
__global__ void k_pc_column_row(int N, int j, const PivState* __restrict__ ps, const double* __restrict__ row,
                                const double* __restrict__ lrow, double* __restrict__ L, double* __restrict__ dres) {
  if (ps->stop) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double acc = row[e];
  for (int l = 0; l < j; ++l) acc -= L[(size_t)l * N + e] * lrow[l];
  const double lj = acc / sqrt(ps->dpiv);
  L[(size_t)j * N + e] = lj;
  double dn = dres[e] - lj * lj;
  if (e == ps->piv) dn = -INFINITY;
  dres[e] = dn;
}

// One pivoted-Cholesky step of a spline-kernel plan (after the arg-max partials).
static dski_status spline_pc_step(dski_plan p, int j, const double* pv, const int* pi, int nblk, double rel_tol,
                                  PivState* ps, int* piv_list, double* L, double* lrow, double* dres,
                                  const int* forced, double* G, double* row, const double* zeros, hipStream_t st) {
  GeoS g = geos_of(p);
  const int vb = (p->N + kBlock - 1) / kBlock;
  k_fill_zero_d<<<(unsigned)std::min<long long>(1024, (p->M + kBlock - 1) / kBlock), kBlock, 0, st>>>(G, p->M);
  if (p->S == kInterpQuintic)
    k_pivot_select_spline<kInterpQuintic><<<1, kBlock, 0, st>>>(g, pv, pi, nblk, j, rel_tol, ps, piv_list, p->cell,
                                                                p->toff, L, lrow, forced, dres, G);
  else
    k_pivot_select_spline<kInterpCubic><<<1, kBlock, 0, st>>>(g, pv, pi, nblk, j, rel_tol, ps, piv_list, p->cell,
                                                              p->toff, L, lrow, forced, dres, G);
  DSKI_HIP(hipGetLastError());
  DSKI_TRY(apply_kuu<double>(p, 1, G, st));
  DSKI_TRY((gather<double, double>(p, 1, G, zeros, p->N, row, p->N, 0.0, 0.0, nullptr, st)));
  k_pc_column_row<<<vb, kBlock, 0, st>>>(p->N, j, ps, row, lrow, L, dres);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// Gram partials of G = D^{-1/2} L: pairs (i <= j) over a chunk of rows.
__global__ void k_gram_partial(const double* __restrict__ L, int N, int n, int k, int rows,
                               double isf, double isg, double* __restrict__ partial) {
  extern __shared__ double sG[];  // rows x k
  int r0 = blockIdx.x * rows;
  int rn = min(rows, N - r0);
  for (int f = threadIdx.x; f < rows * k; f += blockDim.x) {
    int i = f / rows, r = f % rows;
    double v = 0.0;
    if (r < rn) {
      int e = r0 + r;
      v = L[(size_t)i * N + e] * (e < n ? isf : isg);
    }
    sG[(size_t)i * rows + r] = v;
  }
  __syncthreads();
  int npair = k * (k + 1) / 2;
  for (int pidx = threadIdx.x; pidx < npair; pidx += blockDim.x) {
    // decode pidx -> (i, j), j >= i
    int i = 0, rem = pidx;
    while (rem >= k - i) {
      rem -= k - i;
      ++i;
    }
    int jj = i + rem;
    double acc = 0.0;
    for (int r = 0; r < rn; ++r) acc += sG[(size_t)i * rows + r] * sG[(size_t)jj * rows + r];
    partial[(size_t)blockIdx.x * npair + pidx] = acc;
  }
}

// U[:, i] = G V[:, i] / sigma_i  (components with sigma_i = 0 are dropped), stored
// column-major (U) and row-major (Ur).
// (Vs holds V with column i divided by sigma_i.)  One thread per row, outputs in
// groups of 16 so that each L entry is read k/16 times.
__global__ void k_make_u(const double* __restrict__ L, int N, int n, int k, double isf, double isg,
                         const double* __restrict__ sV, double* __restrict__ U, double* __restrict__ Ur) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double sc = e < n ? isf : isg;
  for (int i0 = 0; i0 < k; i0 += 16) {
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    for (int l = 0; l < k; ++l) {
      const double lv = L[(size_t)l * N + e];
      const double* vr = sV + (size_t)l * k + i0;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i0 + i < k) acc[i] += lv * vr[i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i0 + i < k) {
        U[(size_t)(i0 + i) * N + e] = acc[i] * sc;
        Ur[(size_t)e * k + i0 + i] = acc[i] * sc;  // row-major copy for the projections
      }
  }
}

// ------------------------------------------------------------------ apply
// M^{-1} = D^{-1/2} (I - U diag(w) U^T) D^{-1/2},  w = s^2 / (1 + s^2)   (Woodbury,
// U with orthonormal columns, kept in FP64 so that the operator stays SPD);
// C = D^{1/2} (I + U diag(sqrt(1 + s^2) - 1) U^T) with C C^T = M.
// Each application is one projection (wavefront partials, fixed order), one
// reduction that forms the coefficients, and one correction pass.

int vec_blocks(int N) { return (N + kBlock - 1) / kBlock; }

struct PcWork {
  double* partial;  // nblk x k x R
  double* t;
  double* coef;
  int nblk;
};

static dski_status pc_work(dski_precond pc, int R, PcWork& w) {
  dski_plan p = pc->plan;
  int k = pc->k;
  w.nblk = proj_waves(p->N);
  size_t np = std::max((size_t)w.nblk * k * R, (size_t)vec_blocks(p->N) * R);
  DSKI_TRY(pc->work.reserve(sizeof(double) * (np + 2 * (size_t)k * R + 64)));
  double* base = pc->work.as<double>();
  w.partial = base;
  w.t = base + np;
  w.coef = w.t + (size_t)k * R;
  return DSKI_OK;
}

template <typename T>
dski_status precond_apply_tiled(dski_precond pc, int R, const T* Rm, int ld, T* Z, int ldz,
                                double* rz_partial, int* nblk_out, hipStream_t st) {
  dski_plan p = pc->plan;
  int k = pc->k, N = p->N;
  double isf = 1.0 / p->sf, isg = 1.0 / p->sg;
  if (nblk_out) *nblk_out = vec_blocks(N);
  if (R <= 0) return DSKI_OK;
  if (R > kFinalMaxR) {  // independent columns: apply in groups
    for (int c0 = 0; c0 < R; c0 += kFinalMaxR) {
      int rc = std::min(kFinalMaxR, R - c0);
      DSKI_TRY(precond_apply_tiled<T>(pc, rc, Rm + (size_t)c0 * ld, ld, Z + (size_t)c0 * ldz, ldz, nullptr,
                                      nullptr, st));
    }
    return DSKI_OK;
  }
  if (k == 0)
    return launch_final<T>(Rm, ld, N, p->n, R, isf, isg, isf, isg, pc->U, 0, nullptr, Z, ldz, rz_partial, st);
  PcWork w;
  DSKI_TRY(pc_work(pc, R, w));
  DSKI_TRY(launch_proj<T>(Rm, ld, N, p->n, R, isf, isg, pc->Ur, k, w.partial, st));
  RedJob j{w.partial, w.nblk, k * R, R, w.t, pc->w, nullptr, 1.0, w.coef, nullptr};
  DSKI_TRY(launch_reduce(j, nullptr, st));
  return launch_final<T>(Rm, ld, N, p->n, R, isf, isg, isf, isg, pc->U, k, w.coef, Z, ldz, rz_partial, st);
}
template dski_status precond_apply_tiled<float>(dski_precond, int, const float*, int, float*, int,
                                                double*, int*, hipStream_t);
template dski_status precond_apply_tiled<double>(dski_precond, int, const double*, int, double*, int,
                                                 double*, int*, hipStream_t);

// kq[c] = sum_i w_i t_ic^2 with t = t(r_c) the projection of one application.
static __global__ void k_pc_lowrank_quad(const double* __restrict__ t, const double* __restrict__ coef, int k,
                                         int R, double* __restrict__ kq) {
  __shared__ double red[64];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) s += t[(size_t)i * R + c] * coef[(size_t)i * R + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) kq[c] = red[0];
}

dski_status precond_lowrank_quad(dski_precond pc, int R, const double* Rm, int ld, double* kq, hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  if (R > kFinalMaxR) {
    set_error("precond_lowrank_quad: at most %d columns", kFinalMaxR);
    return DSKI_EINVAL;
  }
  dski_plan p = pc->plan;
  const int k = pc->k;
  if (k == 0) {
    DSKI_HIP(hipMemsetAsync(kq, 0, sizeof(double) * (size_t)R, st));
    return DSKI_OK;
  }
  PcWork w;
  DSKI_TRY(pc_work(pc, R, w));
  DSKI_TRY(launch_proj<double>(Rm, ld, p->N, p->n, R, 1.0 / p->sf, 1.0 / p->sg, pc->Ur, k, w.partial, st));
  RedJob j{w.partial, w.nblk, k * R, R, w.t, pc->w, nullptr, 1.0, w.coef, nullptr};
  DSKI_TRY(launch_reduce(j, nullptr, st));
  k_pc_lowrank_quad<<<(unsigned)R, 64, 0, st>>>(w.t, w.coef, k, R, kq);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

template <typename T>
dski_status precond_factor_apply_tiled(dski_precond pc, int R, const T* W, int ld, T* Z, int ldz,
                                       hipStream_t st) {
  dski_plan p = pc->plan;
  int k = pc->k, N = p->N;
  if (R <= 0) return DSKI_OK;
  if (R > kFinalMaxR) {
    for (int c0 = 0; c0 < R; c0 += kFinalMaxR) {
      int rc = std::min(kFinalMaxR, R - c0);
      DSKI_TRY(precond_factor_apply_tiled<T>(pc, rc, W + (size_t)c0 * ld, ld, Z + (size_t)c0 * ldz, ldz, st));
    }
    return DSKI_OK;
  }
  if (k == 0)
    return launch_final<T>(W, ld, N, p->n, R, 1.0, 1.0, p->sf, p->sg, pc->U, 0, nullptr, Z, ldz, nullptr, st);
  PcWork w;
  DSKI_TRY(pc_work(pc, R, w));
  DSKI_TRY(launch_proj<T>(W, ld, N, p->n, R, 1.0, 1.0, pc->Ur, k, w.partial, st));
  RedJob j{w.partial, w.nblk, k * R, R, w.t, pc->rootc, nullptr, -1.0, w.coef, nullptr};
  DSKI_TRY(launch_reduce(j, nullptr, st));
  return launch_final<T>(W, ld, N, p->n, R, 1.0, 1.0, p->sf, p->sg, pc->U, k, w.coef, Z, ldz, nullptr, st);
}
template dski_status precond_factor_apply_tiled<float>(dski_precond, int, const float*, int, float*, int,
                                                       hipStream_t);
template dski_status precond_factor_apply_tiled<double>(dski_precond, int, const double*, int, double*,
                                                        int, hipStream_t);

static void destroy_pc(dski_precond pc) {
  if (!pc) return;
  (void)hipFree(pc->piv_tile);
  (void)hipFree(pc->L);
  (void)hipFree(pc->U);
  (void)hipFree(pc->Ur);
  (void)hipFree(pc->w);
  (void)hipFree(pc->rootc);
  pc->work.release();
  delete pc;
}

static dski_status build_impl(dski_plan p, int k, dski_precond pc, int* rank_host, int* piv_host,
                              const int* forced, hipStream_t st) {
  int N = p->N, n = p->n;
  GeoP g = p->kind == 0 ? geop_of(p) : GeoP{};
  DSKI_HIP(hipMalloc(&pc->piv_tile, sizeof(int) * std::max(k, 1)));
  DSKI_HIP(hipMalloc(&pc->L, sizeof(double) * (size_t)N * std::max(k, 1)));
  // scratch: dres (N), argmax partials, PivState, arow (sum m), lrow (k)
  int nblk = std::min(1024, std::max(1, (N + kBlock - 1) / kBlock));
  int msum = 0;
  if (p->kind == 0)
    for (int a = 0; a < p->d; ++a) msum += p->ax[a].m;
  size_t bytes = sizeof(double) * ((size_t)N + nblk + msum + k + 8) + sizeof(int) * (nblk + 8) +
                 sizeof(PivState) + 256;
  char* scratch = nullptr;
  double* spl_buf = nullptr;  // spline kernel: grid column, zeros and the pivot's row
  DSKI_HIP(hipMalloc(&scratch, bytes));
  double* dres = reinterpret_cast<double*>(scratch);
  double* pv = dres + N;
  double* arow = pv + nblk;
  double* lrow = arow + msum;
  PivState* ps = reinterpret_cast<PivState*>(lrow + k + 8);
  int* pi = reinterpret_cast<int*>(ps + 1);
  dski_status rc = DSKI_OK;
  do {
    int vb = (N + kBlock - 1) / kBlock;
    if (p->kind == 1) {
      rc = dskip_diag(p, dres, st);
      if (rc < 0) break;
    } else if (p->kernel == kKernelSpline) {
      GeoS gs = geos_of(p);
      if (p->S == kInterpQuintic)
        k_pc_diag_spline<kInterpQuintic><<<vb, kBlock, 0, st>>>(gs, p->toff, dres);
      else
        k_pc_diag_spline<kInterpCubic><<<vb, kBlock, 0, st>>>(gs, p->toff, dres);
      if (hipMalloc(&spl_buf, sizeof(double) * ((size_t)p->M + 2 * (size_t)N)) != hipSuccess) {
        spl_buf = nullptr;
        set_error("pivoted Cholesky: allocation failed");
        rc = DSKI_ENOMEM;
        break;
      }
      k_fill_zero_d<<<(unsigned)std::min<long long>(1024, (2 * (long long)N + kBlock - 1) / kBlock), kBlock, 0, st>>>(
          spl_buf + p->M, 2 * (long long)N);
    } else {
      if (p->S == kInterpQuintic)
        k_pc_diag<kInterpQuintic><<<vb, kBlock, 0, st>>>(g, p->cell, p->toff, dres);
      else
        k_pc_diag<kInterpCubic><<<vb, kBlock, 0, st>>>(g, p->cell, p->toff, dres);
    }
    const double rel_tol = 1e-12;
    for (int j = 0; j < k; ++j) {
      k_argmax_partial<<<nblk, kBlock, 0, st>>>(dres, N, pv, pi);
      if (p->kind == 1) {
        rc = dskip_pc_step(p, j, pv, pi, nblk, rel_tol, ps, pc->piv_tile, pc->L, lrow, dres, forced, st);
        if (rc < 0) break;
        continue;
      }
      if (p->kernel == kKernelSpline) {
        // grid column, the pivot's row, and zeros for the gather's noise input
        rc = spline_pc_step(p, j, pv, pi, nblk, rel_tol, ps, pc->piv_tile, pc->L, lrow, dres, forced, spl_buf,
                            spl_buf + p->M + N, spl_buf + p->M, st);
        if (rc < 0) break;
        continue;
      }
      if (p->S == kInterpQuintic) {
        k_pivot_select<kInterpQuintic><<<1, kBlock, 0, st>>>(g, pv, pi, nblk, j, rel_tol, ps, pc->piv_tile, p->cell,
                                                             p->toff, arow, pc->L, lrow, forced, dres);
        k_pc_column<kInterpQuintic><<<vb, kBlock, 0, st>>>(g, j, ps, p->cell, p->toff, arow, lrow, pc->L, dres);
      } else {
        k_pivot_select<kInterpCubic><<<1, kBlock, 0, st>>>(g, pv, pi, nblk, j, rel_tol, ps, pc->piv_tile, p->cell,
                                                           p->toff, arow, pc->L, lrow, forced, dres);
        k_pc_column<kInterpCubic><<<vb, kBlock, 0, st>>>(g, j, ps, p->cell, p->toff, arow, lrow, pc->L, dres);
      }
    }
    if (rc < 0) break;
    if (hipGetLastError() != hipSuccess) {
      set_error("pivoted Cholesky kernel launch failed");
      rc = DSKI_EHIP;
      break;
    }
    PivState hps{};
    if (k > 0) {
      if (hipMemcpyAsync(&hps, ps, sizeof(PivState), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("pivoted Cholesky synchronisation failed");
        rc = DSKI_EHIP;
        break;
      }
    }
    int r = k > 0 ? hps.rank : 0;
    pc->k = r;
    if (rank_host) *rank_host = r;
    if (piv_host && r > 0) {
      std::vector<int> pt(r), perm(n);
      if (hipMemcpy(pt.data(), pc->piv_tile, sizeof(int) * r, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(perm.data(), p->perm, sizeof(int) * n, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("pivot copy failed");
        rc = DSKI_EHIP;
        break;
      }
      for (int j = 0; j < r; ++j) {
        int e = pt[j];
        piv_host[j] = (e / n) * n + perm[e % n];
      }
      for (int j = r; j < k; ++j) piv_host[j] = -1;
    }
    // preconditioner: Gram of G = D^{-1/2} L, eigen-decomposition on the host
    double isf = 1.0 / p->sf, isg = 1.0 / p->sg;
    double logdetD = (double)n * 2.0 * std::log(p->sf) + (double)(N - n) * 2.0 * std::log(p->sg);
    DSKI_HIP(hipMalloc(&pc->U, sizeof(double) * (size_t)N * std::max(r, 1)));
    DSKI_HIP(hipMalloc(&pc->Ur, sizeof(double) * (size_t)N * std::max(r, 1)));
    DSKI_HIP(hipMalloc(&pc->w, sizeof(double) * std::max(r, 1)));
    DSKI_HIP(hipMalloc(&pc->rootc, sizeof(double) * std::max(r, 1)));
    if (r == 0) {
      pc->logdet = logdetD;
      break;
    }
    int rows = std::max(1, 6144 / r);
    int gb = (N + rows - 1) / rows;
    int npair = r * (r + 1) / 2;
    double* gpart = nullptr;
    DSKI_HIP(hipMalloc(&gpart, sizeof(double) * ((size_t)gb * npair + npair)));
    k_gram_partial<<<gb, kBlock, sizeof(double) * rows * r, st>>>(pc->L, N, n, r, rows, isf, isg, gpart);
    dski_status rr = reduce_partials(gpart, gb, npair, gpart + (size_t)gb * npair, st);
    std::vector<double> gram(npair);
    if (rr == DSKI_OK) {
      if (hipMemcpyAsync(gram.data(), gpart + (size_t)gb * npair, sizeof(double) * npair,
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        rr = DSKI_EHIP;
    }
    (void)hipFree(gpart);
    if (rr != DSKI_OK) {
      set_error("Gram matrix of the preconditioner failed");
      rc = DSKI_EHIP;
      break;
    }
    std::vector<double> A((size_t)r * r), V((size_t)r * r), w(r);
    for (int i = 0, pidx = 0; i < r; ++i)
      for (int jj = i; jj < r; ++jj, ++pidx) A[(size_t)i * r + jj] = A[(size_t)jj * r + i] = gram[pidx];
    sym_eig_jacobi(r, A.data(), V.data(), w.data());
    std::vector<double> Vs((size_t)r * r), wd(r), rootc(r);
    double wmax = 0.0;
    for (int i = 0; i < r; ++i) wmax = std::max(wmax, w[i]);
    double ld = logdetD;
    for (int i = 0; i < r; ++i) {
      double s2 = w[i] > 1e-13 * wmax ? w[i] : 0.0;
      double inv = s2 > 0.0 ? 1.0 / std::sqrt(s2) : 0.0;
      for (int l = 0; l < r; ++l) Vs[(size_t)l * r + i] = V[(size_t)l * r + i] * inv;
      wd[i] = s2 / (1.0 + s2);
      rootc[i] = std::sqrt(1.0 + s2) - 1.0;
      ld += std::log1p(s2);
    }
    pc->logdet = ld;
    double* dV = nullptr;
    DSKI_HIP(hipMalloc(&dV, sizeof(double) * (size_t)r * r));
    if (hipMemcpyAsync(dV, Vs.data(), sizeof(double) * r * r, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(pc->w, wd.data(), sizeof(double) * r, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(pc->rootc, rootc.data(), sizeof(double) * r, hipMemcpyHostToDevice, st) !=
            hipSuccess) {
      (void)hipFree(dV);
      set_error("preconditioner upload failed");
      rc = DSKI_EHIP;
      break;
    }
    k_make_u<<<(N + kBlock - 1) / kBlock, kBlock, 0, st>>>(pc->L, N, n, r, isf, isg, dV, pc->U, pc->Ur);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(dV);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      set_error("preconditioner factor kernel failed");
      rc = DSKI_EHIP;
      break;
    }
    if (r < k) rc = DSKI_RANK_TRUNCATED;
  } while (0);
  (void)hipFree(scratch);
  if (spl_buf) (void)hipFree(spl_buf);
  return rc;
}

}  // namespace dski

using namespace dski;

static dski_status build_entry(const char* who, dski_plan p, int k, dski_precond* out, int* rank_host,
                               int* piv_host, const int* forced_user, hipStream_t st) {
  if (!p || !out || k < 0 || k > p->N || k > 1024) {
    set_error("%s: bad arguments (k=%d)", who, k);
    return DSKI_EINVAL;
  }
  if (k > 256) {
    set_error("%s: rank %d too large (at most 256)", who, k);
    return DSKI_ENOTSUP;
  }
  *out = nullptr;
  // forced pivots: user-order N-indices -> tile order, checked on the host
  DevBuf fbuf;
  const int* forced = nullptr;
  if (forced_user && k > 0) {
    const int n = p->n;
    std::vector<int> perm(n), inv(n), ft(k);
    if (p->kind == 0) {
      if (hipMemcpy(perm.data(), p->perm, sizeof(int) * n, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("%s: permutation copy failed", who);
        return DSKI_EHIP;
      }
      for (int i = 0; i < n; ++i) inv[perm[i]] = i;
    } else {
      for (int i = 0; i < n; ++i) inv[i] = i;
    }
    for (int j = 0; j < k; ++j) {
      const int e = forced_user[j];
      if (e < 0 || e >= p->N) {
        set_error("%s: forced pivot %d of step %d is outside 0..N-1", who, e, j);
        return DSKI_EINVAL;
      }
      ft[j] = (e / n) * n + inv[e % n];
    }
    DSKI_TRY(fbuf.reserve(sizeof(int) * k));
    if (hipMemcpyAsync(fbuf.as<int>(), ft.data(), sizeof(int) * k, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      fbuf.release();
      set_error("%s: forced pivot copy failed", who);
      return DSKI_EHIP;
    }
    forced = fbuf.as<int>();
  }
  dski_precond pc = new dski_precond_s();
  pc->plan = p;
  dski_status rc = build_impl(p, k, pc, rank_host, piv_host, forced, st);
  if (forced) {
    // the build has synchronised its stream before returning
    (void)hipStreamSynchronize(st);
    fbuf.release();
  }
  if (rc < 0) {
    destroy_pc(pc);
    return rc;
  }
  *out = pc;
  return rc;
}

extern "C" {

dski_status pivchol_build(dski_plan p, int k, dski_precond* out, int* rank_host, int* piv_host,
                          dski_stream stream) {
  return build_entry("pivchol_build", p, k, out, rank_host, piv_host, nullptr, static_cast<hipStream_t>(stream));
}

dski_status pivchol_build_forced(dski_plan p, int k, const int* forced_piv_host, dski_precond* out,
                                 int* rank_host, int* piv_host, dski_stream stream) {
  if (!forced_piv_host) {
    set_error("pivchol_build_forced: NULL pivot list");
    return DSKI_EINVAL;
  }
  return build_entry("pivchol_build_forced", p, k, out, rank_host, piv_host, forced_piv_host,
                     static_cast<hipStream_t>(stream));
}

dski_status dski_precond_destroy(dski_precond pc) {
  destroy_pc(pc);
  return DSKI_OK;
}

dski_status dski_precond_logdet(dski_precond pc, double* out_host) {
  if (!pc || !out_host) {
    set_error("dski_precond_logdet: NULL argument");
    return DSKI_EINVAL;
  }
  *out_host = pc->logdet;
  return DSKI_OK;
}

}  // extern "C"

template <typename T>
static dski_status precond_apply_user(dski_precond pc, int R, const T* Rm, int ld, T* Z, int ldz,
                                      hipStream_t st) {
  if (!pc || R < 0 || ld < pc->plan->N || ldz < pc->plan->N || (R > 0 && (!Rm || !Z))) {
    set_error("dski_precond_apply: bad arguments");
    return DSKI_EINVAL;
  }
  dski_plan p = pc->plan;
  if (R == 0) return DSKI_OK;
  size_t nr = (size_t)p->N * R;
  DSKI_TRY(p->vin.reserve(sizeof(T) * nr));
  DSKI_TRY(p->vout.reserve(sizeof(T) * nr));
  DSKI_TRY(permute(p, +1, R, Rm, ld, p->vin.as<T>(), p->N, st));
  DSKI_TRY(precond_apply_tiled<T>(pc, R, p->vin.as<T>(), p->N, p->vout.as<T>(), p->N, nullptr, nullptr,
                                  st));
  return permute(p, -1, R, p->vout.as<T>(), p->N, Z, ldz, st);
}

extern "C" {

dski_status dski_precond_apply(dski_precond pc, int R, const float* Rm, int ld, float* Z, int ldz,
                               dski_stream stream) {
  return precond_apply_user<float>(pc, R, Rm, ld, Z, ldz, static_cast<hipStream_t>(stream));
}

dski_status dski_precond_apply_f64(dski_precond pc, int R, const double* Rm, int ld, double* Z, int ldz,
                                   dski_stream stream) {
  return precond_apply_user<double>(pc, R, Rm, ld, Z, ldz, static_cast<hipStream_t>(stream));
}

__global__ void k_factor_out(const double* __restrict__ L, int N, int n, int k,
                             const int* __restrict__ perm, double* __restrict__ out, int ld) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (e >= N || j >= k) return;
  int u = (e / n) * n + perm[e % n];
  out[(size_t)j * ld + u] = L[(size_t)j * N + e];
}

dski_status dski_precond_factor(dski_precond pc, double* Lout, int ld, dski_stream stream) {
  if (!pc || !Lout || ld < pc->plan->N) {
    set_error("dski_precond_factor: bad arguments");
    return DSKI_EINVAL;
  }
  if (pc->k == 0) return DSKI_OK;
  dski_plan p = pc->plan;
  dim3 grid((p->N + kBlock - 1) / kBlock, pc->k);
  k_factor_out<<<grid, kBlock, 0, static_cast<hipStream_t>(stream)>>>(pc->L, p->N, p->n, pc->k, p->perm,
                                                                       Lout, ld);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

}  // extern "C"
