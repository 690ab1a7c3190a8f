// The D-SKI matrix-vector product (Sec. 3.1):
//     Y = [W; dW_1..dW_d] K_UU [W; dW_1..dW_d]^T V + D V
// in three stages over tile-ordered vectors.  The interpolation weights (Keys
// cubic, 4 nodes per axis, or the quintic kernel, 6 nodes per axis) are not
// stored: every stage evaluates them from the points' cell offsets with the
// same FMA Horner routine (interp.h), so the scatter is exactly the transpose
// of the gather.
//   scatter  G = S^T V      owner-computes: one thread per grid node pulls the
//                           contributions of the points whose S^d stencil
//                           covers it, in a fixed order (no atomics, bitwise
//                           reproducible), FP64 accumulation;
//   K_UU     G <- K_UU G    SE kernel: per axis, per grid line, the circulant-
//                           embedded Toeplitz product by a radix-8 Stockham FFT
//                           in registers with LDS exchanges (FP64), two real
//                           lines packed into one complex transform, or a dense
//                           Toeplitz product on the FP64 matrix cores; spline
//                           kernel: the d-dimensional circulant embedding of
//                           the multi-level Toeplitz K_UU (App. A);
//   gather   Y = S G + D V  one thread per point, FP64 accumulation, FP32 store,
//                           optional fused per-block partials of V.Y.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"
#include "interp.h"

namespace dski {

struct GeoK {
  int m[DSKI_MAXD];
  int nc[DSKI_MAXD];
  double invh[DSKI_MAXD];
};

static GeoK geo_of(dski_plan p) {
  GeoK g{};
  for (int a = 0; a < p->d; ++a) {
    g.m[a] = p->ax[a].m;
    g.nc[a] = p->ax[a].ncell;
    g.invh[a] = 1.0 / p->ax[a].h;
  }
  return g;
}

// ------------------------------------------------------------------ scatter
// Grid node j receives sum over points k with j in stencil(k) of
//   w(x_k)_j V_0[k] + sum_q d_q w(x_k)_j V_q[k].
// A point's cell on axis a is its stencil's anchor node c_a (stored 0-based as
// c_a - H, H = S/2 - 1); its S stencil nodes are c_a - H + o, o < S, so node j
// is touched by the cells j - (S - 1 - H) .. j + H (clipped to H .. nc + H - 1)
// at stencil position o = j - c + H.  The weights are computed from the point
// offsets by interp_weights<S>, the function the gather uses too, so the
// scatter applies exactly the transpose of the gather's interpolation.
// The contribution of one point to one node for CR columns: the stencil
// weights of the node on every axis (value wv, derivative wd) form
// w = prod wv and d_q w = wd_q prod_{a != q} wv_a, and each column adds
// w V_0 + sum_q d_q w V_q as one FMA chain (x holds the CR x (D + 1) values,
// column-major by column).  Every scatter form calls this, so all give the
// same bits.
template <int D, int CR, typename VT>
__device__ __forceinline__ void scatter_accum(double (&acc)[CR], const double (&wv)[D], const double (&wd)[D],
                                              const VT* x) {
  double wprod = wv[0];
#pragma unroll
  for (int a = 1; a < D; ++a) wprod *= wv[a];
  double dprod[D];
#pragma unroll
  for (int qq = 0; qq < D; ++qq) {
    double v = qq == 0 ? wd[0] : wv[0];
#pragma unroll
    for (int a = 1; a < D; ++a) v *= (a == qq) ? wd[a] : wv[a];
    dprod[qq] = v;
  }
#pragma unroll
  for (int r = 0; r < CR; ++r) {
    double s = fma(wprod, (double)x[r * (D + 1)], acc[r]);
#pragma unroll
    for (int qq = 0; qq < D; ++qq) s = fma(dprod[qq], (double)x[r * (D + 1) + qq + 1], s);
    acc[r] = s;
  }
}

// Value and derivative weight of stencil position o (o < S) at offset t:
// all S weights are formed as in interp_weights<S> and the one at o selected
// (a select chain, no indexed private array).
template <int S>
__device__ __forceinline__ void interp_weight_at(double t, double ih, int o, double& wv, double& wd) {
  double w[S], dw[S];
  interp_weights<S>(t, ih, w, dw);
  wv = w[0];
  wd = dw[0];
#pragma unroll
  for (int u = 1; u < S; ++u) {
    wv = o == u ? w[u] : wv;
    wd = o == u ? dw[u] : wd;
  }
}

// LDS-staged version: a work-group owns a tile of grid nodes and one chunk of
// CR columns.  It copies into LDS the weights and the CR column values of every
// point in the cells whose stencils reach the tile (the tile's cells plus a
// halo of S - 1 - H below and H above), with a table of each cell's range, then
// every thread sums its node's contributions from LDS in the same fixed order
// as above.  One thread stages one region point; regions of more than PMAX
// points (256 in 1-D and 2-D, 192 in 3-D, whose weight tables are larger: 3-D
// surface regions measured fastest at 192, against 128, 96 and 64) are staged
// PMAX points at a time, each node adding the points of every chunk that fall
// in its cells (same order, same result).
template <int D, int S>
struct TileShape {
  static constexpr int e0 = D == 1 ? 256 : (D == 2 ? 16 : 4);
  static constexpr int e1 = D == 2 ? 16 : 8;
  static constexpr int e2 = 8;
  static constexpr int HALO = S - 1;  // region cells beyond a tile's node extent
  static __host__ __device__ constexpr int ext(int a) { return a == 0 ? e0 : (a == 1 ? e1 : e2); }
  static constexpr int max_cells = D == 1 ? (e0 + HALO)
                                          : (D == 2 ? (e0 + HALO) * (e1 + HALO)
                                                    : (e0 + HALO) * (e1 + HALO) * (e2 + HALO));
  static constexpr int max_rows = D == 1 ? 1 : (D == 2 ? (e0 + HALO) : (e0 + HALO) * (e1 + HALO));
  static constexpr int last_span = ext(D - 1) + HALO;
};

// Region of a tile: the cells whose stencils reach its nodes, as per-axis
// first cell rlo (anchor-node numbering) and span; rows = all region axes but
// the last (their cells are contiguous in the sorted order).
template <int D, int S>
struct TileRegion {
  int origin[D], span[D], rlo[D];
  int nrows, ncells;
  __device__ TileRegion(int tile, const GeoK& g) {
    using TS = TileShape<D, S>;
    constexpr int H = S / 2 - 1;
    int rem = tile;
    for (int a = D - 1; a >= 0; --a) {
      const int nt = (g.m[a] + TS::ext(a) - 1) / TS::ext(a);
      origin[a] = (rem % nt) * TS::ext(a);
      rem /= nt;
    }
    nrows = 1;
    ncells = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int tlast = min(origin[a] + TS::ext(a) - 1, g.m[a] - 1);
      rlo[a] = max(H, origin[a] - (S - 1 - H));
      const int rhi = min(g.nc[a] + H - 1, tlast + H);
      span[a] = rhi - rlo[a] + 1;
      ncells *= span[a];
      if (a < D - 1) nrows *= span[a];
    }
  }
};

// Per-row point ranges of a tile's region in LDS (global first point s_rg0, first
// region cell s_rcb, local offset s_roff, total in s_roff[nrows]); all threads.
template <int D, int S>
__device__ void tile_rows(const TileRegion<D, S>& T, const GeoK& g, const int* __restrict__ cstart, int* s_rg0,
                          int* s_rcb, int* s_rcnt, int* s_roff) {
  constexpr int H = S / 2 - 1;
  const int last = D - 1;
  for (int row = threadIdx.x; row < T.nrows; row += blockDim.x) {
    int rem = row, base = 0;
    int c[D];
    for (int a = last - 1; a >= 0; --a) {
      c[a] = T.rlo[a] + rem % T.span[a];
      rem /= T.span[a];
    }
    for (int a = 0; a < last; ++a) base = base * g.nc[a] + (c[a] - H);
    base = base * g.nc[last] + T.rlo[last] - H;
    const int g0 = cstart[base];
    const int g1 = cstart[base + T.span[last]];
    s_rcb[row] = base;
    s_rg0[row] = g0;
    s_rcnt[row] = g1 - g0;
  }
  __syncthreads();
  // exclusive prefix of the row counts (wavefront 0, 64 rows per step)
  if (threadIdx.x < 64) {
    int carry = 0;
    for (int rb = 0; rb < T.nrows; rb += 64) {
      const int row = rb + threadIdx.x;
      const int v = row < T.nrows ? s_rcnt[row] : 0;
      int incl = v;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if ((int)threadIdx.x >= off) incl += o;
      }
      if (row < T.nrows) s_roff[row] = carry + incl - v;
      carry += __shfl(incl, 63, 64);
    }
    if (threadIdx.x == 0) s_roff[T.nrows] = carry;
  }
  __syncthreads();
}

// Plan set-up, pass 1: the number of points in every tile's region.
template <int D, int S>
__global__ __launch_bounds__(256) void k_tile_count(const int* __restrict__ cstart, GeoK g,
                                                    int* __restrict__ total) {
  using TS = TileShape<D, S>;
  __shared__ int s_rg0[TS::max_rows], s_rcb[TS::max_rows], s_rcnt[TS::max_rows], s_roff[TS::max_rows + 1];
  const TileRegion<D, S> T(blockIdx.x, g);
  tile_rows<D, S>(T, g, cstart, s_rg0, s_rcb, s_rcnt, s_roff);
  if (threadIdx.x == 0) total[blockIdx.x] = s_roff[T.nrows];
}

// Plan set-up, pass 2: every tile's region tables (fixed by the points alone):
// the local point range of each region cell (row-major, last axis fastest), and
// for each local slot q (tile_off[t] + q) the point and its last-axis anchor.
template <int D, int S>
__global__ __launch_bounds__(256) void k_tile_fill(const int* __restrict__ cell, const int* __restrict__ cstart,
                                                   GeoK g, const int* __restrict__ tile_off,
                                                   int* __restrict__ tile_lcs, int* __restrict__ tile_pts,
                                                   int* __restrict__ tile_cl) {
  using TS = TileShape<D, S>;
  constexpr int H = S / 2 - 1;
  __shared__ int s_rg0[TS::max_rows], s_rcb[TS::max_rows], s_rcnt[TS::max_rows], s_roff[TS::max_rows + 1];
  const int last = D - 1;
  const TileRegion<D, S> T(blockIdx.x, g);
  tile_rows<D, S>(T, g, cstart, s_rg0, s_rcb, s_rcnt, s_roff);
  const int total = s_roff[T.nrows];
  int* lcs = tile_lcs + (size_t)blockIdx.x * (TS::max_cells + 1);
  for (int f = threadIdx.x; f < T.nrows * TS::last_span; f += blockDim.x) {
    const int row = f / TS::last_span, cl = f % TS::last_span;
    if (cl < T.span[last]) lcs[row * T.span[last] + cl] = cstart[s_rcb[row] + cl] - s_rg0[row] + s_roff[row];
  }
  if (threadIdx.x == 0) lcs[T.ncells] = total;
  const long long off = tile_off[blockIdx.x];
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    int lo_r = 0, hi_r = T.nrows - 1;  // last row with s_roff[row] <= q
    while (lo_r < hi_r) {
      const int mid = (lo_r + hi_r + 1) >> 1;
      if (s_roff[mid] <= q) lo_r = mid; else hi_r = mid - 1;
    }
    const int kq = s_rg0[lo_r] + q - s_roff[lo_r];
    tile_pts[off + q] = kq;
    tile_cl[off + q] = cell[kq] % g.nc[last] + H;
  }
}

template <int D>
constexpr int scatter_pmax() {
  return D == 3 ? 192 : 256;
}

// Stages region slots [q0, q0 + PMAX) of a tile, one thread one point: its
// last-axis anchor node, its weights (value and derivative per axis, from the
// offsets) and its CR column values (zeros for columns past rc).
template <int D, int S, int CR, typename T>
__device__ __forceinline__ void stage_chunk(int q0, int total, long long off, const int* __restrict__ tile_pts,
                                            const int* __restrict__ tile_cl, const double* __restrict__ toff, int n,
                                            const GeoK& g, const T* __restrict__ V, int ldv, int r0, int rc,
                                            double* s_w, T* s_v, int* s_cl) {
  constexpr int PMAX = scatter_pmax<D>();
  constexpr int WS = 2 * S * D + 1;
  const int q = threadIdx.x;
  if (q < PMAX && q0 + q < total) {
    const int kq = tile_pts[off + q0 + q];
    const int cq = tile_cl[off + q0 + q];
    double tq[D];
#pragma unroll
    for (int a = 0; a < D; ++a) tq[a] = toff[(size_t)a * n + kq];
    T x[CR * (D + 1)];
#pragma unroll
    for (int r = 0; r < CR; ++r)
#pragma unroll
      for (int b = 0; b <= D; ++b)
        x[r * (D + 1) + b] = ld_or0(V, (size_t)(r0 + r) * ldv + (size_t)b * n + kq,
                                    (size_t)r0 * ldv + (size_t)b * n + kq, r < rc);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double w[S], dw[S];
      interp_weights<S>(tq[a], g.invh[a], w, dw);
#pragma unroll
      for (int o = 0; o < S; ++o) {
        s_w[q * WS + a * 2 * S + o] = w[o];
        s_w[q * WS + a * 2 * S + S + o] = dw[o];
      }
    }
#pragma unroll
    for (int e = 0; e < CR * (D + 1); ++e) s_v[q * CR * (D + 1) + e] = x[e];
    s_cl[q] = cq;
  }
}

// Adds the staged points of slots [qs, qe) (chunk-local index slot - q0) of one
// cell row of a node to acc, in slot order, two points per step: both points'
// LDS loads are issued before the first product (the loop is bound by
// dependent LDS latency), then the points are added in order, exactly as one
// at a time.  wo[a]: the LDS offsets of the outer axes' weights in this row;
// jl: the node's index on the last axis.
template <int D, int S, int CR, typename T>
__device__ __forceinline__ void accum_row(double (&acc)[CR], int qs, int qe, int q0, const int (&wo)[D], int jl,
                                          const double* s_w, const T* s_v, const int* s_cl) {
  constexpr int H = S / 2 - 1;
  constexpr int WS = 2 * S * D + 1;
  const int last = D - 1;
  int qq = qs;
  for (; qq + 1 < qe; qq += 2) {
    const int qa = qq - q0, qb = qa + 1;
    const int cla = s_cl[qa], clb = s_cl[qb];
    double wva[D], wda[D], wvb[D], wdb[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int oa = a == last ? last * 2 * S + jl - cla + H : wo[a];
      const int ob = a == last ? last * 2 * S + jl - clb + H : wo[a];
      wva[a] = s_w[qa * WS + oa];
      wda[a] = s_w[qa * WS + S + oa];
      wvb[a] = s_w[qb * WS + ob];
      wdb[a] = s_w[qb * WS + S + ob];
    }
    scatter_accum<D, CR>(acc, wva, wda, s_v + (size_t)qa * CR * (D + 1));
    scatter_accum<D, CR>(acc, wvb, wdb, s_v + (size_t)qb * CR * (D + 1));
  }
  if (qq < qe) {
    const int ql = qq - q0;
    const int cl = s_cl[ql];
    double wv[D], wd[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int o = a == last ? last * 2 * S + jl - cl + H : wo[a];
      wv[a] = s_w[ql * WS + o];
      wd[a] = s_w[ql * WS + S + o];
    }
    scatter_accum<D, CR>(acc, wv, wd, s_v + (size_t)ql * CR * (D + 1));
  }
}

template <int D, int S, int CR, typename T, typename GT>
__global__ __launch_bounds__(256) void k_scatter_lds(const int* __restrict__ cell,
                                                     const double* __restrict__ toff,
                                                     const int* __restrict__ cstart, int n, GeoK g,
                                                     const int* __restrict__ tile_off,
                                                     const int* __restrict__ tile_lcs,
                                                     const int* __restrict__ tile_pts,
                                                     const int* __restrict__ tile_cl,
                                                     const T* __restrict__ V, int ldv, int R, int cr,
                                                     GT* __restrict__ G, long long M) {
  constexpr int PMAX = scatter_pmax<D>();  // one thread stages one region point
  constexpr int H = S / 2 - 1;
  using TS = TileShape<D, S>;
  // weights point-major, 2 S D + 1 doubles per point: lanes reading one point at
  // different stencil offsets hit adjacent banks, different points rarely share one
  constexpr int WS = 2 * S * D + 1;
  __shared__ double s_w[PMAX * WS];
  __shared__ T s_v[PMAX * CR * (D + 1)];
  __shared__ int s_lcs[TS::max_cells + 1];
  __shared__ int s_cl[PMAX];  // last-axis anchor node of every region point
  const int last = D - 1;
  const TileRegion<D, S> TR(blockIdx.x, g);
  int origin[D], span[D], rlo[D], jl[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    origin[a] = TR.origin[a];
    span[a] = TR.span[a];
    rlo[a] = TR.rlo[a];
  }
  if (D == 1) {
    jl[0] = threadIdx.x;
  } else if (D == 2) {
    jl[0] = threadIdx.x / TS::e1;
    jl[1] = threadIdx.x % TS::e1;
  } else {
    jl[0] = threadIdx.x / (TS::e1 * TS::e2);
    jl[1] = (threadIdx.x / TS::e2) % TS::e1;
    jl[2] = threadIdx.x % TS::e2;
  }
  const int r0 = blockIdx.y * cr;
  const int rc = min(cr, R - r0);
  const long long off = tile_off[blockIdx.x];
  const int total = (int)(tile_off[blockIdx.x + 1] - off);
  {
    const int* lcs = tile_lcs + (size_t)blockIdx.x * (TS::max_cells + 1);
    for (int f = threadIdx.x; f <= TR.ncells; f += blockDim.x) s_lcs[f] = lcs[f];
  }
  int j[D];
  bool inside = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    j[a] = origin[a] + jl[a];
    inside = inside && j[a] < g.m[a];
  }
  double acc[CR];
#pragma unroll
  for (int r = 0; r < CR; ++r) acc[r] = 0.0;
  int lo[D], hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = max(H, j[a] - (S - 1 - H));
    hi[a] = min(g.nc[a] + H - 1, j[a] + H);
  }
  int nrow = 1;  // the node's outer cell rows (all axes but the last)
#pragma unroll
  for (int a = 0; a < last; ++a) nrow *= hi[a] - lo[a] + 1;
  // The region's points are staged PMAX at a time, in slot order (one thread
  // per point: its last-axis anchor, weights and column values).  After each
  // chunk every node adds the points of that chunk that lie in its cells: its
  // outer cell rows in odometer order, and in each the contiguous run of cells
  // lo..hi on the last axis.  The node therefore adds its points in the same
  // order whatever the chunking (rows ascending, slots ascending in a row).
  for (int q0 = 0; q0 < total; q0 += PMAX) {
    if (q0 > 0) __syncthreads();  // every node is done with the previous chunk
    stage_chunk<D, S, CR, T>(q0, total, off, tile_pts, tile_cl, toff, n, g, V, ldv, r0, rc, s_w, s_v, s_cl);
    __syncthreads();
    if (!inside) continue;
    const int q1 = min(total, q0 + PMAX);
    for (int row = 0; row < nrow; ++row) {
      int c[D];
      int rem = row, lrow = 0;
#pragma unroll
      for (int a = last - 1; a >= 0; --a) {
        const int sp = hi[a] - lo[a] + 1;
        c[a] = lo[a] + rem % sp;
        rem /= sp;
      }
#pragma unroll
      for (int a = 0; a < last; ++a) lrow = lrow * span[a] + (c[a] - rlo[a]);
      const int qs = max(q0, s_lcs[lrow * span[last] + lo[last] - rlo[last]]);
      const int qe = min(q1, s_lcs[lrow * span[last] + hi[last] - rlo[last] + 1]);
      int wo[D];  // LDS offsets of the outer axes' weights in this row
#pragma unroll
      for (int a = 0; a < last; ++a) wo[a] = a * 2 * S + j[a] - c[a] + H;
      accum_row<D, S, CR, T>(acc, qs, qe, q0, wo, j[last], s_w, s_v, s_cl);
    }
  }
  if (!inside) return;
  long long node = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) node = node * g.m[a] + j[a];
  // Streaming stores (here and in the gather): the next kernel reads the grid
  // after the kernel boundary has written back and invalidated the XCD L2s
  // anyway, so keeping it in L2 gains nothing (scatter and gather about 0.8 us
  // faster each).  The FFT keeps ordinary stores: streaming ones made K_UU
  // slower on the 632^2 and 1000^2 grids and no faster on 200^2.
#pragma unroll
  for (int r = 0; r < CR; ++r)
    if (r < rc) __builtin_nontemporal_store((GT)acc[r], &G[(size_t)(r0 + r) * M + node]);
}

// Columns per work-group of the LDS-tiled scatter: a base chunk (4 columns in
// 1-D and 2-D; 2 FP32 or 1 FP64 in 3-D) times 1, 1.5, 2 or 5 (9 in 3-D, so that
// a 17-column block is one chunk of FP32 columns); wider chunks mean fewer
// work-groups, each staging its region once for more columns.  FP32 and FP64
// column values are tuned separately.  On 3-D surface data the narrow chunks
// win: a node's loop length follows its point count, which varies widely
// within a wavefront (about 15 % of the lanes busy per step on the torus), and
// wide chunks lower the occupancy that hides the LDS latency.
template <int D, int S, typename T, int WIDTH>
constexpr int scatter_cr() {
  constexpr int base = D <= 2 ? 4 : (sizeof(T) == 4 ? 2 : 1);
  constexpr int wide = D == 3 ? 9 : 5;
  int cr = WIDTH == 0 ? base : (WIDTH == 1 ? base + (base + 1) / 2 : (WIDTH == 2 ? 2 * base : wide * base));
  // the staged column values share the 160 KB of LDS with the weights and tables
  using TS = TileShape<D, S>;
  constexpr int P = scatter_pmax<D>();
  while (cr > 1 && P * (2 * S * D + 1) * 8 + P * cr * (D + 1) * (int)sizeof(T) + (TS::max_cells + 1) * 4 +
                       P * 4 > 160 * 1024)
    --cr;
  return cr;
}

template <int D, int S, typename T, typename GT, int WIDTH>
static void launch_scatter(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  GeoK g = geo_of(p);
  using TS = TileShape<D, S>;
  long long tiles = 1;
  for (int a = 0; a < D; ++a) tiles *= (g.m[a] + TS::ext(a) - 1) / TS::ext(a);
  // columns per work-group: at most CR, chunks of equal width but the last
  constexpr int CR = scatter_cr<D, S, T, WIDTH>();
  const int nch = (R + CR - 1) / CR;
  const int cr = (R + nch - 1) / nch;
  dim3 grid((unsigned)tiles, nch);
  k_scatter_lds<D, S, CR, T, GT><<<grid, 256, 0, st>>>(p->cell, p->toff, p->cell_start, p->n, g, p->tile_off,
                                                        p->tile_lcs, p->tile_pts, p->tile_cl, V, ldv, R, cr, G,
                                                        p->M);
}

// Grouped 3-D variant.  On surface data a node's point count, and with it the
// length of its loop, varies widely within a wavefront, and the tiled form
// steps as long as the busiest node of the wavefront in every cell row (about
// one lane pair in twelve busy on the torus).  Here the unit of work is an
// item: one node and one cell c0 of its first axis, i.e. the S cell rows of
// its support with that c0.  At plan set-up the host lists, for every staged
// chunk of a tile, the items with points in that chunk, longest first, so that
// the lanes of a wavefront take items of similar length.  An item continues
// the running sum of its (node, c0) in LDS from chunk to chunk, adding its
// points in the tiled form's order; at the end each node adds its S partial
// sums in c0 order.  The result equals the tiled form's up to that grouping of
// the additions (it is not bitwise equal to the other forms).
template <int S, typename T>
constexpr int scatter_grp_cr() {
  return sizeof(T) == 4 ? 3 : 2;
}

template <int S, int CR, typename T, typename GT>
__global__ __launch_bounds__(256) void k_scatter_grp(const double* __restrict__ toff, int n, GeoK g,
                                                     const int* __restrict__ tile_off,
                                                     const int* __restrict__ tile_lcs,
                                                     const int* __restrict__ tile_pts,
                                                     const int* __restrict__ tile_cl,
                                                     const unsigned short* __restrict__ items,
                                                     const int* __restrict__ chunk_off,
                                                     const int* __restrict__ tile_chunk, const T* __restrict__ V,
                                                     int ldv, int R, int cr, GT* __restrict__ G, long long M) {
  constexpr int D = 3;
  constexpr int PMAX = scatter_pmax<D>();
  constexpr int H = S / 2 - 1;
  using TS = TileShape<D, S>;
  constexpr int WS = 2 * S * D + 1;
  static_assert(TS::e0 * TS::e1 * TS::e2 == 256, "one node per thread at the end");
  __shared__ double s_w[PMAX * WS];
  __shared__ T s_v[PMAX * CR * (D + 1)];
  __shared__ int s_lcs[TS::max_cells + 1];
  __shared__ int s_cl[PMAX];
  __shared__ double s_part[256 * S * CR];  // running sums per (node, c0 - lo0, column)
  const TileRegion<D, S> TR(blockIdx.x, g);
  const int r0 = blockIdx.y * cr;
  const int rc = min(cr, R - r0);
  const long long off = tile_off[blockIdx.x];
  const int total = (int)(tile_off[blockIdx.x + 1] - off);
  {
    const int* lcs = tile_lcs + (size_t)blockIdx.x * (TS::max_cells + 1);
    for (int f = threadIdx.x; f <= TR.ncells; f += blockDim.x) s_lcs[f] = lcs[f];
  }
  for (int f = threadIdx.x; f < 256 * S * CR; f += blockDim.x) s_part[f] = 0.0;
  int ch = tile_chunk[blockIdx.x];
  for (int q0 = 0; q0 < total; q0 += PMAX, ++ch) {
    if (q0 > 0) __syncthreads();  // every item is done with the previous chunk
    stage_chunk<D, S, CR, T>(q0, total, off, tile_pts, tile_cl, toff, n, g, V, ldv, r0, rc, s_w, s_v, s_cl);
    __syncthreads();
    const int q1 = min(total, q0 + PMAX);
    const int ie = chunk_off[ch + 1];
    for (int it = chunk_off[ch] + threadIdx.x; it < ie; it += blockDim.x) {
      const int code = items[it];
      const int node = code >> 3, grp = code & 7;
      int j[D], lo[D], hi[D];
      j[0] = TR.origin[0] + node / (TS::e1 * TS::e2);
      j[1] = TR.origin[1] + (node / TS::e2) % TS::e1;
      j[2] = TR.origin[2] + node % TS::e2;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lo[a] = max(H, j[a] - (S - 1 - H));
        hi[a] = min(g.nc[a] + H - 1, j[a] + H);
      }
      const int c0 = lo[0] + grp;
      double* part = s_part + (size_t)(node * S + grp) * CR;
      double acc[CR];
#pragma unroll
      for (int r = 0; r < CR; ++r) acc[r] = part[r];
      int wo[D];
      wo[0] = j[0] - c0 + H;
      for (int c1 = lo[1]; c1 <= hi[1]; ++c1) {
        const int lrow = (c0 - TR.rlo[0]) * TR.span[1] + (c1 - TR.rlo[1]);
        const int qs = max(q0, s_lcs[lrow * TR.span[2] + lo[2] - TR.rlo[2]]);
        const int qe = min(q1, s_lcs[lrow * TR.span[2] + hi[2] - TR.rlo[2] + 1]);
        wo[1] = 2 * S + j[1] - c1 + H;
        accum_row<D, S, CR, T>(acc, qs, qe, q0, wo, j[2], s_w, s_v, s_cl);
      }
#pragma unroll
      for (int r = 0; r < CR; ++r) part[r] = acc[r];
    }
  }
  __syncthreads();
  int j[D];
  j[0] = TR.origin[0] + threadIdx.x / (TS::e1 * TS::e2);
  j[1] = TR.origin[1] + (threadIdx.x / TS::e2) % TS::e1;
  j[2] = TR.origin[2] + threadIdx.x % TS::e2;
  if (j[0] >= g.m[0] || j[1] >= g.m[1] || j[2] >= g.m[2]) return;
  const int ng = min(g.nc[0] + H - 1, j[0] + H) - max(H, j[0] - (S - 1 - H)) + 1;
  const double* part = s_part + (size_t)threadIdx.x * S * CR;
  const long long node = ((long long)j[0] * g.m[1] + j[1]) * g.m[2] + j[2];
#pragma unroll
  for (int r = 0; r < CR; ++r) {
    double sum = part[r];
    for (int q = 1; q < ng; ++q) sum += part[q * CR + r];
    if (r < rc) __builtin_nontemporal_store((GT)sum, &G[(size_t)(r0 + r) * M + node]);
  }
}

template <int S, typename T, typename GT>
static void launch_scatter_grp(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  GeoK g = geo_of(p);
  using TS = TileShape<3, S>;
  long long tiles = 1;
  for (int a = 0; a < 3; ++a) tiles *= (g.m[a] + TS::ext(a) - 1) / TS::ext(a);
  constexpr int CR = scatter_grp_cr<S, T>();
  const int nch = (R + CR - 1) / CR;
  const int cr = (R + nch - 1) / nch;
  dim3 grid((unsigned)tiles, nch);
  k_scatter_grp<S, CR, T, GT><<<grid, 256, 0, st>>>(p->toff, p->n, g, p->tile_off, p->tile_lcs, p->tile_pts,
                                                     p->tile_cl, p->grp_items, p->grp_chunk_off, p->grp_tile_chunk,
                                                     V, ldv, R, cr, G, p->M);
}

// Direct variant: one thread per (grid node, CRD columns), no LDS; cell ranges,
// offsets and column values are read through the caches (neighbouring nodes
// share points).  Same summation order and weights as the tiled kernel, hence
// the same result.
template <int D, int S, int CRD, typename T, typename GT>
__global__ __launch_bounds__(256) void k_scatter_direct(const int* __restrict__ cell,
                                                        const double* __restrict__ toff,
                                                        const int* __restrict__ cstart, int n, GeoK g,
                                                        const T* __restrict__ V, int ldv, int R,
                                                        GT* __restrict__ G, long long M) {
  constexpr int H = S / 2 - 1;
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= M) return;
  const int r0 = blockIdx.y * CRD;
  const int rc = min(CRD, R - r0);
  const int last = D - 1;
  int j[D];
  {
    long long rem = node;
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      j[a] = (int)(rem % g.m[a]);
      rem /= g.m[a];
    }
  }
  int lo[D], hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = max(H, j[a] - (S - 1 - H));
    hi[a] = min(g.nc[a] + H - 1, j[a] + H);
  }
  int outer_cnt = 1;
#pragma unroll
  for (int a = 0; a < last; ++a) outer_cnt *= hi[a] - lo[a] + 1;
  double acc[CRD];
#pragma unroll
  for (int r = 0; r < CRD; ++r) acc[r] = 0.0;
  for (int oc = 0; oc < outer_cnt; ++oc) {
    int c[D];
    int rem = oc, base = 0;
#pragma unroll
    for (int a = last - 1; a >= 0; --a) {
      int sp = hi[a] - lo[a] + 1;
      c[a] = lo[a] + rem % sp;
      rem /= sp;
    }
#pragma unroll
    for (int a = 0; a < last; ++a) base = base * g.nc[a] + (c[a] - H);
    base *= g.nc[last];
    // the cells lo..hi of the last axis are one contiguous run of points; the
    // stencil position on the last axis changes at each cell boundary
    for (int cl = lo[last]; cl <= hi[last]; ++cl) {
      const int kb = cstart[base + cl - H], ke = cstart[base + cl - H + 1];
      // four points per step: all their loads are issued before the first
      // product; the points are then added in order, exactly as one at a time
      for (int k0 = kb; k0 < ke; k0 += 4) {
        double tq[4][D];
        T x[4][CRD * (D + 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + u < ke ? k0 + u : kb;  // a valid point stands in past the run
#pragma unroll
          for (int a = 0; a < D; ++a) tq[u][a] = toff[(size_t)a * n + k];
#pragma unroll
          for (int r = 0; r < CRD; ++r)
#pragma unroll
            for (int b2 = 0; b2 <= D; ++b2)
              x[u][r * (D + 1) + b2] = ld_or0(V, (size_t)(r0 + r) * ldv + (size_t)b2 * n + k,
                                              (size_t)r0 * ldv + (size_t)b2 * n + k, r < rc);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double wv[D], wd[D];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const int ca = (a == last) ? cl : c[a];
            interp_weight_at<S>(tq[u][a], g.invh[a], j[a] - ca + H, wv[a], wd[a]);
          }
          double t[CRD];
#pragma unroll
          for (int r = 0; r < CRD; ++r) t[r] = acc[r];
          scatter_accum<D, CRD>(t, wv, wd, x[u]);
          const bool ok = k0 + u < ke;
#pragma unroll
          for (int r = 0; r < CRD; ++r) acc[r] = ok ? t[r] : acc[r];
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < CRD; ++r)
    if (r < rc) __builtin_nontemporal_store((GT)acc[r], &G[(size_t)(r0 + r) * M + node]);
}

template <int D, int S, int CRD, typename T, typename GT>
static void launch_scatter_direct(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  GeoK g = geo_of(p);
  dim3 grid((unsigned)((p->M + 255) / 256), (R + CRD - 1) / CRD);
  k_scatter_direct<D, S, CRD, T, GT><<<grid, 256, 0, st>>>(p->cell, p->toff, p->cell_start, p->n, g, V, ldv, R, G,
                                                           p->M);
}

template <int D, int S, typename T, typename GT>
static void scatter_dispatch(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  switch (sizeof(T) == 8 ? p->scatter_variant64 : p->scatter_variant) {
    case 1: launch_scatter_direct<D, S, 1, T, GT>(p, R, V, ldv, G, st); break;
    case 2: launch_scatter_direct<D, S, 2, T, GT>(p, R, V, ldv, G, st); break;
    case 3: launch_scatter<D, S, T, GT, 1>(p, R, V, ldv, G, st); break;
    case 4: launch_scatter<D, S, T, GT, 2>(p, R, V, ldv, G, st); break;
    case 5: launch_scatter<D, S, T, GT, 3>(p, R, V, ldv, G, st); break;
    case 6:  // grouped in 3-D; elsewhere the tiled form of variant 3
      if constexpr (D == 3)
        launch_scatter_grp<S, T, GT>(p, R, V, ldv, G, st);
      else
        launch_scatter<D, S, T, GT, 1>(p, R, V, ldv, G, st);
      break;
    default: launch_scatter<D, S, T, GT, 0>(p, R, V, ldv, G, st); break;
  }
}

template <int S, typename T, typename GT>
static dski_status scatter_s(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  switch (p->d) {
    case 1: scatter_dispatch<1, S, T, GT>(p, R, V, ldv, G, st); break;
    case 2: scatter_dispatch<2, S, T, GT>(p, R, V, ldv, G, st); break;
    case 3: scatter_dispatch<3, S, T, GT>(p, R, V, ldv, G, st); break;
    default: set_error("d=%d not supported", p->d); return DSKI_ENOTSUP;
  }
  return DSKI_OK;
}

template <typename T, typename GT>
dski_status scatter(dski_plan p, int R, const T* V, int ldv, GT* G, hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  DSKI_TRY((p->S == kInterpQuintic ? scatter_s<kInterpQuintic, T, GT>(p, R, V, ldv, G, st)
                                   : scatter_s<kInterpCubic, T, GT>(p, R, V, ldv, G, st)));
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}
template dski_status scatter<float, double>(dski_plan, int, const float*, int, double*, hipStream_t);
template dski_status scatter<double, double>(dski_plan, int, const double*, int, double*, hipStream_t);

// Item lists of the grouped 3-D scatter (see k_scatter_grp), built on the host
// from the cell ranges with the tiles' region geometry: for every chunk of
// PMAX region slots of every tile, the (node, c0) items with points in it, by
// decreasing work (pairs of points per cell row plus one step per row), ties
// in (node, c0) order.
template <int S>
static dski_status build_groups3(dski_plan p, const GeoK& g, long long tiles, const std::vector<int>& off,
                                 hipStream_t st) {
  using TS = TileShape<3, S>;
  constexpr int H = S / 2 - 1, PMAX = scatter_pmax<3>();
  std::vector<int> cs((size_t)p->ncells + 1);
  DSKI_HIP(hipMemcpyAsync(cs.data(), p->cell_start, sizeof(int) * cs.size(), hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  int nt[3];
  for (int a = 0; a < 3; ++a) nt[a] = (g.m[a] + TS::ext(a) - 1) / TS::ext(a);
  std::vector<int> tile_chunk((size_t)tiles + 1), chunk_off(1, 0), lcs;
  std::vector<unsigned short> items;
  std::vector<std::pair<int, int>> list;  // (work, code)
  int nchunks = 0;
  for (long long t = 0; t < tiles; ++t) {
    tile_chunk[(size_t)t] = nchunks;
    const int total = off[(size_t)t + 1] - off[(size_t)t];
    int origin[3], rlo[3], span[3];
    long long rem = t;
    for (int a = 2; a >= 0; --a) {
      origin[a] = (int)(rem % nt[a]) * TS::ext(a);
      rem /= nt[a];
    }
    for (int a = 0; a < 3; ++a) {
      const int tlast = std::min(origin[a] + TS::ext(a) - 1, g.m[a] - 1);
      rlo[a] = std::max(H, origin[a] - (S - 1 - H));
      span[a] = std::min(g.nc[a] + H - 1, tlast + H) - rlo[a] + 1;
    }
    // local slot offsets of the region cells, as k_tile_fill lays them out
    lcs.assign((size_t)span[0] * span[1] * span[2] + 1, 0);
    int pre = 0;
    for (int r0 = 0; r0 < span[0]; ++r0)
      for (int r1 = 0; r1 < span[1]; ++r1) {
        const int row = r0 * span[1] + r1;
        const long long base = ((long long)(rlo[0] + r0 - H) * g.nc[1] + (rlo[1] + r1 - H)) * g.nc[2] + rlo[2] - H;
        for (int k = 0; k < span[2]; ++k) lcs[(size_t)row * span[2] + k] = pre + cs[base + k] - cs[base];
        pre += cs[base + span[2]] - cs[base];
      }
    lcs.back() = pre;
    if (pre != total) {
      set_error("grouped scatter tables: region sizes disagree");
      return DSKI_EINVAL;
    }
    for (int q0 = 0; q0 < total; q0 += PMAX) {
      const int q1 = std::min(total, q0 + PMAX);
      list.clear();
      for (int node = 0; node < 256; ++node) {
        const int j[3] = {origin[0] + node / (TS::e1 * TS::e2), origin[1] + (node / TS::e2) % TS::e1,
                          origin[2] + node % TS::e2};
        if (j[0] >= g.m[0] || j[1] >= g.m[1] || j[2] >= g.m[2]) continue;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max(H, j[a] - (S - 1 - H));
          hi[a] = std::min(g.nc[a] + H - 1, j[a] + H);
        }
        for (int c0 = lo[0]; c0 <= hi[0]; ++c0) {
          int work = 0, pts = 0;
          for (int c1 = lo[1]; c1 <= hi[1]; ++c1) {
            const int lrow = (c0 - rlo[0]) * span[1] + (c1 - rlo[1]);
            const int qs = std::max(q0, lcs[(size_t)lrow * span[2] + lo[2] - rlo[2]]);
            const int qe = std::min(q1, lcs[(size_t)lrow * span[2] + hi[2] - rlo[2] + 1]);
            const int cnt = std::max(0, qe - qs);
            pts += cnt;
            work += (cnt + 1) / 2 + 1;
          }
          if (pts > 0) list.push_back({work, node * 8 + (c0 - lo[0])});
        }
      }
      std::sort(list.begin(), list.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
        return x.first != y.first ? x.first > y.first : x.second < y.second;
      });
      for (const auto& w : list) items.push_back((unsigned short)w.second);
      chunk_off.push_back((int)items.size());
      ++nchunks;
    }
  }
  tile_chunk[(size_t)tiles] = nchunks;
  if (items.empty()) items.push_back(0);
  DSKI_HIP(hipMalloc(&p->grp_items, sizeof(unsigned short) * items.size()));
  DSKI_HIP(hipMalloc(&p->grp_chunk_off, sizeof(int) * chunk_off.size()));
  DSKI_HIP(hipMalloc(&p->grp_tile_chunk, sizeof(int) * tile_chunk.size()));
  DSKI_HIP(hipMemcpyAsync(p->grp_items, items.data(), sizeof(unsigned short) * items.size(), hipMemcpyHostToDevice,
                          st));
  DSKI_HIP(hipMemcpyAsync(p->grp_chunk_off, chunk_off.data(), sizeof(int) * chunk_off.size(),
                          hipMemcpyHostToDevice, st));
  DSKI_HIP(hipMemcpyAsync(p->grp_tile_chunk, tile_chunk.data(), sizeof(int) * tile_chunk.size(),
                          hipMemcpyHostToDevice, st));
  DSKI_HIP(hipStreamSynchronize(st));
  return DSKI_OK;
}

// Region tables of the LDS-tiled scatter, built once per plan: pass 1 counts
// every tile's region points, the host forms the offsets, pass 2 fills the
// tables (see k_tile_fill).
template <int D, int S>
static dski_status build_tiles(dski_plan p, hipStream_t st) {
  using TS = TileShape<D, S>;
  GeoK g = geo_of(p);
  long long tiles = 1;
  for (int a = 0; a < D; ++a) tiles *= (g.m[a] + TS::ext(a) - 1) / TS::ext(a);
  std::vector<int> tot((size_t)tiles), off((size_t)tiles + 1);
  int* d_tot = nullptr;
  DSKI_HIP(hipMalloc(&d_tot, sizeof(int) * (size_t)tiles));
  k_tile_count<D, S><<<(unsigned)tiles, 256, 0, st>>>(p->cell_start, g, d_tot);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(tot.data(), d_tot, sizeof(int) * (size_t)tiles, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_tot);
  DSKI_HIP(e);
  long long slots = 0;
  for (long long t = 0; t < tiles; ++t) {
    off[(size_t)t] = (int)slots;
    slots += tot[(size_t)t];
  }
  if (slots > (1ll << 31) - 1) {
    set_error("scatter region tables too large");
    return DSKI_ENOTSUP;
  }
  off[(size_t)tiles] = (int)slots;
  p->tile_slots = slots;
  DSKI_HIP(hipMalloc(&p->tile_off, sizeof(int) * (size_t)(tiles + 1)));
  DSKI_HIP(hipMalloc(&p->tile_lcs, sizeof(int) * (size_t)tiles * (TS::max_cells + 1)));
  DSKI_HIP(hipMalloc(&p->tile_pts, sizeof(int) * (size_t)std::max(slots, 1ll)));
  DSKI_HIP(hipMalloc(&p->tile_cl, sizeof(int) * (size_t)std::max(slots, 1ll)));
  DSKI_HIP(hipMemcpyAsync(p->tile_off, off.data(), sizeof(int) * (size_t)(tiles + 1), hipMemcpyHostToDevice, st));
  k_tile_fill<D, S><<<(unsigned)tiles, 256, 0, st>>>(p->cell, p->cell_start, g, p->tile_off, p->tile_lcs,
                                                     p->tile_pts, p->tile_cl);
  DSKI_HIP(hipGetLastError());
  DSKI_HIP(hipStreamSynchronize(st));
  if constexpr (D == 3) DSKI_TRY(build_groups3<S>(p, g, tiles, off, st));
  return DSKI_OK;
}

template <int S>
static dski_status scatter_tables_s(dski_plan p, hipStream_t st) {
  switch (p->d) {
    case 1: return build_tiles<1, S>(p, st);
    case 2: return build_tiles<2, S>(p, st);
    case 3: return build_tiles<3, S>(p, st);
    default: set_error("d=%d not supported", p->d); return DSKI_ENOTSUP;
  }
}

dski_status scatter_tables(dski_plan p, hipStream_t st) {
  return p->S == kInterpQuintic ? scatter_tables_s<kInterpQuintic>(p, st) : scatter_tables_s<kInterpCubic>(p, st);
}

// ------------------------------------------------------------------ K_UU by FFT
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i (forward, DIR = +1) or +i (inverse, DIR = -1)
template <int DIR>
__device__ __forceinline__ double2 cmi(double2 a) {
  return DIR > 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// 4-point DFT in registers (DIR = +1: e^{-2 pi i/4}, -1: inverse).
template <int DIR>
__device__ __forceinline__ void dft4(double2& a, double2& b, double2& c, double2& d) {
  double2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = cmi<DIR>(csub(b, d));
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}

// 8-point DFT in registers: two 4-point DFTs on even / odd inputs, then the
// twiddles e^{-+2 pi i k/8}.
template <int DIR>
__device__ __forceinline__ void dft8(double2 v[8]) {
  const double h = 0.70710678118654752440;
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // W^1 = (1 -+ i)/sqrt2, W^2 = -+i, W^3 = (-1 -+ i)/sqrt2
  double2 w1o1 = cscale(cadd(o1, cmi<DIR>(o1)), h);
  double2 w2o2 = cmi<DIR>(o2);
  double2 w3o3 = cscale(csub(cmi<DIR>(o3), o3), h);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1o1);
  v[5] = csub(e1, w1o1);
  v[2] = cadd(e2, w2o2);
  v[6] = csub(e2, w2o2);
  v[3] = cadd(e3, w3o3);
  v[7] = csub(e3, w3o3);
}

// LDS position of element i of a line-pair buffer: one pad element per 8, so
// that the stride-8 accesses of the radix-8 passes spread over the banks.
__device__ __forceinline__ int padi(int i) { return i + (i >> 3); }

// Orders the LDS accesses of one wavefront: lanes exchange values through LDS,
// and the LDS operations of a wavefront complete in issue order, so only the
// compiler has to be kept from moving loads and stores across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work-group index remapped so that consecutive logical blocks run on the same
// XCD (the hardware deals work-groups to the 8 XCDs in turn): blocks that share
// cache lines then share one L2.  A bijection on [0, nb).
__device__ __forceinline__ long long xcd_block(unsigned bid, unsigned nb) {
  const unsigned full = nb & ~7u;
  if (bid >= full) return bid;
  return (long long)(bid & 7u) * (full >> 3) + (bid >> 3);
}

// Shape of the line-pair FFT for L = 2^LG: TPL = L / 8 lanes hold one pair of
// real grid lines as one complex sequence, eight values per lane (one radix-8
// butterfly per pass); 256 / TPL pairs per work-group.  Up to L = 512 a pair
// lives in one wavefront (exchanges need only wavefront ordering); beyond it a
// pair spans 2 or 4 wavefronts and exchanges synchronise the work-group, which
// keeps four work-groups (16 wavefronts) per CU at L = 2048 instead of one.
template <int LG>
struct FftShape {
  static constexpr int L = 1 << LG;
  static constexpr int TPL = L / 8;
  static constexpr bool WIDE = TPL > 64;                   // a pair spans several wavefronts
  static constexpr int E = 8;
  static constexpr int NP = fft_npass(LG);
  static constexpr int PAIRS = 256 / TPL;
  static constexpr int NL = 2 * PAIRS;                      // lines per work-group
  static constexpr int LGNL = 12 - LG;                      // log2(NL)
  static constexpr int LP = L + L / 8 + 1;                  // odd: pair buffers start on different banks
  // The Toeplitz product reads its twiddles and spectrum through the caches
  // (every work-group reads the same small tables; staging them in LDS per
  // work-group was slower: one more round trip and a barrier before the FFT).
  // The multi-level (spline) passes stage the twiddles up to L = 512: there a
  // different spectrum row per line streams through the caches beside them.
  static constexpr bool TW_LDS = L <= 512;
  static constexpr int TW = fft_tw_size(LG);
  static constexpr size_t lds_bytes() { return sizeof(double2) * (size_t)PAIRS * LP; }
  static constexpr size_t lds_bytes_tw() { return sizeof(double2) * ((size_t)PAIRS * LP + (TW_LDS ? TW : 0)); }
};

// Orders the LDS accesses of the lanes that share a line pair.
template <int LG>
__device__ __forceinline__ void pair_sync() {
  if constexpr (FftShape<LG>::WIDE)
    __syncthreads();
  else
    wave_lds_sync();
}

// Radix-RAD butterflies of one pass (stride NS, direction DIR) on the values a
// lane holds: v[b RAD + r] is input r of butterfly jj = lane + b TPL, i.e. the
// sequence element jj + r L / RAD.  Inputs r >= 1 take the pass twiddle of
// k = jj mod NS first (none when NS = 1).
template <int LG, int RAD, int NS, int DIR>
__device__ __forceinline__ void fft_butterflies(double2* v, const double2* __restrict__ tw, int lp) {
  using S = FftShape<LG>;
  constexpr int NB = S::L / RAD / S::TPL;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double2* u = v + b * RAD;
    if (NS > 1) {
      const int k = (lp + b * S::TPL) & (NS - 1);
#pragma unroll
      for (int r = 1; r < RAD; ++r) u[r] = cmul(u[r], tw[(r - 1) * NS + k]);
    }
    if (RAD == 8) {
      dft8<DIR>(u);
    } else if (RAD == 4) {
      dft4<DIR>(u[0], u[1], u[2], u[3]);
    } else {
      const double2 a0 = u[0], a1 = u[1];
      u[0] = cadd(a0, a1);
      u[1] = csub(a0, a1);
    }
  }
}

// Stockham hand-over between two passes through the pair's LDS buffer: the
// outputs of pass (RA, NSA) go to (jj / NSA) RA NSA + jj mod NSA + r NSA, and the
// next pass (RB) reads its inputs jj + r L / RB.
template <int LG, int RA, int NSA, int RB>
__device__ __forceinline__ void fft_exchange(double2* v, double2* __restrict__ buf, int lp) {
  using S = FftShape<LG>;
  constexpr int NBA = S::L / RA / S::TPL, NBB = S::L / RB / S::TPL;
#pragma unroll
  for (int b = 0; b < NBA; ++b) {
    const int jj = lp + b * S::TPL;
    const int o = (jj / NSA) * RA * NSA + (jj & (NSA - 1));
#pragma unroll
    for (int r = 0; r < RA; ++r) buf[padi(o + r * NSA)] = v[b * RA + r];
  }
  pair_sync<LG>();
#pragma unroll
  for (int b = 0; b < NBB; ++b)
#pragma unroll
    for (int r = 0; r < RB; ++r) v[b * RB + r] = buf[padi(lp + b * S::TPL + r * (S::L / RB))];
  pair_sync<LG>();
}

// Passes S0.. of one direction; v enters holding the inputs of pass S0.
template <int LG, int DIR, int S0>
__device__ __forceinline__ void fft_run(double2* v, double2* __restrict__ buf, const double2* __restrict__ tw,
                                        int lp) {
  constexpr int NP = fft_npass(LG);
  constexpr int RAD = fft_radix_dir(LG, S0, DIR), NS = fft_ns(LG, S0, DIR);
  fft_butterflies<LG, RAD, NS, DIR>(v, tw + fft_tw_offset(LG, S0, DIR), lp);
  if constexpr (S0 + 1 < NP) {
    fft_exchange<LG, RAD, NS, fft_radix_dir(LG, S0 + 1, DIR)>(v, buf, lp);
    fft_run<LG, DIR, S0 + 1>(v, buf, tw, lp);
  }
}

// Toeplitz product along one axis for all grid lines of R columns.  Each line
// (m values at stride `inner`) is zero-padded to L, transformed, multiplied by
// the circulant eigenvalues `spec` (scaled by 1/L) and transformed back; two
// lines share one complex FFT (real and imaginary parts), which is exact because
// the spectrum is real and even.  One pair per TPL lanes (see FftShape).  The last forward pass leaves element jj + r L / RAD in the
// lane that the first inverse pass (same radix, NS = 1) needs it in, so the
// spectrum is applied in registers between the two; the first forward pass and
// the last inverse pass touch the elements lane + r L / 8, which contiguous
// lines (inner = 1) load and store straight from and to the grid.  Strided
// lines go through LDS with work-group-wide coalesced loads and stores.
template <int LG, typename GT>
__global__ __launch_bounds__(256) void k_toeplitz(GT* __restrict__ G, long long nlines, int m,
                                                  long long inner, const double2* __restrict__ tw,
                                                  const double* __restrict__ spec) {
  using S = FftShape<LG>;
  constexpr int L = S::L, E = S::E, TPL = S::TPL;
  constexpr int R0 = fft_radix_dir(LG, 0, +1);                 // 8
  constexpr int RL = fft_radix_dir(LG, S::NP - 1, +1);         // radix of the last forward pass
  extern __shared__ double2 smem[];
  __shared__ long long s_base[S::NL];
  const int lp = threadIdx.x % TPL;
  const int pair = threadIdx.x / TPL;
  const long long line0 = xcd_block(blockIdx.x, gridDim.x) * S::NL;
  double2* buf = smem + (size_t)pair * S::LP;
  double2 v[E];
  const long long la = line0 + 2 * pair;
  if (inner == 1) {
    const GT* A = G + la * m;
    const bool va = la < nlines, vb = la + 1 < nlines;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = lp + (e / R0) * TPL + (e % R0) * (L / R0);
      const bool in = pos < m;
      v[e] = make_double2(in && va ? (double)A[pos] : 0.0, in && vb ? (double)A[m + pos] : 0.0);
    }
  } else {
    // line bases of the block: line = q inner + r  ->  q m inner + r
    {
      const long long q0 = line0 / inner;
      const unsigned in = (unsigned)inner, r0 = (unsigned)(line0 - q0 * inner);
      for (int l = threadIdx.x; l < S::NL; l += 256) {  // NL is up to 512
        const unsigned rr = r0 + (unsigned)l;
        s_base[l] = line0 + l < nlines ? (q0 + rr / in) * m * inner + rr % in : -1;
      }
    }
    __syncthreads();
    const int tot = S::NL * m;
    for (int f0 = threadIdx.x; f0 < tot; f0 += 2048) {  // eight branch-free loads in flight per thread
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int f = f0 + 256 * u;
        const long long b = f < tot ? s_base[f & (S::NL - 1)] : -1;
        x[u] = (double)ld_or0(G, (size_t)(b + (long long)(f >> S::LGNL) * inner), 0, b >= 0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int f = f0 + 256 * u;
        if (f < tot) {
          const int l = f & (S::NL - 1);
          reinterpret_cast<double*>(&smem[(size_t)(l >> 1) * S::LP + padi(f >> S::LGNL)])[l & 1] = x[u];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = lp + (e / R0) * TPL + (e % R0) * (L / R0);
      v[e] = pos < m ? buf[padi(pos)] : make_double2(0.0, 0.0);
    }
    pair_sync<LG>();
  }
  fft_run<LG, +1, 0>(v, buf, tw, lp);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cscale(v[e], spec[lp + (e / RL) * TPL + (e % RL) * (L / RL)]);
  fft_run<LG, -1, 0>(v, buf, tw, lp);
  if (inner == 1) {
    GT* A = G + la * m;
    const bool va = la < nlines, vb = la + 1 < nlines;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = lp + (e / R0) * TPL + (e % R0) * (L / R0);
      if (pos < m) {
        if (va) A[pos] = (GT)v[e].x;
        if (vb) A[m + pos] = (GT)v[e].y;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = lp + (e / R0) * TPL + (e % R0) * (L / R0);
      if (pos < m) buf[padi(pos)] = v[e];
    }
    __syncthreads();
    const int tot = S::NL * m;
    for (int f = threadIdx.x; f < tot; f += 256) {
      const int l = f & (S::NL - 1);
      const long long b = s_base[l];
      if (b >= 0)
        G[b + (long long)(f >> S::LGNL) * inner] =
            (GT)reinterpret_cast<const double*>(&smem[(size_t)(l >> 1) * S::LP + padi(f >> S::LGNL)])[l & 1];
    }
  }
}

template <int LG, typename GT>
static dski_status launch_toeplitz(GT* G, long long nlines, int m, long long inner, const double2* tw,
                                   const double* spec, hipStream_t st) {
  using S = FftShape<LG>;
  static_assert(S::lds_bytes() <= 160 * 1024, "LDS");
  static_assert(S::NL == 1 << S::LGNL, "lines per block");
  const size_t sh = S::lds_bytes();
  if (sh > 64 * 1024) {
    static bool done = false;
    if (!done) {
      DSKI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_toeplitz<LG, GT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
      done = true;
    }
  }
  const long long blocks = (nlines + S::NL - 1) / S::NL;
  k_toeplitz<LG, GT><<<(unsigned)blocks, 256, sh, st>>>(G, nlines, m, inner, tw, spec);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// Dense Toeplitz product along one axis on the FP64 matrix cores: for 16 grid
// lines at a time,  Y (m x 16) = T (m x m) X,  T[a][b] = c(|a - b|) with
// c(k) = scale * col[k] (and, for the length-scale derivative, times (k h / ell)^2).
// The 16 lines are staged in LDS (rows padded to a multiple of 4 with zeros);
// each wavefront owns row tiles of 16 and accumulates over b in steps of 4 with
// v_mfma_f64_16x16x4f64 (operands: lane l holds T[a0 + l%16][b0 + l/16] and
// X[b0 + l/16][l%16]; the 16 x 16 result sits in 4 doubles per lane: register r
// of lane l is row l/16 + 4 r, column l%16); the row tiles of a wavefront run
// as independent accumulator chains.
// Results go back through LDS so that the stores follow the memory layout.
// Exact up to rounding; O(m^2) per line against O(L log L) for the FFT, which
// the per-axis tuner weighs.  m <= kDenseMaxM.
typedef double dski_dbl4 __attribute__((ext_vector_type(4)));

template <int NT, typename GT>  // row tiles per wavefront: 4 NT >= ceil(m / 16)
__global__ __launch_bounds__(256) void k_toeplitz_mfma(GT* __restrict__ G, long long nlines, int m,
                                                       long long inner, const double* __restrict__ col,
                                                       double scale, int deriv, double h_over_ell) {
  extern __shared__ double smem_d[];
  __shared__ long long s_base[16];
  const int mp = (m + 3) & ~3;
  double* sX = smem_d;               // mp rows of 16 lines, row stride 17 (banks)
  double* scol = smem_d + (size_t)mp * 17;  // m
  const long long line0 = (long long)blockIdx.x * 16;
  for (int k = threadIdx.x; k < m; k += 256) {
    double v = col[k] * scale;
    if (deriv) {
      const double t = (double)k * h_over_ell;
      v *= t * t;
    }
    scol[k] = v;
  }
  if (threadIdx.x < 16) {
    const long long line = line0 + threadIdx.x;
    s_base[threadIdx.x] = line < nlines ? (line / inner) * ((long long)m * inner) + line % inner : -1;
  }
  __syncthreads();
  const int tot = mp * 16;
  for (int f0 = threadIdx.x; f0 < tot; f0 += 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + 256 * u;
      int l, bb;
      if (inner > 1) {
        l = f % 16;
        bb = f / 16;
      } else {
        bb = f % mp;
        l = f / mp;
      }
      const long long base = f < tot ? s_base[l] : -1;
      v[u] = (base >= 0 && bb < m) ? (double)G[base + (long long)bb * inner] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + 256 * u;
      if (f < tot) {
        const int l = inner > 1 ? f % 16 : f / mp;
        const int bb = inner > 1 ? f / 16 : f % mp;
        sX[bb * 17 + l] = v[u];
      }
    }
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ntiles = (m + 15) / 16;
  // all row tiles of this wavefront advance together: independent accumulator
  // chains that share the X operand of each step.  No branches: rows of X at or
  // beyond m are zero and output rows at or beyond m are discarded, so the
  // Toeplitz index only needs clamping to stay inside the column.
  dski_dbl4 res[NT];
  int arow[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    res[q] = dski_dbl4{0.0, 0.0, 0.0, 0.0};
    arow[q] = (wv + 4 * q) * 16 + r16;
  }
#pragma unroll 2
  for (int k0 = 0; k0 < mp; k0 += 4) {
    const int b = k0 + kq;
    const double xv = sX[b * 17 + r16];
    double av[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int dd = arow[q] > b ? arow[q] - b : b - arow[q];
      av[q] = scol[dd < m ? dd : m - 1];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) res[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], xv, res[q], 0, 0, 0);
  }
  __syncthreads();  // every wavefront has read sX
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int tile = wv + 4 * q;
    if (tile < ntiles) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = tile * 16 + kq + 4 * r;
        if (a < m) sX[a * 17 + r16] = res[q][r];
      }
    }
  }
  __syncthreads();
  const int totm = m * 16;
  for (int f = threadIdx.x; f < totm; f += 256) {
    const int l = inner > 1 ? f % 16 : f / m;
    const int bb = inner > 1 ? f / 16 : f % m;
    const long long base = s_base[l];
    if (base >= 0) G[base + (long long)bb * inner] = (GT)sX[bb * 17 + l];
  }
}

// K_UU factor of one axis (stride `inner`) for R columns, FFT (variant 0) or
// dense matrix-core product (variant 1, m <= kDenseMaxM).
template <typename GT>
dski_status kuu_axis(dski_plan p, int R, GT* G, hipStream_t st, int dwhich, int a, int variant) {
  const Axis& A = p->ax[a];
  long long inner = 1;
  for (int b = a + 1; b < p->d; ++b) inner *= p->ax[b].m;
  const long long nlines = (long long)R * (p->M / A.m);
  if (variant == 1 && A.m <= kDenseMaxM) {
    const int mp = (A.m + 3) & ~3;
    const size_t sh = sizeof(double) * ((size_t)mp * 17 + A.m);
    const double scale = a == 0 ? p->s * p->s : 1.0;
    const unsigned nb = (unsigned)((nlines + 15) / 16);
    const int nt = ((A.m + 15) / 16 + 3) / 4;
    const int dv = a == dwhich ? 1 : 0;
    const double hl = A.h / p->ell[a];
    switch (nt) {
      case 1: k_toeplitz_mfma<1, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      case 2: k_toeplitz_mfma<2, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      case 3: k_toeplitz_mfma<3, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      case 4: k_toeplitz_mfma<4, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      case 5: k_toeplitz_mfma<5, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      case 6: k_toeplitz_mfma<6, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
      default: k_toeplitz_mfma<7, GT><<<nb, 256, sh, st>>>(G, nlines, A.m, inner, A.col, scale, dv, hl); break;
    }
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  }
  const double* spec = (a == dwhich) ? A.dspec : A.spec;
  const double2* tw = reinterpret_cast<const double2*>(A.twiddle);
  switch (A.L) {
    case 8: return launch_toeplitz<3, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 16: return launch_toeplitz<4, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 32: return launch_toeplitz<5, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 64: return launch_toeplitz<6, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 128: return launch_toeplitz<7, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 256: return launch_toeplitz<8, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 512: return launch_toeplitz<9, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 1024: return launch_toeplitz<10, GT>(G, nlines, A.m, inner, tw, spec, st);
    case 2048: return launch_toeplitz<11, GT>(G, nlines, A.m, inner, tw, spec, st);
    default:
      set_error("FFT length %d not supported (grid size per axis 4..1024)", A.L);
      return DSKI_ENOTSUP;
  }
}

template dski_status kuu_axis<double>(dski_plan, int, double*, hipStream_t, int, int, int);

// ------------------------------------------------------------------ K_UU of the spline kernel
// The spline kernel (App. A) is not a product kernel: K_UU is a symmetric
// multi-level Toeplitz matrix (block Toeplitz with Toeplitz blocks in 2-D),
// applied through its d-dimensional circulant embedding of size L_0 x .. x
// L_{d-1} (the per-axis FFT lengths, L_p >= 2 m_p - 1):
//   K_UU G = crop( F^{-1} diag(lambda) F pad(G) ),  lambda = F c,
// with c the embedded generating array (kernel values at the node offsets,
// wrapped, zero outside the band).  lambda is real (c is even on every axis),
// so two real grid columns travel as the real and imaginary parts of one
// complex array.  The transform runs axis by axis with the line FFT of the
// separable case (radix-8 Stockham passes in registers, LDS exchanges):
// forward on axes 0 .. d-2, forward * lambda * inverse on the last
// (contiguous) axis in one kernel, inverse on axes d-2 .. 0.

// Natural position of value e of lane lp (input of a forward transform, output
// of an inverse one), and the frequency it holds after the last forward pass
// (input of the first inverse pass).
template <int LG>
__device__ __forceinline__ int fft_pos_nat(int lp, int e) {
  using S = FftShape<LG>;
  constexpr int R0 = fft_radix_dir(LG, 0, +1);
  return lp + (e / R0) * S::TPL + (e % R0) * (S::L / R0);
}
template <int LG>
__device__ __forceinline__ int fft_pos_freq(int lp, int e) {
  using S = FftShape<LG>;
  constexpr int RL = fft_radix_dir(LG, S::NP - 1, +1);
  return lp + (e / RL) * S::TPL + (e % RL) * (S::L / RL);
}

// The lines an axis pass transforms: line l = (outer index o, inner index i)
// with o = l / ninner over every position of the axes before the axis (and the
// stacked arrays), i = l % ninner over a box of the axes after it, given per
// axis (slowest first) by its count and its stride in the array.  The line
// starts at o * outer_step + sum of digit * stride and steps by `step`; its
// positions from `valid` on are read as zeros (the padding of the embedding,
// which is then never stored).
struct LineMap {
  long long ninner, outer_step, step;
  int nd, valid;
  int cnt[DSKI_MAXD];
  long long stride[DSKI_MAXD];
};

// One complex FFT (DIR = +1 forward, -1 inverse, unnormalised) of each line of
// length L = 2^LG that `map` selects.  A forward transform reads natural order
// and writes frequency order; an inverse one the reverse.  In place (a
// work-group holds its lines in registers between the read and the write).
template <int LG, int DIR>
__global__ __launch_bounds__(256) void k_fft_axis(double2* __restrict__ Z, long long nlines, LineMap map,
                                                  const double2* __restrict__ tw) {
  using S = FftShape<LG>;
  constexpr int E = S::E, TPL = S::TPL, L = S::L;
  extern __shared__ double2 smem[];
  const int lp = threadIdx.x % TPL;
  const int slot = threadIdx.x / TPL;
  double2* buf = smem + (size_t)slot * S::LP;
  const double2* stw = tw;
  if constexpr (S::TW_LDS) {
    double2* t = smem + (size_t)S::PAIRS * S::LP;
    for (int f = threadIdx.x; f < S::TW; f += 256) t[f] = tw[f];
    stw = t;
    __syncthreads();
  }
  const long long line = (long long)blockIdx.x * S::PAIRS + slot;
  const bool ok = line < nlines;
  long long base = 0;
  if (ok) {
    long long rem = line % map.ninner;
    base = (line / map.ninner) * map.outer_step;
    for (int t = map.nd - 1; t >= 0; --t) {
      base += (rem % map.cnt[t]) * map.stride[t];
      rem /= map.cnt[t];
    }
  }
  const long long step = map.step;
  double2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = DIR > 0 ? fft_pos_nat<LG>(lp, e) : fft_pos_freq<LG>(lp, e);
    v[e] = ok && pos < map.valid ? Z[base + (long long)pos * step] : make_double2(0.0, 0.0);
  }
  fft_run<LG, DIR, 0>(v, buf, stw, lp);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = DIR > 0 ? fft_pos_freq<LG>(lp, e) : fft_pos_nat<LG>(lp, e);
      Z[base + (long long)pos * step] = v[e];
    }
  }
}

// Last (contiguous) axis: forward, times lambda (row o = l mod nouter of the
// spectrum, L values), inverse.  Positions from `valid` on are read as zeros.
template <int LG>
__global__ __launch_bounds__(256) void k_fft_last_spec(double2* __restrict__ Z, long long nlines, long long nouter,
                                                       int valid, const double2* __restrict__ tw,
                                                       const double* __restrict__ spec) {
  using S = FftShape<LG>;
  constexpr int E = S::E, TPL = S::TPL, L = S::L;
  extern __shared__ double2 smem[];
  const int lp = threadIdx.x % TPL;
  const int slot = threadIdx.x / TPL;
  double2* buf = smem + (size_t)slot * S::LP;
  const double2* stw = tw;
  if constexpr (S::TW_LDS) {
    double2* t = smem + (size_t)S::PAIRS * S::LP;
    for (int f = threadIdx.x; f < S::TW; f += 256) t[f] = tw[f];
    stw = t;
    __syncthreads();
  }
  const long long line = (long long)blockIdx.x * S::PAIRS + slot;
  const bool ok = line < nlines;
  double2* A = Z + (ok ? line : 0) * L;
  const double* sp = spec + (ok ? line % nouter : 0) * L;
  double2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = fft_pos_nat<LG>(lp, e);
    v[e] = ok && pos < valid ? A[pos] : make_double2(0.0, 0.0);
  }
  fft_run<LG, +1, 0>(v, buf, stw, lp);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cscale(v[e], sp[fft_pos_freq<LG>(lp, e)]);
  fft_run<LG, -1, 0>(v, buf, stw, lp);
  if (ok) {
#pragma unroll
    for (int e = 0; e < E; ++e) A[fft_pos_nat<LG>(lp, e)] = v[e];
  }
}

struct BoxL {
  int d;
  int m[DSKI_MAXD], L[DSKI_MAXD];
  double h[DSKI_MAXD];
};

static BoxL box_of(dski_plan p) {
  BoxL b{};
  b.d = p->d;
  for (int a = 0; a < p->d; ++a) {
    b.m[a] = p->ax[a].m;
    b.L[a] = p->ax[a].L;
    b.h[a] = p->ax[a].h;
  }
  return b;
}

// Spline kernel profile k(r) / s^2 (App. A; a, b as in the header: domain size R).
__device__ __forceinline__ double spline_profile(double r, int d, double R) {
  if (d & 1) return r * r * r - 1.5 * R * r * r + 0.5 * R * R * R;
  const double rl = r > 0.0 ? r * r * log(r) : 0.0;
  return rl - 0.5 * (1.0 + 2.0 * log(R)) * r * r + 0.5 * R * R;
}

// Generating array of the circulant embedding: offset j_p (wrapped) on every
// axis, zero outside the band |offset| < m_p.
__global__ void k_bttb_gen(BoxL b, double R, long long tot, double2* __restrict__ Z) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < tot;
       j += (long long)gridDim.x * blockDim.x) {
    long long rem = j;
    double r2 = 0.0;
    bool band = true;
    for (int a = b.d - 1; a >= 0; --a) {
      const int ja = (int)(rem % b.L[a]);
      rem /= b.L[a];
      const int off = ja < b.m[a] ? ja : (ja > b.L[a] - b.m[a] ? b.L[a] - ja : -1);
      band = band && off >= 0;
      const double x = (double)off * b.h[a];
      r2 += x * x;
    }
    Z[j] = make_double2(band ? spline_profile(sqrt(r2), b.d, R) : 0.0, 0.0);
  }
}

__global__ void k_bttb_spec(const double2* __restrict__ Z, long long tot, double scale, double* __restrict__ spec) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < tot;
       j += (long long)gridDim.x * blockDim.x)
    spec[j] = Z[j].x * scale;
}

// Embedded position (last axis fastest, L box) of grid node `node` (m box).
__device__ __forceinline__ long long bttb_pos(long long node, const BoxL& b) {
  long long rem = node, j = 0, stride = 1;
  for (int a = b.d - 1; a >= 0; --a) {
    j += (rem % b.m[a]) * stride;
    rem /= b.m[a];
    stride *= b.L[a];
  }
  return j;
}

// Z[c2] = G[2 c2] + i G[2 c2 + 1] on the m box.  The rest of the embedded
// array is not written: the transforms read it as zeros.
__global__ void k_bttb_pack(const double* __restrict__ G, long long M, int R, BoxL b, long long tot,
                            double2* __restrict__ Z) {
  const int c2 = blockIdx.y;
  const int ca = 2 * c2, cb = 2 * c2 + 1;
  for (long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x; node < M;
       node += (long long)gridDim.x * blockDim.x) {
    double2 v;
    v.x = G[(size_t)ca * M + node];
    v.y = cb < R ? G[(size_t)cb * M + node] : 0.0;
    Z[(size_t)c2 * tot + bttb_pos(node, b)] = v;
  }
}

// G[2 c2] = scale Re Z[c2], G[2 c2 + 1] = scale Im Z[c2] on the m box.
__global__ void k_bttb_unpack(const double2* __restrict__ Z, long long M, int R, BoxL b, long long tot,
                              double scale, double* __restrict__ G) {
  const int c2 = blockIdx.y;
  const int ca = 2 * c2, cb = 2 * c2 + 1;
  for (long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x; node < M;
       node += (long long)gridDim.x * blockDim.x) {
    const double2 v = Z[(size_t)c2 * tot + bttb_pos(node, b)];
    G[(size_t)ca * M + node] = scale * v.x;
    if (cb < R) G[(size_t)cb * M + node] = scale * v.y;
  }
}

template <int LG, int DIR>
static dski_status launch_fft_axis(double2* Z, long long nlines, const LineMap& map, const double2* tw,
                                   hipStream_t st) {
  using S = FftShape<LG>;
  const size_t sh = S::lds_bytes_tw();
  if (sh > 64 * 1024) {
    static bool done = false;
    if (!done) {
      DSKI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_axis<LG, DIR>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
      done = true;
    }
  }
  const long long blocks = (nlines + S::PAIRS - 1) / S::PAIRS;
  k_fft_axis<LG, DIR><<<(unsigned)blocks, 256, sh, st>>>(Z, nlines, map, tw);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

template <int LG>
static dski_status launch_fft_last(double2* Z, long long nlines, long long nouter, int valid, const double2* tw,
                                   const double* spec, hipStream_t st) {
  using S = FftShape<LG>;
  const size_t sh = S::lds_bytes_tw();
  if (sh > 64 * 1024) {
    static bool done = false;
    if (!done) {
      DSKI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_last_spec<LG>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
      done = true;
    }
  }
  const long long blocks = (nlines + S::PAIRS - 1) / S::PAIRS;
  k_fft_last_spec<LG><<<(unsigned)blocks, 256, sh, st>>>(Z, nlines, nouter, valid, tw, spec);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

static int log2_exact(int L) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  return lg;
}

static dski_status fft_axis(double2* Z, int L, int dir, long long nlines, const LineMap& map, const double2* tw,
                            hipStream_t st) {
#define DSKI_FA(LGV)                                                                          \
  case LGV:                                                                                   \
    return dir > 0 ? launch_fft_axis<LGV, +1>(Z, nlines, map, tw, st)                         \
                   : launch_fft_axis<LGV, -1>(Z, nlines, map, tw, st);
  switch (log2_exact(L)) {
    DSKI_FA(3)
    DSKI_FA(4)
    DSKI_FA(5)
    DSKI_FA(6)
    DSKI_FA(7)
    DSKI_FA(8)
    DSKI_FA(9)
    DSKI_FA(10)
    DSKI_FA(11)
    default:
      set_error("FFT length %d not supported", L);
      return DSKI_ENOTSUP;
  }
#undef DSKI_FA
}

static dski_status fft_last(double2* Z, int L, long long nlines, long long nouter, int valid, const double2* tw,
                            const double* spec, hipStream_t st) {
  switch (log2_exact(L)) {
    case 3: return launch_fft_last<3>(Z, nlines, nouter, valid, tw, spec, st);
    case 4: return launch_fft_last<4>(Z, nlines, nouter, valid, tw, spec, st);
    case 5: return launch_fft_last<5>(Z, nlines, nouter, valid, tw, spec, st);
    case 6: return launch_fft_last<6>(Z, nlines, nouter, valid, tw, spec, st);
    case 7: return launch_fft_last<7>(Z, nlines, nouter, valid, tw, spec, st);
    case 8: return launch_fft_last<8>(Z, nlines, nouter, valid, tw, spec, st);
    case 9: return launch_fft_last<9>(Z, nlines, nouter, valid, tw, spec, st);
    case 10: return launch_fft_last<10>(Z, nlines, nouter, valid, tw, spec, st);
    case 11: return launch_fft_last<11>(Z, nlines, nouter, valid, tw, spec, st);
    default:
      set_error("FFT length %d not supported", L);
      return DSKI_ENOTSUP;
  }
}

static long long bttb_total(dski_plan p) {
  long long tot = 1;
  for (int a = 0; a < p->d; ++a) tot *= p->ax[a].L;
  return tot;
}

// Lines along axis a of `stack` embedded arrays (last axis fastest): every
// position of the axes before a, and on the axes after it either every position
// (full) or only the first m_b (the grid box).  Restricting a forward pass so
// skips lines that are still all zero (the box was padded with zeros and no
// pass has touched the later axes yet: their transforms would be exact zeros);
// restricting an inverse pass skips lines whose outputs the crop to the box
// discards.  Either way the values the crop keeps are the same bits.
static LineMap line_map(dski_plan p, int a, long long stack, bool box, long long* nlines) {
  LineMap m{};
  long long inner_full = 1;
  for (int b = p->d - 1; b > a; --b) inner_full *= p->ax[b].L;
  m.step = inner_full;
  m.outer_step = inner_full * p->ax[a].L;
  m.valid = p->ax[a].L;
  long long outer = stack;
  for (int b = 0; b < a; ++b) outer *= p->ax[b].L;
  m.nd = 0;
  m.ninner = 1;
  long long stride = inner_full;
  for (int b = a + 1; b < p->d; ++b) {
    stride /= p->ax[b].L;
    m.cnt[m.nd] = box ? p->ax[b].m : p->ax[b].L;
    m.stride[m.nd] = stride;
    m.ninner *= m.cnt[m.nd];
    ++m.nd;
  }
  *nlines = outer * m.ninner;
  return m;
}

// Spectrum of the spline kernel's K_UU (without s^2): lambda / prod L_p, in
// the natural frequency order of the embedded array.  Independent of the
// hyper-parameters (s enters as a factor at application).
dski_status bttb_build_spectrum(dski_plan p, hipStream_t st) {
  const long long tot = bttb_total(p);
  double R2 = 0.0;
  for (int a = 0; a < p->d; ++a) {
    const double ext = (p->ax[a].m - 1) * p->ax[a].h;
    R2 += ext * ext;
  }
  p->spline_R = 2.0 * std::sqrt(R2);
  if (!p->bttb_spec) DSKI_HIP(hipMalloc(&p->bttb_spec, sizeof(double) * (size_t)tot));
  DevBuf work;
  DSKI_TRY(work.reserve(sizeof(double2) * (size_t)tot));
  double2* Z = work.as<double2>();
  BoxL b = box_of(p);
  const unsigned nb = (unsigned)std::min<long long>(4096, (tot + 255) / 256);
  k_bttb_gen<<<nb, 256, 0, st>>>(b, p->spline_R, tot, Z);
  DSKI_HIP(hipGetLastError());
  for (int a = p->d - 1; a >= 0; --a) {
    long long nl = 0;
    const LineMap map = line_map(p, a, 1, false, &nl);
    DSKI_TRY(fft_axis(Z, p->ax[a].L, +1, nl, map, reinterpret_cast<const double2*>(p->ax[a].twiddle), st));
  }
  // the last-axis kernel expects each spectrum row in natural frequency order
  // too, so this is lambda in the layout both passes index
  k_bttb_spec<<<nb, 256, 0, st>>>(Z, tot, 1.0 / (double)tot, p->bttb_spec);
  DSKI_HIP(hipGetLastError());
  DSKI_HIP(hipStreamSynchronize(st));
  work.release();
  return DSKI_OK;
}

// G <- s^2 K_spl G for R FP64 grid columns.
static dski_status bttb_apply(dski_plan p, int R, double* G, hipStream_t st, double scale) {
  const long long tot = bttb_total(p);
  const int R2 = (R + 1) / 2;
  DSKI_TRY(p->bttb_work.reserve(sizeof(double2) * (size_t)tot * R2));
  double2* Z = p->bttb_work.as<double2>();
  BoxL b = box_of(p);
  const unsigned nb = (unsigned)std::min<long long>(2048, (p->M + 255) / 256);
  k_bttb_pack<<<dim3(nb, R2), 256, 0, st>>>(G, p->M, R, b, tot, Z);
  DSKI_HIP(hipGetLastError());
  const int d = p->d;
  // all R2 arrays stacked; forward passes on axes 0 .. d-2 over the lines whose
  // later axes lie in the grid box (each reading past m_a as zeros: the pack
  // wrote only the box), inverse passes over the lines the crop keeps
  const long long lines_of = tot * R2;
  for (int a = 0; a < d - 1; ++a) {
    long long nl = 0;
    LineMap map = line_map(p, a, R2, true, &nl);
    map.valid = p->ax[a].m;
    DSKI_TRY(fft_axis(Z, p->ax[a].L, +1, nl, map, reinterpret_cast<const double2*>(p->ax[a].twiddle), st));
  }
  const int Ll = p->ax[d - 1].L;
  DSKI_TRY(fft_last(Z, Ll, lines_of / Ll, tot / Ll, p->ax[d - 1].m,
                    reinterpret_cast<const double2*>(p->ax[d - 1].twiddle), p->bttb_spec, st));
  for (int a = d - 2; a >= 0; --a) {
    long long nl = 0;
    const LineMap map = line_map(p, a, R2, true, &nl);
    DSKI_TRY(fft_axis(Z, p->ax[a].L, -1, nl, map, reinterpret_cast<const double2*>(p->ax[a].twiddle), st));
  }
  k_bttb_unpack<<<dim3(nb, R2), 256, 0, st>>>(Z, p->M, R, b, tot, scale, G);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// G <- K_UU G for R columns; dwhich = p (0..d-1) uses d T_p / dlog ell_p on axis p.
// Every transform computes in FP64 whatever the grid's storage type GT.
template <typename GT>
dski_status apply_kuu(dski_plan p, int R, GT* G, hipStream_t st, int dwhich) {
  if (R <= 0) return DSKI_OK;
  if (p->kernel == kKernelSpline) {
    if constexpr (std::is_same<GT, double>::value) {
      // no length scale: a derivative along one is zero
      return bttb_apply(p, R, G, st, dwhich >= 0 && dwhich < p->d ? 0.0 : p->s * p->s);
    } else {
      set_error("spline kernel: FP64 grids only");
      return DSKI_ENOTSUP;
    }
  }
  for (int a = 0; a < p->d; ++a) DSKI_TRY(kuu_axis<GT>(p, R, G, st, dwhich, a, p->kuu_variant[a]));
  return DSKI_OK;
}
template dski_status apply_kuu<double>(dski_plan, int, double*, hipStream_t, int);

// ------------------------------------------------------------------ gather + noise
// One thread per (point, group of CG columns): the point's weights are formed
// once for the group (interp_weights<S> from its offsets, as in the scatter),
// the S^d grid values of each column give the value and all d derivative rows.
// Y = S G + D V with FP64 accumulation; optional per-block partials of V.Y per
// column (p^T q of CG), stored output-major: pq_partial[column * blocks +
// block].  The 1-D grid is laid out so that all column groups of one block of
// points run on the same XCD (the hardware deals work-groups to the 8 XCDs in
// turn): the points' offsets are fetched into one L2.  The number of point
// blocks is padded to a multiple of 8; padded blocks write zero partials.
// The S x S grid values of one stencil plane are loaded together before they
// are combined (S^d values for d <= 2, one plane at a time in 3-D).
template <int D, int S, int CG, typename T, typename GT>
__global__ __launch_bounds__(256) void k_gather(const int* __restrict__ cell,
                                                const double* __restrict__ toff, int n, GeoK g,
                                                const GT* __restrict__ G, long long M,
                                                const T* __restrict__ V, int ldv,
                                                T* __restrict__ Y, int ldy, int R, int ngy, double nv,
                                                double ng, double* __restrict__ pq_partial) {
  constexpr int H = S / 2 - 1;
  const unsigned bid = blockIdx.x, xcd = bid & 7u, sq = bid >> 3;
  const int bx = (int)(xcd + 8u * (sq / (unsigned)ngy));   // point block
  const int r0 = (int)(sq % (unsigned)ngy) * CG;          // first column of the group
  const int nbx = (int)(gridDim.x / (unsigned)ngy);       // point blocks (multiple of 8)
  const int k = bx * 256 + threadIdx.x;
  double dot[CG];
#pragma unroll
  for (int j = 0; j < CG; ++j) dot[j] = 0.0;
  if (k < n) {
    double w[D][S], dw[D][S];
    int c[D];
    int rem = cell[k];
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      c[a] = rem % g.nc[a];      // first stencil node (anchor - H)
      rem /= g.nc[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) interp_weights<S>(toff[(size_t)a * n + k], g.invh[a], w[a], dw[a]);
    long long base = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) base = base * g.m[a] + c[a];
    long long stride[D];
    stride[D - 1] = 1;
#pragma unroll
    for (int a = D - 2; a >= 0; --a) stride[a] = stride[a + 1] * g.m[a + 1];
    T vin_t[CG][D + 1];
#pragma unroll
    for (int j = 0; j < CG; ++j)
#pragma unroll
      for (int q = 0; q <= D; ++q)
        vin_t[j][q] = ld_or0(V, (size_t)(r0 + j) * ldv + (size_t)q * n + k, (size_t)r0 * ldv + (size_t)q * n + k,
                             r0 + j < R);
    double acc[CG][D + 1];
#pragma unroll
    for (int j = 0; j < CG; ++j)
#pragma unroll
      for (int q = 0; q <= D; ++q) acc[j][q] = 0.0;
    if constexpr (D <= 2) {
      constexpr int NG = D == 1 ? S : S * S;
      double gv[CG][NG];
#pragma unroll
      for (int j = 0; j < CG; ++j) {
        const bool ok = r0 + j < R;
        const GT* Gr = G + (size_t)(ok ? r0 + j : r0) * M + base;
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          const long long off = D == 1 ? f : (f / S) * stride[0] + (f % S);
          gv[j][f] = ok ? (double)Gr[off] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < CG; ++j) {
        if constexpr (D == 1) {
#pragma unroll
          for (int o0 = 0; o0 < S; ++o0) {
            acc[j][0] += w[0][o0] * gv[j][o0];
            acc[j][1] += dw[0][o0] * gv[j][o0];
          }
        } else {
#pragma unroll
          for (int o0 = 0; o0 < S; ++o0) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int o1 = 0; o1 < S; ++o1) {
              const double x = gv[j][o0 * S + o1];
              s0 += w[1][o1] * x;
              s1 += dw[1][o1] * x;
            }
            acc[j][0] += w[0][o0] * s0;
            acc[j][1] += dw[0][o0] * s0;
            acc[j][2] += w[0][o0] * s1;
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < CG; ++j) {
        const bool ok = r0 + j < R;
        const GT* Gr = G + (size_t)(ok ? r0 + j : r0) * M + base;
#pragma unroll
        for (int o0 = 0; o0 < S; ++o0) {
          double gv[S * S];
#pragma unroll
          for (int f = 0; f < S * S; ++f)
            gv[f] = ok ? (double)Gr[o0 * stride[0] + (f / S) * stride[1] + (f % S)] : 0.0;
          double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
          for (int o1 = 0; o1 < S; ++o1) {
            double s0 = 0.0, s2 = 0.0;
#pragma unroll
            for (int o2 = 0; o2 < S; ++o2) {
              const double x = gv[o1 * S + o2];
              s0 += w[2][o2] * x;
              s2 += dw[2][o2] * x;
            }
            t0 += w[1][o1] * s0;
            t1 += dw[1][o1] * s0;
            t2 += w[1][o1] * s2;
          }
          acc[j][0] += w[0][o0] * t0;
          acc[j][1] += dw[0][o0] * t0;
          acc[j][2] += w[0][o0] * t1;
          acc[j][3] += w[0][o0] * t2;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CG; ++j) {
      if (r0 + j < R) {
        T* yy = Y + (size_t)(r0 + j) * ldy + k;
#pragma unroll
        for (int q = 0; q <= D; ++q) {
          const double vin = (double)vin_t[j][q];
          const T out = (T)(acc[j][q] + (q == 0 ? nv : ng) * vin);
          __builtin_nontemporal_store(out, &yy[(size_t)q * n]);
          dot[j] += vin * (double)out;
        }
      }
    }
  }
  if (pq_partial) {
    __shared__ double red[CG][4];
#pragma unroll
    for (int j = 0; j < CG; ++j) {
      double d = dot[j];
      for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
      if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = d;
    }
    __syncthreads();
    if (threadIdx.x < CG && r0 + (int)threadIdx.x < R) {
      const int j = threadIdx.x;
      pq_partial[(size_t)(r0 + j) * nbx + bx] = red[j][0] + red[j][1] + red[j][2] + red[j][3];
    }
  }
}

static int gather_point_blocks(dski_plan p) { return (((p->n + 255) / 256) + 7) & ~7; }
int gather_blocks(dski_plan p) { return p->kind == 1 ? (p->N + 255) / 256 : gather_point_blocks(p); }

template <int D, int S, int CG, typename T, typename GT>
static void launch_gather_cg(dski_plan p, int R, const GT* G, const T* V, int ldv, T* Y, int ldy, double nv,
                             double ng, double* pq_partial, hipStream_t st) {
  GeoK g = geo_of(p);
  const int ngy = (R + CG - 1) / CG;
  const unsigned nb = (unsigned)(gather_point_blocks(p) * ngy);
  k_gather<D, S, CG, T, GT><<<nb, 256, 0, st>>>(p->cell, p->toff, p->n, g, G, p->M, V, ldv, Y, ldy, R, ngy, nv,
                                                ng, pq_partial);
}

template <int D, int S, typename T, typename GT>
static void launch_gather(dski_plan p, int R, const GT* G, const T* V, int ldv, T* Y, int ldy,
                          double nv, double ng, double* pq_partial, hipStream_t st) {
  if constexpr (D == 3) {  // S^3 grid values per column: one column per thread
    launch_gather_cg<D, S, 1, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st);
  } else {
    switch (p->gather_variant) {
      case 1: launch_gather_cg<D, S, 1, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
      case 2: launch_gather_cg<D, S, 4, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
      default: launch_gather_cg<D, S, 2, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
    }
  }
}

template <int S, typename T, typename GT>
static dski_status gather_s(dski_plan p, int R, const GT* G, const T* V, int ldv, T* Y, int ldy, double nv,
                            double ng, double* pq_partial, hipStream_t st) {
  switch (p->d) {
    case 1: launch_gather<1, S, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
    case 2: launch_gather<2, S, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
    case 3: launch_gather<3, S, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st); break;
    default: set_error("d=%d not supported", p->d); return DSKI_ENOTSUP;
  }
  return DSKI_OK;
}

template <typename T, typename GT>
dski_status gather(dski_plan p, int R, const GT* G, const T* V, int ldv, T* Y, int ldy, double nv,
                   double ng, double* pq_partial, hipStream_t st) {
  if (R <= 0 || p->n == 0) return DSKI_OK;
  DSKI_TRY((p->S == kInterpQuintic
                ? gather_s<kInterpQuintic, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st)
                : gather_s<kInterpCubic, T, GT>(p, R, G, V, ldv, Y, ldy, nv, ng, pq_partial, st)));
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}
template dski_status gather<float, double>(dski_plan, int, const double*, const float*, int, float*, int,
                                           double, double, double*, hipStream_t);
template dski_status gather<double, double>(dski_plan, int, const double*, const double*, int, double*, int,
                                            double, double, double*, hipStream_t);

// The three stages on a caller-chosen grid workspace G (M x R doubles).  The
// grid stays FP64 beside FP32 vectors: an FP32 grid between the stages was
// measured to move the terrain MVM 1.6e-5 away from the FP64 product (3e-8
// with the FP64 grid) and to cost the FP32 block PCG 21 % more iterations,
// because the gather's derivative weights (of order 1/h) difference nearby
// grid values.
template <typename T>
static dski_status mvm_tiled_on(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double* pq_partial,
                                double* G, hipStream_t st) {
  DSKI_TRY((scatter<T, double>(p, R, V, ldv, G, st)));
  DSKI_TRY(apply_kuu<double>(p, R, G, st));
  return gather<T, double>(p, R, G, V, ldv, Y, ldy, p->sf * p->sf, p->sg * p->sg, pq_partial, st);
}

template <typename T>
dski_status mvm_tiled(dski_plan p, int R, const T* V, int ldv, T* Y, int ldy, double* pq_partial,
                      hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  if (p->kind == 1) return dskip_mvm<T>(p, R, V, ldv, Y, ldy, pq_partial, st);
  DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)p->M * R));
  return mvm_tiled_on<T>(p, R, V, ldv, Y, ldy, pq_partial, p->grid.as<double>(), st);
}

// ------------------------------------------------------------------ fixed workspace
// The grid workspace of dski_mvm_tiled_noalloc: a file-scope device array of
// kNoAllocBytes, one copy on every GPU the library is loaded on, held until
// the process ends.  Host code must not pass the array's name to a kernel (on
// the host it is only a stand-in for the symbol): its device address is looked
// up once per device with hipGetSymbolAddress and kept in noalloc_ptr.
constexpr size_t kNoAllocBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];
static std::mutex noalloc_mu;
static double* noalloc_ptr[kMaxDevices];

static dski_status noalloc_workspace(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("dski_mvm_tiled_noalloc: no current device (or device id %d beyond %d)", dev, kMaxDevices);
    return DSKI_EHIP;
  }
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("dski_mvm_tiled_noalloc: hipGetSymbolAddress of the workspace failed on device %d: %s", dev,
                hipGetErrorString(e));
      return DSKI_EHIP;
    }
    noalloc_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = noalloc_ptr[dev];
  return DSKI_OK;
}
template dski_status mvm_tiled<float>(dski_plan, int, const float*, int, float*, int, double*,
                                      hipStream_t);
template dski_status mvm_tiled<double>(dski_plan, int, const double*, int, double*, int, double*,
                                       hipStream_t);

template <typename T>
__global__ void k_noise_deriv(const T* __restrict__ V, int ldv, T* __restrict__ Y, int ldy, int n,
                              int N, int R, double cv, double cg) {
  size_t tot = (size_t)N * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e % N);
    int r = (int)(e / N);
    double c = i < n ? cv : cg;
    Y[(size_t)r * ldy + i] = (T)(c * (double)V[(size_t)r * ldv + i]);
  }
}

// Y = dK~/dtheta_which V on tile-ordered vectors: for ell_p the derivative
// spectrum on axis p, for s the factor 2 of K_UU, for the noise levels the
// diagonal 2 sigma^2 on the value or gradient rows.
template <typename T>
dski_status mvm_dtheta(dski_plan p, int which, int R, const T* V, int ldv, T* Y, int ldy,
                       hipStream_t st) {
  if (R <= 0) return DSKI_OK;
  int d = p->d;
  size_t tot = (size_t)p->N * R;
  int blocks = (int)std::min<size_t>((tot + 255) / 256, 65535 * 8);
  if (p->kind == 1 && which < d) {
    set_error("D-SKIP: length-scale derivatives of the Lanczos factors are not available");
    return DSKI_ENOTSUP;
  }
  if (p->kind == 1 && which == d)  // dK~/dlog s = 2 K
    return dskip_apply<T>(p, R, V, ldv, Y, ldy, 2.0 * p->s * p->s, 0.0, 0.0, nullptr, st);
  if (which <= d) {
    DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)p->M * R));
    double* G = p->grid.as<double>();
    DSKI_TRY((scatter<T, double>(p, R, V, ldv, G, st)));
    DSKI_TRY(apply_kuu<double>(p, R, G, st, which < d ? which : -1));
    DSKI_TRY((gather<T, double>(p, R, G, V, ldv, Y, ldy, 0.0, 0.0, nullptr, st)));
    if (which == d) {
      k_noise_deriv<T><<<blocks, 256, 0, st>>>(Y, ldy, Y, ldy, p->N, p->N, R, 2.0, 2.0);
      DSKI_HIP(hipGetLastError());
    }
    return DSKI_OK;
  }
  double cv = which == d + 1 ? 2.0 * p->sf * p->sf : 0.0;
  double cg = which == d + 2 ? 2.0 * p->sg * p->sg : 0.0;
  k_noise_deriv<T><<<blocks, 256, 0, st>>>(V, ldv, Y, ldy, p->n, p->N, R, cv, cg);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

template dski_status mvm_dtheta<float>(dski_plan, int, int, const float*, int, float*, int,
                                       hipStream_t);
template dski_status mvm_dtheta<double>(dski_plan, int, int, const double*, int, double*, int,
                                        hipStream_t);

}  // namespace dski

using namespace dski;

static dski_status check_mvm_args(dski_plan p, int R, const void* V, int ldv, const void* Y,
                                  int ldy) {
  if (!p || R < 0 || (R > 0 && (!V || !Y)) || ldv < p->N || ldy < p->N) {
    set_error("bad MVM arguments (R=%d, ldv=%d, ldy=%d, N=%d)", R, ldv, ldy, p ? p->N : -1);
    return DSKI_EINVAL;
  }
  return DSKI_OK;
}

template <typename T>
static dski_status mvm_user(dski_plan p, int which, int R, const T* V, int ldv, T* Y, int ldy,
                            hipStream_t st) {
  DSKI_TRY(check_mvm_args(p, R, V, ldv, Y, ldy));
  if (which < -1 || which > p->d + 2) {
    set_error("which=%d out of range 0..%d", which, p->d + 2);
    return DSKI_EINVAL;
  }
  if (R == 0 || p->N == 0) return DSKI_OK;
  size_t nr = (size_t)p->N * R;
  DSKI_TRY(p->vin.reserve(sizeof(T) * nr));
  DSKI_TRY(p->vout.reserve(sizeof(T) * nr));
  T* vi = p->vin.as<T>();
  T* vo = p->vout.as<T>();
  DSKI_TRY(permute(p, +1, R, V, ldv, vi, p->N, st));
  if (which < 0)
    DSKI_TRY(mvm_tiled<T>(p, R, vi, p->N, vo, p->N, nullptr, st));
  else
    DSKI_TRY(mvm_dtheta<T>(p, which, R, vi, p->N, vo, p->N, st));
  return permute(p, -1, R, vo, p->N, Y, ldy, st);
}

extern "C" {

dski_status dski_mvm_tiled(dski_plan p, int R, const float* V, int ldv, float* Y, int ldy,
                           dski_stream stream) {
  DSKI_TRY(check_mvm_args(p, R, V, ldv, Y, ldy));
  return mvm_tiled<float>(p, R, V, ldv, Y, ldy, nullptr, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_tiled_f64(dski_plan p, int R, const double* V, int ldv, double* Y, int ldy,
                               dski_stream stream) {
  DSKI_TRY(check_mvm_args(p, R, V, ldv, Y, ldy));
  return mvm_tiled<double>(p, R, V, ldv, Y, ldy, nullptr, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_tiled_noalloc(dski_plan p, int R, const float* V, int ldv, float* Y, int ldy,
                                   dski_stream stream) {
  DSKI_TRY(check_mvm_args(p, R, V, ldv, Y, ldy));
  if (p->kind != 0 || p->kernel != kKernelSE) {
    set_error("dski_mvm_tiled_noalloc: D-SKIP plans and the spline kernel are not supported (they need more "
              "workspace than the grid)");
    return DSKI_ENOTSUP;
  }
  if (R == 0 || p->n == 0) return DSKI_OK;
  const size_t need = sizeof(double) * (size_t)p->M * (size_t)R;
  if (need > kNoAllocBytes) {
    set_error("dski_mvm_tiled_noalloc: %d columns on %lld grid nodes need %zu bytes of grid workspace; the "
              "fixed workspace holds %zu (grid nodes x columns <= %zu)",
              R, (long long)p->M, need, kNoAllocBytes, kNoAllocBytes / sizeof(double));
    return DSKI_EINVAL;
  }
  double* G = nullptr;
  DSKI_TRY(noalloc_workspace(&G));
  return mvm_tiled_on<float>(p, R, V, ldv, Y, ldy, nullptr, G, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_stage(dski_plan p, int stage, int R, const float* V, int ldv, float* Y, int ldy,
                           dski_stream stream) {
  if (!p || R < 0 || stage < 0 || stage > 2 || (stage != 1 && (!V || ldv < p->N)) ||
      (stage == 2 && (!Y || ldy < p->N))) {
    set_error("dski_mvm_stage: bad arguments");
    return DSKI_EINVAL;
  }
  if (R == 0) return DSKI_OK;
  if (p->kind != 0) {
    set_error("dski_mvm_stage: a D-SKIP plan has no grid stages");
    return DSKI_ENOTSUP;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (stage == 0) DSKI_TRY(p->grid.reserve(sizeof(double) * (size_t)p->M * R));
  if (p->grid.bytes < sizeof(double) * (size_t)p->M * R) {
    set_error("dski_mvm_stage: run stage 0 with at least R columns first");
    return DSKI_EINVAL;
  }
  double* G = p->grid.as<double>();
  if (stage == 0) return scatter<float, double>(p, R, V, ldv, G, st);
  if (stage == 1) return apply_kuu<double>(p, R, G, st);
  return gather<float, double>(p, R, G, V, ldv, Y, ldy, p->sf * p->sf, p->sg * p->sg, nullptr, st);
}

dski_status dski_mvm(dski_plan p, int R, const float* V, int ldv, float* Y, int ldy,
                     dski_stream stream) {
  return mvm_user<float>(p, -1, R, V, ldv, Y, ldy, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_f64(dski_plan p, int R, const double* V, int ldv, double* Y, int ldy,
                         dski_stream stream) {
  return mvm_user<double>(p, -1, R, V, ldv, Y, ldy, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_dtheta(dski_plan p, int which, int R, const float* V, int ldv, float* Y,
                            int ldy, dski_stream stream) {
  if (which < 0) {
    set_error("which=%d out of range", which);
    return DSKI_EINVAL;
  }
  return mvm_user<float>(p, which, R, V, ldv, Y, ldy, static_cast<hipStream_t>(stream));
}

dski_status dski_mvm_dtheta_f64(dski_plan p, int which, int R, const double* V, int ldv, double* Y,
                                int ldy, dski_stream stream) {
  if (which < 0) {
    set_error("which=%d out of range", which);
    return DSKI_EINVAL;
  }
  return mvm_user<double>(p, which, R, V, ldv, Y, ldy, static_cast<hipStream_t>(stream));
}

}  // extern "C"
