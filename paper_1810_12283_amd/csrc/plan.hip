// Plan set-up: grid geometry, per-point interpolation cells, tile order,
// circulant spectra of the Toeplitz factors of K_UU; utilities shared by
// the solvers (errors, buffers, permutations, reductions, probes).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"
#include "interp.h"

namespace dski {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

dski_status DevBuf::reserve(size_t want) {
  if (want <= bytes) return DSKI_OK;
  release();
  size_t sz = want + want / 4 + 256;
  if (hipMalloc(&p, sz) != hipSuccess) {
    p = nullptr;
    bytes = 0;
    set_error("device allocation of %zu bytes failed", sz);
    return DSKI_ENOMEM;
  }
  bytes = sz;
  return DSKI_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

struct Geo {
  int d;
  int S;  // stencil nodes per axis
  int m[DSKI_MAXD];
  int nc[DSKI_MAXD];
  double lo[DSKI_MAXD];
  double h[DSKI_MAXD];
};

// Cell index and offset of every point (user order), histogram of cells.
// With S stencil nodes per axis and H = S/2 - 1, the anchor node is
// i_p = clamp(floor(s_p), H, m_p - S + H), s_p = (x_p - lo_p) / h_p, so the
// stencil nodes i_p - H .. i_p - H + S - 1 lie in the grid; t_p = s_p - i_p;
// the cell id on the axis is i_p - H (its first stencil node).
__global__ void k_cells(const double* __restrict__ X, int n, Geo g, int* __restrict__ cell_u,
                        double* __restrict__ t_u, int* __restrict__ counts, int* __restrict__ err) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int H = g.S / 2 - 1;
  int lin = 0;
  for (int p = 0; p < g.d; ++p) {
    double x = X[(size_t)u * g.d + p];
    double s = (x - g.lo[p]) / g.h[p];
    const double smin = (double)H, smax = (double)(g.m[p] - g.S + H + 1);
    if (!(s >= smin - 1e-9 && s <= smax + 1e-9)) {
      atomicOr(err, 1);
      s = fmin(fmax(s, smin), smax);
    }
    int i = (int)floor(s);
    const int imax = g.m[p] - g.S + H;
    i = i < H ? H : (i > imax ? imax : i);
    double t = s - (double)i;
    t = fmin(fmax(t, 0.0), 1.0);
    t_u[(size_t)p * n + u] = t;
    lin = lin * g.nc[p] + (i - H);
  }
  cell_u[u] = lin;
  atomicAdd(&counts[lin], 1);
}

// Exclusive scan of counts[0..len) into out[0..len] with one work-group.
__global__ void k_scan_single(const int* __restrict__ counts, int len, int* __restrict__ out) {
  __shared__ int buf[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < len; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < len ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int a = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < len) out[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[len] = carry;
}

__global__ void k_place(const int* __restrict__ cell_u, int n, const int* __restrict__ start,
                        int* __restrict__ fill, int* __restrict__ perm) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int c = cell_u[u];
  int pos = start[c] + atomicAdd(&fill[c], 1);
  perm[pos] = u;
}

// Deterministic order inside a cell: ascending user index.
__global__ void k_sort_cells(const int* __restrict__ start, int ncells, int* __restrict__ perm) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int a = start[c], b = start[c + 1];
  for (int i = a + 1; i < b; ++i) {
    int v = perm[i];
    int j = i - 1;
    while (j >= a && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

__global__ void k_gather_points(const int* __restrict__ perm, int n, int d,
                                const int* __restrict__ cell_u, const double* __restrict__ t_u,
                                int* __restrict__ cell, double* __restrict__ toff) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int u = perm[k];
  cell[k] = cell_u[u];
  for (int p = 0; p < d; ++p) toff[(size_t)p * n + k] = t_u[(size_t)p * n + u];
}

// Pass twiddles of the length-2^lg FFT in the layout of the radix plan
// (forward passes e^{-2 pi i r k / (radix Ns)}, then inverse passes with +).
__global__ void k_twiddle(int lg, double* __restrict__ tw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= fft_tw_size(lg)) return;
  const int np = fft_npass(lg);
  for (int dir = 1; dir >= -1; dir -= 2)
    for (int s = 0; s < np; ++s) {
      const int off = fft_tw_offset(lg, s, dir), rad = fft_radix_dir(lg, s, dir), ns = fft_ns(lg, s, dir);
      if (e < off || e >= off + (rad - 1) * ns) continue;
      const int r = 1 + (e - off) / ns, k = (e - off) % ns;
      double sn, cs;
      sincospi(2.0 * (double)(r * k) / (double)(rad * ns), &sn, &cs);
      tw[2 * e] = cs;
      tw[2 * e + 1] = dir > 0 ? -sn : sn;
    }
}

// Circulant eigenvalues of the embedding [c_0..c_{m-1}, 0.., c_{m-1}..c_1] of the
// symmetric Toeplitz factor c_j = exp(-(j h)^2 / (2 ell^2)) (SE kernel on the grid):
// lambda_k = c_0 + 2 sum_{j>=1} c_j cos(2 pi j k / L); also those of the derivative
// factor with c'_j = c_j (j h / ell)^2 (d/dlog ell).  Both carry `scale` (= s^2 / L
// on axis 0, 1 / L elsewhere, so that the inverse FFT needs no normalisation).
__global__ void k_spectrum(int m, int L, double h, double ell, double scale,
                           double* __restrict__ spec, double* __restrict__ dspec,
                           double* __restrict__ col) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) {
    double r = (double)k * h / ell;
    col[k] = exp(-0.5 * r * r);
  }
  if (k >= L) return;
  double acc = 0.0, dacc = 0.0;
  for (int j = 0; j < m; ++j) {
    double r = (double)j * h / ell;
    double c = exp(-0.5 * r * r);
    long long ph = ((long long)j * (long long)k) % L;
    double cs = cospi(2.0 * (double)ph / (double)L);
    double w = j == 0 ? 1.0 : 2.0;
    acc += w * c * cs;
    dacc += w * c * r * r * cs;
  }
  spec[k] = acc * scale;
  dspec[k] = dacc * scale;
}

// Permutation between user order and tile order for R vectors of N = n(d+1).
template <typename T>
__global__ void k_permute(const int* __restrict__ perm, int n, int nb, int R, int dir,
                          const T* __restrict__ in, int ldi, T* __restrict__ out, int ldo) {
  size_t tot = (size_t)n * nb * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int k = (int)(e % n);
    size_t rest = e / n;
    int b = (int)(rest % nb);
    int r = (int)(rest / nb);
    int u = perm[k];
    if (dir > 0)
      out[(size_t)r * ldo + (size_t)b * n + k] = in[(size_t)r * ldi + (size_t)b * n + u];
    else
      out[(size_t)r * ldo + (size_t)b * n + u] = in[(size_t)r * ldi + (size_t)b * n + k];
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): output k = mix64(seed + (k + 1) * golden).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_rademacher(uint64_t seed, int col0, int ncols, int N, T* __restrict__ out, int ld) {
  size_t tot = (size_t)N * ncols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e % N);
    int c = (int)(e / N);
    uint64_t ctr = (uint64_t)(col0 + c) * (uint64_t)N + (uint64_t)i;
    uint64_t z = mix64(seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull);
    out[(size_t)c * ld + i] = (z >> 63) ? (T)-1 : (T)1;
  }
}

// out[c] = sum_b partial[b * ncol + c], fixed order (one work-group per column).
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int ncol,
                                  double* __restrict__ out) {
  __shared__ double buf[kBlock];
  int c = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += partial[(size_t)b * ncol + c];
  buf[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) buf[threadIdx.x] += buf[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = buf[0];
}

dski_status reduce_partials(const double* partial, int nblk, int ncol, double* out,
                            hipStream_t st) {
  if (ncol <= 0) return DSKI_OK;
  k_reduce_partials<<<ncol, kBlock, 0, st>>>(partial, nblk, ncol, out);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

static int grid1d(size_t work, int block = kBlock) {
  size_t g = (work + block - 1) / block;
  if (g > 65535 * 8) g = 65535 * 8;
  return (int)(g == 0 ? 1 : g);
}

template <typename T>
static dski_status permute_t(dski_plan p, int dir, int R, const T* in, int ldi, T* out, int ldo,
                             hipStream_t st) {
  size_t tot = (size_t)p->N * R;
  if (tot == 0) return DSKI_OK;
  k_permute<T><<<grid1d(tot), kBlock, 0, st>>>(p->perm, p->n, p->d + 1, R, dir, in, ldi, out, ldo);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

dski_status permute(dski_plan p, int dir, int R, const float* in, int ldi, float* out, int ldo,
                    hipStream_t st) {
  return permute_t<float>(p, dir, R, in, ldi, out, ldo, st);
}

dski_status permute(dski_plan p, int dir, int R, const double* in, int ldi, double* out, int ldo,
                    hipStream_t st) {
  return permute_t<double>(p, dir, R, in, ldi, out, ldo, st);
}

template <typename T>
dski_status rademacher(uint64_t seed, int col0, int ncols, int N, T* out, int ld, hipStream_t st) {
  size_t tot = (size_t)N * ncols;
  if (tot == 0) return DSKI_OK;
  k_rademacher<T><<<grid1d(tot), kBlock, 0, st>>>(seed, col0, ncols, N, out, ld);
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}
template dski_status rademacher<float>(uint64_t, int, int, int, float*, int, hipStream_t);
template dski_status rademacher<double>(uint64_t, int, int, int, double*, int, hipStream_t);

static int fft_len(int m) {
  int L = 8;
  while (L < 2 * m - 1) L <<= 1;
  return L;
}

}  // namespace dski

using namespace dski;

extern "C" {

const char* dski_last_error(void) { return g_last_error.c_str(); }

const char* dski_version(void) { return "dski-gfx950 " __DATE__; }

dski_status dski_plan_destroy(dski_plan p) {
  if (!p) return DSKI_OK;
  if (p->kind == 1) dskip_destroy(p);
  (void)hipFree(p->perm);
  (void)hipFree(p->cell);
  (void)hipFree(p->toff);
  (void)hipFree(p->cell_start);
  (void)hipFree(p->tile_off);
  (void)hipFree(p->tile_lcs);
  (void)hipFree(p->tile_pts);
  (void)hipFree(p->tile_cl);
  (void)hipFree(p->grp_items);
  (void)hipFree(p->grp_chunk_off);
  (void)hipFree(p->grp_tile_chunk);
  (void)hipFree(p->bttb_spec);
  p->bttb_work.release();
  for (int a = 0; a < (p->kind == 0 ? p->d : 0); ++a) {
    (void)hipFree(p->ax[a].twiddle);
    (void)hipFree(p->ax[a].spec);
    (void)hipFree(p->ax[a].dspec);
    (void)hipFree(p->ax[a].col);
  }
  p->grid.release();
  p->vin.release();
  p->vout.release();
  p->partial.release();
  p->scal.release();
  delete p;
  return DSKI_OK;
}

static dski_status plan_create_impl(dski_plan p, const double* X, const int* grid_m,
                                    const double* lo, const double* hi, hipStream_t st) {
  int n = p->n, d = p->d;
  const int S = p->S, H = S / 2 - 1;
  Geo g{};
  g.d = d;
  g.S = S;
  std::vector<double> blo(d), bhi(d);
  if (lo && hi) {
    for (int a = 0; a < d; ++a) {
      blo[a] = lo[a];
      bhi[a] = hi[a];
    }
  } else {
    // bounding box of X
    std::vector<double> hx((size_t)n * d);
    DSKI_HIP(hipMemcpyAsync(hx.data(), X, hx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    DSKI_HIP(hipStreamSynchronize(st));
    for (int a = 0; a < d; ++a) {
      blo[a] = INFINITY;
      bhi[a] = -INFINITY;
    }
    for (int u = 0; u < n; ++u)
      for (int a = 0; a < d; ++a) {
        blo[a] = std::fmin(blo[a], hx[(size_t)u * d + a]);
        bhi[a] = std::fmax(bhi[a], hx[(size_t)u * d + a]);
      }
  }
  long long M = 1;
  long long nc = 1;
  for (int a = 0; a < d; ++a) {
    Axis& A = p->ax[a];
    if (grid_m[a] < S) {
      set_error("grid size %d on axis %d: need >= %d (the interpolation stencil)", grid_m[a], a, S);
      return DSKI_EINVAL;
    }
    if (!(bhi[a] > blo[a]) || !std::isfinite(blo[a]) || !std::isfinite(bhi[a])) {
      set_error("degenerate or non-finite data box on axis %d", a);
      return DSKI_EINVAL;
    }
    A.m = grid_m[a];
    A.ncell = A.m - S + 1;
    A.h = (bhi[a] - blo[a]) / (double)A.ncell;
    A.lo = blo[a] - H * A.h;
    A.L = fft_len(A.m);
    if (A.L > (1 << kFftMaxLog2)) {
      set_error("grid size %d on axis %d exceeds the FFT limit (m <= 1024)", A.m, a);
      return DSKI_ENOTSUP;
    }
    g.m[a] = A.m;
    g.nc[a] = A.ncell;
    g.lo[a] = A.lo;
    g.h[a] = A.h;
    M *= A.m;
    nc *= A.ncell;
  }
  if (M > (1ll << 31) || nc > (1ll << 30)) {
    set_error("grid too large");
    return DSKI_ENOTSUP;
  }
  p->M = M;
  p->ncells = (int)nc;
  DSKI_HIP(hipMalloc(&p->perm, sizeof(int) * (size_t)std::max(n, 1)));
  DSKI_HIP(hipMalloc(&p->cell, sizeof(int) * (size_t)std::max(n, 1)));
  DSKI_HIP(hipMalloc(&p->toff, sizeof(double) * (size_t)std::max(n, 1) * d));
  DSKI_HIP(hipMalloc(&p->cell_start, sizeof(int) * (size_t)(nc + 1)));
  for (int a = 0; a < d; ++a) {
    Axis& A = p->ax[a];
    int lg = 0;
    while ((1 << lg) < A.L) ++lg;
    DSKI_HIP(hipMalloc(&A.twiddle, sizeof(double) * 2 * fft_tw_size(lg)));
    DSKI_HIP(hipMalloc(&A.spec, sizeof(double) * A.L));
    DSKI_HIP(hipMalloc(&A.dspec, sizeof(double) * A.L));
    DSKI_HIP(hipMalloc(&A.col, sizeof(double) * A.m));
    k_twiddle<<<(fft_tw_size(lg) + kBlock - 1) / kBlock, kBlock, 0, st>>>(lg, A.twiddle);
    DSKI_HIP(hipGetLastError());
  }
  // temporaries
  int *cell_u = nullptr, *counts = nullptr, *err = nullptr;
  double* t_u = nullptr;
  size_t tmp_bytes = sizeof(double) * (size_t)std::max(n, 1) * d + sizeof(int) * (size_t)std::max(n, 1) +
                     sizeof(int) * (size_t)(2 * nc + 2) + 128;
  char* tmp = nullptr;
  DSKI_HIP(hipMalloc(&tmp, tmp_bytes));
  t_u = reinterpret_cast<double*>(tmp);
  cell_u = reinterpret_cast<int*>(t_u + (size_t)std::max(n, 1) * d);
  counts = cell_u + std::max(n, 1);
  int* fill = counts + nc + 1;
  err = fill + nc + 1;
  dski_status rc = DSKI_OK;
  int herr = 0;
  do {
    if (hipMemsetAsync(counts, 0, sizeof(int) * (size_t)(2 * nc + 2) + sizeof(int), st) != hipSuccess) {
      set_error("hipMemsetAsync failed");
      rc = DSKI_EHIP;
      break;
    }
    if (n > 0) {
      k_cells<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(X, n, g, cell_u, t_u, counts, err);
    }
    k_scan_single<<<1, 1024, 0, st>>>(counts, (int)nc, p->cell_start);
    if (n > 0) {
      k_place<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(cell_u, n, p->cell_start, fill, p->perm);
      k_sort_cells<<<(int)((nc + kBlock - 1) / kBlock), kBlock, 0, st>>>(p->cell_start, (int)nc, p->perm);
      k_gather_points<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(p->perm, n, d, cell_u, t_u, p->cell,
                                                                   p->toff);
    }
    if (hipGetLastError() != hipSuccess) {
      set_error("set-up kernel launch failed");
      rc = DSKI_EHIP;
      break;
    }
    if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("set-up synchronisation failed");
      rc = DSKI_EHIP;
      break;
    }
    if (herr) {
      set_error("a point lies outside the interpolation box (or is not finite)");
      rc = DSKI_EINVAL;
      break;
    }
    rc = scatter_tables(p, st);
  } while (0);
  (void)hipFree(tmp);
  return rc;
}

dski_status dski_plan_create(dski_plan* out, int n, int d, const double* X, const int* grid_m_host,
                             const double* lo_host, const double* hi_host, int interp, dski_stream stream) {
  if (!out) {
    set_error("out is NULL");
    return DSKI_EINVAL;
  }
  *out = nullptr;
  if (n < 0 || d < 1 || d > DSKI_MAXD || !grid_m_host || (n > 0 && !X) ||
      ((lo_host == nullptr) != (hi_host == nullptr)) || (n == 0 && !lo_host)) {
    set_error("dski_plan_create: bad arguments (n=%d, d=%d; d must be 1..%d; box required when n=0)",
              n, d, DSKI_MAXD);
    return DSKI_EINVAL;
  }
  if ((long long)n * (d + 1) > (1ll << 31) - 1) {
    set_error("n too large");
    return DSKI_EINVAL;
  }
  if (interp != DSKI_INTERP_CUBIC && interp != DSKI_INTERP_QUINTIC) {
    set_error("dski_plan_create: interp must be DSKI_INTERP_CUBIC (0) or DSKI_INTERP_QUINTIC (1), got %d", interp);
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  dski_plan p = new dski_plan_s();
  p->n = n;
  p->d = d;
  p->N = n * (d + 1);
  p->S = interp == DSKI_INTERP_QUINTIC ? kInterpQuintic : kInterpCubic;
  dski_status rc = plan_create_impl(p, X, grid_m_host, lo_host, hi_host, st);
  if (rc < 0) {
    dski_plan_destroy(p);
    return rc;
  }
  double le[DSKI_MAXD] = {0, 0, 0};
  rc = dski_set_hypers(p, le, 0.0, std::log(0.1), std::log(0.1), stream);
  if (rc < 0) {
    dski_plan_destroy(p);
    return rc;
  }
  *out = p;
  return DSKI_OK;
}

dski_status dski_plan_info(dski_plan p, int* n, int* d, int* N, long long* grid_nodes, int* m_host,
                           int* fft_len_host, double* h_host, double* lo_host) {
  if (!p) {
    set_error("plan is NULL");
    return DSKI_EINVAL;
  }
  if (n) *n = p->n;
  if (d) *d = p->d;
  if (N) *N = p->N;
  if (grid_nodes) *grid_nodes = p->M;
  for (int a = 0; a < (p->kind == 0 ? p->d : 0); ++a) {
    if (m_host) m_host[a] = p->ax[a].m;
    if (fft_len_host) fft_len_host[a] = p->ax[a].L;
    if (h_host) h_host[a] = p->ax[a].h;
    if (lo_host) lo_host[a] = p->ax[a].lo;
  }
  return DSKI_OK;
}

dski_status dski_set_hypers(dski_plan p, const double* log_ell_host, double log_s,
                            double log_sigma_f, double log_sigma_g, dski_stream stream) {
  if (!p || !log_ell_host) {
    set_error("dski_set_hypers: NULL argument");
    return DSKI_EINVAL;
  }
  for (int a = 0; a < p->d; ++a)
    if (!std::isfinite(log_ell_host[a])) {
      set_error("non-finite log length scale");
      return DSKI_EINVAL;
    }
  if (!std::isfinite(log_s) || !std::isfinite(log_sigma_f) || !std::isfinite(log_sigma_g)) {
    set_error("non-finite hyper-parameter");
    return DSKI_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->s = std::exp(log_s);
  p->sf = std::exp(log_sigma_f);
  p->sg = std::exp(log_sigma_g);
  if (p->kind == 1) return dskip_set_hypers(p, log_ell_host, st);  // rebuilds the factors when ell moves
  for (int a = 0; a < p->d; ++a) {
    Axis& A = p->ax[a];
    p->ell[a] = std::exp(log_ell_host[a]);
    double scale = (a == 0 ? p->s * p->s : 1.0) / (double)A.L;
    int work = std::max(A.L, A.m);
    k_spectrum<<<(work + kBlock - 1) / kBlock, kBlock, 0, st>>>(A.m, A.L, A.h, p->ell[a], scale, A.spec,
                                                                A.dspec, A.col);
    DSKI_HIP(hipGetLastError());
  }
  return DSKI_OK;
}

dski_status dski_permute(dski_plan p, int dir, int R, const float* in, int ldi, float* out, int ldo,
                         dski_stream stream) {
  if (!p || (dir != 1 && dir != -1) || R < 0 || (R > 0 && (!in || !out)) || ldi < p->N ||
      ldo < p->N) {
    set_error("dski_permute: bad arguments");
    return DSKI_EINVAL;
  }
  return permute(p, dir, R, in, ldi, out, ldo, static_cast<hipStream_t>(stream));
}

dski_status dski_permute_f64(dski_plan p, int dir, int R, const double* in, int ldi, double* out,
                             int ldo, dski_stream stream) {
  if (!p || (dir != 1 && dir != -1) || R < 0 || (R > 0 && (!in || !out)) || ldi < p->N ||
      ldo < p->N) {
    set_error("dski_permute_f64: bad arguments");
    return DSKI_EINVAL;
  }
  return permute(p, dir, R, in, ldi, out, ldo, static_cast<hipStream_t>(stream));
}

dski_status dski_set_kernel(dski_plan p, int kernel, dski_stream stream) {
  if (!p || (kernel != DSKI_KERNEL_SE && kernel != DSKI_KERNEL_SPLINE)) {
    set_error("dski_set_kernel: kernel must be DSKI_KERNEL_SE (0) or DSKI_KERNEL_SPLINE (1)");
    return DSKI_EINVAL;
  }
  if (p->kind != 0) {
    set_error("dski_set_kernel: D-SKIP plans carry the SE product kernel only");
    return DSKI_ENOTSUP;
  }
  if (kernel == DSKI_KERNEL_SPLINE) DSKI_TRY(bttb_build_spectrum(p, static_cast<hipStream_t>(stream)));
  p->kernel = kernel == DSKI_KERNEL_SPLINE ? kKernelSpline : kKernelSE;
  return DSKI_OK;
}

dski_status dski_plan_set_precision(dski_plan p, int bits) {
  if (!p || (bits != 32 && bits != 64)) {
    set_error("dski_plan_set_precision: bits must be 32 or 64");
    return DSKI_EINVAL;
  }
  p->precision = bits;
  return DSKI_OK;
}

dski_status dski_tile_order(dski_plan p, int* perm_host) {
  if (!p || !perm_host) {
    set_error("dski_tile_order: NULL argument");
    return DSKI_EINVAL;
  }
  DSKI_HIP(hipMemcpy(perm_host, p->perm, sizeof(int) * (size_t)p->n, hipMemcpyDeviceToHost));
  return DSKI_OK;
}

dski_status dski_rademacher(uint64_t seed, int col0, int ncols, int N, float* out, int ld,
                            dski_stream stream) {
  if (col0 < 0 || ncols < 0 || N < 0 || ld < N || (ncols > 0 && N > 0 && !out)) {
    set_error("dski_rademacher: bad arguments");
    return DSKI_EINVAL;
  }
  return rademacher<float>(seed, col0, ncols, N, out, ld, static_cast<hipStream_t>(stream));
}

}  // extern "C"
