// Preconditioned conjugate gradients on a block of R right-hand sides (Sec. 2,
// Sec. 3.3).  The columns are independent CG runs that share every MVM (the
// block is not a block-Krylov method, so each column keeps its own Lanczos
// tridiagonal for quadrature).  Vectors are FP32 (or FP64) in tile order, the
// iterate x is accumulated in FP64, all inner products and scalars are FP64 and
// live on the device; the host only polls the number of active columns.
//
// One iteration is 9 launches (10 with the FFT of a 3-D grid):
//   scatter | K_UU per axis | gather (+ partials of p.q)
//   update:  alpha (every block reduces the p.q partials itself, same order),
//            x += alpha p, r -= alpha q, partials of r.r and of U^T D^{-1/2} r
//   reduce:  t1 = U^T r', coef1 = c .* t1; r.r
//   project: t2 = U^T (r' - U coef1)
//   reduce:  coef2 = c .* (t1 + t2)
//   final:   z = D^{-1/2}(r' - U coef2) (+ partials of r.z)
//   beta:    beta (every block reduces the r.z partials), convergence test,
//            p = z + beta p.
// Scalars that one kernel both reads in every block and updates (rz, the
// active flags) are double-buffered by iteration parity.
#include <cmath>

#include "internal.h"
#include "tskinny.h"

namespace dski {

constexpr int kPcgMaxR = 32;  // columns per fused PCG (larger blocks run in groups)

struct PcgScal {
  double* rz;     // [2][R] r^T M^{-1} r, by parity
  double* rr;     // [R] r^T r (current)
  double* bb;     // [R] b^T b
  double* alpha;  // [R]
  double* tol2;   // [R]
  int* active;    // [2][R] by parity
  int* iters;     // [R]
  int* flags;     // [0] active columns, [1] breakdown
};

constexpr int kVecChunk = 1024;  // rows per work-group in the streaming vector kernels

static int nchunks(int N) { return (N + kVecChunk - 1) / kVecChunk; }


// R = B, X = 0, partials of b.b (block = kVecChunk rows, all columns)
template <typename T>
__global__ void k_pcg_init(const T* __restrict__ B, int ldb, T* __restrict__ Rr, double* __restrict__ Xd,
                           int N, int R, double* __restrict__ partial) {
  __shared__ double red[4];
  const int e0 = blockIdx.x * kVecChunk;
  for (int c = 0; c < R; ++c) {
    double acc = 0.0;
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x) {
      T b = B[(size_t)c * ldb + e];
      Rr[(size_t)c * N + e] = b;
      Xd[(size_t)c * N + e] = 0.0;
      acc += (double)b * (double)b;
    }
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

// After the initial preconditioner application (parity 0): rz, bb, rr, active.
// One wavefront per column (partials are output-major).
__global__ void k_pcg_init_scal(const double* __restrict__ bb_part, int nb_b, const double* __restrict__ rz_part,
                                int nb_z, int R, int fixed_iters, PcgScal s, double* __restrict__ rz0) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wv; c < R; c += nw) {
    double bb = wave_out_sum(bb_part, nb_b, c);
    double rz = rz_part ? wave_out_sum(rz_part, nb_z, c) : bb;
    if ((threadIdx.x & 63) != 0) continue;
  s.bb[c] = bb;
  s.rr[c] = bb;
  s.rz[c] = rz;
  s.rz[R + c] = rz;
  rz0[c] = rz;
  s.iters[c] = 0;
  int act = bb > 0.0 && (fixed_iters > 0 || bb > s.tol2[c] * bb);
  s.active[c] = act;
  s.active[R + c] = act;
  if (act) atomicAdd(&s.flags[0], 1);
  }
}

// alpha, x and r updates, partials of r.r and of U^T D^{-1/2} r (row tile of RT rows).
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update(const T* __restrict__ P, const T* __restrict__ Q,
                                                    T* __restrict__ Rr, double* __restrict__ Xd, int N, int n,
                                                    int R, PcgScal s, int par, const double* __restrict__ pq_part,
                                                    int nb_pq, double* __restrict__ rr_part,
                                                    const T* __restrict__ U, int k, double isf, double isg,
                                                    int RT, ProjLds L, double* __restrict__ t_part,
                                                    double* __restrict__ hist, int max_iter) {
  extern __shared__ __align__(16) char smem[];
  T* sU = reinterpret_cast<T*>(smem + L.oU);
  double* sx = reinterpret_cast<double*>(smem + L.ox);
  double* sred = reinterpret_cast<double*>(smem + L.ored);
  __shared__ double s_alpha[kPcgMaxR];
  __shared__ int s_act[kPcgMaxR];
  const int* act = s.active + par * R;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = wv; c < R; c += 4) {  // one wavefront per column
    int on = act[c];
    double pq = on ? wave_out_sum(pq_part, nb_pq, c) : 0.0;
    if (lane == 0) {
      double a = 0.0;
      if (on) {
        if (!(pq > 0.0) || !isfinite(pq)) {
          if (blockIdx.x == 0) s.flags[1] = 1;
        } else {
          a = s.rz[par * R + c] / pq;
        }
        if (blockIdx.x == 0 && hist && s.iters[c] < max_iter) hist[(size_t)c * max_iter + s.iters[c]] = a;
      }
      if (blockIdx.x == 0) s.alpha[c] = a;
      s_alpha[c] = a;
      s_act[c] = on;
    }
  }
  const int e0 = blockIdx.x * RT;
  const int rn = min(RT, N - e0);
  if (k > 0) tile_load_u<T>(U, N, k, e0, rn, RT, sU);
  __syncthreads();
  for (int f = threadIdx.x; f < RT * R; f += blockDim.x) {
    int r = f % RT, c = f / RT;
    double v = 0.0;
    if (r < rn) {
      size_t i = (size_t)c * N + e0 + r;
      double rv = (double)Rr[i];
      if (s_act[c]) {
        double a = s_alpha[c];
        Xd[i] += a * (double)P[i];
        T rnew = (T)(rv - a * (double)Q[i]);
        Rr[i] = rnew;
        rv = (double)rnew;
      }
      v = rv;
    }
    sx[r * R + c] = v;
  }
  __syncthreads();
  for (int c = wv; c < R; c += 4) {
    double acc = 0.0;
    for (int r = lane; r < rn; r += 64) {
      double v = sx[r * R + c];
      acc += v * v;
    }
    acc = wave_sum64(acc);
    if (lane == 0) rr_part[(size_t)c * gridDim.x + blockIdx.x] = acc;
  }
  if (k == 0) return;
  __syncthreads();
  for (int f = threadIdx.x; f < rn * R; f += blockDim.x) {
    int r = f / R;
    sx[f] *= (e0 + r < n ? isf : isg);
  }
  __syncthreads();
  tile_proj<T>(sU, sx, rn, RT, k, R, sred, t_part);
}

// Wavefront-shuffle variant of the update: grid (row blocks of 256, column
// groups of cgs); one thread per row for its group's columns.
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update_shfl(const T* __restrict__ P, const T* __restrict__ Q,
                                                         T* __restrict__ Rr, double* __restrict__ Xd, int N, int n,
                                                         int R, PcgScal s, int par,
                                                         const double* __restrict__ pq_part, int nb_pq,
                                                         double* __restrict__ rr_part, const T* __restrict__ U,
                                                         int k, double isf, double isg, int cgs,
                                                         double* __restrict__ t_part, double* __restrict__ hist,
                                                         int max_iter) {
  __shared__ double red[4][kShflChunk][kShflGroup];
  __shared__ double s_alpha[kShflGroup];
  __shared__ int s_act[kShflGroup];
  const int c0 = blockIdx.y * cgs;
  const int cg = min(cgs, R - c0);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wv < cg) {  // one wavefront per column of the group
    const int c = c0 + wv;
    int on = s.active[par * R + c];
    double pq = on ? wave_out_sum(pq_part, nb_pq, c) : 0.0;
    if (lane == 0) {
      double a = 0.0;
      if (on) {
        if (!(pq > 0.0) || !isfinite(pq)) {
          if (blockIdx.x == 0) s.flags[1] = 1;
        } else {
          a = s.rz[par * R + c] / pq;
        }
        if (blockIdx.x == 0 && hist && s.iters[c] < max_iter) hist[(size_t)c * max_iter + s.iters[c]] = a;
      }
      if (blockIdx.x == 0) s.alpha[c] = a;
      s_alpha[wv] = a;
      s_act[wv] = on;
    }
  }
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double v[kShflGroup];
#pragma unroll
  for (int c = 0; c < kShflGroup; ++c) v[c] = 0.0;
  if (e < N) {
#pragma unroll
    for (int c = 0; c < kShflGroup; ++c) {
      if (c < cg) {
        size_t i = (size_t)(c0 + c) * N + e;
        double rv = (double)Rr[i];
        if (s_act[c]) {
          double a = s_alpha[c];
          Xd[i] += a * (double)P[i];
          T rnew = (T)(rv - a * (double)Q[i]);
          Rr[i] = rnew;
          rv = (double)rnew;
        }
        v[c] = rv;
      }
    }
  }
  // partials of r.r
#pragma unroll
  for (int c = 0; c < kShflGroup; ++c) {
    if (c < cg) {
      double sm = wave_sum64(v[c] * v[c]);
      if (lane == 0) red[wv][0][c] = sm;
    }
  }
  __syncthreads();
  if (threadIdx.x < cg) {
    int c = threadIdx.x;
    rr_part[(size_t)(c0 + c) * gridDim.x + blockIdx.x] = red[0][0][c] + red[1][0][c] + red[2][0][c] + red[3][0][c];
  }
  __syncthreads();
  if (k == 0) return;
  const double pre = e < n ? isf : isg;
#pragma unroll
  for (int c = 0; c < kShflGroup; ++c) v[c] *= pre;
  shfl_project<T>(U, N, e, k, R, c0, cg, v, red, t_part);
}

// beta, history, convergence test, p = z + beta p.  Grid (row chunks of 256, R):
// every block recomputes its column's beta from the r.z partials (same order);
// block (0, c) writes the column's next-parity state.
template <typename T>
__global__ void k_pcg_beta(const T* __restrict__ Z, T* __restrict__ P, int N, int R, PcgScal s, int par,
                           const double* __restrict__ rz_part, int nb_rz, double* __restrict__ hist,
                           int max_iter, int fixed_iters) {
  __shared__ double s_beta;
  __shared__ int s_on;
  const int c = blockIdx.y;
  const int on = s.active[par * R + c];
  if (!on) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      s.rz[(1 - par) * R + c] = s.rz[par * R + c];
      s.active[(1 - par) * R + c] = 0;
    }
    return;
  }
  if (threadIdx.x < 64) {
    double rzs = rz_part ? wave_out_sum(rz_part, nb_rz, c) : 0.0;
    if (threadIdx.x == 0) {
      double rz_old = s.rz[par * R + c];
      double rzn = rz_part ? rzs : s.rr[c];
      if (!(rzn >= 0.0) || !isfinite(rzn)) {
        if (blockIdx.x == 0) s.flags[1] = 1;
      }
      double b = rz_old > 0.0 ? rzn / rz_old : 0.0;
      if (blockIdx.x == 0) {
        int it = s.iters[c];
        bool done = fixed_iters > 0 ? (it + 1 >= fixed_iters) : (s.rr[c] <= s.tol2[c] * s.bb[c]);
        if (hist && it < max_iter) hist[(size_t)R * max_iter + (size_t)c * max_iter + it] = b;
        s.iters[c] = it + 1;
        if (done) atomicSub(&s.flags[0], 1);
        s.rz[(1 - par) * R + c] = rzn;
        s.active[(1 - par) * R + c] = done ? 0 : 1;
      }
      s_beta = b;
    }
  }
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) {
    size_t i = (size_t)c * N + e;
    P[i] = (T)((double)Z[i] + s_beta * (double)P[i]);
  }
}

// True residual r = b - y (y = K~ x from the FP64-storage operator): stored into Rr
// for the columns flagged in `verify`, partials of |r|^2 (output-major).
template <typename T>
__global__ void k_true_resid(const T* __restrict__ B, int ldb, const double* __restrict__ Y, T* __restrict__ Rr,
                             int N, int R, const int* __restrict__ verify, double* __restrict__ partial) {
  __shared__ double red[4];
  const int e0 = blockIdx.x * kVecChunk;
  for (int c = 0; c < R; ++c) {
    double acc = 0.0;
    const bool ver = verify[c] != 0;
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x) {
      double r = (double)B[(size_t)c * ldb + e] - Y[(size_t)c * N + e];
      if (ver) Rr[(size_t)c * N + e] = (T)r;
      acc += r * r;
    }
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)c * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

// Restart of the columns in `restart`: rz from the new M^{-1} r, active again.
__global__ void k_pcg_restart_scal(const double* __restrict__ rr_part, int nb_r, const double* __restrict__ rz_part,
                                   int nb_z, int R, const int* __restrict__ restart, PcgScal s) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wv; c < R; c += nw) {
    double rr = wave_out_sum(rr_part, nb_r, c);
    double rz = rz_part ? wave_out_sum(rz_part, nb_z, c) : rr;
    if ((threadIdx.x & 63) != 0) continue;
    s.rr[c] = rr;
    if (restart[c]) {
      s.rz[c] = rz;
      s.rz[R + c] = rz;
      s.active[c] = 1;
      s.active[R + c] = 1;
      atomicAdd(&s.flags[0], 1);
    }
  }
}

template <typename T>
__global__ void k_copy_cols_masked(const T* __restrict__ a, T* __restrict__ b, int N, int R,
                                   const int* __restrict__ mask) {
  const int e0 = blockIdx.x * kVecChunk;
  for (int c = 0; c < R; ++c) {
    if (!mask[c]) continue;
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x)
      b[(size_t)c * N + e] = a[(size_t)c * N + e];
  }
}

template <typename T>
__global__ void k_copy_cols(const T* __restrict__ a, T* __restrict__ b, int N, int R) {
  const int e0 = blockIdx.x * kVecChunk;
  for (int c = 0; c < R; ++c)
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x)
      b[(size_t)c * N + e] = a[(size_t)c * N + e];
}

template <typename TO>
__global__ void k_x_out(const double* __restrict__ Xd, int N, int R, TO* __restrict__ X, int ldx) {
  const int e0 = blockIdx.x * kVecChunk;
  for (int c = 0; c < R; ++c)
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x)
      X[(size_t)c * ldx + e] = (TO)Xd[(size_t)c * N + e];
}

// One PCG on R <= kPcgMaxR columns (history layout [alpha: R x max_iter][beta: R x max_iter]).
template <typename T>
static dski_status pcg_group(dski_plan p, dski_precond pc, int R, const T* B, int ldb, T* X, int ldx,
                             const double* tol_host, int max_iter, int fixed_iters, double* hist,
                             PcgResult& res, int res_c0, hipStream_t st, double* X64, int ldx64,
                             const int* verify_mask) {
  const int N = p->N, n = p->n;
  const int k = pc ? pc->k : 0;
  const size_t nr = (size_t)N * R;
  const int nbv = nchunks(N), nbg = gather_blocks(p), nbz = vec_blocks(N);
  ProjLds L = proj_lds(k, R, sizeof(T));
  const bool shfl = p->proj_variant == 1;
  const int ngs = (R + kShflGroup - 1) / kShflGroup;
  const int cgs = (R + ngs - 1) / ngs;
  const int nbt = shfl ? (N + 255) / 256 : (N + L.RT - 1) / L.RT;
  const size_t npart = (size_t)std::max(std::max(nbv, nbg), std::max(nbz, nbt)) * R;
  const size_t ntp = (size_t)nbt * std::max(k, 1) * R;
  // workspace: Rr, Z, P, Q (T), Xd, partials, t partials, t1, t2, coef, scalars
  size_t tb = ((sizeof(T) * nr * 4) + 63) / 64 * 64;
  size_t db = sizeof(double) * (nr + 3 * npart + ntp + 3 * (size_t)k * R + 12 * (size_t)R + 16);
  size_t ib = sizeof(int) * (4 * (size_t)R + 8);
  DSKI_TRY(p->vin.reserve(tb + db + ib + 512));
  char* base = p->vin.as<char>();
  T* Rr = reinterpret_cast<T*>(base);
  T* Z = Rr + nr;
  T* P = Z + nr;
  T* Q = P + nr;
  double* Xd = reinterpret_cast<double*>(base + tb);
  double* pq_part = Xd + nr;
  double* rr_part = pq_part + npart;
  double* rz_part = rr_part + npart;
  double* t_part = rz_part + npart;
  double* t1 = t_part + ntp;
  double* t2 = t1 + (size_t)k * R;
  double* coef = t2 + (size_t)k * R;
  PcgScal s;
  s.rz = coef + (size_t)k * R;
  s.rr = s.rz + 2 * R;
  s.bb = s.rr + R;
  s.alpha = s.bb + R;
  s.tol2 = s.alpha + R;
  double* rz0 = s.tol2 + R;
  s.active = reinterpret_cast<int*>(rz0 + R + 2);
  s.iters = s.active + 2 * R;
  s.flags = s.iters + R;
  std::vector<double> tol2(R);
  for (int r = 0; r < R; ++r) tol2[r] = tol_host ? tol_host[r] * tol_host[r] : 0.0;
  DSKI_HIP(hipMemcpyAsync(s.tol2, tol2.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
  DSKI_HIP(hipMemsetAsync(s.flags, 0, sizeof(int) * 2, st));
  k_pcg_init<T><<<nbv, kBlock, 0, st>>>(B, ldb, Rr, Xd, N, R, rr_part);
  const double* rzp = nullptr;
  const T* Zuse = Rr;
  if (pc) {
    DSKI_TRY(precond_apply_tiled<T>(pc, R, Rr, N, Z, N, rz_part, nullptr, st));
    rzp = rz_part;
    Zuse = Z;
  }
  k_copy_cols<T><<<nbv, kBlock, 0, st>>>(Zuse, P, N, R);
  k_pcg_init_scal<<<1, 256, 0, st>>>(rr_part, nbv, rzp, nbz, R, fixed_iters, s, rz0);
  DSKI_HIP(hipGetLastError());
  int* hflags = nullptr;
  DSKI_HIP(hipHostMalloc(&hflags, sizeof(int) * 2, hipHostMallocDefault));
  const T* U = pc ? u_of<T>(pc) : nullptr;
  const double isf = 1.0 / p->sf, isg = 1.0 / p->sg;
  dski_status rc = DSKI_OK;
  const int limit = fixed_iters > 0 ? fixed_iters : max_iter;
  int it = 0;
  auto run = [&]() -> dski_status {
    int check = 1;
    while (it < limit) {
      int burst = std::min(check, limit - it);
      for (int b = 0; b < burst; ++b) {
        const int par = (it + b) & 1;
        DSKI_TRY(mvm_tiled<T>(p, R, P, N, Q, N, pq_part, st));
        if (shfl)
          k_pcg_update_shfl<T><<<dim3(nbt, ngs), kBlock, 0, st>>>(P, Q, Rr, Xd, N, n, R, s, par, pq_part, nbg,
                                                                  rr_part, U, k, isf, isg, cgs, t_part, hist,
                                                                  max_iter);
        else
          k_pcg_update<T><<<nbt, kBlock, L.bytes, st>>>(P, Q, Rr, Xd, N, n, R, s, par, pq_part, nbg, rr_part, U,
                                                         k, isf, isg, L.RT, L, t_part, hist, max_iter);
        RedJob jr{rr_part, nbt, R, R, s.rr, nullptr, nullptr, 0.0, nullptr, s.active + par * R};
        if (pc && k > 0) {
          RedJob jt{t_part, nbt, k * R, R, t1, pc->c, nullptr, 1.0, coef, nullptr};
          DSKI_TRY(launch_reduce(jt, &jr, st));
          if (shfl) {
            int nbx = 0;
            launch_proj_shfl<T>(Rr, N, N, n, R, isf, isg, U, k, coef, t_part, &nbx, st);
          } else {
            k_ts_proj<T><<<nbt, kBlock, L.bytes, st>>>(Rr, N, N, n, R, isf, isg, U, k, coef, L.RT, L, t_part);
          }
          RedJob j2{t_part, nbt, k * R, R, t2, pc->c, t1, 1.0, coef, nullptr};
          DSKI_TRY(launch_reduce(j2, nullptr, st));
          launch_final<T>(Rr, N, N, n, R, isf, isg, isf, isg, U, k, coef, Z, N, rz_part, st);
        } else {
          DSKI_TRY(launch_reduce(jr, nullptr, st));
          if (pc)  // rank-0 preconditioner: M = D
            launch_final<T>(Rr, N, N, n, R, isf, isg, isf, isg, U, 0, nullptr, Z, N,
                                                 rz_part, st);
        }
        k_pcg_beta<T><<<dim3(nbz, R), kBlock, 0, st>>>(pc ? Z : Rr, P, N, R, s, par, pc ? rz_part : nullptr,
                                                       nbz, hist, max_iter, fixed_iters);
      }
      it += burst;
      DSKI_HIP(hipGetLastError());
      DSKI_HIP(hipMemcpyAsync(hflags, s.flags, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
      DSKI_HIP(hipStreamSynchronize(st));
      if (hflags[1]) {
        set_error("PCG breakdown: p^T K p <= 0 or r^T M^{-1} r < 0");
        return DSKI_EBREAKDOWN;
      }
      if (hflags[0] <= 0) break;
      check = std::min(check * 2, 32);
    }
    return DSKI_OK;
  };
  rc = run();
  // True-residual verification: columns that met the tolerance on the recurrence
  // residual are checked with b - K~ x (FP64 iterate, FP64-storage operator) and
  // resumed from x if still above it (at most 3 rounds).
  std::vector<int> ver(R, 0);
  bool any_ver = false;
  for (int r = 0; r < R; ++r) {
    ver[r] = verify_mask ? verify_mask[r] : 0;
    any_ver = any_ver || ver[r];
  }
  std::vector<double> true_rr;
  if (rc == DSKI_OK && fixed_iters <= 0 && any_ver) {
    DevBuf ybuf;
    int* dmask = nullptr;
    for (int round = 0; round < 3 && rc == DSKI_OK; ++round) {
      if (ybuf.reserve(sizeof(double) * nr + sizeof(int) * 2 * (size_t)R + 64) < 0) {
        rc = DSKI_ENOMEM;
        break;
      }
      double* Y = ybuf.as<double>();
      dmask = reinterpret_cast<int*>(Y + nr);
      int* drestart = dmask + R;
      rc = mvm_tiled<double>(p, R, Xd, N, Y, N, nullptr, st);
      if (rc < 0) break;
      DSKI_HIP(hipMemcpyAsync(dmask, ver.data(), sizeof(int) * R, hipMemcpyHostToDevice, st));
      k_true_resid<T><<<nbv, kBlock, 0, st>>>(B, ldb, Y, Rr, N, R, dmask, rr_part);
      std::vector<double> hrt(R), hbb(R);
      RedJob jq{rr_part, nbv, R, R, t2, nullptr, nullptr, 0.0, nullptr, nullptr};
      DSKI_TRY(launch_reduce(jq, nullptr, st));
      DSKI_HIP(hipMemcpyAsync(hrt.data(), t2, sizeof(double) * R, hipMemcpyDeviceToHost, st));
      DSKI_HIP(hipMemcpyAsync(hbb.data(), s.bb, sizeof(double) * R, hipMemcpyDeviceToHost, st));
      DSKI_HIP(hipStreamSynchronize(st));
      true_rr = hrt;
      std::vector<int> restart(R, 0);
      int nre = 0;
      for (int r = 0; r < R; ++r) {
        if (ver[r] && hrt[r] > tol2[r] * hbb[r] * (1.0 + 1e-12)) {
          restart[r] = 1;
          ++nre;
        }
      }
      if (nre == 0 || it >= limit) break;
      DSKI_HIP(hipMemcpyAsync(drestart, restart.data(), sizeof(int) * R, hipMemcpyHostToDevice, st));
      // r (true, already in Rr for verified columns), z = M^{-1} r, p = z for the restarted columns
      const double* rzp2 = nullptr;
      const T* Zuse2 = Rr;
      if (pc) {
        rc = precond_apply_tiled<T>(pc, R, Rr, N, Z, N, rz_part, nullptr, st);
        if (rc < 0) break;
        rzp2 = rz_part;
        Zuse2 = Z;
      }
      k_copy_cols_masked<T><<<nbv, kBlock, 0, st>>>(Zuse2, P, N, R, drestart);
      DSKI_HIP(hipMemsetAsync(s.flags, 0, sizeof(int) * 2, st));
      k_pcg_restart_scal<<<1, 256, 0, st>>>(rr_part, nbv, rzp2, nbz, R, drestart, s);
      DSKI_HIP(hipGetLastError());
      rc = run();
    }
    ybuf.release();
  }
  (void)hipHostFree(hflags);
  if (rc < 0 && rc != DSKI_EBREAKDOWN) return rc;
  if (X) k_x_out<T><<<nbv, kBlock, 0, st>>>(Xd, N, R, X, ldx);
  if (X64) k_x_out<double><<<nbv, kBlock, 0, st>>>(Xd, N, R, X64, ldx64);
  DSKI_HIP(hipGetLastError());
  std::vector<double> hrr(R), hbb(R), hrz0(R);
  std::vector<int> hit(R);
  DSKI_HIP(hipMemcpyAsync(hit.data(), s.iters, sizeof(int) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hrr.data(), s.rr, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hbb.data(), s.bb, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hrz0.data(), rz0, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  bool notconv = false;
  for (int r = 0; r < R; ++r) {
    res.iters[res_c0 + r] = hit[r];
    res.rz0[res_c0 + r] = hrz0[r];
    double rr = (!true_rr.empty() && ver[r]) ? true_rr[r] : hrr[r];
    res.relres[res_c0 + r] = hbb[r] > 0 ? std::sqrt(std::max(rr, 0.0) / hbb[r]) : 0.0;
    if (fixed_iters <= 0 && tol_host && res.relres[res_c0 + r] > tol_host[r]) notconv = true;
  }
  if (rc == DSKI_EBREAKDOWN) {
    res.breakdown = true;
    return rc;
  }
  return notconv ? DSKI_NOT_CONVERGED : DSKI_OK;
}

template <typename T>
dski_status pcg_tiled(dski_plan p, dski_precond pc, int R, const T* B, int ldb, T* X, int ldx,
                      const double* tol_host, int max_iter, int fixed_iters, double* alpha_beta,
                      PcgResult& res, hipStream_t st, double* X64, const int* verify_mask) {
  res.iters.assign(R, 0);
  res.relres.assign(R, 0.0);
  res.rz0.assign(R, 0.0);
  if (R <= 0) return DSKI_OK;
  if (R > kPcgMaxR && alpha_beta) {
    set_error("PCG with a CG-coefficient history supports at most %d columns per call", kPcgMaxR);
    return DSKI_ENOTSUP;
  }
  dski_status worst = DSKI_OK;
  for (int c0 = 0; c0 < R; c0 += kPcgMaxR) {
    int rg = std::min(kPcgMaxR, R - c0);
    dski_status rc = pcg_group<T>(p, pc, rg, B + (size_t)c0 * ldb, ldb, X ? X + (size_t)c0 * ldx : nullptr, ldx,
                                  tol_host + c0, max_iter, fixed_iters, alpha_beta, res, c0, st,
                                  X64 ? X64 + (size_t)c0 * ldx : nullptr, ldx,
                                  verify_mask ? verify_mask + c0 : nullptr);
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
  }
  return worst;
}
template dski_status pcg_tiled<float>(dski_plan, dski_precond, int, const float*, int, float*, int,
                                      const double*, int, int, double*, PcgResult&, hipStream_t, double*,
                                      const int*);
template dski_status pcg_tiled<double>(dski_plan, dski_precond, int, const double*, int, double*, int,
                                       const double*, int, int, double*, PcgResult&, hipStream_t,
                                       double*, const int*);

}  // namespace dski

using namespace dski;

template <typename T>
static dski_status pcg_user(dski_plan p, dski_precond pc, int R, const T* B, int ldb, double* X, int ldx,
                            const double* tol_host, int max_iter, int* iters_host, double* relres_host,
                            double* alpha_beta, hipStream_t st) {
  if (!p || R < 0 || ldb < p->N || ldx < p->N || (R > 0 && (!B || !X || !tol_host)) || max_iter < 0 ||
      (pc && pc->plan != p)) {
    set_error("pcg_solve: bad arguments");
    return DSKI_EINVAL;
  }
  if (R == 0 || p->N == 0) return DSKI_OK;
  size_t nr = (size_t)p->N * R;
  // user -> tile order (B and X in vout; the PCG itself uses vin as workspace)
  DSKI_TRY(p->vout.reserve(sizeof(T) * nr + sizeof(double) * nr + 64));
  T* Bt = p->vout.as<T>();
  double* Xt = reinterpret_cast<double*>(p->vout.as<char>() + ((sizeof(T) * nr + 63) / 64) * 64);
  DSKI_TRY(permute(p, +1, R, B, ldb, Bt, p->N, st));
  PcgResult res;
  // without a CG-coefficient history every column gets the true-residual check
  std::vector<int> verify(R, alpha_beta ? 0 : 1);
  dski_status rc = pcg_tiled<T>(p, pc, R, Bt, p->N, nullptr, p->N, tol_host, max_iter, 0, alpha_beta, res, st,
                                Xt, verify.data());
  if (rc < 0 && rc != DSKI_EBREAKDOWN) return rc;
  DSKI_TRY(permute(p, -1, R, Xt, p->N, X, ldx, st));
  DSKI_HIP(hipStreamSynchronize(st));
  for (int r = 0; r < R; ++r) {
    if (iters_host) iters_host[r] = res.iters[r];
    if (relres_host) relres_host[r] = res.relres[r];
  }
  return rc;
}

extern "C" {

dski_status pcg_solve(dski_plan p, dski_precond pc, int R, const float* B, int ldb, double* X, int ldx,
                      const double* tol_host, int max_iter, int* iters_host, double* relres_host,
                      double* alpha_beta, dski_stream stream) {
  return pcg_user<float>(p, pc, R, B, ldb, X, ldx, tol_host, max_iter, iters_host, relres_host, alpha_beta,
                         static_cast<hipStream_t>(stream));
}

dski_status pcg_solve_f64(dski_plan p, dski_precond pc, int R, const double* B, int ldb, double* X,
                          int ldx, const double* tol_host, int max_iter, int* iters_host,
                          double* relres_host, double* alpha_beta, dski_stream stream) {
  return pcg_user<double>(p, pc, R, B, ldb, X, ldx, tol_host, max_iter, iters_host, relres_host,
                          alpha_beta, static_cast<hipStream_t>(stream));
}

}  // extern "C"
