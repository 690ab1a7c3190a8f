// Preconditioned conjugate gradients on a block of R right-hand sides (Sec. 2,
// Sec. 3.3).  The columns are independent CG runs that share every MVM (the
// block is not a block-Krylov method, so each column keeps its own Lanczos
// tridiagonal for quadrature).  Vectors are FP32 (or FP64) in tile order, the iterate x
// is accumulated in FP64, all inner products and scalars are FP64 and live on
// the device; the host only polls the number of active columns every few
// iterations.
#include <cmath>

#include "internal.h"

namespace dski {

struct PcgScal {
  double* rz;     // r^T M^{-1} r
  double* rr;     // r^T r
  double* bb;     // b^T b
  double* alpha;
  double* beta;
  double* tol2;
  int* active;
  int* iters;
  int* flags;     // [0] number of active columns, [1] breakdown
};

constexpr int kVecChunk = 1024;  // elements per work-group in the vector kernels

static int nchunks(int N) { return (N + kVecChunk - 1) / kVecChunk; }

// R = B, X = 0, partials of b.b
template <typename T>
__global__ void k_pcg_init(const T* __restrict__ B, int ldb, T* __restrict__ Rr,
                           double* __restrict__ Xd, int N, int R, double* __restrict__ partial) {
  int r = blockIdx.y;
  int e0 = blockIdx.x * kVecChunk;
  double acc = 0.0;
  for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x) {
    T b = B[(size_t)r * ldb + e];
    Rr[(size_t)r * N + e] = b;
    Xd[(size_t)r * N + e] = 0.0;
    acc += (double)b * (double)b;
  }
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * R + r] = red[0] + red[1] + red[2] + red[3];
}

__device__ double block_sum_col(const double* __restrict__ partial, int nblk, int R, int r) {
  __shared__ double buf[kBlock];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) a += partial[(size_t)b * R + r];
  buf[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) buf[threadIdx.x] += buf[threadIdx.x + off];
    __syncthreads();
  }
  double v = buf[0];
  __syncthreads();
  return v;
}

// After the initial preconditioner application: rz, bb, rr, active flags.
__global__ void k_pcg_init_scal(const double* __restrict__ bb_part, int nb_b,
                                const double* __restrict__ rz_part, int nb_z, int R,
                                int fixed_iters, PcgScal s, double* __restrict__ rz0) {
  int r = blockIdx.x;
  double bb = block_sum_col(bb_part, nb_b, R, r);
  double rz = rz_part ? block_sum_col(rz_part, nb_z, R, r) : bb;
  if (threadIdx.x == 0) {
    s.bb[r] = bb;
    s.rr[r] = bb;
    s.rz[r] = rz;
    rz0[r] = rz;
    s.iters[r] = 0;
    int act = bb > 0.0 && (fixed_iters > 0 || bb > s.tol2[r] * bb);
    s.active[r] = act;
    if (act) atomicAdd(&s.flags[0], 1);
  }
}

// alpha = r^T z / p^T q
__global__ void k_pcg_alpha(const double* __restrict__ pq_part, int nblk, int R, PcgScal s,
                            double* __restrict__ hist, int max_iter) {
  int r = blockIdx.x;
  double pq = block_sum_col(pq_part, nblk, R, r);
  if (threadIdx.x == 0) {
    double a = 0.0;
    if (s.active[r]) {
      if (!(pq > 0.0) || !isfinite(pq)) {
        s.flags[1] = 1;
      } else {
        a = s.rz[r] / pq;
      }
      if (hist && s.iters[r] < max_iter) hist[(size_t)r * max_iter + s.iters[r]] = a;
    }
    s.alpha[r] = a;
  }
}

// x += alpha p (FP64), r -= alpha q; partials of r.r
template <typename T>
__global__ void k_pcg_update_xr(const T* __restrict__ P, const T* __restrict__ Q,
                                T* __restrict__ Rr, double* __restrict__ Xd, int N, int R,
                                PcgScal s, double* __restrict__ partial) {
  int r = blockIdx.y;
  int e0 = blockIdx.x * kVecChunk;
  double acc = 0.0;
  if (s.active[r]) {
    double a = s.alpha[r];
    for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x) {
      size_t i = (size_t)r * N + e;
      Xd[i] += a * (double)P[i];
      T rn = (T)((double)Rr[i] - a * (double)Q[i]);
      Rr[i] = rn;
      acc += (double)rn * (double)rn;
    }
  }
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * R + r] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_pcg_rr(const double* __restrict__ part, int nblk, int R, PcgScal s) {
  int r = blockIdx.x;
  double v = block_sum_col(part, nblk, R, r);
  if (threadIdx.x == 0 && s.active[r]) s.rr[r] = v;
}

// beta = r'^T z' / r^T z, history, convergence test, active count
__global__ void k_pcg_beta(const double* __restrict__ rz_part, int nblk, int R, PcgScal s,
                           double* __restrict__ hist, int max_iter, int fixed_iters) {
  int r = blockIdx.x;
  double rzn = rz_part ? block_sum_col(rz_part, nblk, R, r) : 0.0;
  if (threadIdx.x == 0) {
    if (!rz_part) rzn = s.rr[r];
    double b = 0.0;
    if (s.active[r]) {
      if (!(rzn >= 0.0) || !isfinite(rzn)) s.flags[1] = 1;
      b = s.rz[r] > 0.0 ? rzn / s.rz[r] : 0.0;
      int it = s.iters[r];
      if (hist && it < max_iter) hist[(size_t)R * max_iter + (size_t)r * max_iter + it] = b;
      s.iters[r] = it + 1;
      s.rz[r] = rzn;
      bool done = fixed_iters > 0 ? (it + 1 >= fixed_iters) : (s.rr[r] <= s.tol2[r] * s.bb[r]);
      if (done) {
        s.active[r] = 0;
        atomicSub(&s.flags[0], 1);
      }
    }
    s.beta[r] = b;
  }
}

template <typename T>
__global__ void k_pcg_update_p(const T* __restrict__ Z, T* __restrict__ P, int N, PcgScal s) {
  int r = blockIdx.y;
  if (!s.active[r]) return;
  double b = s.beta[r];
  int e0 = blockIdx.x * kVecChunk;
  for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x) {
    size_t i = (size_t)r * N + e;
    P[i] = (T)((double)Z[i] + b * (double)P[i]);
  }
}

template <typename T>
__global__ void k_copy_f(const T* __restrict__ a, T* __restrict__ b, int N, int R) {
  int r = blockIdx.y;
  int e0 = blockIdx.x * kVecChunk;
  for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x)
    b[(size_t)r * N + e] = a[(size_t)r * N + e];
}

template <typename TO>
__global__ void k_x_out(const double* __restrict__ Xd, int N, TO* __restrict__ X, int ldx) {
  int r = blockIdx.y;
  int e0 = blockIdx.x * kVecChunk;
  for (int e = e0 + threadIdx.x; e < min(N, e0 + kVecChunk); e += blockDim.x)
    X[(size_t)r * ldx + e] = (TO)Xd[(size_t)r * N + e];
}

template <typename T>
dski_status pcg_tiled(dski_plan p, dski_precond pc, int R, const T* B, int ldb, T* X, int ldx,
                      const double* tol_host, int max_iter, int fixed_iters, double* alpha_beta,
                      PcgResult& res, hipStream_t st, double* X64) {
  int N = p->N;
  res.iters.assign(R, 0);
  res.relres.assign(R, 0.0);
  res.rz0.assign(R, 0.0);
  if (R <= 0) return DSKI_OK;
  // workspace: Rr, Z, P, Q (FP32), Xd (FP64), partials, scalars
  size_t nr = (size_t)N * R;
  int nbv = nchunks(N);
  int nbg = gather_blocks(p);
  int nbz = vec_blocks(N);
  int npart = std::max(nbv, std::max(nbg, nbz));
  size_t fbytes = sizeof(T) * nr * 4;
  size_t dbytes = sizeof(double) * (nr + (size_t)npart * R * 2 + 8 * (size_t)R + 8);
  size_t ibytes = sizeof(int) * (2 * (size_t)R + 8);
  DevBuf& wb = p->vin;  // shares the plan's vector workspace
  DSKI_TRY(wb.reserve(fbytes + dbytes + ibytes + 512));
  char* base = wb.as<char>();
  T* Rr = reinterpret_cast<T*>(base);
  T* Z = Rr + nr;
  T* P = Z + nr;
  T* Q = P + nr;
  double* Xd = reinterpret_cast<double*>(Q + nr);
  double* part1 = Xd + nr;
  double* part2 = part1 + (size_t)npart * R;
  PcgScal s;
  s.rz = part2 + (size_t)npart * R;
  s.rr = s.rz + R;
  s.bb = s.rr + R;
  s.alpha = s.bb + R;
  s.beta = s.alpha + R;
  s.tol2 = s.beta + R;
  double* rz0 = s.tol2 + R;
  s.active = reinterpret_cast<int*>(rz0 + R + 1);
  s.iters = s.active + R;
  s.flags = s.iters + R;
  std::vector<double> tol2(R);
  for (int r = 0; r < R; ++r) tol2[r] = tol_host ? tol_host[r] * tol_host[r] : 0.0;
  DSKI_HIP(hipMemcpyAsync(s.tol2, tol2.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
  DSKI_HIP(hipMemsetAsync(s.flags, 0, sizeof(int) * 2, st));
  dim3 vg(nbv, R);
  k_pcg_init<T><<<vg, kBlock, 0, st>>>(B, ldb, Rr, Xd, N, R, part1);
  // z = M^{-1} r, p = z
  const double* rzp = nullptr;
  T* Zuse = Rr;
  int nbzz = 0;
  if (pc) {
    DSKI_TRY(precond_apply_tiled<T>(pc, R, Rr, N, Z, N, part2, &nbzz, st));
    rzp = part2;
    Zuse = Z;
  }
  k_copy_f<T><<<vg, kBlock, 0, st>>>(Zuse, P, N, R);
  k_pcg_init_scal<<<R, kBlock, 0, st>>>(part1, nbv, rzp, nbzz, R, fixed_iters, s, rz0);
  DSKI_HIP(hipGetLastError());
  int* hflags = nullptr;
  DSKI_HIP(hipHostMalloc(&hflags, sizeof(int) * 2, hipHostMallocDefault));
  dski_status rc = DSKI_OK;
  int limit = fixed_iters > 0 ? fixed_iters : max_iter;
  int it = 0;
  int check = 1;
  while (it < limit) {
    int burst = std::min(check, limit - it);
    for (int b = 0; b < burst; ++b) {
      rc = mvm_tiled<T>(p, R, P, N, Q, N, part1, st);
      if (rc < 0) break;
      k_pcg_alpha<<<R, kBlock, 0, st>>>(part1, nbg, R, s, alpha_beta, max_iter);
      k_pcg_update_xr<T><<<vg, kBlock, 0, st>>>(P, Q, Rr, Xd, N, R, s, part2);
      k_pcg_rr<<<R, kBlock, 0, st>>>(part2, nbv, R, s);
      if (pc) {
        rc = precond_apply_tiled<T>(pc, R, Rr, N, Z, N, part1, &nbzz, st);
        if (rc < 0) break;
        k_pcg_beta<<<R, kBlock, 0, st>>>(part1, nbzz, R, s, alpha_beta, max_iter, fixed_iters);
        k_pcg_update_p<T><<<vg, kBlock, 0, st>>>(Z, P, N, s);
      } else {
        k_pcg_beta<<<R, kBlock, 0, st>>>(nullptr, 0, R, s, alpha_beta, max_iter, fixed_iters);
        k_pcg_update_p<T><<<vg, kBlock, 0, st>>>(Rr, P, N, s);
      }
    }
    if (rc < 0) break;
    it += burst;
    if (hipGetLastError() != hipSuccess) {
      set_error("PCG kernel launch failed");
      rc = DSKI_EHIP;
      break;
    }
    if (hipMemcpyAsync(hflags, s.flags, sizeof(int) * 2, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("PCG synchronisation failed");
      rc = DSKI_EHIP;
      break;
    }
    if (hflags[1]) {
      set_error("PCG breakdown: p^T K p <= 0 or r^T M^{-1} r < 0");
      rc = DSKI_EBREAKDOWN;
      break;
    }
    if (hflags[0] <= 0) break;
    check = std::min(check * 2, 32);
  }
  (void)hipHostFree(hflags);
  if (rc < 0 && rc != DSKI_EBREAKDOWN) return rc;
  if (X) k_x_out<T><<<vg, kBlock, 0, st>>>(Xd, N, X, ldx);
  if (X64) k_x_out<double><<<vg, kBlock, 0, st>>>(Xd, N, X64, ldx);
  DSKI_HIP(hipGetLastError());
  std::vector<double> hrr(R), hbb(R), hrz0(R);
  DSKI_HIP(hipMemcpyAsync(res.iters.data(), s.iters, sizeof(int) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hrr.data(), s.rr, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(hbb.data(), s.bb, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipMemcpyAsync(res.rz0.data(), rz0, sizeof(double) * R, hipMemcpyDeviceToHost, st));
  DSKI_HIP(hipStreamSynchronize(st));
  bool notconv = false;
  for (int r = 0; r < R; ++r) {
    res.relres[r] = hbb[r] > 0 ? std::sqrt(std::max(hrr[r], 0.0) / hbb[r]) : 0.0;
    if (fixed_iters <= 0 && tol_host && res.relres[r] > tol_host[r]) notconv = true;
  }
  if (rc == DSKI_EBREAKDOWN) {
    res.breakdown = true;
    return rc;
  }
  return notconv ? DSKI_NOT_CONVERGED : DSKI_OK;
}

template dski_status pcg_tiled<float>(dski_plan, dski_precond, int, const float*, int, float*, int,
                                      const double*, int, int, double*, PcgResult&, hipStream_t, double*);
template dski_status pcg_tiled<double>(dski_plan, dski_precond, int, const double*, int, double*, int,
                                       const double*, int, int, double*, PcgResult&, hipStream_t,
                                       double*);

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
  dski_status rc =
      pcg_tiled<T>(p, pc, R, Bt, p->N, nullptr, p->N, tol_host, max_iter, 0, alpha_beta, res, st, Xt);
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
