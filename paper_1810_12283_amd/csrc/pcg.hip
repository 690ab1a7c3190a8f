// Preconditioned conjugate gradients on a block of R right-hand sides (Sec. 2,
// Sec. 3.3).  The columns are independent CG runs that share every MVM (the
// block is not a block-Krylov method, so each column keeps its own Lanczos
// tridiagonal for quadrature).  Vectors are FP32 (or FP64) in tile order, the
// iterate x is accumulated in FP64, all inner products and scalars are FP64 and
// live on the device; the host only polls the number of active columns.
//
// One iteration is 8 launches (9 with the FFT of a 3-D grid):
//   scatter | K_UU per axis | gather (+ partials of p.q)
//   update:  alpha (every block reduces the p.q partials itself, same order),
//            x += alpha p, r -= alpha q, partials of r.r and of U^T D^{-1/2} r
//   reduce:  t = U^T r', coef = w .* t; r.r
//   final:   z = D^{-1/2}(r' - U coef) (+ partials of r.z)
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
  double* rrd;    // [R] |D^{-1/2} r|^2 (current), right after rr: one reduction writes both
  double* bb;     // [R] b^T b
  double* alpha;  // [R]
  double* tol2;   // [R]
  int* active;    // [2][R] by parity
  int* iters;     // [R]
  int* flags;     // [0] active columns, [1] breakdown
};

constexpr int kVecChunk = 1024;  // rows per work-group in the streaming vector kernels
constexpr int kGraphIters = 8;   // PCG iterations per captured HIP graph
constexpr int kReplaceEvery = 256;  // iterations between residual replacements (FP32 vectors)

// Captured iterations of one solve (side stream, ordering events, graph).
struct PcgGraph {
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int par0 = -1;
  void reset_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    par0 = -1;
  }
  ~PcgGraph() {
    if (stream) (void)hipStreamSynchronize(stream);
    reset_graph();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

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

// alpha, the r update, partials of r.r, |D^{-1/2} r|^2 and U^T D^{-1/2} r.  A wavefront
// takes 32 rows (each lane one row and half of the columns), keeps the new r in
// LDS and projects it on the FP64 matrix cores (the first 16 columns, and the
// next 16 when RB > 20) with up to 4 remaining columns on the vector ALU.  Four
// wavefronts form a work-group of 128 rows, and two work-groups share a CU, so
// that one's loads overlap the other's products.  The four wavefronts' partials
// are added in LDS in a fixed order and written once per work-group,
// block-major (t_part[b k R + i R + c], rr_part[b 2 R + c] and [b 2 R + R + c]).
// RB = R padded to a multiple of 4.
constexpr int kPqRegs = 16;  // p.q partials per lane held in registers (8 lanes: 128 blocks)
constexpr int kUpdRows = 32;   // rows per wavefront
constexpr int kUpdWaves = 4;   // wavefronts per work-group
static int upd_blocks(int N) { return (N + kUpdRows * kUpdWaves - 1) / (kUpdRows * kUpdWaves); }

template <int RB>
struct UpdShape {
  static constexpr int MB = RB <= 20 ? 1 : 2;           // matrix-core column blocks
  static constexpr int VR = RB > 16 && RB <= 20 ? RB - 16 : 0;  // vector-ALU columns
  static constexpr int CW = RB > 16 * MB ? RB : 16 * MB;  // columns held per row (zeros beyond R)
  static constexpr int HC = CW / 2;                     // columns per lane (two lanes per row)
  static constexpr int XP = CW + 1;                     // LDS row stride of the new r
  static constexpr int TB = 64 * CW;                    // one group of 64 outputs i per column
  template <typename T>
  static constexpr size_t bytes() {
    return kUpdWaves * sizeof(T) * (size_t)kUpdRows * XP + sizeof(double) * kUpdWaves * (size_t)TB;
  }
};

template <typename T, int RB, bool PC>
__global__ __launch_bounds__(256, 2) void k_pcg_update(const T* __restrict__ Q, T* __restrict__ Rr, int N, int n,
                                                       int R, PcgScal s, int par,
                                                       const double* __restrict__ pq_part, int nb_pq,
                                                       double* __restrict__ rr_part,
                                                       const double* __restrict__ Ur, int k, double isf, double isg,
                                                       double* __restrict__ t_part, double* __restrict__ hist,
                                                       int max_iter) {
  using S = UpdShape<RB>;
  constexpr int XP = S::XP, MB = S::MB, VR = S::VR, CW = S::CW, HC = S::HC, UR = kUpdRows, NS = UR / 4;
  static_assert(kUpdWaves * 64 == kBlock, "one work-group of kBlock threads");
  extern __shared__ __align__(16) char smem[];
  T* sx = reinterpret_cast<T*>(smem) + (size_t)(threadIdx.x >> 6) * UR * XP;
  double* st = reinterpret_cast<double*>(smem + kUpdWaves * sizeof(T) * (size_t)UR * XP);  // kUpdWaves x TB
  __shared__ double s_alpha[kPcgMaxR];
  __shared__ int s_act[kPcgMaxR];
  __shared__ double s_rr[kUpdWaves][RB], s_rrd[kUpdWaves][RB];
  const int* act = s.active + par * R;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int e0 = (blockIdx.x * kUpdWaves + wv) * UR;
  const int rl = lane & (UR - 1), hh = lane / UR;  // this lane's row and half of the columns
  const int e = e0 + rl;
  // Every load of the kernel is issued before the first wait, in the order
  // their values are needed (loads complete in order): the column state and
  // the p.q partials for alpha, this lane's row of r and q, then the
  // projection's operands.
  // alpha: 8 lanes per column; lane j adds blocks j, j + 8, ... in order
  const int c_al = threadIdx.x >> 3, j_al = threadIdx.x & 7;
  const bool col = c_al < R;
  const int on_al = col ? act[c_al] : 0;
  const double rz_al = col ? s.rz[par * R + c_al] : 0.0;
  const double* pqc = pq_part + (size_t)(col ? c_al : 0) * nb_pq;
  double pqv[kPqRegs];
#pragma unroll
  for (int u = 0; u < kPqRegs; ++u) pqv[u] = ld_or0(pqc, (size_t)(j_al + 8 * u), 0, col && j_al + 8 * u < nb_pq);
  const bool in = e < N;  // rows past N (and wavefronts past the last row) act as zeros
  // r and q of this lane's row, its half of the columns (q of a finished
  // column is read and not used)
  T rv[HC], qv[HC];
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;
    const size_t idx = (size_t)(c < R ? c : 0) * N + (in ? e : 0);
    rv[j] = Rr[idx];
    qv[j] = Q[idx];
  }
  // A operands of the projection (U rows e0 + 4 s + kq, columns i0 + 16 b +
  // l % 16).  The indices are clamped into U instead of masked: a row past N
  // meets a zero B row, and an output i >= k is never written, so whatever
  // finite entry of U stands in adds nothing that is kept.
  double aop[NS][4];
  const size_t nk_last = (size_t)N * (size_t)(k > 0 ? k : 1) - 1;
  auto load_u = [&](int i0) {  // row-major U: 4 rows x 16 consecutive columns per load
#pragma unroll
    for (int s4 = 0; s4 < NS; ++s4) {
      const int er = e0 + 4 * s4 + kq;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const size_t i = (size_t)er * k + (size_t)(i0 + 16 * b + r16);
        aop[s4][b] = Ur[i < nk_last ? i : nk_last];
      }
    }
  };
  // (PC: k > 0, a compile-time branch, so that the loads stay in one basic
  // block and the wait for the partials below does not cover them)
  if (PC) load_u(0);
  {
    double pq = 0.0;
#pragma unroll
    for (int u = 0; u < kPqRegs; ++u) pq += pqv[u];
    for (int b = j_al + 8 * kPqRegs; b < nb_pq; b += 8) pq += ld_or0(pqc, (size_t)b, 0, col);
    pq += __shfl_xor(pq, 1, 64);
    pq += __shfl_xor(pq, 2, 64);
    pq += __shfl_xor(pq, 4, 64);
    if (col && j_al == 0) {
      const int c = c_al;
      double a = 0.0;
      if (on_al) {
        if (!(pq > 0.0) || !isfinite(pq)) {
          if (blockIdx.x == 0) s.flags[1] = 1;
        } else {
          a = rz_al / pq;
        }
        if (blockIdx.x == 0 && hist && s.iters[c] < max_iter) hist[(size_t)c * max_iter + s.iters[c]] = a;
      }
      if (blockIdx.x == 0) s.alpha[c] = a;
      s_alpha[c] = a;
      s_act[c] = on_al;
    }
  }
  __syncthreads();
  // r -= alpha q on this lane's row and columns (x += alpha p is done by the
  // beta kernel, which reads p anyway); every column below CW goes to LDS
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;
    const bool ok = in && c < R;
    if (ok && s_act[c]) {
      const T rnew = (T)((double)rv[j] - s_alpha[c] * (double)qv[j]);
      Rr[(size_t)c * N + e] = rnew;
      rv[j] = rnew;
    }
    sx[rl * XP + c] = ok ? rv[j] : (T)0;
  }
  wave_lds_fence();
  {  // |r|^2 and |D^{-1/2} r|^2 of every column over the 32 rows: lane c + 32 h sums rows 16 h ..
    const int c = lane & 31, h = lane >> 5;
    const double isf2 = isf * isf, isg2 = isg * isg;
    double acc = 0.0, accd = 0.0;
    if (c < RB) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double v = (double)sx[(16 * h + j) * XP + c], vv = v * v;
        acc += vv;
        accd += vv * (e0 + 16 * h + j < n ? isf2 : isg2);
      }
    }
    acc += __shfl_xor(acc, 32, 64);
    accd += __shfl_xor(accd, 32, 64);
    if (h == 0 && c < RB) {
      s_rr[wv][c] = acc;
      s_rrd[wv][c] = accd;
    }
  }
  // scaled B operands of the projection: rows 4 s + kq of the 32
  double bop[NS][MB], rsc[NS];
#pragma unroll
  for (int s4 = 0; s4 < NS; ++s4) {
    const int row = 4 * s4 + kq;
    rsc[s4] = e0 + row < n ? isf : isg;
#pragma unroll
    for (int cb = 0; cb < MB; ++cb) bop[s4][cb] = rsc[s4] * (double)sx[row * XP + 16 * cb + r16];
  }
  __syncthreads();  // s_rr complete
  if (threadIdx.x < R) {  // block-major, 2 R per block: |r|^2, then |D^{-1/2} r|^2
    const int c = threadIdx.x;
    rr_part[(size_t)blockIdx.x * 2 * R + c] = (s_rr[0][c] + s_rr[1][c]) + (s_rr[2][c] + s_rr[3][c]);
    rr_part[(size_t)blockIdx.x * 2 * R + R + c] = (s_rrd[0][c] + s_rrd[1][c]) + (s_rrd[2][c] + s_rrd[3][c]);
  }
  const int KR = k * R;
  for (int i0 = 0; PC && i0 < k; i0 += 64) {  // groups of four 16-column blocks of U
    dski_pdbl4 acc[4][MB];
    double vacc[4][VR > 0 ? VR : 1];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int cb = 0; cb < MB; ++cb) acc[b][cb] = dski_pdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int v = 0; v < VR; ++v) vacc[b][v] = 0.0;
    }
    if (i0 > 0) load_u(i0);
#pragma unroll
    for (int s4 = 0; s4 < NS; ++s4) {
      double vop[VR > 0 ? VR : 1];
#pragma unroll
      for (int v = 0; v < VR; ++v) vop[v] = rsc[s4] * (double)sx[(4 * s4 + kq) * XP + 16 + v];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int cb = 0; cb < MB; ++cb)
          acc[b][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[s4][b], bop[s4][cb], acc[b][cb], 0, 0, 0);
#pragma unroll
        for (int v = 0; v < VR; ++v) vacc[b][v] += aop[s4][b] * vop[v];
      }
    }
    // this wavefront's 64 x RB block of t: matrix-core part (register r of lane
    // l: i = 16 b + l / 16 + 4 r, c = 16 cb + l % 16), vector part summed over
    // the four lanes that share i
    double* mine = st + (size_t)wv * S::TB;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int cb = 0; cb < MB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[(16 * b + kq + 4 * r) * CW + 16 * cb + r16] = acc[b][cb][r];
#pragma unroll
      for (int v = 0; v < VR; ++v) {
        double x = vacc[b][v];
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        if (kq == 0) mine[(16 * b + r16) * CW + 16 + v] = x;
      }
    }
    __syncthreads();
    // the block's partial, four wavefronts in a fixed order, written coalesced
    for (int f = threadIdx.x; f < 64 * R; f += 256) {
      const int il = f / R, c = f - il * R, i = i0 + il;
      if (i < k) {
        const int o = il * CW + c;
        t_part[(size_t)blockIdx.x * KR + (size_t)i * R + c] =
            (st[o] + st[S::TB + o]) + (st[2 * S::TB + o] + st[3 * S::TB + o]);
      }
    }
    __syncthreads();
  }
}

template <typename T, int RB>
static dski_status launch_update_rb(int nb, const T* Q, T* Rr, int N, int n, int R,
                                    const PcgScal& s, int par, const double* pq_part, int nb_pq, double* rr_part,
                                    const double* Ur, int k, double isf, double isg, double* t_part, double* hist,
                                    int max_iter, hipStream_t st) {
  constexpr size_t sh = UpdShape<RB>::template bytes<T>();
  static bool done_pc = false, done_plain = false;
  if (k > 0) {
    DSKI_TRY(lds_limit(&k_pcg_update<T, RB, true>, sh, done_pc));
    k_pcg_update<T, RB, true><<<nb, kBlock, sh, st>>>(Q, Rr, N, n, R, s, par, pq_part, nb_pq, rr_part, Ur, k, isf,
                                                      isg, t_part, hist, max_iter);
  } else {
    DSKI_TRY(lds_limit(&k_pcg_update<T, RB, false>, sh, done_plain));
    k_pcg_update<T, RB, false><<<nb, kBlock, sh, st>>>(Q, Rr, N, n, R, s, par, pq_part, nb_pq, rr_part, Ur, k,
                                                       isf, isg, t_part, hist, max_iter);
  }
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

// Partials are per update work-group: nb = upd_blocks(N) blocks.
template <typename T>
static dski_status launch_update(int nb, const T* Q, T* Rr, int N, int n, int R,
                                 const PcgScal& s, int par, const double* pq_part, int nb_pq, double* rr_part,
                                 const double* Ur, int k, double isf, double isg, double* t_part, double* hist,
                                 int max_iter, hipStream_t st) {
#define DSKI_UPD(V)                                                                                          \
  case V:                                                                                                    \
    return launch_update_rb<T, V>(nb, Q, Rr, N, n, R, s, par, pq_part, nb_pq, rr_part, Ur, k, isf, isg, t_part, \
                                  hist, max_iter, st);
  switch (pad4(R)) {
    DSKI_UPD(4)
    DSKI_UPD(8)
    DSKI_UPD(12)
    DSKI_UPD(16)
    DSKI_UPD(20)
    DSKI_UPD(24)
    DSKI_UPD(28)
    DSKI_UPD(32)
    default:
      set_error("at most %d columns per fused PCG", kPcgMaxR);
      return DSKI_ENOTSUP;
  }
#undef DSKI_UPD
}

// Without a preconditioner (z = r): beta = r.r / r.r_old from the reduced norms
// (every thread forms it, the same value), history (hist = the beta rows),
// convergence test, x += alpha p and then p = r + beta p (p of this iteration
// is read once for both).  Grid (row chunks of 256, R); block (0, c) writes the
// column's next-parity state.
template <typename T>
__global__ void k_pcg_beta(const T* __restrict__ Rr, T* __restrict__ P, double* __restrict__ Xd, int N, int R,
                           PcgScal s, int par, double* __restrict__ hist, int max_iter, int fixed_iters) {
  const int c = blockIdx.y;
  const int on = s.active[par * R + c];
  const double rz_old = s.rz[par * R + c], rzn = s.rr[c];
  if (!on) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      s.rz[(1 - par) * R + c] = rz_old;
      s.active[(1 - par) * R + c] = 0;
    }
    return;
  }
  const double b = rz_old > 0.0 ? rzn / rz_old : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!(rzn >= 0.0) || !isfinite(rzn)) s.flags[1] = 1;
    const int it = s.iters[c];
    const bool done = fixed_iters > 0 ? (it + 1 >= fixed_iters) : (rzn <= s.tol2[c] * s.bb[c]);
    if (hist && it < max_iter) hist[(size_t)c * max_iter + it] = b;
    s.iters[c] = it + 1;
    if (done) atomicSub(&s.flags[0], 1);
    s.rz[(1 - par) * R + c] = rzn;
    s.active[(1 - par) * R + c] = done ? 0 : 1;
  }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) {
    const size_t ip = (size_t)c * N + e;
    const double pv = (double)P[ip];
    Xd[ip] = Xd[ip] + s.alpha[c] * pv;  // x += alpha p with this iteration's p
    P[ip] = (T)((double)Rr[ip] + b * pv);
  }
}

// The rest of an iteration with a preconditioner M = D + L L^T, after the
// reductions of t = U^T D^{-1/2} r (coef = w o t, the Woodbury form
// z = D^{-1/2}(D^{-1/2} r - U coef)) and of |r|^2, |D^{-1/2} r|^2:
//   r.z = |D^{-1/2} r|^2 - sum_i coef_i t_i   (the same quantity as r^T z),
//   beta = r.z / r.z_old, x += alpha p, p = z + beta p,
// so that z never leaves registers.  Every work-group forms each column's r.z
// from the reduced values in one fixed order (16 lanes per column), so all agree;
// work-group 0 records the column's next state (beta history, iteration count,
// convergence, next-parity r.z and flag).  Rows as in k_ts_final: eight 32-row
// wavefronts per work-group, U coef on the FP64 matrix cores (CB blocks of 16
// columns, VC more on the vector ALU), coef staged in LDS per 64-column chunk of
// U, every load but x's issued before the first wait (the column scalars first,
// then the rows of r and p, then the first chunk).  PC: rank k > 0.
template <typename T, int CB, int VC, bool PC>
__global__ __launch_bounds__(512) void k_pcg_step(const T* __restrict__ Rr, T* __restrict__ P,
                                                  double* __restrict__ Xd, int N, int n, int R, double isf,
                                                  double isg, const double* __restrict__ U, int k,
                                                  const double* __restrict__ coef, const double* __restrict__ tv,
                                                  PcgScal s, int par, double* __restrict__ hist, int max_iter,
                                                  int fixed_iters) {
  constexpr int FR = kFinalRows, EB = FR / 16, CW = 16 * CB + VC, XP = CW + 1, HC = (CW + 1) / 2;
  constexpr int NT = 64 * kFinalWaves, CF = (64 * CW + NT - 1) / NT, QL = 16, QW = 4;  // QL lanes per column
  static_assert(CW <= kPcgMaxR, "columns per launch");
  extern __shared__ __align__(16) char smem[];
  __shared__ double s_coef[64 * XP];
  __shared__ double s_alpha[kPcgMaxR], s_beta[kPcgMaxR];
  __shared__ int s_on[kPcgMaxR];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int e0 = (blockIdx.x * kFinalWaves + wv) * FR;
  double* sz = reinterpret_cast<double*>(smem) + (size_t)wv * FR * XP;
  const int rl = lane & (FR - 1), hh = lane / FR;  // this lane's row and half of the columns
  const int e = e0 + rl;
  const bool in = e < N;
  // column scalars: QL lanes per column, lane j takes the entries i = j, j + QL, ...
  static_assert(NT / QL >= kPcgMaxR, "a lane group per column");
  const int c_q = threadIdx.x / QL, j_q = threadIdx.x % QL;
  const bool colq = c_q < R;
  const int cq = colq ? c_q : 0;
  const int on_q = s.active[par * R + cq];
  const double rzo_q = s.rz[par * R + cq], rr_q = s.rr[cq], rrd_q = s.rrd[cq], al_q = s.alpha[cq];
  double tq[QW], cq_[QW];
#pragma unroll
  for (int u = 0; u < QW; ++u) {
    const int i = j_q + QL * u;
    const bool ok = PC && colq && i < k;
    tq[u] = ld_or0(tv, (size_t)i * R + cq, 0, ok);
    cq_[u] = ld_or0(coef, (size_t)i * R + cq, 0, ok);
  }
  // this lane's rows of r and p (clamped indices; finished columns are read and
  // left alone); x is read at the end, where registers are free
  T rv[HC], pv[HC];
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;
    const size_t idx = (size_t)(c < R ? c : R - 1) * N + (in ? e : 0);
    rv[j] = Rr[idx];
    pv[j] = P[idx];
  }
  // a chunk of coef (to LDS) and this wavefront's U operands; U indices are
  // clamped instead of masked (a column i >= k meets a zero coefficient, a row
  // past N is never stored)
  const size_t nk_last = (size_t)N * (size_t)(k > 0 ? k : 1) - 1;
  double cf[CF], av[16][EB];
  auto load_chunk = [&](int i0) {
#pragma unroll
    for (int u = 0; u < CF; ++u) {
      const int f = threadIdx.x + NT * u, il = f / CW, c = f - il * CW;
      cf[u] = ld_or0(coef, (size_t)(i0 + il) * R + c, 0, f < 64 * CW && i0 + il < k && c < R);
    }
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int i = i0 + 4 * st + kq;
#pragma unroll
      for (int eb = 0; eb < EB; ++eb) {
        const size_t o = (size_t)i * N + (size_t)(e0 + 16 * eb + r16);
        av[st][eb] = U[o < nk_last ? o : nk_last];
      }
    }
  };
  if (PC) load_chunk(0);
  {
    double q = 0.0;  // sum_i coef_i t_i of column c_q
#pragma unroll
    for (int u = 0; u < QW; ++u) q += cq_[u] * tq[u];
    for (int i = j_q + QL * QW; PC && i < k; i += QL)
      if (colq) q += coef[(size_t)i * R + cq] * tv[(size_t)i * R + cq];
    q += __shfl_xor(q, 1, 64);
    q += __shfl_xor(q, 2, 64);
    q += __shfl_xor(q, 4, 64);
    q += __shfl_xor(q, 8, 64);
    if (colq && j_q == 0) {
      const int c = c_q;
      double beta = 0.0;
      if (on_q) {
        const double rzn = rrd_q - q;
        if (!(rzn >= 0.0) || !isfinite(rzn)) {
          if (blockIdx.x == 0) s.flags[1] = 1;
        }
        beta = rzo_q > 0.0 ? rzn / rzo_q : 0.0;
        if (blockIdx.x == 0) {
          const int it = s.iters[c];
          const bool done = fixed_iters > 0 ? (it + 1 >= fixed_iters) : (rr_q <= s.tol2[c] * s.bb[c]);
          if (hist && it < max_iter) hist[(size_t)c * max_iter + it] = beta;
          s.iters[c] = it + 1;
          if (done) atomicSub(&s.flags[0], 1);
          s.rz[(1 - par) * R + c] = rzn;
          s.active[(1 - par) * R + c] = done ? 0 : 1;
        }
      } else if (blockIdx.x == 0) {
        s.rz[(1 - par) * R + c] = rzo_q;
        s.active[(1 - par) * R + c] = 0;
      }
      s_alpha[c] = al_q;
      s_beta[c] = beta;
      s_on[c] = on_q;
    }
  }
  dski_pdbl4 acc[EB][CB];
  double vacc[EB][VC > 0 ? VC : 1];
#pragma unroll
  for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[eb][cb] = dski_pdbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < VC; ++v) vacc[eb][v] = 0.0;
  }
  if (!PC) __syncthreads();  // the column scalars
  for (int i0 = 0; PC && i0 < k; i0 += 64) {
    if (i0 > 0) {
      __syncthreads();  // every wavefront is done with the previous chunk
      load_chunk(i0);
    }
#pragma unroll
    for (int u = 0; u < CF; ++u) {
      const int f = threadIdx.x + NT * u, il = f / CW, c = f - il * CW;
      if (f < 64 * CW) s_coef[il * XP + c] = cf[u];
    }
    __syncthreads();  // (the first one also publishes the column scalars)
    const int steps = min(16, (k - i0 + 3) / 4);  // steps holding a column i < k
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      if (st < steps) {
        const double* crow = s_coef + (4 * st + kq) * XP;
        double bv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) bv[cb] = crow[16 * cb + r16];
#pragma unroll
        for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[eb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st][eb], bv[cb], acc[eb][cb], 0, 0, 0);
#pragma unroll
          for (int v = 0; v < VC; ++v) vacc[eb][v] += av[st][eb] * crow[16 * CB + v];
        }
      }
    }
  }
  // U coef through LDS (layout as in k_ts_final), then z, x and p per row
#pragma unroll
  for (int eb = 0; eb < EB; ++eb) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) sz[(16 * eb + kq + 4 * r) * XP + 16 * cb + r16] = acc[eb][cb][r];
#pragma unroll
    for (int v = 0; v < VC; ++v) {
      double x = vacc[eb][v];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (kq == 0) sz[(16 * eb + r16) * XP + 16 * CB + v] = x;
    }
  }
  wave_lds_fence();
  double xv[HC];
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;
    xv[j] = Xd[(size_t)(c < R ? c : R - 1) * N + (in ? e : 0)];
  }
  const double dsc = e < n ? isf : isg;  // D^{-1/2} of this row
#pragma unroll
  for (int j = 0; j < HC; ++j) {
    const int c = hh * HC + j;
    if (in && c < R && s_on[c]) {
      const double z = dsc * (dsc * (double)rv[j] - sz[rl * XP + c]);
      const double pold = (double)pv[j];
      const size_t idx = (size_t)c * N + e;
      Xd[idx] = xv[j] + s_alpha[c] * pold;  // x += alpha p with this iteration's p
      P[idx] = (T)(z + s_beta[c] * pold);
    }
  }
}

template <typename T, int CB, int VC>
static dski_status launch_step_cw(const T* Rr, T* P, double* Xd, int N, int n, int R, double isf, double isg,
                                  const double* U, int k, const double* coef, const double* tv, const PcgScal& s,
                                  int par, double* hist, int max_iter, int fixed_iters, hipStream_t st) {
  constexpr size_t sh = sizeof(double) * kFinalWaves * kFinalRows * (16 * CB + VC + 1);
  constexpr int rows = kFinalRows * kFinalWaves;
  const int nb = (N + rows - 1) / rows;
  if (k > 0) {
    static bool done = false;
    DSKI_TRY(lds_limit(&k_pcg_step<T, CB, VC, true>, sh, done));
    k_pcg_step<T, CB, VC, true><<<nb, 64 * kFinalWaves, sh, st>>>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, tv, s,
                                                                  par, hist, max_iter, fixed_iters);
  } else {
    static bool done = false;
    DSKI_TRY(lds_limit(&k_pcg_step<T, CB, VC, false>, sh, done));
    k_pcg_step<T, CB, VC, false><<<nb, 64 * kFinalWaves, sh, st>>>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, tv,
                                                                   s, par, hist, max_iter, fixed_iters);
  }
  DSKI_HIP(hipGetLastError());
  return DSKI_OK;
}

template <typename T>
static dski_status launch_step(const T* Rr, T* P, double* Xd, int N, int n, int R, double isf, double isg,
                               const double* U, int k, const double* coef, const double* tv, const PcgScal& s,
                               int par, double* hist, int max_iter, int fixed_iters, hipStream_t st) {
  if (R <= 16)
    return launch_step_cw<T, 1, 0>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, tv, s, par, hist, max_iter,
                                   fixed_iters, st);
  if (R <= 20)
    return launch_step_cw<T, 1, 4>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, tv, s, par, hist, max_iter,
                                   fixed_iters, st);
  return launch_step_cw<T, 2, 0>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, tv, s, par, hist, max_iter, fixed_iters,
                                 st);
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

// Residual replacement of the columns in `mask` (the active ones): r.r and r.z
// of the replaced residual for the next iteration (parity par); p, the
// iteration counts and the active flags stay.
__global__ void k_pcg_replace_scal(const double* __restrict__ rr_part, int nb_r, const double* __restrict__ rz_part,
                                   int nb_z, int R, const int* __restrict__ mask, PcgScal s, int par) {
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wv; c < R; c += nw) {
    double rr = wave_out_sum(rr_part, nb_r, c);
    double rz = rz_part ? wave_out_sum(rz_part, nb_z, c) : rr;
    if ((threadIdx.x & 63) != 0 || !mask[c]) continue;
    s.rr[c] = rr;
    s.rz[par * R + c] = rz;
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

// One PCG on R <= kPcgMaxR columns; alpha of column c at hist[c max_iter + j], beta at
// hist_b[c max_iter + j] (both may be NULL).
template <typename T>
static dski_status pcg_group(dski_plan p, dski_precond pc, int R, const T* B, int ldb, T* X, int ldx,
                             const double* tol_host, int max_iter, int fixed_iters, double* hist, double* hist_b,
                             PcgResult& res, int res_c0, hipStream_t st, double* X64, int ldx64,
                             const int* verify_mask) {
  const int N = p->N, n = p->n;
  const int k = pc ? pc->k : 0;
  const size_t nr = (size_t)N * R;
  const int nbv = nchunks(N), nbg = gather_blocks(p), nbz = vec_blocks(N);
  const int nbt = upd_blocks(N);  // update work-groups (their partials of t and r.r)
  const size_t npart = (size_t)std::max(std::max(nbv, nbg), std::max(nbz, 2 * nbt)) * R;  // rr_part: 2 R per block
  const size_t ntp = (size_t)nbt * std::max(k, 1) * R;
  // workspace: Rr, Z, P, Q (T), Xd, partials, t partials, t1, scratch (R), coef, scalars
  const size_t kr = (size_t)std::max(k, 1) * R;
  size_t tb = ((sizeof(T) * nr * 4) + 63) / 64 * 64;
  size_t db = sizeof(double) * (nr + 3 * npart + ntp + 3 * kr + 12 * (size_t)R + 16);
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
  double* t2 = t1 + kr;  // R doubles of scratch (true-residual norms)
  double* coef = t2 + kr;
  PcgScal s;
  s.rz = coef + kr;
  s.rr = s.rz + 2 * R;
  s.rrd = s.rr + R;
  s.bb = s.rrd + R;
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
  const double* U = pc ? pc->U : nullptr;
  const double* Ur = pc ? pc->Ur : nullptr;
  const double isf = 1.0 / p->sf, isg = 1.0 / p->sg;
  dski_status rc = DSKI_OK;
  const int limit = fixed_iters > 0 ? fixed_iters : max_iter;
  int it = 0;
  // one iteration, all launches on stream `q`
  auto iterate = [&](int par, hipStream_t q) -> dski_status {
    DSKI_TRY(mvm_tiled<T>(p, R, P, N, Q, N, pq_part, q));
    DSKI_TRY(launch_update<T>(nbt, Q, Rr, N, n, R, s, par, pq_part, nbg, rr_part, Ur, pc ? k : 0, isf, isg, t_part,
                              hist, max_iter, q));
    // |r|^2 to s.rr and |D^{-1/2} r|^2 to s.rrd (2 R outputs), for active columns
    RedJob jr{rr_part, nbt, 2 * R, R, s.rr, nullptr, nullptr, 0.0, nullptr, s.active + par * R};
    if (pc) {
      if (k > 0) {
        RedJob jt{t_part, nbt, k * R, R, t1, pc->w, nullptr, 1.0, coef, nullptr};
        DSKI_TRY(launch_reduce_bm(jt, &jr, q));
      } else {
        DSKI_TRY(launch_reduce_bm(jr, nullptr, q));
      }
      DSKI_TRY(launch_step<T>(Rr, P, Xd, N, n, R, isf, isg, U, k, coef, t1, s, par, hist_b, max_iter, fixed_iters,
                              q));
    } else {
      DSKI_TRY(launch_reduce_bm(jr, nullptr, q));
      k_pcg_beta<T><<<dim3(nbz, R), kBlock, 0, q>>>(Rr, P, Xd, N, R, s, par, hist_b, max_iter, fixed_iters);
    }
    DSKI_HIP(hipGetLastError());
    return DSKI_OK;
  };
  // Bursts of kGraphIters iterations are replayed from a HIP graph captured once
  // per solve on a side stream (ordered after and before `st` by events); the
  // first iterations run eagerly, which also sizes every workspace.
  PcgGraph gr;
  auto graph_burst = [&](int nrep) -> dski_status {
    const int par0 = it & 1;
    if (!gr.exec || gr.par0 != par0) {
      if (!gr.stream) {
        DSKI_HIP(hipStreamCreateWithFlags(&gr.stream, hipStreamNonBlocking));
        DSKI_HIP(hipEventCreateWithFlags(&gr.ev0, hipEventDisableTiming));
        DSKI_HIP(hipEventCreateWithFlags(&gr.ev1, hipEventDisableTiming));
      }
      gr.reset_graph();
      DSKI_HIP(hipStreamBeginCapture(gr.stream, hipStreamCaptureModeRelaxed));
      dski_status cr = DSKI_OK;
      for (int j = 0; j < kGraphIters && cr == DSKI_OK; ++j) cr = iterate((par0 + j) & 1, gr.stream);
      hipGraph_t g = nullptr;
      hipError_t ec = hipStreamEndCapture(gr.stream, &g);
      if (cr < 0) {
        if (g) (void)hipGraphDestroy(g);
        return cr;
      }
      if (ec != hipSuccess) {
        set_error("PCG graph capture failed: %s", hipGetErrorString(ec));
        return DSKI_EHIP;
      }
      gr.graph = g;
      DSKI_HIP(hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0));
      gr.par0 = par0;
    }
    DSKI_HIP(hipEventRecord(gr.ev0, st));
    DSKI_HIP(hipStreamWaitEvent(gr.stream, gr.ev0, 0));
    for (int j = 0; j < nrep; ++j) DSKI_HIP(hipGraphLaunch(gr.exec, gr.stream));
    DSKI_HIP(hipEventRecord(gr.ev1, gr.stream));
    DSKI_HIP(hipStreamWaitEvent(st, gr.ev1, 0));
    return DSKI_OK;
  };
  // Residual replacement (FP32 vectors only): every kReplaceEvery iterations the
  // recurrence residual of the active columns is replaced by b - K~ x (FP64
  // iterate, FP64-storage operator), z and r.z are recomputed and p is kept, so
  // that the recurrence cannot drift away from the true residual (which would
  // otherwise end in a restart that discards the Krylov space).
  DevBuf repbuf;
  int last_rep = 0;
  auto replace = [&]() -> dski_status {
    DSKI_TRY(repbuf.reserve(sizeof(double) * nr + 64));
    double* Y = repbuf.as<double>();
    DSKI_TRY(mvm_tiled<double>(p, R, Xd, N, Y, N, nullptr, st));
    const int par = it & 1;
    const int* mask = s.active + par * R;
    k_true_resid<T><<<nbv, kBlock, 0, st>>>(B, ldb, Y, Rr, N, R, mask, rr_part);
    DSKI_HIP(hipGetLastError());
    if (pc) DSKI_TRY(precond_apply_tiled<T>(pc, R, Rr, N, Z, N, rz_part, nullptr, st));
    k_pcg_replace_scal<<<1, 256, 0, st>>>(rr_part, nbv, pc ? rz_part : nullptr, nbz, R, mask, s, par);
    DSKI_HIP(hipGetLastError());
    last_rep = it;
    return DSKI_OK;
  };
  const bool replacing = sizeof(T) == 4 && fixed_iters <= 0;
  auto run = [&]() -> dski_status {
    int check = 1;
    while (it < limit) {
      int burst = std::min(check, limit - it);
      int b = 0;
      if (p->use_graph && burst >= kGraphIters) {
        const int nrep = burst / kGraphIters;
        DSKI_TRY(graph_burst(nrep));
        b = nrep * kGraphIters;
      }
      for (; b < burst; ++b) DSKI_TRY(iterate((it + b) & 1, st));
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
      if (replacing && it - last_rep >= kReplaceEvery) DSKI_TRY(replace());
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
  dski_status worst = DSKI_OK;
  // columns run in independent groups of at most kPcgMaxR; history layout
  // [alpha: R x max_iter][beta: R x max_iter] over all R columns
  for (int c0 = 0; c0 < R; c0 += kPcgMaxR) {
    int rg = std::min(kPcgMaxR, R - c0);
    double* ha = alpha_beta ? alpha_beta + (size_t)c0 * max_iter : nullptr;
    double* hb = alpha_beta ? alpha_beta + ((size_t)R + c0) * max_iter : nullptr;
    dski_status rc = pcg_group<T>(p, pc, rg, B + (size_t)c0 * ldb, ldb, X ? X + (size_t)c0 * ldx : nullptr, ldx,
                                  tol_host + c0, max_iter, fixed_iters, ha, hb, res, c0, st,
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
