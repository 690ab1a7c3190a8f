// Pivot selection of the greedy pivoted Cholesky (Sec. 3.3), shared by the
// D-SKI and D-SKIP row providers.
#pragma once

#include "internal.h"

namespace dski {

// Final arg-max over the per-block partials (largest residual diagonal, lowest
// index among exact ties), the stop test (residual <= rel_tol * largest initial
// diagonal, or not positive) and the bookkeeping of step j.  Called by every
// thread of one work-group of kBlock threads; returns the pivot (tile-order
// N-index) to all of them, or -1 once the factorisation has stopped.  With a
// forced list the pivot of step j is forced[j] instead of the arg-max (the
// stop test still looks at the largest residual, and a forced pivot whose
// residual diagonal dres is not positive stops the factorisation).
__device__ inline int pivot_select_block(const double* __restrict__ pv, const int* __restrict__ pi,
                                         int nblk, int j, double rel_tol, PivState* __restrict__ ps,
                                         int* __restrict__ piv_list, const int* __restrict__ forced,
                                         const double* __restrict__ dres) {
  __shared__ double sv[kBlock];
  __shared__ int si[kBlock];
  __shared__ int s_piv;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    double v = pv[b];
    int i = pi[b];
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
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
    if (j == 0) {
      ps->dmax0 = sv[0];
      ps->stop = 0;
      ps->rank = 0;
    }
    int stop = ps->stop;
    if (!stop && !(sv[0] > rel_tol * ps->dmax0 && sv[0] > 0.0)) stop = 1;
    int pick = si[0];
    double dpick = sv[0];
    if (forced && !stop) {
      pick = forced[j];
      dpick = dres[pick];
      if (!(dpick > 0.0)) stop = 1;
    }
    ps->stop = stop;
    s_piv = stop ? -1 : pick;
    if (!stop) {
      ps->piv = pick;
      ps->dpiv = dpick;
      piv_list[j] = pick;
      ps->rank = j + 1;
    }
  }
  __syncthreads();
  return s_piv;
}

}  // namespace dski
