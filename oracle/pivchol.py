"""Truncated pivoted Cholesky K ~ (Pi L)(Pi L)^T (FP64).

Follows Sec. 3.3: the low-rank factor of the preconditioner comes from a
pivoted Cholesky factorisation truncated at rank k, which needs only the
diagonal of K and the rows at the chosen pivots (greedy choice of the largest
remaining diagonal entry, Harbrecht, Peters, Schneider 2012).

Readings:
* The factored matrix is the noise-free K (the noise is the sigma^2 I part of
  M = sigma^2 I + F F^T); F = L is N x k (the paper writes n x m).
* Ties: the lowest index among exactly equal maxima (numpy.argmax, which is
  also LAPACK dpstrf's choice).
* Early stop when the largest remaining diagonal entry is <= rel_tol times the
  largest initial diagonal entry (default 1e-12); the rank is then < k.
* ``forced`` lets a caller dictate the pivot sequence (used to follow another
  implementation's choices at near-ties); ``near_tie`` then reports, for each
  step, how far the forced pivot's residual diagonal fell below the maximum.
"""
import numpy as np


def pivoted_cholesky(diag, row, k, rel_tol=1e-12, forced=None):
    """diag: (N,) diagonal of K; row(i) -> (N,) row i of K.

    Returns (L (N x r), piv (r,), gaps (r,)) where gaps[j] =
    (max residual diag - residual diag at the chosen pivot) / max initial diag."""
    d = np.array(diag, dtype=np.float64, copy=True)
    N = d.shape[0]
    dmax0 = float(d.max())
    L = np.zeros((N, k))
    piv = []
    gaps = []
    chosen = np.zeros(N, dtype=bool)
    for j in range(k):
        dm = np.where(chosen, -np.inf, d)
        best = int(np.argmax(dm))
        i = best if forced is None else int(forced[j])
        if dm[best] <= rel_tol * dmax0 or d[i] <= 0.0:
            break
        gaps.append((dm[best] - d[i]) / dmax0)
        r = np.asarray(row(i), dtype=np.float64)
        col = (r - L[:, :j] @ L[i, :j]) / np.sqrt(d[i])
        L[:, j] = col
        d -= col * col
        chosen[i] = True
        piv.append(i)
    r = len(piv)
    return L[:, :r], np.array(piv, dtype=np.int64), np.array(gaps)
