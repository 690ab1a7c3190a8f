"""Squared-exponential kernel and the exact derivative kernel (FP64, dense).

Follows Sec. 2 (multi-output GP for values and gradients, the block kernel
k^grad = [[k, (d_x' k)^T], [d_x k, d^2 k]]), App. A (SE kernel) and App. B
(closed-form first and second derivatives of the SE kernel).

Readings:
* Derivatives are unscaled, i.e. raw partial derivatives d f / d x_p, which
  is the form App. B writes (Sec. 2 mentions an optional length-scale scaling).
* Length scales are per-dimension (ARD): k(x, x') = s^2 exp(-sum_p
  (x_p - x'_p)^2 / (2 ell_p^2)).  The isotropic App. A kernel is the case of
  equal ell_p.

Block layout of vectors: [f(x_1..x_n); d_1 f(x_1..x_n); ...; d_d f(...)].
"""
import numpy as np


def se(X1, X2, ell, s):
    """SE kernel matrix s^2 exp(-|(x - x')/ell|^2 / 2) between rows of X1, X2."""
    ell = np.broadcast_to(np.asarray(ell, dtype=np.float64), (X1.shape[1],))
    # direct differences for accuracy (the matrices here are small)
    diff = (X1[:, None, :] - X2[None, :, :]) / ell
    r2 = (diff * diff).sum(-1)
    return s * s * np.exp(-0.5 * r2)


def dse_dense(X, ell, s, X2=None):
    """Exact derivative-SE covariance matrix of size n(d+1) x n2(d+1).

    Entries (App. B, ARD-extended), with Delta_p = x_ip - x'_jp:
      Cov(f_i,      f'_j)       = k
      Cov(f_i,      d_q f'_j)   = + Delta_q / ell_q^2 * k
      Cov(d_p f_i,  f'_j)       = - Delta_p / ell_p^2 * k
      Cov(d_p f_i,  d_q f'_j)   = (delta_pq / ell_p^2 - Delta_p Delta_q / (ell_p^2 ell_q^2)) * k
    """
    if X2 is None:
        X2 = X
    n, d = X.shape
    n2 = X2.shape[0]
    ell = np.broadcast_to(np.asarray(ell, dtype=np.float64), (d,))
    K = se(X, X2, ell, s)
    Dl = X[:, None, :] - X2[None, :, :]          # n x n2 x d
    out = np.zeros((n * (d + 1), n2 * (d + 1)))
    out[:n, :n2] = K
    for q in range(d):
        out[:n, (q + 1) * n2:(q + 2) * n2] = Dl[:, :, q] / ell[q] ** 2 * K
        out[(q + 1) * n:(q + 2) * n, :n2] = -Dl[:, :, q] / ell[q] ** 2 * K
    for p in range(d):
        for q in range(d):
            blk = -Dl[:, :, p] * Dl[:, :, q] / (ell[p] ** 2 * ell[q] ** 2)
            if p == q:
                blk = blk + 1.0 / ell[p] ** 2
            out[(p + 1) * n:(p + 2) * n, (q + 1) * n2:(q + 2) * n2] = blk * K
    return out


def noise_diag(n, d, sigma_f, sigma_g):
    """Diagonal D = diag(sigma_f^2 1_n, sigma_g^2 1_{nd}): one noise level for
    values and one for gradients, as in the terrain experiment of Sec. 4."""
    out = np.full(n * (d + 1), sigma_g ** 2)
    out[:n] = sigma_f ** 2
    return out
