"""Thin-plate spline kernel under SKI / D-SKI (FP64, dense K_UU).

Follows App. A, which gives the spline kernels
    k(x, y) = s^2 (r^3 + a r^2 + b)            d odd,
    k(x, y) = s^2 (r^2 log r + a r^2 + b)      d even,     r = |x - y|,
with a, b "chosen to make the kernel symmetric and positive definite on the
given domain", and Sec. 4.3, which fits an implicit surface with SKI and this
kernel on a 3-D grid.  The spline kernel is not a product kernel, so D-SKIP
does not apply (Sec. 4); under D-SKI the kernel enters only through K_UU, the
kernel on the grid nodes (a symmetric multi-level Toeplitz matrix), and the
derivative rows come from the interpolation weights as for the SE kernel
(Sec. 3.1).

Readings (the paper does not give a, b):
* a and b are those of the thin-plate covariances of Williams and Fitzgibbon
  (Gaussian process implicit surfaces, 2007), written with a domain size R:
      d odd:  k = s^2 (r^3 - (3/2) R r^2 + R^3 / 2)             = (s^2/2)(2 r^3 - 3 R r^2 + R^3)
      d even: k = s^2 (r^2 log r - ((1 + 2 log R)/2) r^2 + R^2 / 2)
  with R twice the diameter of the grid (the largest distance between two
  grid nodes).  With R equal to the diameter the odd form is slightly
  indefinite on 3-D grids; at twice the diameter both forms are positive
  definite on every grid tried (the pins check it).
* Hyper-parameters: s and the two noise levels; the kernel has no length
  scale, so the gradient entries for log ell_p are zero.

The oracle forms K_UU densely from the kernel function (no FFT, small grids
only) and reuses the CSR interpolation matrices of ``interp``.
"""
import numpy as np

from . import interp
from .kernels import noise_diag


def spline_k(r, d, R):
    """The spline kernel profile k(r) / s^2 for dimension d and domain size R."""
    r = np.asarray(r, dtype=np.float64)
    if d % 2 == 1:
        return r ** 3 - 1.5 * R * r ** 2 + 0.5 * R ** 3
    with np.errstate(divide="ignore", invalid="ignore"):
        rlog = np.where(r > 0, r * r * np.log(np.where(r > 0, r, 1.0)), 0.0)
    return rlog - 0.5 * (1.0 + 2.0 * np.log(R)) * r * r + 0.5 * R * R


def grid_domain_size(grid):
    """R = twice the largest distance between two grid nodes."""
    return 2.0 * float(np.linalg.norm((grid.m - 1) * grid.h))


class SplineDSKI:
    """D-SKI operator with the spline kernel: K~ = S (s^2 K_spl) S^T + D.

    theta: log_s, log_sigma_f, log_sigma_g (the length scales of the SE
    operator's signature are accepted and ignored)."""

    def __init__(self, X, grid_m, lo_box, hi_box, log_s, log_sigma_f, log_sigma_g, interp_kind="cubic"):
        self.X = np.asarray(X, dtype=np.float64)
        self.n, self.d = self.X.shape
        self.N = self.n * (self.d + 1)
        self.grid = interp.Grid(lo_box, hi_box, grid_m, interp_kind)
        self.S = interp.interp_matrices(self.X, self.grid)
        self.ST = self.S.T.tocsr()
        self.R = grid_domain_size(self.grid)
        nodes = np.stack(np.meshgrid(*[self.grid.nodes(p) for p in range(self.d)], indexing="ij"),
                         -1).reshape(-1, self.d)
        dist = np.linalg.norm(nodes[:, None, :] - nodes[None, :, :], axis=-1)
        self.Kspl = spline_k(dist, self.d, self.R)
        self.set_hypers(log_s, log_sigma_f, log_sigma_g)

    def set_hypers(self, log_s, log_sigma_f, log_sigma_g):
        self.s = np.exp(float(log_s))
        self.sigma_f = np.exp(float(log_sigma_f))
        self.sigma_g = np.exp(float(log_sigma_g))
        self.Dn = noise_diag(self.n, self.d, self.sigma_f, self.sigma_g)

    def kuu_apply(self, G):
        return self.s ** 2 * (self.Kspl @ G)

    def matvec_K(self, V):
        V2 = V.reshape(self.N, -1)
        return (self.S @ self.kuu_apply(self.ST @ V2)).reshape(V.shape)

    def matvec(self, V):
        V2 = V.reshape(self.N, -1)
        out = self.S @ self.kuu_apply(self.ST @ V2) + self.Dn[:, None] * V2
        return out.reshape(V.shape)

    def matvec_dtheta(self, which, V):
        """dK~/dtheta V, which in 0..d+2 in the SE order (log ell_1..d: zero,
        log s, log sigma_f, log sigma_g)."""
        V2 = V.reshape(self.N, -1)
        if which < self.d:
            out = np.zeros_like(V2)
        elif which == self.d:
            out = 2.0 * (self.S @ self.kuu_apply(self.ST @ V2))
        elif which == self.d + 1:
            out = np.zeros_like(V2)
            out[:self.n] = 2 * self.sigma_f ** 2 * V2[:self.n]
        elif which == self.d + 2:
            out = np.zeros_like(V2)
            out[self.n:] = 2 * self.sigma_g ** 2 * V2[self.n:]
        else:
            raise ValueError(which)
        return out.reshape(V.shape)

    def diag_K(self):
        """diag(S K_UU S^T)_i = w_i^T K_UU[stencil, stencil] w_i over row i's nonzeros."""
        S = self.S
        out = np.empty(self.N)
        for i in range(self.N):
            c = S.indices[S.indptr[i]:S.indptr[i + 1]]
            w = S.data[S.indptr[i]:S.indptr[i + 1]]
            out[i] = self.s ** 2 * (w @ self.Kspl[np.ix_(c, c)] @ w)
        return out

    def row_K(self, i):
        e = np.zeros((self.N, 1))
        e[i, 0] = 1.0
        return self.matvec_K(e)[:, 0]

    def dense_K(self):
        Sd = self.S.toarray()
        return Sd @ self.kuu_apply(Sd.T)

    def dense(self):
        return self.dense_K() + np.diag(self.Dn)
