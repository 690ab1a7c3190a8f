"""D-SKI operator (FP64): K~ = [W; dW] K_UU [W; dW]^T + D.

Follows Sec. 3.1 (the D-SKI block form: value block W K_UU W^T, cross blocks
W K_UU dW^T and dW K_UU W^T, gradient block dW K_UU dW^T, with K_UU applied
through its Kronecker/Toeplitz structure) and Sec. 2 (SKI).  The noise enters
through D = diag(sigma_f^2 1_n, sigma_g^2 1_{nd}) (two noise levels, as the
terrain experiment of Sec. 4 fits them).

K_UU = s^2 T_1 (x) T_2 (x) ... (x) T_d with the symmetric Toeplitz factors
(T_p)_{ab} = exp(-((a - b) h_p)^2 / (2 ell_p^2)) of the SE kernel (App. A) on
the grid.  The oracle applies K_UU by dense mode-p products (no FFT).

Readings: mean function mu = 0; the matrix the preconditioner factors is the
noise-free K = S K_UU S^T (the noise enters only through M, Sec. 3.3).
"""
import numpy as np

from . import interp
from .kernels import noise_diag


def toeplitz_factor(m, h, ell):
    """(T)_{ab} = exp(-((a-b) h)^2 / (2 ell^2)), a, b < m (dense)."""
    j = np.arange(m)
    D = (j[:, None] - j[None, :]) * h
    return np.exp(-0.5 * (D / ell) ** 2)


def toeplitz_factor_dlogell(m, h, ell):
    """d T / d log(ell) = T * ((a-b) h / ell)^2."""
    j = np.arange(m)
    D = (j[:, None] - j[None, :]) * h
    r2 = (D / ell) ** 2
    return np.exp(-0.5 * r2) * r2


def mode_product(G, mats):
    """Apply (mats[0] (x) ... (x) mats[d-1]) to columns of G (m x R), C order."""
    shape = [M.shape[0] for M in mats]
    R = G.shape[1]
    T = G.reshape(shape + [R])
    for p, M in enumerate(mats):
        T = np.moveaxis(np.tensordot(M, T, axes=([1], [p])), 0, p)
    return T.reshape(-1, R)


class DSKI:
    """The D-SKI operator for points X on a grid, with hyper-parameters theta.

    theta: log_ell (d,), log_s, log_sigma_f, log_sigma_g (natural logs)."""

    def __init__(self, X, grid_m, lo_box, hi_box, log_ell, log_s, log_sigma_f, log_sigma_g, interp_kind="cubic"):
        self.X = np.asarray(X, dtype=np.float64)
        self.n, self.d = self.X.shape
        self.N = self.n * (self.d + 1)
        self.grid = interp.Grid(lo_box, hi_box, grid_m, interp_kind)
        self.S = interp.interp_matrices(self.X, self.grid)
        self.ST = self.S.T.tocsr()
        self.set_hypers(log_ell, log_s, log_sigma_f, log_sigma_g)

    def set_hypers(self, log_ell, log_s, log_sigma_f, log_sigma_g):
        self.log_ell = np.broadcast_to(np.asarray(log_ell, dtype=np.float64), (self.d,)).copy()
        self.ell = np.exp(self.log_ell)
        self.log_s = float(log_s)
        self.s = np.exp(self.log_s)
        self.sigma_f = np.exp(float(log_sigma_f))
        self.sigma_g = np.exp(float(log_sigma_g))
        self.T = [toeplitz_factor(self.grid.m[p], self.grid.h[p], self.ell[p]) for p in range(self.d)]
        self.Dn = noise_diag(self.n, self.d, self.sigma_f, self.sigma_g)

    # --- K_UU and its derivatives ------------------------------------------------
    def kuu_apply(self, G):
        return self.s ** 2 * mode_product(G, self.T)

    def kuu_dtheta_apply(self, which, G):
        """d K_UU / d theta_which applied to G; which < d: log ell_p; which == d: log s."""
        if which < self.d:
            mats = list(self.T)
            mats[which] = toeplitz_factor_dlogell(self.grid.m[which], self.grid.h[which], self.ell[which])
            return self.s ** 2 * mode_product(G, mats)
        if which == self.d:
            return 2.0 * self.kuu_apply(G)
        raise ValueError(which)

    # --- operator products -------------------------------------------------------
    def matvec_K(self, V):
        """Noise-free K V = S (K_UU (S^T V)); V is N x R (or N)."""
        V2 = V.reshape(self.N, -1)
        out = self.S @ self.kuu_apply(self.ST @ V2)
        return out.reshape(V.shape)

    def matvec(self, V):
        """(K + D) V."""
        V2 = V.reshape(self.N, -1)
        out = self.S @ self.kuu_apply(self.ST @ V2) + self.Dn[:, None] * V2
        return out.reshape(V.shape)

    def matvec_dtheta(self, which, V):
        """dK~/dtheta_which V for which in 0..d+2 (log ell_1..d, log s, log sigma_f, log sigma_g)."""
        V2 = V.reshape(self.N, -1)
        if which <= self.d:
            out = self.S @ self.kuu_dtheta_apply(which, self.ST @ V2)
        elif which == self.d + 1:
            out = np.zeros_like(V2)
            out[:self.n] = 2 * self.sigma_f ** 2 * V2[:self.n]
        elif which == self.d + 2:
            out = np.zeros_like(V2)
            out[self.n:] = 2 * self.sigma_g ** 2 * V2[self.n:]
        else:
            raise ValueError(which)
        return out.reshape(V.shape)

    # --- entries of K --------------------------------------------------------------
    def diag_K(self):
        """diag(S K_UU S^T)_i = sum_{a,b} S_ia (K_UU)_ab S_ib over the nonzeros of row i."""
        S = self.S
        out = np.empty(self.N)
        indptr, indices, data = S.indptr, S.indices, S.data
        shape = tuple(self.grid.m)
        for i0 in range(0, self.N, 4096):
            i1 = min(self.N, i0 + 4096)
            lens = np.diff(indptr[i0:i1 + 1])
            nnz = lens.max()
            if not np.all(lens == nnz):
                # rare: rows with merged duplicates; fall back row by row
                for i in range(i0, i1):
                    c = indices[indptr[i]:indptr[i + 1]]
                    w = data[indptr[i]:indptr[i + 1]]
                    mi = np.unravel_index(c, shape)
                    Kb = np.full((len(c), len(c)), self.s ** 2)
                    for p in range(self.d):
                        Kb = Kb * self.T[p][np.ix_(mi[p], mi[p])]
                    out[i] = w @ Kb @ w
                continue
            c = indices[indptr[i0]:indptr[i1]].reshape(i1 - i0, nnz)
            w = data[indptr[i0]:indptr[i1]].reshape(i1 - i0, nnz)
            mi = np.unravel_index(c, shape)
            Kb = np.full((i1 - i0, nnz, nnz), self.s ** 2)
            for p in range(self.d):
                Kb *= self.T[p][mi[p][:, :, None], mi[p][:, None, :]]
            out[i0:i1] = np.einsum("ia,iab,ib->i", w, Kb, w)
        return out

    def row_K(self, i):
        """Row i of K = S K_UU S^T (the column S^T e_i pushed through K_UU and S)."""
        e = np.zeros((self.N, 1))
        e[i, 0] = 1.0
        return self.matvec_K(e)[:, 0]

    def dense_K(self, chunk=512):
        """Dense S K_UU S^T (small problems only), assembled `chunk` columns
        at a time so that the grid-sized intermediate K_UU S^T stays small."""
        out = np.empty((self.N, self.N))
        for c0 in range(0, self.N, chunk):
            c1 = min(self.N, c0 + chunk)
            out[:, c0:c1] = self.S @ self.kuu_apply(self.ST[:, c0:c1].toarray())
        return out

    def dense(self):
        return self.dense_K() + np.diag(self.Dn)
