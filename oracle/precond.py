"""Low-rank-plus-diagonal preconditioner M = D + L L^T (FP64).

Follows Sec. 3.3: M = sigma^2 I + F F^T is applied through the economy QR
factorisation [F; sigma I] = [Q_1; Q_2] R instead of Sherman-Morrison-Woodbury,
which is inaccurate for small sigma; then M^{-1} b = sigma^{-2}(b - Q_1 Q_1^T b).

Readings:
* The paper's formula applies the projection to "f"; it is the right-hand
  side b.
* Two noise levels: with D = diag(sigma_f^2 1_n, sigma_g^2 1_{nd}), scale
  G = D^{-1/2} L, so M = D^{1/2} (I + G G^T) D^{1/2}; the QR of [G; I_k] gives
  (I + G G^T)^{-1} = I - Q_1 Q_1^T and M^{-1} b = D^{-1/2}(b' - Q_1 Q_1^T b')
  with b' = D^{-1/2} b.  With a single sigma this is the paper's formula.
* log det M = sum log D_ii + 2 sum log |R_jj|.
* Square-root form (same operator): with the thin SVD G = U Sigma V^T,
  M^{-1} = D^{-1/2} B B D^{-1/2}, B = I - U diag(c) U^T,
  c_i = 1 - (1 + sigma_i^2)^{-1/2}, and a factor C with C C^T = M is
  C = D^{1/2} (I + U diag(sqrt(1 + sigma_i^2) - 1) U^T).  C maps Rademacher
  driving vectors w to probes z = C w with covariance M.
"""
import numpy as np


class Precond:
    def __init__(self, L, Dn):
        self.L = np.asarray(L, dtype=np.float64)
        self.Dn = np.asarray(Dn, dtype=np.float64)
        N, k = self.L.shape
        self.k = k
        self.dh = np.sqrt(self.Dn)
        G = self.L / self.dh[:, None]
        self.G = G
        A = np.vstack([G, np.eye(k)])
        Q, R = np.linalg.qr(A, mode="reduced")      # Householder (LAPACK geqrf)
        self.Q1 = Q[:N]
        self.R = R
        U, sv, _ = np.linalg.svd(G, full_matrices=False)
        self.U = U
        self.sv = sv
        self.c = 1.0 - 1.0 / np.sqrt(1.0 + sv ** 2)
        self.root_c = np.sqrt(1.0 + sv ** 2) - 1.0

    def solve(self, B):
        """M^{-1} B via the QR form."""
        B2 = B.reshape(self.L.shape[0], -1)
        Bp = B2 / self.dh[:, None]
        Z = Bp - self.Q1 @ (self.Q1.T @ Bp)
        return (Z / self.dh[:, None]).reshape(B.shape)

    def solve_sqrt_form(self, B):
        """M^{-1} B via the square-root form D^{-1/2} B B D^{-1/2}."""
        B2 = B.reshape(self.L.shape[0], -1)
        W = B2 / self.dh[:, None]
        for _ in range(2):
            W = W - self.U @ (self.c[:, None] * (self.U.T @ W))
        return (W / self.dh[:, None]).reshape(B.shape)

    def factor_apply(self, W):
        """C W with C C^T = M (maps driving vectors to probes of covariance M)."""
        W2 = W.reshape(self.L.shape[0], -1)
        Z = W2 + self.U @ (self.root_c[:, None] * (self.U.T @ W2))
        return (Z * self.dh[:, None]).reshape(W.shape)

    def logdet(self):
        return float(np.sum(np.log(self.Dn)) + 2.0 * np.sum(np.log(np.abs(np.diag(self.R)))))

    def dense(self):
        return np.diag(self.Dn) + self.L @ self.L.T
