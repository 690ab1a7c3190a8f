"""D-SKIP: the derivative kernel matrix as a Hadamard product of 1-D factors (FP64).

Follows Sec. 3.2: for a product kernel, the SKI matrix with derivatives is the
Hadamard product over dimensions of one-dimensional SKI matrices, where the
(alpha, beta) block of the factor for axis p uses derivative interpolation
weights on the side whose observation is the derivative along p (eq. (skip)
shows d = 2); each factor is then replaced by a rank-r Lanczos decomposition
Q_p T_p Q_p^T and the product is applied through the SKIP reduction (Gardner
et al. 2018).

Readings:
* The factor of axis p is the full N x N matrix (N = n(d+1))
      Khat_p[(a, i), (b, j)] = [W_p^{(a==p)} T_p W_p^{(b==p)T}]_{ij},
  i.e. Khat_p = S_p G_p S_p^T with G_p the 2n x 2n 1-D D-SKI matrix of
  coordinate p and S_p selecting its derivative rows for block a == p and its
  value rows otherwise.  Lanczos runs on Khat_p itself.
* s^2 multiplies the product once; the noise D is added to the product.
* Lanczos: r steps, full re-orthogonalisation, start vector the normalised
  Rademacher column ``node`` of the SplitMix64 stream ``seed`` (leaves are
  nodes 0..d-1, internal nodes are numbered on from d level by level).
* d > 2: binary tree, pairs (0,1), (2,3), ... level by level (an odd factor
  moves up unchanged); every internal node except the root is recompressed by
  r Lanczos steps on the Hadamard product of its children; the root is kept as
  the exact Hadamard product of its two rank-r children.
* Hadamard MVM of two low-rank factors A = Qa Ta Qa^T, B = Qb Tb Qb^T:
      (A o B) v = rowsum((Qa Ta) o ((Qb Tb) C^T)),   C = Qa^T diag(v) Qb.
Parity unpinned: the tree shape and pairing for d > 2 (no value in the paper).
"""
import numpy as np

from . import rng
from .dski import DSKI
from .kernels import noise_diag


class AxisFactor:
    """Khat_p = S_p G_p S_p^T for coordinate p of n points in d dimensions."""

    def __init__(self, x, p, d, m, lo, hi, log_ell):
        self.p, self.d = p, d
        self.n = x.shape[0]
        self.N = self.n * (d + 1)
        self.op = DSKI(x[:, None], [m], [lo], [hi], [log_ell], 0.0, 0.0, 0.0)

    def compress(self, V):
        """S_p^T: (d+1)n -> 2n (value part sums the blocks a != p)."""
        n, d, p = self.n, self.d, self.p
        V = V.reshape(self.N, -1)
        blocks = V.reshape(d + 1, n, -1)
        val = blocks.sum(axis=0) - blocks[p + 1]
        return np.concatenate([val, blocks[p + 1]], axis=0)

    def expand(self, U):
        """S_p: 2n -> (d+1)n."""
        n, d, p = self.n, self.d, self.p
        U = U.reshape(2 * n, -1)
        out = np.repeat(U[None, :n], d + 1, axis=0)
        out[p + 1] = U[n:]
        return out.reshape(self.N, -1)

    def matvec(self, V):
        shp = V.shape
        return self.expand(self.op.matvec_K(self.compress(V))).reshape(shp)

    def dense(self):
        return self.matvec(np.eye(self.N))


def lanczos_full(matvec, N, r, seed, node):
    """r Lanczos steps with full re-orthogonalisation from the normalised
    Rademacher start vector; returns (Q N x r', T r' x r') with r' <= r."""
    q = rng.rademacher(seed, node, 1, N)[:, 0]
    q /= np.linalg.norm(q)
    Q = np.zeros((N, r))
    alpha, beta = [], []
    b = 0.0
    q_prev = np.zeros(N)
    for j in range(r):
        Q[:, j] = q
        w = matvec(q)
        a = float(q @ w)
        alpha.append(a)
        w = w - a * q - b * q_prev
        for _ in range(2):  # full re-orthogonalisation, twice
            w = w - Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        b = float(np.linalg.norm(w))
        if j == r - 1 or b <= 1e-12 * max(abs(a), 1.0):
            break
        beta.append(b)
        q_prev = q
        q = w / b
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    return Q[:, :k], T


def hadamard_matvec(Qa, Ta, Qb, Tb, V):
    """(Qa Ta Qa^T o Qb Tb Qb^T) V via the SKIP reduction."""
    V = V.reshape(Qa.shape[0], -1)
    Aa = Qa @ Ta
    Ab = Qb @ Tb
    out = np.empty_like(V)
    for c in range(V.shape[1]):
        C = Qa.T @ (V[:, c:c + 1] * Qb)
        out[:, c] = np.sum(Aa * (Ab @ C.T), axis=1)
    return out


class DSKIP:
    """The D-SKIP operator K~ = s^2 (o_p Khat_p, Lanczos-compressed) + D."""

    def __init__(self, X, m, lo, hi, log_ell, log_s, log_sigma_f, log_sigma_g, r, seed):
        X = np.asarray(X, dtype=np.float64)
        self.n, self.d = X.shape
        self.N = self.n * (self.d + 1)
        self.s2 = np.exp(2.0 * log_s)
        le = np.broadcast_to(np.asarray(log_ell, dtype=np.float64), (self.d,))
        self.Dn = noise_diag(self.n, self.d, np.exp(log_sigma_f), np.exp(log_sigma_g))
        self.factors = [AxisFactor(X[:, p], p, self.d, m, lo[p], hi[p], le[p]) for p in range(self.d)]
        node = 0
        level = []
        for f in self.factors:
            level.append(lanczos_full(f.matvec, self.N, r, seed, node))
            node += 1
        while len(level) > 2:
            nxt = []
            for i in range(0, len(level) - 1, 2):
                (Qa, Ta), (Qb, Tb) = level[i], level[i + 1]
                mv = (lambda Qa, Ta, Qb, Tb: (lambda v: hadamard_matvec(Qa, Ta, Qb, Tb, v)[:, 0]))(Qa, Ta, Qb, Tb)
                nxt.append(lanczos_full(mv, self.N, r, seed, node))
                node += 1
            if len(level) % 2:
                nxt.append(level[-1])
            level = nxt
        self.root = level

    def matvec_K(self, V):
        V2 = V.reshape(self.N, -1)
        if len(self.root) == 1:
            Q, T = self.root[0]
            out = Q @ (T @ (Q.T @ V2))
        else:
            (Qa, Ta), (Qb, Tb) = self.root
            out = hadamard_matvec(Qa, Ta, Qb, Tb, V2)
        return (self.s2 * out).reshape(V.shape)

    def matvec(self, V):
        V2 = V.reshape(self.N, -1)
        return (self.matvec_K(V2) + self.Dn[:, None] * V2).reshape(V.shape)

    def diag_K(self):
        if len(self.root) == 1:
            Q, T = self.root[0]
            return self.s2 * np.sum((Q @ T) * Q, axis=1)
        (Qa, Ta), (Qb, Tb) = self.root
        return self.s2 * np.sum((Qa @ Ta) * Qa, axis=1) * np.sum((Qb @ Tb) * Qb, axis=1)

    def row_K(self, i):
        if len(self.root) == 1:
            Q, T = self.root[0]
            return self.s2 * (Q @ (T @ Q[i]))
        (Qa, Ta), (Qb, Tb) = self.root
        return self.s2 * (Qa @ (Ta @ Qa[i])) * (Qb @ (Tb @ Qb[i]))
