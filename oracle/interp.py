"""Uniform inducing grid and Keys cubic-convolution weights (FP64).

Follows Sec. 2 (SKI: K_XX ~ W K_UU W^T with sparse local cubic interpolation
weights on a uniform grid U) and Sec. 3.1 (D-SKI: differentiate the
interpolation scheme, grad k(x, x') ~ sum_i grad w_i(x) k(x_i, x')).

Readings (the paper names cubic convolution, Keys 1981, and is silent on the
rest):
* Keys' kernel with a = -1/2 (the third-order accurate member of the family):
      u(r) = (a+2)|r|^3 - (a+3)|r|^2 + 1          for |r| <= 1
      u(r) = a|r|^3 - 5a|r|^2 + 8a|r| - 4a         for 1 < |r| < 2
      u(r) = 0                                     otherwise
  A coordinate x gets weight u((x - u_j)/h) on grid node u_j and derivative
  weight u'((x - u_j)/h)/h.
* Grid placement: for a data box [a_p, b_p] on axis p with m_p nodes,
  h_p = (b_p - a_p)/(m_p - 3) and the first node is lo_p = a_p - h_p, so every
  point of the box has all four stencil nodes inside the grid.
* Tensor-product interpolation in d dimensions; node multi-index
  (j_1, ..., j_d) is linearised in C order (j_1 slowest).

The oracle evaluates Keys' kernel on every node within distance 2 of the
point; it never forms the cubic polynomials per cell offset.
"""
import numpy as np
import scipy.sparse as sp

KEYS_A = -0.5


def keys_u(r, a=KEYS_A):
    """Keys' cubic convolution kernel u(r)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    m1 = r <= 1.0
    m2 = (r > 1.0) & (r < 2.0)
    out[m1] = (a + 2) * r[m1] ** 3 - (a + 3) * r[m1] ** 2 + 1.0
    out[m2] = a * r[m2] ** 3 - 5 * a * r[m2] ** 2 + 8 * a * r[m2] - 4 * a
    return out


def keys_du(r, a=KEYS_A):
    """Derivative u'(r) of Keys' kernel (odd function of r)."""
    r = np.asarray(r, dtype=np.float64)
    ar = np.abs(r)
    sg = np.sign(r)
    out = np.zeros_like(r)
    m1 = ar <= 1.0
    m2 = (ar > 1.0) & (ar < 2.0)
    out[m1] = 3 * (a + 2) * ar[m1] ** 2 - 2 * (a + 3) * ar[m1]
    out[m2] = 3 * a * ar[m2] ** 2 - 10 * a * ar[m2] + 8 * a
    return out * sg


class Grid:
    """Uniform grid: per axis (lo_p, h_p, m_p); nodes lo_p + j h_p."""

    def __init__(self, lo_box, hi_box, m):
        self.m = np.asarray(m, dtype=np.int64)
        a = np.asarray(lo_box, dtype=np.float64)
        b = np.asarray(hi_box, dtype=np.float64)
        self.h = (b - a) / (self.m - 3)
        self.lo = a - self.h
        self.d = len(self.m)

    @property
    def size(self):
        return int(np.prod(self.m))

    def nodes(self, p):
        return self.lo[p] + np.arange(self.m[p]) * self.h[p]


def axis_weights(x, lo, h, m):
    """1-D Keys weights of coordinates x (n,) on the grid lo + j h, j < m.

    Returns (idx, w, dw): n x 4 node indices and their value / derivative
    weights.  The candidate nodes are floor(s)-1 .. floor(s)+2 with
    s = (x - lo)/h, shifted to stay inside [0, m) at the box edges (there the
    node that drops out is at distance 2, where Keys' kernel vanishes).
    Points outside the data box (s outside [1, m-2] beyond rounding) raise."""
    s = (np.asarray(x, dtype=np.float64) - lo) / h
    if np.any(s < 1.0 - 1e-9) or np.any(s > m - 2 + 1e-9):
        raise ValueError("point outside the interpolation box")
    base = np.clip(np.floor(s).astype(np.int64) - 1, 0, m - 4)
    idx = base[:, None] + np.arange(4)[None, :]
    r = s[:, None] - idx                       # distance in grid units
    w = keys_u(r)
    dw = keys_du(r) / h
    return idx, w, dw


def interp_matrices(X, grid):
    """Sparse S = [W; d_1 W; ...; d_d W] (N x m, CSR, FP64), N = n(d+1).

    Row i of W holds prod_p w_p(x_ip) on the 4^d tensor nodes; row i of d_q W
    holds the same product with axis q's factor replaced by its derivative."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    per = [axis_weights(X[:, p], grid.lo[p], grid.h[p], grid.m[p]) for p in range(d)]
    # tensor product over the 4^d stencil
    combos = np.stack(np.meshgrid(*([np.arange(4)] * d), indexing="ij"), -1).reshape(-1, d)
    nnz = combos.shape[0]
    cols = np.zeros((n, nnz), dtype=np.int64)
    for p in range(d):
        cols = cols * grid.m[p] + per[p][0][:, combos[:, p]]
    blocks = []
    for blk in range(d + 1):
        val = np.ones((n, nnz))
        for p in range(d):
            src = per[p][2] if blk == p + 1 else per[p][1]
            val = val * src[:, combos[:, p]]
        blocks.append(sp.csr_matrix((val.ravel(), cols.ravel(),
                                     np.arange(0, n * nnz + 1, nnz)),
                                    shape=(n, grid.size)))
    S = sp.vstack(blocks).tocsr()
    S.sum_duplicates()
    return S
