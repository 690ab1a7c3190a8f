"""Uniform inducing grid, Keys cubic and quintic convolution weights (FP64).

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
* Quintic interpolation (Sec. 3.1 names the quintic kernel of Meijering et
  al. 1999 as the default; its coefficients are not printed): the kernel is
  taken as the piecewise quintic u on [-3, 3], even, zero for |r| >= 3, that
  interpolates (u(0) = 1, u(+-1) = u(+-2) = 0), has continuous first and
  second derivatives everywhere (including |r| = 3, where it meets zero), and
  reproduces polynomials of degree <= 4 (sum_k u(t - k) (k - t)^j = [j = 0]
  for j <= 4 and all t).  These linear conditions on the 18 coefficients of
  the three pieces have exactly one solution, which ``quintic_pieces``
  computes in exact rational arithmetic.  Six nodes per axis; grid
  h_p = (b_p - a_p)/(m_p - 5), first node a_p - 2 h_p.

The oracle evaluates the kernel on every node within its support radius of
the point; it never forms the polynomials per cell offset.
"""
from fractions import Fraction
from functools import lru_cache
from math import comb

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


def _solve_exact(rows, rhs, nunk):
    """Unique solution of the square-or-overdetermined consistent system
    rows x = rhs in exact fractions (Gauss-Jordan); raises if it is not unique
    or not consistent."""
    A = [list(r) + [b] for r, b in zip(rows, rhs)]
    piv = []
    r = 0
    for c in range(nunk):
        pr = next((i for i in range(r, len(A)) if A[i][c] != 0), None)
        if pr is None:
            continue
        A[r], A[pr] = A[pr], A[r]
        pv = A[r][c]
        A[r] = [x / pv for x in A[r]]
        for i in range(len(A)):
            if i != r and A[i][c] != 0:
                f = A[i][c]
                A[i] = [x - f * y for x, y in zip(A[i], A[r])]
        piv.append(c)
        r += 1
    if len(piv) != nunk:
        raise ArithmeticError("quintic kernel conditions do not fix the kernel")
    if any(all(x == 0 for x in row[:nunk]) and row[nunk] != 0 for row in A):
        raise ArithmeticError("quintic kernel conditions are inconsistent")
    x = [Fraction(0)] * nunk
    for i, c in enumerate(piv):
        x[c] = A[i][nunk]
    return x


@lru_cache(maxsize=None)
def quintic_pieces():
    """Coefficients c[p][i] (Fractions) of the quintic kernel on |r| in [p, p+1],
    u(r) = sum_i c[p][i] |r|^i, p = 0, 1, 2, from the conditions stated in the
    module docstring."""
    nunk = 18

    def at(p, x, der=0):
        row = [Fraction(0)] * nunk
        for i in range(der, 6):
            f = Fraction(1)
            for k in range(der):
                f *= i - k
            row[6 * p + i] = f * Fraction(x) ** (i - der)
        return row

    rows, rhs = [], []

    def eq(row, b):
        rows.append(row)
        rhs.append(Fraction(b))

    # interpolation and compact support
    for p, x, b in ((0, 0, 1), (0, 1, 0), (1, 1, 0), (1, 2, 0), (2, 2, 0), (2, 3, 0)):
        eq(at(p, x), b)
    # smoothness: u' = 0 at 0 (even kernel); u', u'' continuous at 1, 2; zero at 3
    eq(at(0, 0, 1), 0)
    for der in (1, 2):
        eq([a - b for a, b in zip(at(0, 1, der), at(1, 1, der))], 0)
        eq([a - b for a, b in zip(at(1, 2, der), at(2, 2, der))], 0)
        eq(at(2, 3, der), 0)
    # reproduction of degree <= 4: for t in [0, 1) the nodes k = -2..3 sit at
    # distance |t - k| in pieces 2, 1, 0, 0, 1, 2 (argument a + s t)
    nodes = ((-2, 2, 2, 1), (-1, 1, 1, 1), (0, 0, 0, 1), (1, 0, 1, -1), (2, 1, 2, -1), (3, 2, 3, -1))
    for j in range(5):
        poly = [[Fraction(0)] * nunk for _ in range(11)]   # coefficient of t^e, e <= 10
        for k, p, a, sgn in nodes:
            for i in range(6):
                for e1 in range(i + 1):                      # (a + sgn t)^i
                    ci = comb(i, e1) * Fraction(a) ** (i - e1) * Fraction(sgn) ** e1
                    for e2 in range(j + 1):                  # (k - t)^j
                        cj = comb(j, e2) * Fraction(k) ** (j - e2) * Fraction(-1) ** e2
                        poly[e1 + e2][6 * p + i] += ci * cj
        for e in range(11):
            eq(poly[e], 1 if (j == 0 and e == 0) else 0)
    x = _solve_exact(rows, rhs, nunk)
    return tuple(tuple(x[6 * p + i] for i in range(6)) for p in range(3))


def quintic_u(r):
    """The quintic convolution kernel u(r) (support |r| < 3)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    for p, c in enumerate(quintic_pieces()):
        m = r < 1 if p == 0 else ((r >= 1) & (r < 2) if p == 1 else (r >= 2) & (r < 3))
        out[m] = sum(float(ci) * r[m] ** i for i, ci in enumerate(c))
    return out


def quintic_du(r):
    """Derivative u'(r) of the quintic kernel (odd function of r)."""
    r = np.asarray(r, dtype=np.float64)
    ar = np.abs(r)
    out = np.zeros_like(r)
    for p, c in enumerate(quintic_pieces()):
        m = ar < 1 if p == 0 else ((ar >= 1) & (ar < 2) if p == 1 else (ar >= 2) & (ar < 3))
        out[m] = sum(i * float(ci) * ar[m] ** (i - 1) for i, ci in enumerate(c) if i > 0)
    return out * np.sign(r)


# kernel by name: (u, u', stencil nodes S)
KERNELS = {"cubic": (keys_u, keys_du, 4), "quintic": (quintic_u, quintic_du, 6)}


class Grid:
    """Uniform grid: per axis (lo_p, h_p, m_p); nodes lo_p + j h_p.  With S
    stencil nodes per axis (4 cubic, 6 quintic) and H = S/2 - 1,
    h_p = (b_p - a_p)/(m_p - S + 1) and lo_p = a_p - H h_p."""

    def __init__(self, lo_box, hi_box, m, interp="cubic"):
        self.interp = interp
        self.S = KERNELS[interp][2]
        H = self.S // 2 - 1
        self.m = np.asarray(m, dtype=np.int64)
        a = np.asarray(lo_box, dtype=np.float64)
        b = np.asarray(hi_box, dtype=np.float64)
        self.h = (b - a) / (self.m - self.S + 1)
        self.lo = a - H * self.h
        self.d = len(self.m)

    @property
    def size(self):
        return int(np.prod(self.m))

    def nodes(self, p):
        return self.lo[p] + np.arange(self.m[p]) * self.h[p]


def axis_weights(x, lo, h, m, interp="cubic"):
    """1-D interpolation weights of coordinates x (n,) on the grid lo + j h, j < m.

    Returns (idx, w, dw): n x S node indices and their value / derivative
    weights (S = 4 cubic, 6 quintic; H = S/2 - 1).  The candidate nodes are
    floor(s) - H .. floor(s) - H + S - 1 with s = (x - lo)/h, shifted to stay
    inside [0, m) at the box edges (there the node that drops out is at the
    support radius, where the kernel vanishes).  Points outside the data box
    (s outside [H, m - S + H + 1] beyond rounding) raise."""
    u, du, S = KERNELS[interp]
    H = S // 2 - 1
    s = (np.asarray(x, dtype=np.float64) - lo) / h
    if np.any(s < H - 1e-9) or np.any(s > m - S + H + 1 + 1e-9):
        raise ValueError("point outside the interpolation box")
    base = np.clip(np.floor(s).astype(np.int64) - H, 0, m - S)
    idx = base[:, None] + np.arange(S)[None, :]
    r = s[:, None] - idx                       # distance in grid units
    w = u(r)
    dw = du(r) / h
    return idx, w, dw


def interp_matrices(X, grid):
    """Sparse S = [W; d_1 W; ...; d_d W] (N x m, CSR, FP64), N = n(d+1).

    Row i of W holds prod_p w_p(x_ip) on the S^d tensor nodes; row i of d_q W
    holds the same product with axis q's factor replaced by its derivative."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    per = [axis_weights(X[:, p], grid.lo[p], grid.h[p], grid.m[p], grid.interp) for p in range(d)]
    # tensor product over the S^d stencil
    combos = np.stack(np.meshgrid(*([np.arange(grid.S)] * d), indexing="ij"), -1).reshape(-1, d)
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
