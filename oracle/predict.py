"""Posterior mean of f and of its gradient at test points (FP64).

ORACLE -- test infrastructure only: the tests, the smoke check and the bench's
CPU baseline use it; the library never does.

Sec. 1 (contributions): learning costs O(nd) and prediction O(1) per test
point.  With alpha = K~^{-1} y (eq. (1)), the posterior mean of the test
observations [f(x*); grad f(x*)] is K_{*X} alpha.  Under D-SKI (Sec. 3.1)
K_{*X} = S_* K_UU S^T with S_* = [W_*; d_1 W_*; ...; d_d W_*] the value and
derivative interpolation rows of the test points, so the grid vector
g = K_UU S^T alpha is formed once and each test point interpolates it on its
cubic stencil: mean = S_* g (4^d nodes per test point, whatever n).

Readings (the paper states the complexity, not the steps):
* the mean of every test observation, value and all d partial derivatives,
  is returned, as the training observations are value and gradient;
* test points must lie in the interpolation box of the training grid.
"""
import numpy as np

from . import interp
from .kernels import dse_dense, noise_diag


def grid_vector(op, alpha):
    """g = K_UU S^T alpha (m,) for the D-SKI operator `op` (oracle.dski.DSKI)."""
    a = np.asarray(alpha, dtype=np.float64).reshape(op.N, 1)
    return np.asarray(op.kuu_apply(op.ST @ a)).reshape(-1)


def predict_mean(op, g, Xs):
    """Posterior means at the test points Xs (n* x d): an n* x (d + 1) array,
    column 0 the value, column 1 + p the derivative along axis p."""
    Xs = np.asarray(Xs, dtype=np.float64)
    ns, d = Xs.shape
    S_star = interp.interp_matrices(Xs, op.grid)
    return (S_star @ g).reshape(d + 1, ns).T


def exact_predict_mean(X, y, Xs, ell, s, sigma_f, sigma_g):
    """The same posterior means with the exact derivative-SE kernel (dense
    solve; small problems): K_{*X} (K + D)^{-1} y."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    K = dse_dense(X, ell, s) + np.diag(noise_diag(n, d, sigma_f, sigma_g))
    alpha = np.linalg.solve(K, y)
    Ks = dse_dense(np.asarray(Xs, dtype=np.float64), ell, s, X2=X)
    return (Ks @ alpha).reshape(d + 1, -1).T
