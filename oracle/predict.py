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

Predictive variance (Sec. 4.4, first approach): with the pivoted-Cholesky
preconditioner M = D + L L^T in place of K~,
    v^(x) = k(x, x) - K_{xX} M^{-1} K_{Xx}
for the value f(x) at a test point (the paper writes the single-noise QR form
sigma^{-2}(||K_{Xx}||^2 - ||Q_1^T K_{Xx}||^2) of the same quantity).

Randomized variance (Sec. 4.4, second approach): the pivoted-Cholesky
estimate as a control variate for a diagonal estimator with probes z over the
test points,
    v = v^ - E_z[ z .* (K_{X'X} (K~^{-1} - M^{-1}) K_{XX'} z) ],
unbiased when E[z z^T] = I; the mean over the caller's probes replaces E_z.

Readings (the paper states the complexity and the formula, not the steps):
* the mean of every test observation, value and all d partial derivatives,
  is returned, as the training observations are value and gradient;
* test points must lie in the interpolation box of the training grid;
* k(x, x) and K_{Xx} are those of the D-SKI kernel (w_x^T K_UU w_x and
  S K_UU w_x, w_x the test point's value stencil), so that v^ is the variance
  of the approximate model;
* the printed randomized formula subtracts v^ and starts from diag(K_{X'X'});
  read as the control-variate form above (v^ plus the estimate of
  diag(K_{X'X} (M^{-1} - K~^{-1}) K_{XX'}) with the opposite sign), the only
  form whose expectation is v;
* the paper calls v^ a small overestimate of v; since pivoted Cholesky gives
  L L^T <= K, M <= K~ and v^ <= v: v^ underestimates v, and equals it when L
  has full rank (both checked by the pins).
"""
import numpy as np

from . import interp
from .kernels import dse_dense, noise_diag
from .precond import Precond


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


def prior_cov(op, Xs):
    """(k(x, x) per test point, K_{Xx} as N x n*) of the D-SKI kernel: with w_x
    the value stencil, w_x^T K_UU w_x and S K_UU w_x."""
    Xs = np.asarray(Xs, dtype=np.float64)
    ns = Xs.shape[0]
    Wv = interp.interp_matrices(Xs, op.grid)[:ns]            # value stencils, n* x m
    H = np.asarray(op.kuu_apply(Wv.T.toarray()))              # K_UU w_x, m x n*
    kxx = np.asarray((Wv.multiply(H.T)).sum(axis=1)).ravel()
    return kxx, op.S @ H


def predictive_variance(op, L, Xs):
    """v^(x) = k(x, x) - K_{xX} M^{-1} K_{Xx} of f(x) at each test point, with
    M = D + L L^T (L: N x k pivoted-Cholesky factor of the noise-free K)."""
    kxx, Kx = prior_cov(op, Xs)
    return kxx - np.sum(Kx * Precond(L, op.Dn).solve(Kx), axis=0)


def exact_variance(op, Xs):
    """v(x) = k(x, x) - K_{xX} K~^{-1} K_{Xx} with the dense D-SKI matrix."""
    kxx, Kx = prior_cov(op, Xs)
    return kxx - np.sum(Kx * np.linalg.solve(op.dense(), Kx), axis=0)


def predictive_variance_probes(op, L, Xs, Zp):
    """Randomized predictive variance of f at the test points Xs with the
    pivoted-Cholesky estimate as control variate; Zp (R x n*) holds the probes
    (row r = probe r over the test points)."""
    Zp = np.asarray(Zp, dtype=np.float64)
    R = Zp.shape[0]
    vhat = predictive_variance(op, L, Xs)
    _, Kx = prior_cov(op, Xs)                       # K_{XX'}, N x n*
    b = Kx @ Zp.T                                   # K_{XX'} z, N x R
    u = np.linalg.solve(op.dense(), b) - Precond(L, op.Dn).solve(b)
    e = Kx.T @ u                                    # K_{X'X} (K~^{-1} - M^{-1}) K_{XX'} z, n* x R
    return vhat - np.sum(Zp.T * e, axis=1) / R
