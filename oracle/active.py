"""Active-subspace dimension reduction (FP64).

ORACLE -- test infrastructure only: the tests, the smoke check and the bench's
CPU baseline use it; the library never does.

Sec. 3.4 (dimensionality reduction): the active subspace of f: R^D -> R is
spanned by the dominant eigenvectors of C = int grad f grad f^T, estimated by
Monte Carlo over the sample points; with P (D x d, orthonormal columns) the GP
works with the kernel k(P^T x, P^T x').  Readings:
* C is the sample mean (1/n) sum_i g_i g_i^T of the n gradient observations;
* the reduced data are u_i = P^T x_i with value f_i and gradient P^T g_i (the
  gradient of u -> f(P u), as f(x) ~ f(P P^T x));
* each eigenvector's sign is fixed so that its entry of largest magnitude is
  positive (the lowest index on a tie), which makes P unique when the
  eigenvalues are distinct.
"""
import numpy as np


def gradient_covariance(G):
    """C = (1/n) G^T G for the n x D gradient samples G (row i = grad f(x_i))."""
    G = np.asarray(G, dtype=np.float64)
    return G.T @ G / G.shape[0]


def active_subspace(G, d):
    """(P, eigenvalues): the d dominant eigenvectors of C as columns of the
    D x d matrix P, and all D eigenvalues of C in decreasing order."""
    lam, V = np.linalg.eigh(gradient_covariance(G))
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V[:, :d].copy(), lam


def project(X, G, P):
    """Reduced data: U = X P (n x d) and the reduced gradients G P (n x d)."""
    return np.asarray(X, dtype=np.float64) @ P, np.asarray(G, dtype=np.float64) @ P
