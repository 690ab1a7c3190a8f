"""Log marginal likelihood, eq. (1), and its hyper-parameter gradient (FP64).

eq. (1) with the n(d+1) observations of values and gradients:
    L(theta) = -1/2 [ y^T alpha + log|K~| + N log(2 pi) ],  alpha = K~^{-1} y,
with mean mu = 0.  Its derivative with respect to a hyper-parameter theta_j is
    dL/dtheta_j = 1/2 alpha^T (dK~/dtheta_j) alpha - 1/2 tr(K~^{-1} dK~/dtheta_j).

Sec. 3 ("differentiate the approximate kernel"): the derivative is that of the
D-SKI matrix itself, so the interpolation weights stay fixed and only K_UU
(through ell_p and s) and the noise D (through sigma_f, sigma_g) move.

Parameters are natural logs, ordered (log ell_1..log ell_d, log s,
log sigma_f, log sigma_g).

The stochastic trace uses the probes of the log-det estimator: with
z ~ (Cov M), u = K~^{-1} z and v = M^{-1} z, E[u^T K' v] = tr(K~^{-1} K').

Two variants:
* ``exact``: dense Cholesky (small problems): the textbook definitions.
* ``stochastic``: the iterative method -- one batched PCG on [y, z_1..z_t],
  SLQ log det from the same PCG coefficients, stochastic trace for the gradient.
"""
import math

import numpy as np
import scipy.linalg as sla

from . import krylov, rng, slq
from .precond import Precond


def exact(op, y):
    """Dense mll and gradient of the D-SKI model (Cholesky; N up to a few thousand)."""
    A = op.dense()
    cf = sla.cho_factor(A, lower=True)
    return exact_from_dense(op, A, cf, y)


def exact_from_dense(op, A, cf, y):
    alpha = sla.cho_solve(cf, y)
    logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
    N = A.shape[0]
    mll = -0.5 * (y @ alpha + logdet + N * math.log(2 * math.pi))
    Ainv = sla.cho_solve(cf, np.eye(N))
    grad = np.empty(op.d + 3)
    chunk = 512
    for j in range(op.d + 3):
        # tr(K~^{-1} dK) = sum_i (K~^{-1} dK)_ii, over column chunks of dK = dK I
        tr = 0.0
        for c0 in range(0, N, chunk):
            c1 = min(N, c0 + chunk)
            E = np.zeros((N, c1 - c0))
            E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            dKc = op.matvec_dtheta(j, E)
            tr += np.sum(Ainv[c0:c1, :] * dKc.T)
        grad[j] = 0.5 * alpha @ op.matvec_dtheta(j, alpha) - 0.5 * tr
    return dict(mll=mll, grad=grad, logdet=logdet, alpha=alpha)


def stochastic(op, y, L, num_probes, seed, tol, max_iter=10000, probes=None):
    """The iterative estimator; L is the pivoted-Cholesky factor (N x k).

    Returns dict(mll, grad, logdet, logdet_stderr, quads, weights, pcg)."""
    N = op.N
    P = Precond(L, op.Dn)
    W = rng.rademacher(seed, 0, num_probes, N) if probes is None else probes
    Z = P.factor_apply(W)
    B = np.concatenate([y[:, None], Z], axis=1)
    res = krylov.pcg(op.matvec, B, precond=P.solve, tol=tol, max_iter=max_iter)
    X = res["x"]
    alpha = X[:, 0]
    U = X[:, 1:]
    V = P.solve(Z)
    quads, weights = [], []
    for i in range(num_probes):
        dg, of = krylov.cg_tridiag(res["alpha"][1 + i], res["beta"][1 + i])
        quads.append(slq.quad_from_tridiag(dg, of))
        weights.append(float(Z[:, i] @ V[:, i]))
    logdet, se = slq.estimate(quads, weights, P.logdet())
    mll = -0.5 * (y @ alpha + logdet + N * math.log(2 * math.pi))
    grad = np.empty(op.d + 3)
    for j in range(op.d + 3):
        ka = op.matvec_dtheta(j, alpha)
        kv = op.matvec_dtheta(j, V)
        grad[j] = 0.5 * alpha @ ka - 0.5 * np.mean(np.sum(U * kv, axis=0))
    return dict(mll=mll, grad=grad, logdet=logdet, logdet_stderr=se, quads=np.array(quads),
                weights=np.array(weights), pcg=res, precond=P)
