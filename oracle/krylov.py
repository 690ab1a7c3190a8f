"""Batched preconditioned CG and Lanczos (FP64).

Follows Sec. 2: linear systems with K~ are solved by conjugate gradients using
only MVMs, and the Lanczos connection supplies the tridiagonal matrices that
stochastic Lanczos quadrature needs (Gauss quadrature, Ubaru et al.; Dong et
al.).  Textbook PCG (Saad, Iterative Methods for Sparse Linear Systems,
Alg. 9.1) run on every column of a block independently; the columns share
each MVM but not their Krylov spaces.

Readings:
* x_0 = 0; a column stops when its recurrence residual satisfies
  ||r_j|| <= tol ||b|| (2-norm, unpreconditioned); the true residual
  ||b - K~ x|| / ||b|| is reported beside it.
* The Lanczos tridiagonal of the preconditioned operator from the CG
  coefficients (Saad Sec. 6.7.3): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
  T_{j,j+1} = sqrt(beta_j)/alpha_j (beta_{-1} = 0).
"""
import numpy as np


def pcg(matvec, B, precond=None, tol=1e-6, max_iter=10000, fixed_iters=None):
    """Independent PCG on each column of B (N x R).

    precond(R) -> M^{-1} R (None = identity).  With fixed_iters, every column
    runs exactly that many iterations (no tolerance test).

    Returns dict(x, iters, relres (recurrence), alpha, beta) where alpha/beta
    are lists (per column) of the CG coefficients."""
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    N, R = B.shape
    apply_m = (lambda V: V) if precond is None else precond
    X = np.zeros_like(B)
    Rr = B.copy()
    Z = apply_m(Rr)
    P = Z.copy()
    rz = np.sum(Rr * Z, axis=0)
    bnorm = np.linalg.norm(B, axis=0)
    bnorm[bnorm == 0] = 1.0
    active = np.ones(R, dtype=bool)
    if fixed_iters is None:
        active &= np.linalg.norm(Rr, axis=0) > tol * bnorm
    iters = np.zeros(R, dtype=np.int64)
    alphas = [[] for _ in range(R)]
    betas = [[] for _ in range(R)]
    limit = fixed_iters if fixed_iters is not None else max_iter
    for it in range(limit):
        if not active.any():
            break
        Q = matvec(P)
        pq = np.sum(P * Q, axis=0)
        alpha = np.where(active, rz / np.where(pq != 0, pq, 1.0), 0.0)
        X += alpha * P
        Rr -= alpha * Q
        Z = apply_m(Rr)
        rz_new = np.sum(Rr * Z, axis=0)
        beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        for c in np.nonzero(active)[0]:
            alphas[c].append(alpha[c])
            betas[c].append(beta[c])
            iters[c] += 1
        P = np.where(active, Z + beta * P, P)
        rz = np.where(active, rz_new, rz)
        if fixed_iters is None:
            active &= np.linalg.norm(Rr, axis=0) > tol * bnorm
    relres = np.linalg.norm(Rr, axis=0) / bnorm
    return dict(x=X, iters=iters, relres=relres, alpha=alphas, beta=betas)


def true_relres(matvec, B, X):
    B = B.reshape(B.shape[0], -1)
    X = X.reshape(B.shape)
    return np.linalg.norm(B - matvec(X), axis=0) / np.linalg.norm(B, axis=0)


def cg_tridiag(alpha, beta):
    """Lanczos tridiagonal (diag, offdiag) from CG coefficients of one column."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    J = len(a)
    diag = 1.0 / a
    diag[1:] += b[:J - 1] / a[:J - 1]
    off = np.sqrt(b[:J - 1]) / a[:J - 1]
    return diag, off


def lanczos(matvec, v0, steps, precond_solve=None, reorth=False):
    """Lanczos on M^{-1} K~ in the M-inner product (plain Lanczos when
    precond_solve is None), started from r0 = v0 (r-space vector).

    Builds T with the recurrence on residual-space vectors q_j (M-orthonormal
    after preconditioning): z_j = M^{-1} q_j.  Returns (diag, offdiag, ||v0||_{M^{-1}}^2).
    With reorth, full re-orthogonalisation against all previous vectors."""
    solve = (lambda V: V) if precond_solve is None else precond_solve
    r = np.asarray(v0, dtype=np.float64).copy()
    z = solve(r)
    nrm2 = float(r @ z)
    beta_prev = np.sqrt(nrm2)
    qs, zs = [], []
    q_prev = np.zeros_like(r)
    z_prev = np.zeros_like(r)
    diag, off = [], []
    q = r / beta_prev
    zq = z / beta_prev
    b = 0.0
    for j in range(steps):
        qs.append(q)
        zs.append(zq)
        w = matvec(zq)                  # K~ M^{-1} q  (residual space)
        a = float(zq @ w)
        diag.append(a)
        w = w - a * q - b * q_prev
        if reorth:
            for qq, zz in zip(qs, zs):
                w = w - (zz @ w) * qq
        wz = solve(w)
        b_new = float(np.sqrt(max(w @ wz, 0.0)))
        if j == steps - 1 or b_new == 0.0:
            break
        off.append(b_new)
        q_prev, z_prev = q, zq
        q = w / b_new
        zq = wz / b_new
        b = b_new
    return np.array(diag), np.array(off), nrm2
