"""Stochastic Lanczos quadrature for log det K~ (FP64).

Follows Sec. 2: log|K~| = tr(log K~) is estimated with probe vectors and the
Gauss-quadrature connection of Lanczos (Ubaru, Chen, Saad; Dong et al.), which
needs only MVMs and a few probes.

With a preconditioner M = C C^T (Sec. 3.3):
    log det K~ = log det M + tr log(C^{-1} K~ C^{-T})
and for a probe z with C^{-1} z = w,
    w^T log(C^{-1} K~ C^{-T}) w ~ (z^T M^{-1} z) e_1^T log(T) e_1,
where T is the Lanczos tridiagonal of the preconditioned operator started
from z (equivalently, from the PCG coefficients of the solve K~ x = z).

Readings:
* Probes: Rademacher driving vectors w (SplitMix64 stream, see ``rng``) mapped
  to z = C w with the square-root-form factor, so Cov(z) = M; without a
  preconditioner z = w.
* The estimate is log det M + (1/t) sum_i (z_i^T M^{-1} z_i) e_1^T log(T_i) e_1.
* A fixed number of Lanczos steps (the small FP64 configuration's "30 Lanczos
  steps") runs the explicit Lanczos process of the preconditioned operator in
  the M-inner product from z = C w, with full re-orthogonalisation against all
  earlier Lanczos vectors (``fixed_step_logdet``).  In exact arithmetic its
  tridiagonal is the one CG's coefficients give; in floating point a short
  Lanczos run without re-orthogonalisation loses orthogonality and its value
  moves by about 1e-3 relative under rounding-level perturbations of K~ or
  M^{-1}, while the re-orthogonalised run does not.
* ``quad_from_tridiag`` evaluates e_1^T log(T) e_1 through the symmetric
  eigen-decomposition T = V diag(theta) V^T: sum_k V_1k^2 log theta_k.  T is
  written out densely and decomposed by LAPACK's divide-and-conquer driver
  (syevd via scipy), whose cost stays a few seconds for the thousands of
  steps of a converged solve (the tridiagonal QL driver accumulates the
  eigenvectors in O(J^3) scalar rotations: 45 s at J = 3,000).
"""
import numpy as np
import scipy.linalg as sla

from . import krylov


def quad_from_tridiag(diag, off):
    """e_1^T log(T) e_1 for the symmetric tridiagonal T = tridiag(off, diag, off)."""
    diag = np.asarray(diag, dtype=np.float64)
    off = np.asarray(off, dtype=np.float64)
    if diag.size == 1:
        return float(np.log(diag[0]))
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    theta, V = sla.eigh(T, driver="evd")
    if np.any(theta <= 0):
        raise FloatingPointError("non-positive Ritz value in SLQ")
    return float(np.sum(V[0, :] ** 2 * np.log(theta)))


def estimate(quads, weights, logdet_M=0.0):
    """Combine per-probe quadratures: logdet_M + mean(weight_i * quad_i); also
    the standard error of the mean."""
    vals = np.asarray(weights, dtype=np.float64) * np.asarray(quads, dtype=np.float64)
    t = vals.size
    se = float(np.std(vals, ddof=1) / np.sqrt(t)) if t > 1 else float("nan")
    return float(logdet_M + vals.mean()), se


def fixed_step_logdet(matvec, P, W, steps):
    """log det K~ from `steps` Lanczos steps per probe with full
    re-orthogonalisation: for each Rademacher column w of W, z = C w (P's
    square-root factor, C C^T = M), the Lanczos tridiagonal T of the
    preconditioned operator started from z, and the weight ||z||^2_{M^{-1}};
    returns (estimate, standard error) as ``estimate`` combines them with
    log det M."""
    Z = P.factor_apply(np.asarray(W, dtype=np.float64))
    quads, weights = [], []
    for i in range(Z.shape[1]):
        dg, of, nrm2 = krylov.lanczos(matvec, Z[:, i], steps, P.solve, reorth=True)
        quads.append(quad_from_tridiag(dg, of))
        weights.append(nrm2)
    return estimate(quads, weights, P.logdet())
