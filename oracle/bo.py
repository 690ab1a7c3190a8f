"""Expected-improvement acquisition (FP64).

ORACLE -- test infrastructure only: the tests, the smoke check and the bench's
CPU baseline use it; the library never does.

Sec. 4.4 (Bayesian optimisation with derivatives, Alg. 1): the next sample
maximises the EI acquisition over the reduced space, built from the GP's
posterior mean and predictive variance.  Readings:
* the test functions are minimised, so the improvement at a candidate is
  max(f_best - xi - Y, 0) with Y ~ N(mu, sigma^2) the posterior of f there and
  xi >= 0 an exploration margin (0 in the plain criterion);
* sigma = sqrt(max(v, 0)): a variance estimate below zero (possible for the
  pivoted-Cholesky estimate) counts as no uncertainty;
* the acquisition is maximised over a caller-supplied candidate set (the first
  index on a tie).
"""
import math

import numpy as np


def expected_improvement(mu, var, f_best, xi=0.0):
    """EI = (f_best - xi - mu) Phi(z) + sigma phi(z), z = (f_best - xi - mu) / sigma;
    max(f_best - xi - mu, 0) where sigma = 0."""
    mu = np.asarray(mu, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    out = np.empty_like(mu)
    for j in range(mu.size):
        s = math.sqrt(max(var[j], 0.0))
        imp = f_best - xi - mu[j]
        if s == 0.0:
            out[j] = max(imp, 0.0)
        else:
            z = imp / s
            Phi = 0.5 * math.erfc(-z / math.sqrt(2.0))
            phi = math.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
            out[j] = imp * Phi + s * phi
    return out


def best_candidate(mu, var, f_best, xi=0.0):
    """(index, value) of the largest EI over the candidates (first on a tie)."""
    ei = expected_improvement(mu, var, f_best, xi)
    j = int(np.argmax(ei))
    return j, float(ei[j])
