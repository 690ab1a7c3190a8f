"""Pins of the oracle's expected improvement (Sec. 4.4): the defining
expectation by numerical quadrature, the zero-variance limit, monotonicity in
the variance, and the first-index tie rule."""
import numpy as np
from scipy import integrate

from oracle import bo


def test_ei_is_the_expected_improvement_by_quadrature():
    r = np.random.default_rng(2)
    mu = r.normal(0.0, 1.0, 12)
    var = r.uniform(0.01, 4.0, 12)
    f_best, xi = 0.3, 0.05
    ei = bo.expected_improvement(mu, var, f_best, xi)
    for j in range(12):
        s = np.sqrt(var[j])
        dens = lambda y: np.exp(-0.5 * ((y - mu[j]) / s) ** 2) / (s * np.sqrt(2 * np.pi))
        q, _ = integrate.quad(lambda y: (f_best - xi - y) * dens(y), -np.inf, f_best - xi, epsabs=1e-13,
                              epsrel=1e-12)
        assert abs(ei[j] - q) <= 1e-10 * max(1.0, q)


def test_zero_and_negative_variance_give_the_plain_improvement():
    ei = bo.expected_improvement([0.0, 1.0, 2.0], [0.0, -3.0, 0.0], 1.5)
    assert np.array_equal(ei, [1.5, 0.5, 0.0])
    # the limit sigma -> 0 agrees with it
    small = bo.expected_improvement([0.0, 2.0], [1e-20, 1e-20], 1.5)
    assert np.abs(small - [1.5, 0.0]).max() < 1e-9


def test_ei_grows_with_the_variance_and_the_tie_rule():
    var = np.linspace(0.0, 5.0, 30)
    ei = bo.expected_improvement(np.full(30, 0.7), var, 0.2)
    assert (np.diff(ei) > 0).all()
    j, v = bo.best_candidate([1.0, 0.0, 0.0, 2.0], [1.0, 1.0, 1.0, 0.0], 0.5)
    assert j == 1 and v > 0
