"""Pins of the oracle's posterior mean at test points (Sec. 1, O(1) prediction;
mean = K_{*X} alpha with alpha = K~^{-1} y).  Not the formula retyped: the
identity at the training points, the exact derivative-SE posterior mean as the
grid is refined, and finite differences of the predicted value."""
import numpy as np

from oracle import dski as odski, predict
from oracle.kernels import dse_dense, noise_diag


def small_problem(n=40, d=2, m=20, seed=5):
    r = np.random.default_rng(seed)
    X = r.uniform(0.0, 1.0, (n, d))
    y = r.standard_normal(n * (d + 1))
    le, ls, lf, lg = np.log([0.3] * d), 0.2, np.log(0.05), np.log(0.1)
    op = odski.DSKI(X, [m] * d, np.zeros(d), np.ones(d), le, ls, lf, lg)
    return X, y, op, (np.exp(le), np.exp(ls), np.exp(lf), np.exp(lg))


def test_mean_at_training_points_is_y_minus_noise_times_alpha():
    """At the training points S_* = S, so S K_UU S^T alpha = (K~ - D) alpha = y - D alpha."""
    X, y, op, _ = small_problem()
    alpha = np.linalg.solve(op.dense(), y)
    mu = predict.predict_mean(op, predict.grid_vector(op, alpha), X)
    want = (y - op.Dn * alpha).reshape(X.shape[1] + 1, -1).T
    assert np.abs(mu - want).max() <= 1e-10 * np.abs(want).max()


def test_dski_mean_tends_to_the_exact_derivative_se_mean():
    """With the grid refined, the D-SKI posterior mean (value and gradient) at
    test points approaches the exact derivative-SE one (cubic interpolation
    error O(h^3) in the kernel)."""
    r = np.random.default_rng(11)
    n, d = 30, 2
    X = r.uniform(0.0, 1.0, (n, d))
    y = r.standard_normal(n * (d + 1))
    Xs = r.uniform(0.05, 0.95, (25, d))
    ell, s, sf, sg = 0.3, np.exp(0.2), 0.05, 0.1
    exact = predict.exact_predict_mean(X, y, Xs, [ell] * d, s, sf, sg)
    errs = []
    for m in (30, 60, 120):
        op = odski.DSKI(X, [m] * d, np.zeros(d), np.ones(d), np.log([ell] * d), 0.2, np.log(sf), np.log(sg))
        alpha = np.linalg.solve(op.dense(), y)
        mu = predict.predict_mean(op, predict.grid_vector(op, alpha), Xs)
        errs.append(np.abs(mu - exact).max() / np.abs(exact).max())
    assert errs[2] < 5e-3  # measured 9.4e-2, 8.0e-3, 2.1e-3
    assert errs[2] < errs[1] < errs[0]


def test_gradient_rows_are_derivatives_of_the_value_row():
    X, y, op, _ = small_problem()
    alpha = np.linalg.solve(op.dense(), y)
    g = predict.grid_vector(op, alpha)
    r = np.random.default_rng(2)
    Xs = r.uniform(0.1, 0.9, (10, 2))
    mu = predict.predict_mean(op, g, Xs)
    h = 1e-6
    for p in range(2):
        e = np.zeros(2)
        e[p] = h
        fd = (predict.predict_mean(op, g, Xs + e)[:, 0] - predict.predict_mean(op, g, Xs - e)[:, 0]) / (2 * h)
        assert np.abs(fd - mu[:, 1 + p]).max() <= 1e-6 * np.abs(mu[:, 1 + p]).max()


def test_variance_equals_exact_with_full_rank_and_underestimates_otherwise():
    """v^ uses M = D + L L^T for K~: with a full-rank pivoted Cholesky M = K~ and
    v^ is the exact D-SKI posterior variance; with rank k < N, L L^T <= K so
    v^ <= v (the paper's 'overestimate' is read as this inequality's other
    side); the exact variance itself lies in [0, k(x, x)]."""
    from oracle import pivchol
    X, y, op, _ = small_problem(n=30, m=16)
    r = np.random.default_rng(9)
    Xs = r.uniform(0.05, 0.95, (12, 2))
    K = op.dense_K()
    v = predict.exact_variance(op, Xs)
    Lf, piv, _ = pivchol.pivoted_cholesky(np.diag(K), lambda i: K[i], op.N, rel_tol=0.0)
    # full rank up to the numerical rank of K: M = D + L L^T reproduces K~
    vf = predict.predictive_variance(op, Lf, Xs)
    assert np.abs(vf - v).max() <= 1e-8 * np.abs(v).max() + 1e-12
    L5, _, _ = pivchol.pivoted_cholesky(np.diag(K), lambda i: K[i], 5)
    v5 = predict.predictive_variance(op, L5, Xs)
    assert (v5 <= v + 1e-12).all()
    assert (v >= -1e-12).all()
    kxx, _ = predict.prior_cov(op, Xs)
    assert (v <= kxx + 1e-12).all()


def test_prior_covariances_tend_to_the_exact_derivative_se_ones():
    """k(x, x) and K_{Xx} of the D-SKI kernel approach the exact derivative-SE
    covariances of f(x) with the training values and gradients as the grid is
    refined (App. B entries, cubic interpolation error O(h^3))."""
    r = np.random.default_rng(12)
    n, d = 25, 2
    X = r.uniform(0.0, 1.0, (n, d))
    Xs = r.uniform(0.05, 0.95, (10, d))
    ell, ls = 0.3, 0.2
    ref = dse_dense(Xs, [ell] * d, np.exp(ls), X2=X)[:len(Xs)].T     # N x n*: Cov(obs, f(x*))
    kref = np.diag(dse_dense(Xs, [ell] * d, np.exp(ls))[:len(Xs), :len(Xs)])
    errs = []
    for m in (20, 40, 80):
        op = odski.DSKI(X, [m] * d, np.zeros(d), np.ones(d), np.log([ell] * d), ls, np.log(0.05), np.log(0.1))
        kxx, Kx = predict.prior_cov(op, Xs)
        errs.append(max(np.abs(kxx - kref).max() / kref.max(), np.abs(Kx - ref).max() / np.abs(ref).max()))
    assert errs[-1] < 2e-3 and errs[2] < errs[1] < errs[0], errs


def test_randomized_variance_is_exact_with_scaled_unit_probes_and_unbiased():
    """With the n* probes sqrt(n*) e_j (E[z z^T] = I exactly over the set) the
    diagonal estimate is exact and the result is the exact D-SKI variance; with
    many Rademacher probes it approaches it, from a control variate far from it."""
    from oracle import pivchol
    X, y, op, _ = small_problem(n=30, m=16)
    r = np.random.default_rng(21)
    Xs = r.uniform(0.05, 0.95, (8, 2))
    K = op.dense_K()
    L, _, _ = pivchol.pivoted_cholesky(np.diag(K), lambda i: K[i], 10)
    v = predict.exact_variance(op, Xs)
    vhat = predict.predictive_variance(op, L, Xs)
    ns = len(Xs)
    ve = predict.predictive_variance_probes(op, L, Xs, np.sqrt(ns) * np.eye(ns))
    assert np.abs(ve - v).max() <= 1e-9 * np.abs(vhat - v).max()
    Zr = r.choice([-1.0, 1.0], (4000, ns))
    vr = predict.predictive_variance_probes(op, L, Xs, Zr)
    assert np.abs(vr - v).max() <= 0.1 * np.abs(vhat - v).max()
