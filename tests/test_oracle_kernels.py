"""Pins of the oracle's kernels, grid weights, RNG and D-SKI operator.

Every check compares the oracle with something other than itself: published
values (tests/golden), finite differences, closed forms, brute force on tiny
inputs, or a library routine.
"""
import os

import numpy as np
import pytest

from oracle import dski, interp, kernels, rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- SplitMix64
def test_splitmix64_reference_vector():
    want = [int(r[0]) for r in _gold("splitmix64_seed1234567.txt")]
    got = rng.splitmix64(1234567, np.arange(5)).tolist()
    assert got == want


def test_rademacher_counter_layout():
    a = rng.rademacher(99, 0, 3, 50)
    b = rng.rademacher(99, 1, 2, 50)
    assert set(np.unique(a)) <= {-1.0, 1.0}
    assert np.array_equal(a[:, 1:], b)           # column c uses counters c*N + i
    z = rng.splitmix64(99, np.arange(50, 100))
    assert np.array_equal(a[:, 1], np.where(z >> np.uint64(63), -1.0, 1.0))
    assert abs(a.mean()) < 0.3


# ---------------------------------------------------------------- SE / D-SE
def _fd_grad_k(x, xp, ell, s, h=1e-5):
    d = len(x)
    g = np.zeros(d)
    for p in range(d):
        e = np.zeros(d); e[p] = h
        g[p] = (kernels.se(x[None] + e, xp[None], ell, s) - kernels.se(x[None] - e, xp[None], ell, s))[0, 0] / (2 * h)
    return g


def test_dse_first_derivatives_match_finite_differences():
    r = np.random.default_rng(0)
    ell = np.array([0.3, 0.5, 0.2]); s = 1.3
    X = r.random((2, 3))
    K = kernels.dse_dense(X, ell, s)
    n = 2
    for i in range(n):
        for j in range(n):
            # Cov(d_p f_i, f_j) = d/dx_ip k(x_i, x_j)
            g = _fd_grad_k(X[i], X[j], ell, s)
            for p in range(3):
                assert K[(p + 1) * n + i, j] == pytest.approx(g[p], rel=1e-7, abs=1e-9)
            # Cov(f_i, d_q f_j) = d/dx_jq k(x_i, x_j)
            g2 = _fd_grad_k(X[j], X[i], ell, s)
            for q in range(3):
                assert K[i, (q + 1) * n + j] == pytest.approx(g2[q], rel=1e-7, abs=1e-9)


def test_dse_second_derivatives_match_finite_differences():
    r = np.random.default_rng(1)
    ell = np.array([0.4, 0.25]); s = 0.7
    X = r.random((3, 2))
    n = 3
    K = kernels.dse_dense(X, ell, s)
    h = 1e-4
    for i in range(n):
        for j in range(n):
            for p in range(2):
                for q in range(2):
                    ep = np.zeros(2); ep[p] = h
                    eq = np.zeros(2); eq[q] = h
                    k = lambda a, b: kernels.se(a[None], b[None], ell, s)[0, 0]
                    fd = (k(X[i] + ep, X[j] + eq) - k(X[i] + ep, X[j] - eq)
                          - k(X[i] - ep, X[j] + eq) + k(X[i] - ep, X[j] - eq)) / (4 * h * h)
                    assert K[(p + 1) * n + i, (q + 1) * n + j] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_dse_symmetric_psd_and_1d_spectral_form():
    r = np.random.default_rng(2)
    X = r.random((40, 2))
    K = kernels.dse_dense(X, [0.3, 0.3], 1.0)
    assert np.array_equal(K, K.T) or np.abs(K - K.T).max() < 1e-14
    lam = np.linalg.eigvalsh(K)
    assert lam.min() >= -1e-10 * lam.max()
    # d = 1: k(x,x') = s^2 E_w[cos(w (x - x'))], w ~ N(0, 1/ell^2), so
    # Cov(f'(x), f'(x')) = s^2 E[w^2 cos(w r)] (Bochner).  Gauss-Hermite quadrature
    # evaluates the expectation independently of the closed form.
    ell, s = 0.35, 1.2
    x = np.array([[0.1], [0.45]])
    Kd = kernels.dse_dense(x, [ell], s)
    gh, wts = np.polynomial.hermite_e.hermegauss(80)
    w = gh / ell
    norm = wts.sum()
    rr = x[0, 0] - x[1, 0]
    e_cos = s * s * np.sum(wts * np.cos(w * rr)) / norm
    e_w2cos = s * s * np.sum(wts * w * w * np.cos(w * rr)) / norm
    e_wsin = s * s * np.sum(wts * w * np.sin(w * rr)) / norm
    assert Kd[0, 1] == pytest.approx(e_cos, rel=1e-12)
    assert Kd[2, 3] == pytest.approx(e_w2cos, rel=1e-10)
    # Cov(f'(x_0), f(x_1)) = d/dx_0 k = -s^2 E[w sin(w (x_0 - x_1))]
    assert Kd[2, 1] == pytest.approx(-e_wsin, rel=1e-10)


# ---------------------------------------------------------------- Keys weights
def test_keys_golden_weights():
    for row in _gold("keys_catmull_rom.txt"):
        t, *w = map(float, row)
        got = interp.keys_u(np.array([1 + t, t, 1 - t, 2 - t]))
        np.testing.assert_allclose(got, w, atol=1e-15)


def test_keys_partition_of_unity_and_derivative_sum():
    t = np.linspace(0, 1, 101)
    r = np.stack([1 + t, t, t - 1, t - 2], 1)
    w = interp.keys_u(r)
    dw = interp.keys_du(r)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)
    np.testing.assert_allclose(dw.sum(1), 0.0, atol=1e-14)


def test_keys_reproduces_quadratics_and_derivatives():
    g = interp.Grid([0.0], [1.0], [20])
    u = g.nodes(0)
    poly = lambda x: 0.3 - 1.7 * x + 2.2 * x * x
    dpoly = lambda x: -1.7 + 4.4 * x
    x = np.random.default_rng(3).random(200)
    idx, w, dw = interp.axis_weights(x, g.lo[0], g.h[0], g.m[0])
    np.testing.assert_allclose((w * poly(u[idx])).sum(1), poly(x), atol=1e-13)
    np.testing.assert_allclose((dw * poly(u[idx])).sum(1), dpoly(x), atol=1e-11)


def test_keys_on_grid_point_and_c1_continuity():
    g = interp.Grid([0.0], [1.0], [13])
    u = g.nodes(0)
    idx, w, dw = interp.axis_weights(np.array([u[5]]), g.lo[0], g.h[0], g.m[0])
    full = np.zeros(13); dfull = np.zeros(13)
    np.add.at(full, idx[0], w[0]); np.add.at(dfull, idx[0], dw[0])
    e = np.zeros(13); e[5] = 1
    np.testing.assert_allclose(full, e, atol=1e-15)
    cd = np.zeros(13); cd[4] = -0.5 / g.h[0]; cd[6] = 0.5 / g.h[0]
    np.testing.assert_allclose(dfull, cd, atol=1e-12)
    # derivative weights continuous across a cell boundary
    for eps in (1e-9,):
        a = interp.axis_weights(np.array([u[5] - eps, u[5] + eps]), g.lo[0], g.h[0], g.m[0])
        fa = np.zeros((2, 13))
        for k in range(2):
            np.add.at(fa[k], a[0][k], a[2][k])
        assert np.abs(fa[0] - fa[1]).max() < 1e-6 / g.h[0]


def test_grid_placement_keeps_stencil_inside():
    g = interp.Grid([0.0, -1.0], [1.0, 2.0], [10, 17])
    assert g.h[0] == pytest.approx(1 / 7) and g.lo[0] == pytest.approx(-1 / 7)
    x = np.array([0.0, 1.0])
    idx, w, dw = interp.axis_weights(x, g.lo[0], g.h[0], g.m[0])
    assert idx.min() >= 0 and idx.max() <= 9
