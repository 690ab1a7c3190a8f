"""Pins of the oracle's quintic interpolation (Sec. 3.1; the six-point quintic
convolution kernel of Meijering et al. 1999, derived in oracle/interp.py from
its defining conditions) by what fixes it from outside the derivation:
partition of unity, exact reproduction of polynomials up to degree four (and
not five) with their derivatives, the identity row on grid nodes, smoothness
across cell boundaries, and a convergence order against the exact
derivative-SE kernel above that of cubic convolution."""
import numpy as np
import pytest

from oracle import dski, interp, kernels


def _weights(x, m=24):
    g = interp.Grid([0.0], [1.0], [m], "quintic")
    idx, w, dw = interp.axis_weights(x, g.lo[0], g.h[0], g.m[0], "quintic")
    return g, idx, w, dw


def test_quintic_grid_placement():
    g = interp.Grid([0.0, -1.0], [1.0, 2.0], [10, 17], "quintic")
    assert g.S == 6
    assert g.h[0] == pytest.approx(1 / 5) and g.lo[0] == pytest.approx(-2 / 5)
    assert g.h[1] == pytest.approx(3 / 12) and g.lo[1] == pytest.approx(-1.5)
    idx, w, dw = interp.axis_weights(np.array([0.0, 1.0, 0.5]), g.lo[0], g.h[0], g.m[0], "quintic")
    assert idx.shape == (3, 6) and idx.min() >= 0 and idx.max() <= 9
    with pytest.raises(ValueError):
        interp.axis_weights(np.array([1.01]), g.lo[0], g.h[0], g.m[0], "quintic")


def test_quintic_partition_of_unity():
    x = np.random.default_rng(1).random(500)
    g, idx, w, dw = _weights(x)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(dw.sum(1), 0.0, atol=1e-10)


@pytest.mark.parametrize("deg", [1, 2, 3, 4])
def test_quintic_reproduces_polynomials_up_to_degree_four(deg):
    r = np.random.default_rng(deg)
    c = r.standard_normal(deg + 1)
    poly = np.polynomial.Polynomial(c)
    x = r.random(300)
    g, idx, w, dw = _weights(x)
    u = g.nodes(0)
    np.testing.assert_allclose((w * poly(u[idx])).sum(1), poly(x), atol=1e-11)
    np.testing.assert_allclose((dw * poly(u[idx])).sum(1), poly.deriv()(x), atol=1e-8)


def test_quintic_does_not_reproduce_degree_five():
    x = np.random.default_rng(9).random(300)
    g, idx, w, dw = _weights(x)
    u = g.nodes(0)
    err = np.abs((w * u[idx] ** 5).sum(1) - x ** 5).max()
    assert err > 1e-7


def test_quintic_on_grid_nodes_and_smoothness():
    g, _, _, _ = _weights(np.array([0.5]), m=20)
    u = g.nodes(0)
    idx, w, dw = interp.axis_weights(np.array([u[7]]), g.lo[0], g.h[0], g.m[0], "quintic")
    full = np.zeros(20)
    np.add.at(full, idx[0], w[0])
    e = np.zeros(20)
    e[7] = 1.0
    np.testing.assert_allclose(full, e, atol=1e-13)
    # value and derivative weights continuous across a cell boundary
    eps = 1e-9
    a = interp.axis_weights(np.array([u[9] - eps, u[9] + eps]), g.lo[0], g.h[0], g.m[0], "quintic")
    fw, fd = np.zeros((2, 20)), np.zeros((2, 20))
    for k in range(2):
        np.add.at(fw[k], a[0][k], a[1][k])
        np.add.at(fd[k], a[0][k], a[2][k])
    assert np.abs(fw[0] - fw[1]).max() < 1e-7
    assert np.abs(fd[0] - fd[1]).max() < 1e-6 / g.h[0]
    # the kernel itself: interpolating and zero beyond its support
    np.testing.assert_allclose(interp.quintic_u(np.array([0.0, 1.0, 2.0, -1.0, 3.0, 3.5])),
                               [1, 0, 0, 0, 0, 0], atol=1e-13)


def test_quintic_dski_converges_faster_than_cubic():
    """h -> h/2 against the exact D-SE kernel: value block about fifth order
    (quartics reproduced), blocks with derivatives about fourth order, and
    below the cubic error on the same grid."""
    r = np.random.default_rng(8)
    X = 0.1 + 0.8 * r.random((60, 2))
    ell, s, n = 0.2, 1.0, 60
    E = kernels.dse_dense(X, [ell, ell], s)
    errs, cub = [], []
    for m in (17, 29, 53, 101):
        for kind, out in (("quintic", errs), ("cubic", cub)):
            op = dski.DSKI(X, [m, m], [0, 0], [1, 1], np.log([ell, ell]), np.log(s), -3, -3, kind)
            K = op.dense_K()
            ev = np.linalg.norm(K[:n, :n] - E[:n, :n]) / np.linalg.norm(E[:n, :n])
            eg = np.linalg.norm(K[n:, n:] - E[n:, n:]) / np.linalg.norm(E[n:, n:])
            out.append((ev, eg))
    errs, cub = np.array(errs), np.array(cub)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders[1:, 0] > 4.2)          # value block
    assert np.all(orders[1:, 1] > 3.2)          # gradient block
    assert np.all(errs[1:] < cub[1:])
    assert errs[-1, 0] < 1e-7 and errs[-1, 1] < 1e-5
