"""Pins of the oracle's D-SKI operator (Sec. 3.1) against brute force,
closed forms and convergence order."""
import numpy as np
import pytest

from oracle import dski, interp, kernels


def _small_op(n=60, m=(9, 11), ell=(0.3, 0.45), s=1.1, sf=0.05, sg=0.1, seed=0):
    r = np.random.default_rng(seed)
    X = r.random((n, len(m)))
    op = dski.DSKI(X, m, np.zeros(len(m)), np.ones(len(m)), np.log(ell), np.log(s),
                   np.log(sf), np.log(sg))
    return op


def test_mode_product_equals_kron():
    r = np.random.default_rng(0)
    mats = [r.standard_normal((4, 4)), r.standard_normal((3, 3)), r.standard_normal((5, 5))]
    G = r.standard_normal((60, 2))
    K = np.kron(np.kron(mats[0], mats[1]), mats[2])
    np.testing.assert_allclose(dski.mode_product(G, mats), K @ G, rtol=1e-13, atol=1e-13)


def test_toeplitz_circulant_embedding_fft():
    # the circulant embedding of length L >= 2m-1 reproduces the Toeplitz product
    m, h, ell = 37, 0.05, 0.21
    T = dski.toeplitz_factor(m, h, ell)
    for L in (2 * m - 1, 2 * m, 128):
        c = np.zeros(L)
        c[:m] = T[0]
        c[L - m + 1:] = T[0, 1:][::-1]
        lam = np.fft.fft(c).real
        v = np.random.default_rng(L).standard_normal(m)
        pad = np.zeros(L); pad[:m] = v
        out = np.fft.ifft(lam * np.fft.fft(pad)).real[:m]
        np.testing.assert_allclose(out, T @ v, rtol=1e-12, atol=1e-13)
        assert lam.min() > -1e-12 * lam.max()


def _brute_dski(op):
    """Brute force: sum_ab dw_a(x_i) k(u_a, u_b) dw_b(x_j) with the SE kernel
    evaluated directly on node coordinates and the weights taken from Keys'
    kernel node by node (no sparse matrices, no Kronecker structure)."""
    X, g, d, n = op.X, op.grid, op.d, op.n
    nodes = np.stack(np.meshgrid(*[g.nodes(p) for p in range(d)], indexing="ij"), -1).reshape(-1, d)
    Kuu = kernels.se(nodes, nodes, op.ell, op.s)
    # weights of every point on every node (dense, from the kernel definition)
    Wd = np.ones((d + 1, n, nodes.shape[0]))
    for p in range(d):
        r = (X[:, p][:, None] - nodes[:, p][None, :]) / g.h[p]
        for blk in range(d + 1):
            Wd[blk] *= interp.keys_du(r) / g.h[p] if blk == p + 1 else interp.keys_u(r)
    Sd = Wd.reshape((d + 1) * n, -1)
    return Sd @ Kuu @ Sd.T


def test_dski_matches_brute_force():
    op = _small_op(n=40, m=(8, 10))
    Kb = _brute_dski(op)
    np.testing.assert_allclose(op.dense_K(), Kb, rtol=1e-11, atol=1e-11 * np.abs(Kb).max())
    v = np.random.default_rng(1).standard_normal((op.N, 3))
    np.testing.assert_allclose(op.matvec(v), Kb @ v + op.Dn[:, None] * v,
                               rtol=1e-10, atol=1e-10 * np.abs(Kb @ v).max())


def test_dski_3d_matches_brute_force():
    r = np.random.default_rng(4)
    X = r.random((25, 3))
    op = dski.DSKI(X, (7, 6, 8), np.zeros(3), np.ones(3), np.log([0.4, 0.3, 0.5]), 0.2,
                   np.log(0.01), np.log(0.05))
    Kb = _brute_dski(op)
    np.testing.assert_allclose(op.dense_K(), Kb, atol=1e-11 * np.abs(Kb).max())


def test_dski_separable_entries():
    """An entry of the D-SKI matrix is the product over axes of 1-D SKI entries
    (Sec. 3.2): block (alpha, beta) uses the derivative weights on axis p
    exactly when alpha (resp. beta) is the derivative in direction p."""
    op = _small_op(n=30, m=(9, 12))
    K = op.dense_K()
    n, d = op.n, op.d
    per = [interp.axis_weights(op.X[:, p], op.grid.lo[p], op.grid.h[p], op.grid.m[p]) for p in range(d)]
    T = op.T
    r = np.random.default_rng(5)
    for _ in range(40):
        i, j = r.integers(0, n, 2)
        a, b = r.integers(0, d + 1, 2)
        val = op.s ** 2
        for p in range(d):
            idx, w, dw = per[p]
            wi = dw[i] if a == p + 1 else w[i]
            wj = dw[j] if b == p + 1 else w[j]
            val *= wi @ T[p][np.ix_(idx[i], idx[j])] @ wj
        assert K[a * n + i, b * n + j] == pytest.approx(val, rel=1e-11, abs=1e-12)


def test_dski_on_grid_points_value_block_is_exact_se():
    g = interp.Grid([0, 0], [1, 1], [12, 12])
    r = np.random.default_rng(6)
    ii = r.integers(1, 11, (30, 2))
    X = np.stack([g.nodes(0)[ii[:, 0]], g.nodes(1)[ii[:, 1]]], 1)
    X = np.clip(X, 0, 1)
    op = dski.DSKI(X, [12, 12], [0, 0], [1, 1], np.log([0.3, 0.3]), 0.0, -3, -3)
    K = op.dense_K()
    n = op.n
    Kse = kernels.se(op.X, op.X, op.ell, op.s)
    np.testing.assert_allclose(K[:n, :n], Kse, atol=1e-14)


def test_dski_symmetric_psd_adjoint():
    op = _small_op(n=80, m=(10, 10))
    K = op.dense()
    assert np.abs(K - K.T).max() < 1e-12 * np.abs(K).max()
    lam = np.linalg.eigvalsh(op.dense_K())
    assert lam.min() > -1e-10 * lam.max()
    r = np.random.default_rng(7)
    u, v = r.standard_normal(op.N), r.standard_normal(op.N)
    assert u @ op.matvec(v) == pytest.approx(v @ op.matvec(u), rel=1e-12)


def test_dski_converges_to_dse_with_expected_orders():
    """Refining the grid h -> h/2 shrinks the error against the exact D-SE
    kernel at the orders of cubic convolution: value block ~h^3 (Keys), blocks
    with derivatives ~h^2."""
    r = np.random.default_rng(8)
    X = 0.1 + 0.8 * r.random((60, 2))
    ell, s = 0.2, 1.0
    E = kernels.dse_dense(X, [ell, ell], s)
    n = 60
    errs = []
    for m in (15, 27, 51, 99):
        op = dski.DSKI(X, [m, m], [0, 0], [1, 1], np.log([ell, ell]), np.log(s), -3, -3)
        K = op.dense_K()
        ev = np.linalg.norm(K[:n, :n] - E[:n, :n]) / np.linalg.norm(E[:n, :n])
        eg = np.linalg.norm(K[n:, n:] - E[n:, n:]) / np.linalg.norm(E[n:, n:])
        errs.append((ev, eg))
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders[1:, 0] > 2.6)        # value block, third order
    assert np.all(orders[1:, 1] > 1.7)        # gradient block, second order
    assert errs[-1, 0] < 1e-5 and errs[-1, 1] < 1e-3


def test_diag_and_rows_match_dense():
    op = _small_op(n=50, m=(9, 9))
    K = op.dense_K()
    np.testing.assert_allclose(op.diag_K(), np.diag(K), rtol=1e-12)
    for i in (0, 17, op.N - 1):
        np.testing.assert_allclose(op.row_K(i), K[i], atol=1e-13 * np.abs(K).max())


def test_dtheta_matches_finite_differences():
    op = _small_op(n=30, m=(9, 10))
    v = np.random.default_rng(9).standard_normal(op.N)
    base = [op.log_ell.copy(), op.log_s, np.log(op.sigma_f), np.log(op.sigma_g)]
    h = 1e-5
    for which in range(op.d + 3):
        def mv(delta):
            le, ls, lf, lg = base[0].copy(), base[1], base[2], base[3]
            if which < op.d:
                le[which] += delta
            elif which == op.d:
                ls += delta
            elif which == op.d + 1:
                lf += delta
            else:
                lg += delta
            op.set_hypers(le, ls, lf, lg)
            return op.matvec(v)
        fd = (mv(h) - mv(-h)) / (2 * h)
        op.set_hypers(*base)
        np.testing.assert_allclose(op.matvec_dtheta(which, v), fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
