"""Pins of the oracle's D-SKIP operator (Sec. 3.2): untruncated D-SKIP equals
D-SKI on the tensor grid, the SKIP reduction equals the dense Hadamard
product, and the result is positive semi-definite (Schur product theorem)."""
import numpy as np
import pytest

from oracle import dski, dskip, rng


def _setup(n, d, m, seed=0):
    r = np.random.default_rng(seed)
    X = r.uniform(-1, 1, (n, d))
    lo, hi = -np.ones(d), np.ones(d)
    le = np.log(np.linspace(0.4, 0.7, d))
    return X, lo, hi, le


def test_axis_factor_block_structure():
    """Khat_p[(a,i),(b,j)] uses derivative weights exactly on the sides whose
    observation is the derivative along p (eq. (skip) for d = 2)."""
    X, lo, hi, le = _setup(6, 3, 8)
    p = 1
    F = dskip.AxisFactor(X[:, p], p, 3, 8, lo[p], hi[p], le[p])
    K = F.dense()
    G = F.op.dense_K()          # 2n x 2n: [W; dW] T [W; dW]^T of coordinate p
    n = 6
    for a in range(4):
        for b in range(4):
            ra = slice(n, 2 * n) if a == p + 1 else slice(0, n)
            rb = slice(n, 2 * n) if b == p + 1 else slice(0, n)
            np.testing.assert_allclose(K[a * n:(a + 1) * n, b * n:(b + 1) * n], G[ra, rb], atol=1e-14)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_untruncated_dskip_equals_tensor_grid_dski(d):
    n, m = 5, 6
    X, lo, hi, le = _setup(n, d, m, seed=d)
    N = n * (d + 1)
    op = dskip.DSKIP(X, m, lo, hi, le, 0.3, np.log(0.05), np.log(0.1), r=N, seed=7)
    K = op.matvec_K(np.eye(N))
    ref = dski.DSKI(X, [m] * d, lo, hi, le, 0.3, np.log(0.05), np.log(0.1)).dense_K()
    assert np.linalg.norm(K - ref) / np.linalg.norm(ref) < 1e-9
    np.testing.assert_allclose(op.diag_K(), np.diag(ref), rtol=1e-8, atol=1e-10 * np.abs(ref).max())
    np.testing.assert_allclose(op.row_K(3), ref[3], atol=1e-9 * np.abs(ref).max())


def test_skip_reduction_equals_dense_hadamard():
    r = np.random.default_rng(1)
    N, k = 40, 6
    Qa, _ = np.linalg.qr(r.standard_normal((N, k)))
    Qb, _ = np.linalg.qr(r.standard_normal((N, k)))
    Ta = np.diag(r.random(k)) + np.diag(r.random(k - 1), 1)
    Ta = Ta + Ta.T
    Tb = np.diag(r.random(k)) + np.diag(r.random(k - 1), 1)
    Tb = Tb + Tb.T
    V = r.standard_normal((N, 3))
    dense = (Qa @ Ta @ Qa.T) * (Qb @ Tb @ Qb.T)
    np.testing.assert_allclose(dskip.hadamard_matvec(Qa, Ta, Qb, Tb, V), dense @ V, atol=1e-12)


def test_truncated_dskip_is_psd_and_accurate():
    n, d, m = 60, 2, 20
    X, lo, hi, le = _setup(n, d, m, seed=3)
    N = n * (d + 1)
    ref = dski.DSKI(X, [m] * d, lo, hi, le, 0.0, np.log(0.05), np.log(0.1)).dense_K()
    errs = []
    for r in (8, 16, 32):
        op = dskip.DSKIP(X, m, lo, hi, le, 0.0, np.log(0.05), np.log(0.1), r=r, seed=11)
        K = op.matvec_K(np.eye(N))
        lam = np.linalg.eigvalsh(0.5 * (K + K.T))
        assert lam.min() > -1e-10 * lam.max()
        errs.append(np.linalg.norm(K - ref) / np.linalg.norm(ref))
    assert errs[2] < errs[0] and errs[2] < 1e-2


def test_lanczos_start_vector_is_the_rademacher_stream():
    F = lambda v: 2.0 * v
    Q, T = dskip.lanczos_full(F, 10, 1, seed=5, node=3)
    z = rng.rademacher(5, 3, 1, 10)[:, 0]
    np.testing.assert_allclose(Q[:, 0], z / np.linalg.norm(z), atol=1e-15)
    assert T[0, 0] == pytest.approx(2.0)
