"""Pins of the oracle's spline kernel under D-SKI (App. A; Sec. 4.3) by what
fixes it from outside its own code: the paper's form s^2 (r^3 + a r^2 + b) /
s^2 (r^2 log r + a r^2 + b) recovered from kernel values, symmetry and
positive definiteness of K_UU on grids (the property a and b are chosen for),
the multi-level Toeplitz product by d-dimensional circulant embedding and FFT
(numpy) equal to the dense one, brute-force D-SKI entries, adjointness, and
convergence of the value block to the exact spline kernel matrix as the grid
is refined."""
import numpy as np
import pytest

from oracle import interp, spline


def _op(d, m, n=40, seed=0, box=None):
    r = np.random.default_rng(seed)
    hi = np.ones(d) if box is None else np.asarray(box, dtype=np.float64)
    X = r.random((n, d)) * hi
    return spline.SplineDSKI(X, [m] * d, np.zeros(d), hi, np.log(0.7), np.log(0.05), np.log(0.1))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_spline_profile_has_the_paper_form(d):
    """k(r)/s^2 - r^3 (d odd) or - r^2 log r (d even) is a quadratic a r^2 + b
    in r, with the b of the reading (R^3/2 or R^2/2)."""
    R = 2.7
    r = np.linspace(0.1, 2.0, 9)
    base = r ** 3 if d % 2 == 1 else r * r * np.log(r)
    rest = spline.spline_k(r, d, R) - base
    coef = np.polyfit(r, rest, 2)
    np.testing.assert_allclose(coef[1], 0.0, atol=1e-10)
    assert coef[2] == pytest.approx(R ** 3 / 2 if d % 2 == 1 else R * R / 2, rel=1e-12)
    assert spline.spline_k(0.0, d, R) == pytest.approx(coef[2], rel=1e-12)


@pytest.mark.parametrize("d,m", [(1, 40), (2, 14), (3, 8)])
def test_spline_kuu_symmetric_positive_definite(d, m):
    for box in (None, [0.3, 1.7, 0.9][:d]):
        op = _op(d, m, box=box)
        K = op.Kspl
        assert np.array_equal(K, K.T)
        ev = np.linalg.eigvalsh(K)
        assert ev.min() > 1e-12 * ev.max()


@pytest.mark.parametrize("d,m", [(2, 9), (3, 6)])
def test_spline_kuu_by_circulant_embedding_fft(d, m):
    """K_UU is symmetric multi-level Toeplitz: embedding its first column in a
    d-dimensional circulant of 2m per axis and multiplying through numpy's FFT
    gives the dense product."""
    op = _op(d, m)
    G = np.random.default_rng(1).standard_normal((op.grid.size, 3))
    ref = op.Kspl @ G
    L = [2 * mm for mm in op.grid.m]
    idx = np.meshgrid(*[np.arange(Lp) for Lp in L], indexing="ij")
    dist2 = np.zeros(L)
    for p in range(d):
        j = np.minimum(idx[p], L[p] - idx[p])
        dist2 = dist2 + (j * op.grid.h[p]) ** 2
    c = spline.spline_k(np.sqrt(dist2), d, op.R)
    for p in range(d):  # the index m_p itself is outside the Toeplitz band
        sl = [slice(None)] * d
        sl[p] = op.grid.m[p]
        c[tuple(sl)] = 0.0
    lam = np.fft.fftn(c).real
    out = np.empty_like(G)
    for k in range(G.shape[1]):
        pad = np.zeros(L)
        pad[tuple(slice(0, mm) for mm in op.grid.m)] = G[:, k].reshape(op.grid.m)
        y = np.fft.ifftn(lam * np.fft.fftn(pad)).real
        out[:, k] = y[tuple(slice(0, mm) for mm in op.grid.m)].ravel()
    np.testing.assert_allclose(out, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_spline_dski_brute_force_and_adjoint():
    op = _op(2, 9, n=25)
    Sd = op.S.toarray()
    Kb = Sd @ (op.s ** 2 * op.Kspl) @ Sd.T + np.diag(op.Dn)
    V = np.random.default_rng(2).standard_normal((op.N, 2))
    np.testing.assert_allclose(op.matvec(V), Kb @ V, rtol=1e-12, atol=1e-12 * np.abs(Kb @ V).max())
    u, v = V[:, 0], V[:, 1]
    assert u @ op.matvec(v) == pytest.approx(v @ op.matvec(u), rel=1e-12)
    np.testing.assert_allclose(op.diag_K(), np.diag(Kb) - op.Dn, rtol=1e-12)
    np.testing.assert_allclose(op.row_K(7), Kb[7] - np.eye(op.N)[7] * op.Dn[7], rtol=1e-12, atol=1e-12)


def test_spline_dski_value_block_converges_to_exact_kernel():
    """Sec. 4: SKI with the spline kernel approximates the kernel matrix as well
    as with the SE kernel; the value block's error falls under grid refinement."""
    r = np.random.default_rng(4)
    X = 0.1 + 0.8 * r.random((40, 3))
    errs = []
    for m in (8, 12, 18):
        op = spline.SplineDSKI(X, [m] * 3, [0, 0, 0], [1, 1, 1], 0.0, -3.0, -3.0)
        D = np.linalg.norm(X[:, None] - X[None], axis=-1)
        E = spline.spline_k(D, 3, op.R)
        K = op.dense_K()[:40, :40]
        errs.append(np.linalg.norm(K - E) / np.linalg.norm(E))
    errs = np.array(errs)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3
