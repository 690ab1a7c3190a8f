"""Host-side checks of the C-ABI library (no GPU needed): it loads, it
exports every function include/dski.h declares, and its host numerics agree
with the oracle."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dski.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"if", "sizeof"})


def _lib():
    from paper_1810_12283_amd import dski
    if not os.path.exists(dski.LIB_PATH):
        pytest.skip("libdski.so not built (run python -m paper_1810_12283_amd.build)")
    return dski


def test_library_exports_every_declared_symbol():
    dski = _lib()
    L = dski.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(dski.EXPORTS)


def test_version_and_last_error_are_strings():
    dski = _lib()
    assert dski.version().startswith("dski-gfx950")
    assert isinstance(dski.last_error(), str)


def test_lanczos_quadrature_matches_oracle():
    """The host Golub-Welsch quadrature against the oracle's LAPACK path on CG
    coefficients of a real preconditioned solve."""
    dski = _lib()
    from oracle import dski as odski, krylov, pivchol, precond, rng, slq
    r = np.random.default_rng(0)
    X = r.random((60, 2))
    op = odski.DSKI(X, (10, 10), [0, 0], [1, 1], np.log([0.3, 0.3]), 0.0, np.log(0.05), np.log(0.1))
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 10)
    P = precond.Precond(L, op.Dn)
    z = rng.rademacher(3, 0, 1, op.N)[:, 0]
    res = krylov.pcg(op.matvec, z, P.solve, fixed_iters=40)
    a, b = res["alpha"][0], res["beta"][0]
    want = slq.quad_from_tridiag(*krylov.cg_tridiag(a, b))
    got = dski.lanczos_quad_log(a, b[:-1])
    assert got == pytest.approx(want, rel=1e-10, abs=1e-12)
    # a 1x1 tridiagonal is log(1/alpha)
    assert dski.lanczos_quad_log([0.25], []) == pytest.approx(np.log(4.0), rel=1e-15)


@pytest.mark.parametrize("J,seed", [(2, 1), (7, 2), (300, 3), (3000, 4)])
def test_lanczos_quadrature_random_cg_coefficients(J, seed):
    """The host quadrature against LAPACK (the oracle's tridiagonal
    eigen-solver) on CG coefficients of a random SPD spectrum: Lanczos
    tridiagonals up to the lengths of a terrain solve, a spread of four
    decades and a tight cluster of ten eigenvalues."""
    dski = _lib()
    from oracle import krylov, slq
    r = np.random.default_rng(seed)
    lam = np.concatenate([np.geomspace(1e-2, 1e2, 3990), 2.0 + 1e-9 * np.arange(10)])
    lam = lam[r.permutation(lam.size)]
    z = r.choice([-1.0, 1.0], lam.size)
    res = krylov.pcg(lambda V: lam[:, None] * V, z, fixed_iters=J)
    a, b = res["alpha"][0], res["beta"][0]
    want = slq.quad_from_tridiag(*krylov.cg_tridiag(a, b))
    got = dski.lanczos_quad_log(a, b[:-1])
    assert got == pytest.approx(want, rel=1e-10, abs=1e-12)



def test_lanczos_quadrature_against_high_precision():
    """The integral-form quadrature (tridiagonals longer than 64) against a
    30-digit eigen-decomposition (mpmath) of an 80-step CG tridiagonal of a
    spectrum over ten decades, and both forms against each other at the
    switch-over length."""
    mp = pytest.importorskip("mpmath")
    dski = _lib()
    from oracle import krylov
    r = np.random.default_rng(0)
    lam = np.geomspace(1e-6, 1e4, 3000)
    z = r.choice([-1.0, 1.0], lam.size)
    res = krylov.pcg(lambda V: lam[:, None] * V, z, fixed_iters=80)
    a, b = res["alpha"][0], res["beta"][0]
    J = len(a)
    diag = [1.0 / a[j] + (b[j - 1] / a[j - 1] if j > 0 else 0.0) for j in range(J)]
    off = [np.sqrt(b[j]) / a[j] for j in range(J - 1)]
    mp.mp.dps = 30
    T = mp.matrix(J, J)
    for i in range(J):
        T[i, i] = mp.mpf(diag[i])
        if i + 1 < J:
            T[i, i + 1] = T[i + 1, i] = mp.mpf(off[i])
    E, Q = mp.eighe(T)
    want = float(sum(Q[0, k] ** 2 * mp.log(E[k]) for k in range(J)))
    got = dski.lanczos_quad_log(a, b[:-1])
    assert got == pytest.approx(want, rel=1e-13)
    # the QR form at J = 64 and the integral form at J = 65 describe the same rule
    # family: each against LAPACK on its own leading block
    from oracle import slq
    for Jc in (64, 65):
        w = slq.quad_from_tridiag(*krylov.cg_tridiag(a[:Jc], b[:Jc]))
        assert dski.lanczos_quad_log(a[:Jc], b[:Jc - 1]) == pytest.approx(w, rel=1e-10)
