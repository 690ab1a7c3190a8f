"""Pins of the oracle's pivoted Cholesky, preconditioner, PCG, Lanczos, SLQ
and marginal-likelihood code against LAPACK, dense linear algebra, exactness
special cases, statistics and finite differences."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import workloads
from oracle import dski, krylov, mll, pivchol, precond, rng, slq


def _op(n=80, m=(10, 10), ell=0.3, s=1.0, sf=0.05, sg=0.1, seed=0):
    r = np.random.default_rng(seed)
    X = r.random((n, 2))
    return dski.DSKI(X, m, [0, 0], [1, 1], np.log([ell, ell]), np.log(s), np.log(sf), np.log(sg))


# ---------------------------------------------------------------- pivoted Cholesky
def test_pivchol_pivots_match_lapack_dpstrf():
    r = np.random.default_rng(1)
    B = r.standard_normal((12, 7))
    A = B @ B.T + np.diag(r.random(12))
    L, piv, _ = pivchol.pivoted_cholesky(np.diag(A), lambda i: A[i], 12)
    c, p, rank, info = lapack.dpstrf(A, lower=1, tol=-1.0)
    assert np.array_equal(piv, p[:len(piv)] - 1)
    np.testing.assert_allclose(L @ L.T, A, rtol=1e-12, atol=1e-12)


def test_pivchol_lowest_index_on_exact_ties():
    A = np.array([[2.0, 0.5, 0.1], [0.5, 2.0, 0.3], [0.1, 0.3, 2.0]])
    _, piv, _ = pivchol.pivoted_cholesky(np.diag(A), lambda i: A[i], 1)
    c, p, rank, info = lapack.dpstrf(A, lower=1)
    assert piv[0] == 0 == p[0] - 1


def test_pivchol_full_rank_and_monotone_trace():
    op = _op(n=20, m=(6, 6))            # rank(K) <= 36 < N = 60
    K = op.dense_K()
    L, piv, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 60, rel_tol=1e-13)
    np.testing.assert_allclose(L @ L.T, K, atol=1e-9 * np.abs(K).max())
    resid = np.trace(K) - np.cumsum(np.sum(L * L, axis=0))
    assert np.all(np.diff(resid) <= 1e-9)
    assert len(piv) <= 36


def test_pivchol_forced_pivots_and_gaps():
    op = _op(n=30, m=(8, 8))
    L, piv, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 10)
    assert np.all(gaps == 0)
    forced = list(piv[:5]) + [int(np.argsort(op.diag_K())[len(piv)])] + list(piv[6:])
    L2, piv2, gaps2 = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 10, forced=forced)
    assert list(piv2[:6]) == forced[:6]
    assert gaps2[5] >= 0


# ---------------------------------------------------------------- preconditioner
def test_precond_solve_and_logdet_match_dense():
    op = _op()
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 15)
    P = precond.Precond(L, op.Dn)
    Md = P.dense()
    b = np.random.default_rng(2).standard_normal((op.N, 3))
    ref = np.linalg.solve(Md, b)
    np.testing.assert_allclose(P.solve(b), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    np.testing.assert_allclose(P.solve_sqrt_form(b), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    assert P.logdet() == pytest.approx(np.linalg.slogdet(Md)[1], rel=1e-12)
    C = P.factor_apply(np.eye(op.N))
    np.testing.assert_allclose(C @ C.T, Md, atol=1e-10 * np.abs(Md).max())


def test_precond_equals_paper_formula_for_single_sigma():
    """With sigma_f = sigma_g = sigma, M^{-1} b = sigma^{-2}(b - Q_1 Q_1^T b) from
    the QR of [F; sigma I] (Sec. 3.3)."""
    op = _op(sf=0.07, sg=0.07)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 12)
    sig = 0.07
    Q, R = np.linalg.qr(np.vstack([L, sig * np.eye(L.shape[1])]))
    Q1 = Q[:op.N]
    b = np.random.default_rng(3).standard_normal(op.N)
    paper = (b - Q1 @ (Q1.T @ b)) / sig ** 2
    P = precond.Precond(L, op.Dn)
    np.testing.assert_allclose(P.solve(b), paper, rtol=1e-9, atol=1e-9 * np.abs(paper).max())


# ---------------------------------------------------------------- PCG
def test_pcg_matches_cholesky_solve():
    W = workloads.small2d()
    op = dski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, W.rank)
    P = precond.Precond(L, op.Dn)
    res = krylov.pcg(op.matvec, W.y, P.solve, tol=1e-8, max_iter=5000)
    A = op.dense()
    x = sla.cho_solve(sla.cho_factor(A), W.y)
    assert res["relres"][0] <= 1e-8
    assert krylov.true_relres(op.matvec, W.y, res["x"])[0] < 1e-7
    assert np.linalg.norm(res["x"][:, 0] - x) / np.linalg.norm(x) < 1e-4


def test_pcg_one_iteration_when_preconditioner_is_exact():
    """If rank(K) <= k the pivoted Cholesky is exact, M = K~ and PCG converges
    in one iteration."""
    op = _op(n=20, m=(6, 6))
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 60, rel_tol=1e-14)
    P = precond.Precond(L, op.Dn)
    b = np.random.default_rng(4).standard_normal((op.N, 2))
    res = krylov.pcg(op.matvec, b, P.solve, tol=1e-8)
    assert np.all(res["iters"] == 1)


def test_preconditioning_cuts_iterations():
    """Analog of the App. C study: CG vs pivoted-Cholesky PCG to 1e-4."""
    W = workloads.small2d(n=300, grid=30)
    op = dski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 50)
    P = precond.Precond(L, op.Dn)
    r_pcg = krylov.pcg(op.matvec, W.y, P.solve, tol=1e-4, max_iter=3000)
    r_cg = krylov.pcg(op.matvec, W.y, None, tol=1e-4, max_iter=3000)
    assert r_pcg["relres"][0] <= 1e-4
    assert r_pcg["iters"][0] * 5 < r_cg["iters"][0]


# ---------------------------------------------------------------- Lanczos / SLQ
def test_cg_tridiagonal_equals_explicit_lanczos():
    op = _op(n=60)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 10)
    P = precond.Precond(L, op.Dn)
    z = rng.rademacher(11, 0, 1, op.N)[:, 0]
    # (12 steps: before finite-precision CG loses orthogonality on this operator)
    res = krylov.pcg(op.matvec, z, P.solve, fixed_iters=12)
    dg, of = krylov.cg_tridiag(res["alpha"][0], res["beta"][0])
    ld, lo, nrm2 = krylov.lanczos(op.matvec, z, 12, P.solve, reorth=True)
    np.testing.assert_allclose(dg, ld, rtol=1e-9)
    np.testing.assert_allclose(of, lo, rtol=1e-9)
    assert nrm2 == pytest.approx(z @ P.solve(z), rel=1e-13)


def test_slq_exact_with_unit_probes_and_full_krylov():
    """Lanczos run to exhaustion makes Gauss quadrature exact, so with the unit
    probes e_1..e_N the estimate is tr log A = log det A."""
    r = np.random.default_rng(5)
    B = r.standard_normal((14, 14))
    A = B @ B.T + 0.5 * np.eye(14)
    tot = 0.0
    for i in range(14):
        e = np.zeros(14); e[i] = 1.0
        dg, of, nrm2 = krylov.lanczos(lambda v: A @ v, e, 14, reorth=True)
        tot += nrm2 * slq.quad_from_tridiag(dg, of)
    assert tot == pytest.approx(np.linalg.slogdet(A)[1], rel=1e-10)


def test_slq_statistical_and_preconditioned_exactness():
    op = _op(n=40, m=(8, 8))
    A = op.dense()
    exact = np.linalg.slogdet(A)[1]
    # plain Hutchinson + Lanczos with many probes: within 4 standard errors
    t = 400
    Z = rng.rademacher(21, 0, t, op.N)
    q = []
    for i in range(t):
        dg, of, nrm2 = krylov.lanczos(op.matvec, Z[:, i], 40)
        q.append(nrm2 * slq.quad_from_tridiag(dg, of))
    est, se = slq.estimate(q, np.ones(t))
    assert abs(est - exact) < 4 * se
    # preconditioned with an exact preconditioner: the estimate is exact
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, op.N, rel_tol=1e-14)
    P = precond.Precond(L, op.Dn)
    assert P.logdet() == pytest.approx(exact, rel=1e-8)


def test_stochastic_mll_matches_exact_within_error():
    W = workloads.small2d(n=200, grid=30)
    op = dski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    ex = mll.exact(op, W.y)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 40)
    st = mll.stochastic(op, W.y, L, 16, 0x181012283, 1e-8)
    assert abs(st["logdet"] - ex["logdet"]) < 4 * st["logdet_stderr"] + 1e-6 * abs(ex["logdet"])
    # the data-fit term is deterministic
    assert W.y @ st["pcg"]["x"][:, 0] == pytest.approx(W.y @ ex["alpha"], rel=1e-6)


def test_exact_gradient_matches_finite_differences():
    """Central differences (h = 1e-3 in log-theta) of the dense D-SKI mll."""
    W = workloads.small2d(n=120, grid=20)
    op = dski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    base = list(W.hypers())
    g = mll.exact(op, W.y)["grad"]
    h = 1e-3
    for j in range(op.d + 3):
        vals = []
        for sgn in (1, -1):
            le, ls, lf, lg = base[0].copy(), base[1], base[2], base[3]
            if j < op.d:
                le[j] += sgn * h
            elif j == op.d:
                ls += sgn * h
            elif j == op.d + 1:
                lf += sgn * h
            else:
                lg += sgn * h
            op.set_hypers(le, ls, lf, lg)
            vals.append(mll.exact(op, W.y)["mll"])
        op.set_hypers(*base)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g).max())


def test_stochastic_gradient_unbiased_for_trace_term():
    """E[(K~^{-1} z)^T K' (M^{-1} z)] = tr(K~^{-1} K') for z ~ Cov M."""
    op = _op(n=40, m=(8, 8))
    A = op.dense()
    Ainv = np.linalg.inv(A)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, 10)
    P = precond.Precond(L, op.Dn)
    for j in (0, op.d, op.d + 2):
        dK = op.matvec_dtheta(j, np.eye(op.N))
        ex = np.sum(Ainv * dK.T)
        Wr = rng.rademacher(31, 0, 3000, op.N)
        Z = P.factor_apply(Wr)
        vals = np.sum((Ainv @ Z) * (dK @ P.solve(Z)), axis=0)
        assert abs(vals.mean() - ex) < 4 * vals.std() / math.sqrt(vals.size)


def test_fixed_step_slq_is_well_conditioned_and_exact_with_exact_preconditioner():
    """The fixed-step estimate with full re-orthogonalisation: (i) symmetric
    perturbations of K~ and M^{-1} at 1e-13 of their largest entries move it by
    less than 1e-8 relative, where the same 30 steps from CG's coefficients (no
    re-orthogonalisation) move by ~1e-4..1e-3; (ii) with an exact preconditioner
    (full-rank pivoted Cholesky) it is log det M = log det K~."""
    W = workloads.small2d()
    op = dski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, W.rank)
    P = precond.Precond(L, op.Dn)
    Wr = rng.rademacher(0x181012283, 0, 4, op.N)
    base, _ = slq.fixed_step_logdet(op.matvec, P, Wr, 30)
    Minv = P.solve(np.eye(op.N))
    K = op.dense()
    r = np.random.default_rng(3)
    E = r.standard_normal((op.N, op.N))
    E = (E + E.T) * (1e-13 * np.abs(Minv).max())
    F = r.standard_normal((op.N, op.N))
    F = (F + F.T) * (1e-13 * np.abs(K).max())
    Pp = type("Pp", (), {"solve": staticmethod(lambda B: P.solve(B) + E @ B),
                         "factor_apply": staticmethod(P.factor_apply), "logdet": staticmethod(P.logdet)})
    pert, _ = slq.fixed_step_logdet(lambda B: op.matvec(B) + F @ B, Pp, Wr, 30)
    assert abs(pert - base) < 1e-8 * abs(base)
    # (ii) exact preconditioner
    op2 = _op(n=30, m=(7, 7))
    L2, _, _ = pivchol.pivoted_cholesky(op2.diag_K(), op2.row_K, op2.N, rel_tol=1e-15)
    P2 = precond.Precond(L2, op2.Dn)
    est, _ = slq.fixed_step_logdet(op2.matvec, P2, rng.rademacher(5, 0, 3, op2.N), 5)
    assert est == pytest.approx(np.linalg.slogdet(op2.dense())[1], rel=1e-9)
