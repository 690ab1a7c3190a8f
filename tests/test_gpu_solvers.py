"""GPU parity of pivoted Cholesky, preconditioner, PCG, SLQ and the marginal
likelihood with its gradient against the FP64 oracle (same probes, same
pivots).  Bars: pivot order equal except at near-ties (the GPU pick is within
tau = 1e-4 x max initial diagonal of the oracle's best); factor 1e-4; log det
M 1e-5; solves 1e-4 true relative residual (oracle's FP64 operator); log det
1e-3; mll gradient 1e-3 relative to its norm."""
import math

import numpy as np
import scipy.linalg as sla
import pytest
import torch

import workloads
from oracle import dski as odski, krylov, mll as omll, pivchol, precond, rng as orng, slq
from tests.gpu_common import SEED, from_gpu, make, need_gpu, rel_cols, say, to_gpu

pytestmark = pytest.mark.gpu

TAU = 1e-4


def _pivchol_pair(W, k):
    plan, op = make(W)
    pc = plan.pivchol(k)
    piv = pc.pivots
    dg = op.diag_K()
    L, opiv, gaps = pivchol.pivoted_cholesky(dg, op.row_K, len(piv), forced=piv)
    return plan, op, pc, L, gaps


@pytest.mark.parametrize("name,k", [("small2d", 20), ("terrain_small", 50), ("torus_small", 30)])
def test_pivchol_matches_oracle(name, k):
    W = {"small2d": workloads.small2d(), "terrain_small": workloads.terrain(n=3000, grid=60),
         "torus_small": workloads.torus(n=700, grid=14)}[name]
    say("pivchol", name, k)
    plan, op, pc, L, gaps = _pivchol_pair(W, k)
    assert pc.rank == k
    say("  max gap", gaps.max())
    assert gaps.max() <= TAU
    Lg = pc.factor().cpu().numpy().T
    err = np.linalg.norm(Lg - L) / np.linalg.norm(L)
    say("  factor rel err", err)
    assert err < 1e-4
    P = precond.Precond(L, op.Dn)
    assert pc.logdet() == pytest.approx(P.logdet(), rel=1e-5)
    # preconditioner application
    B = np.random.default_rng(1).standard_normal((op.N, 3)).astype(np.float32).astype(np.float64)
    Z = from_gpu(pc.apply(to_gpu(B)))
    e2 = rel_cols(Z, P.solve(B)).max()
    say("  apply rel err", e2)
    assert e2 < 1e-4


def test_pivchol_exact_low_rank_and_truncation():
    """rank(K) <= grid size: asking for more columns stops early (rank
    truncated) and then M = K~, so PCG converges in one step."""
    dski = need_gpu()
    say("pivchol low rank")
    r = np.random.default_rng(3)
    X = r.random((20, 2))
    plan = dski.Plan(torch.tensor(X, device="cuda"), [6, 6], [0, 0], [1, 1])
    plan.set_hypers(np.log([0.3, 0.3]), 0.0, np.log(0.05), np.log(0.1))
    pc = plan.pivchol(60)
    assert pc.status == dski.RANK_TRUNCATED
    assert pc.rank <= 36
    B = to_gpu(r.standard_normal((60, 2)))
    X_, iters, relres, st, _ = plan.pcg(B, pc, tol=1e-3, max_iter=50)
    say("  iters", iters, relres)
    assert max(iters) <= 2


@pytest.mark.parametrize("name,bits,variant", [("small2d", 32, 1), ("terrain_small", 32, 4), ("small2d", 64, 3),
                                              ("terrain_small", 32, 0), ("small2d", 32, 5),
                                              ("terrain_small", 32, 2), ("small2d", 64, 4)])
def test_pcg_true_residual(name, bits, variant):
    W = {"small2d": workloads.small2d(), "terrain_small": workloads.terrain(n=3000, grid=60)}[name]
    say("pcg", name, bits, "scatter variant", variant)
    plan, op = make(W)
    plan.set_variants(variant, variant % 3)  # every scatter and gather form
    pc = plan.pivchol(W.rank)
    Wr = orng.rademacher(SEED, 0, 2, op.N)
    B = np.concatenate([W.y[:, None], Wr], axis=1).astype(np.float32).astype(np.float64)
    Bg = to_gpu(B) if bits == 32 else to_gpu(B).double()
    X, iters, relres, st, _ = plan.pcg(Bg, pc, tol=1e-4, max_iter=20000)
    say("  iters", iters, "relres", relres, "status", st)
    assert st == 0
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  true relres (oracle FP64 operator)", tr)
    assert tr.max() <= 1e-4
    # unpreconditioned CG on the same system needs more iterations
    X2, it2, rr2, st2, _ = plan.pcg(to_gpu(B[:, :1]), None, tol=1e-4, max_iter=max(iters) * 10)
    say("  CG iters", it2, rr2)
    assert it2[0] > 1.5 * iters[0]


def test_pcg_not_converged_status():
    W = workloads.small2d()
    say("pcg max_iter")
    plan, op = make(W)
    X, iters, relres, st, _ = plan.pcg(to_gpu(W.y), None, tol=1e-8, max_iter=5)
    assert st == 1 and iters == [5] and relres[0] > 1e-8


def _oracle_slq_pcg(op, P, Z, steps=None, tol=None):
    """SLQ from the FP64 oracle's own PCG coefficients (the CG->Lanczos reading)."""
    q, w = [], []
    for i in range(Z.shape[1]):
        if steps:
            res = krylov.pcg(op.matvec, Z[:, i], P.solve, fixed_iters=steps)
        else:
            res = krylov.pcg(op.matvec, Z[:, i], P.solve, tol=tol, max_iter=20000)
        q.append(slq.quad_from_tridiag(*krylov.cg_tridiag(res["alpha"][0], res["beta"][0])))
        w.append(Z[:, i] @ P.solve(Z[:, i]))
    return slq.estimate(q, w, P.logdet())


def test_slq_fixed_steps_matches_oracle():
    """small2d (the FP64 configuration): 10 probes x 30 Lanczos steps, the
    explicit preconditioned Lanczos process with full re-orthogonalisation on
    both sides, same probes and pivots as the oracle: log det within 1e-3
    relative (the log-determinant bar; without re-orthogonalisation a 30-step run
    is ill-conditioned and this bar could not be held).  Also checked with
    FP32 plan storage (the fixed-step path keeps FP64 vectors) and against the
    exact log det within the truncation bias of 30 steps (7 % here)."""
    W = workloads.small2d()
    say("slq small2d, 30 re-orthogonalised Lanczos steps")
    plan, op, pc, L, gaps = _pivchol_pair(W, W.rank)
    P = precond.Precond(L, op.Dn)
    Wr = orng.rademacher(SEED, 0, W.num_probes, op.N)
    ld_or, se_or = slq.fixed_step_logdet(op.matvec, P, Wr, W.lanczos_steps)
    exact = np.linalg.slogdet(op.dense())[1]
    for bits in (64, 32):
        plan.set_precision(bits)
        ld_gpu, se_gpu = plan.slq_logdet(pc, W.num_probes, W.lanczos_steps, seed=SEED)
        rel = abs(ld_gpu - ld_or) / abs(ld_or)
        say("  bits", bits, "gpu", ld_gpu, se_gpu, "oracle", ld_or, se_or, "rel", rel, "exact", exact)
        assert rel <= 1e-3
        assert abs(se_gpu - se_or) <= 1e-3 * se_or
    assert abs(ld_gpu - exact) < 0.1 * abs(exact)
    # a probe block whose Krylov space is exhausted early (6 x 6 grid, rank 36:
    # the preconditioner is exact) ends after one step: log det M
    dski = need_gpu()
    r = np.random.default_rng(3)
    X = r.random((20, 2))
    plan2 = dski.Plan(torch.tensor(X, device="cuda"), [6, 6], [0, 0], [1, 1])
    plan2.set_hypers(np.log([0.3, 0.3]), 0.0, np.log(0.05), np.log(0.1))
    pc2 = plan2.pivchol(60)
    ld2, _ = plan2.slq_logdet(pc2, 3, 10, seed=SEED)
    assert ld2 == pytest.approx(pc2.logdet(), rel=1e-10)


@pytest.mark.parametrize("bits", [32, 64])
def test_slq_converged_matches_oracle_and_exact(bits):
    W = workloads.small2d()
    say("slq small2d converged", bits)
    plan, op, pc, L, gaps = _pivchol_pair(W, W.rank)
    plan.set_precision(bits)
    ld_gpu, se_gpu = plan.slq_logdet(pc, W.num_probes, 0, tol=1e-6, max_iter=5000, seed=SEED)
    P = precond.Precond(L, op.Dn)
    Z = P.factor_apply(orng.rademacher(SEED, 0, W.num_probes, op.N))
    ld_or, se_or = _oracle_slq_pcg(op, P, Z, tol=1e-6)
    exact = np.linalg.slogdet(op.dense())[1]
    say("  gpu", ld_gpu, se_gpu, "oracle", ld_or, se_or, "exact", exact)
    assert ld_gpu == pytest.approx(ld_or, rel=1e-3)
    assert abs(ld_gpu - exact) < 4 * se_gpu + 1e-3 * abs(exact)


@pytest.mark.parametrize("bits", [32, 64])
def test_mll_and_grad_matches_oracle_small(bits):
    W = workloads.small2d(n=400, grid=40)
    say("mll small2d", bits)
    plan, op, pc, L, gaps = _pivchol_pair(W, 30)
    t = 16
    yg = to_gpu(W.y.astype(np.float32))
    if bits == 64:
        yg = yg.double()
    res = plan.mll_and_grad(yg, pc, num_probes=t, seed=SEED, tol=1e-6, max_iter=5000)
    ref = omll.stochastic(op, W.y.astype(np.float32).astype(np.float64), L, t, SEED, 1e-6)
    say("  gpu", res["mll"], res["logdet"], res["grad"])
    say("  orc", ref["mll"], ref["logdet"], ref["grad"])
    assert res["logdet"] == pytest.approx(ref["logdet"], rel=1e-3)
    assert res["mll"] == pytest.approx(ref["mll"], rel=1e-3, abs=1e-3 * abs(ref["logdet"]))
    g, gr = res["grad"], ref["grad"]
    assert np.linalg.norm(g - gr) / np.linalg.norm(gr) < 1e-3
    # and against the dense exact gradient within the stochastic error
    ex = omll.exact(op, W.y.astype(np.float32).astype(np.float64))
    say("  exact", ex["mll"], ex["grad"])
    assert abs(res["logdet"] - ex["logdet"]) < 5e-2 * abs(ex["logdet"])


def test_mll_warm_start_matches_cold():
    """mll_and_grad_warm: a zero start reproduces the cold call; a start from
    the alpha of nearby hyper-parameters meets the same oracle true residual
    with fewer data-column iterations, and the probe columns (which always
    start at zero) give the same log det."""
    W = workloads.terrain(n=3000, grid=60)
    say("mll warm start terrain", W.n, W.grid_m)
    plan, op = make(W)
    y = to_gpu(W.y.astype(np.float32)).contiguous()
    k, t, tol = 30, 4, 1e-5
    cold0 = plan.mll_and_grad(y, None, k=k, num_probes=t, seed=SEED, tol=tol)
    z = plan.mll_and_grad(y, None, k=k, num_probes=t, seed=SEED, tol=tol, want_alpha=True)
    assert z["mll"] == pytest.approx(cold0["mll"], rel=1e-12)
    assert z["iters"] == cold0["iters"]
    le, ls, lf, lg = W.hypers()
    step = np.array([0.02, -0.02])
    h1 = (le + step, ls + 0.02, lf - 0.02, lg + 0.02)
    plan.set_hypers(*h1)
    op.set_hypers(*h1)
    cold = plan.mll_and_grad(y, None, k=k, num_probes=t, seed=SEED, tol=tol)
    warm = plan.mll_and_grad(y, None, k=k, num_probes=t, seed=SEED, tol=tol, x0=z["alpha"], want_alpha=True)
    say("  data-column iterations: cold", cold["iters"][0], "warm", warm["iters"][0])
    say("  mll cold", cold["mll"], "warm", warm["mll"], " log det", cold["logdet"], warm["logdet"])
    y64 = W.y.astype(np.float32).astype(np.float64)
    a = warm["alpha"].cpu().numpy()
    rel = np.linalg.norm(y64 - op.matvec(a[:, None])[:, 0]) / np.linalg.norm(y64)
    say("  oracle true residual of the warm alpha", rel)
    assert rel <= 1.05 * tol
    assert warm["iters"][0] < cold["iters"][0]
    assert warm["iters"][1:] == cold["iters"][1:]
    assert warm["logdet"] == pytest.approx(cold["logdet"], rel=1e-9)
    assert warm["mll"] == pytest.approx(cold["mll"], rel=1e-4, abs=1e-6 * abs(cold["logdet"]))
    g, gc = warm["grad"], cold["grad"]
    assert np.linalg.norm(g - gc) / np.linalg.norm(gc) < 1e-3
    with pytest.raises(TypeError):
        plan.mll_and_grad(y.double(), None, k=k, num_probes=0, tol=tol, want_alpha=True)
    plan.close()


def test_autograd_mll_on_the_implicit_surface():
    """torch.autograd through MarginalLikelihood returns the adjoint gradient of
    mll_and_grad (bitwise); on a small torus (d = 3) that gradient matches the
    oracle's stochastic gradient with the same 64 probes to 1e-3, and the
    central differences (h = 1e-3 in log-theta) of the oracle's dense exact mll
    within 4 standard errors of the probe average (plus 1e-3 relative)."""
    dski = need_gpu()
    W = workloads.torus(n=500, grid=14)
    say("autograd mll torus", W.n)
    plan, op = make(W)
    y = to_gpu(W.y.astype(np.float32))
    le, ls, lf, lg = W.hypers()
    t, k = 64, 60
    theta = torch.tensor(np.concatenate([le, [ls, lf, lg]]), dtype=torch.float64, requires_grad=True)
    mll = dski.MarginalLikelihood.apply(theta, plan, y, k, t, SEED, 1e-6, 5000)  # 65 columns: 3 PCG groups
    (g,) = torch.autograd.grad(mll, theta)
    direct = plan.mll_and_grad(y, None, k=k, num_probes=t, seed=SEED, tol=1e-6, max_iter=5000)
    assert mll.item() == direct["mll"]
    np.testing.assert_array_equal(g.numpy(), direct["grad"])
    yd = W.y.astype(np.float32).astype(np.float64)
    # the same estimator (same pivots, preconditioner and probes) with the
    # solves done by a dense Cholesky factorisation
    pc = plan.pivchol(k)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    P = precond.Precond(L, op.Dn)
    Z = P.factor_apply(orng.rademacher(SEED, 0, t, op.N))
    cf = sla.cho_factor(op.dense(), lower=True)
    al, U, V = sla.cho_solve(cf, yd), sla.cho_solve(cf, Z), P.solve(Z)
    ref = np.empty(W.d + 3)
    se = np.empty(W.d + 3)
    for j in range(W.d + 3):
        samples = np.sum(U * op.matvec_dtheta(j, V), axis=0)
        ref[j] = 0.5 * al @ op.matvec_dtheta(j, al) - 0.5 * samples.mean()
        se[j] = 0.5 * samples.std(ddof=1) / np.sqrt(t)
    e_same = np.linalg.norm(g.numpy() - ref) / np.linalg.norm(ref)
    h = 1e-3
    fd = np.empty(W.d + 3)
    th0 = theta.detach().numpy()
    for j in range(W.d + 3):
        vals = []
        for sgn in (1, -1):
            th = th0.copy()
            th[j] += sgn * h
            o = odski.DSKI(W.X, W.grid_m, W.lo, W.hi, th[:W.d], th[W.d], th[W.d + 1], th[W.d + 2])
            vals.append(omll.exact(o, yd)["mll"])
        fd[j] = (vals[0] - vals[1]) / (2 * h)
    say("  gpu", g.numpy(), "\n  orc", ref, "\n  fd ", fd, "\n  se ", se, "same-probe rel", e_same)
    assert e_same < 1e-3
    assert np.all(np.abs(g.numpy() - fd) <= 4 * se + 1e-3 * np.abs(fd))


@pytest.mark.parametrize("name", ["terrain_small", "ridge_dskip"])
def test_pcg_graph_replay_equals_eager(name):
    """Bursts of PCG iterations replayed from a captured HIP graph (many
    replays per solve, with host synchronisations between bursts) give the same
    bits as launching every kernel directly: iterate, iteration counts and
    residuals."""
    dski = need_gpu()
    say("pcg graph vs eager", name)
    if name == "terrain_small":
        W = workloads.terrain(n=3000, grid=60)
        plan, op = make(W)
        k = W.rank
    else:
        from tests.test_gpu_dskip import SMALL, make_skip
        W = workloads.ridge8d(**SMALL["d8"])
        plan, op = make_skip(W)
        k = 60
    pc = plan.pivchol(k)
    B = to_gpu(np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, 4, op.N)], axis=1))
    out = {}
    for on in (False, True):
        plan.set_graph(on)
        X, iters, relres, st, _ = plan.pcg(B, pc, tol=1e-5, max_iter=20000)
        out[on] = (X.cpu().numpy(), iters, relres, st)
    say("  iters", out[True][1], "status", out[True][3])
    assert max(out[True][1]) > 40  # several graph bursts
    assert out[True][1] == out[False][1] and out[True][3] == out[False][3]
    np.testing.assert_array_equal(out[True][2], out[False][2])
    np.testing.assert_array_equal(out[True][0], out[False][0])


@pytest.mark.parametrize("k", [1, 17, 65, 100])
def test_precond_apply_column_widths_and_ranks(k):
    """The tall-skinny products at ranks around the 16- and 64-column blocks of
    the matrix-core kernels and at every padded width (R = 1 .. 40, the last in
    groups of 32): FP32 storage to 1e-4, FP64 storage to 1e-8 against the oracle's
    M^{-1} on the same factor."""
    W = workloads.terrain(n=3000, grid=60)
    say("precond widths, rank", k)
    plan, op, pc, L, gaps = _pivchol_pair(W, k)
    P = precond.Precond(L, op.Dn)
    rng = np.random.default_rng(41 + k)
    for R in (1, 5, 16, 17, 20, 21, 30, 40):
        B = rng.standard_normal((op.N, R)).astype(np.float32).astype(np.float64)
        ref = P.solve(B)
        e32 = rel_cols(from_gpu(pc.apply(to_gpu(B))), ref).max()
        Z64 = pc.apply(torch.tensor(B.T.copy(), device="cuda")).cpu().numpy().T
        e64 = rel_cols(Z64, ref).max()
        say("  R", R, "fp32", e32, "fp64", e64)
        assert e32 < 1e-4 and e64 < 1e-8


@pytest.mark.parametrize("R,k", [(6, 70), (13, 33), (24, 70)])
def test_pcg_true_residual_column_widths(R, k):
    """The fused PCG iteration at padded widths 8, 16 and 24 (one or two
    matrix-core column blocks) and ranks off the 16-column blocks."""
    W = workloads.terrain(n=3000, grid=60)
    say("pcg widths", R, k)
    plan, op = make(W)
    pc = plan.pivchol(k)
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, R - 1, op.N)], axis=1)
    B = B.astype(np.float32).astype(np.float64)
    X, iters, relres, st, _ = plan.pcg(to_gpu(B), pc, tol=1e-4, max_iter=20000)
    assert st == 0
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  iters", max(iters), "true relres", tr.max())
    assert tr.max() <= 1e-4


def test_pcg_rank0_preconditioner_against_jacobi_oracle():
    """A rank-0 pivoted-Cholesky preconditioner is M = D, the noise diagonal
    (the fused iteration without its low-rank term), on 17 columns (one
    matrix-core column block plus vector columns): with FP64 vectors the
    iteration counts follow the oracle's PCG with the same diagonal
    preconditioner (within 2 % + 3), and with FP32 and FP64 vectors the
    oracle's FP64 true residual meets the tolerance."""
    W = workloads.terrain(n=3000, grid=60)
    say("pcg rank 0")
    plan, op = make(W)
    pc = plan.pivchol(0)
    assert pc.rank == 0
    R, tol = 17, 1e-3
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, R - 1, op.N)], axis=1)
    B = B.astype(np.float32).astype(np.float64)
    ref = krylov.pcg(op.matvec, B[:, :3], lambda V: V / op.Dn.reshape((-1,) + (1,) * (V.ndim - 1)), tol=tol,
                     max_iter=20000)
    X64, it64, _, st64, _ = plan.pcg(torch.tensor(B.T.copy(), device="cuda"), pc, tol=tol, max_iter=20000)
    X32, it32, _, st32, _ = plan.pcg(to_gpu(B), pc, tol=tol, max_iter=20000)
    tr64 = krylov.true_relres(op.matvec, B, X64.cpu().numpy().T)
    tr32 = krylov.true_relres(op.matvec, B, from_gpu(X32))
    say("  iters oracle", list(ref["iters"]), "fp64", it64[:3], "fp32", max(it32), "true relres", tr64.max(),
        tr32.max())
    assert st64 == 0 and st32 == 0
    assert tr64.max() <= tol and tr32.max() <= tol
    for c in range(3):
        assert abs(it64[c] - ref["iters"][c]) <= 0.02 * ref["iters"][c] + 3
