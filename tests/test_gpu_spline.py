"""GPU parity of the thin-plate spline kernel under D-SKI (App. A; the
implicit surface of Sec. 4.3) against the FP64 oracle, which forms K_UU
densely from the kernel function: the multi-level Toeplitz K_UU product by
d-dimensional circulant FFTs inside the MVM in 1-D, 2-D (ragged grids) and
3-D (FP32 storage to 1e-5, 2-norm and element-wise; FP64 storage), its
derivatives (s and the noise levels; zero for length scales), the pivoted
Cholesky on the kernel's own diagonal and rows, the block PCG to an oracle
true residual of 1e-4, mll and gradient against the oracle's same-probe
estimator, and the posterior mean."""
import numpy as np
import pytest
import torch

import workloads
from oracle import krylov, mll as omll, pivchol, predict as opred, rng as orng, spline
from tests.gpu_common import SEED, from_gpu, mvm_errors, need_gpu, rel_cols, say, to_gpu

pytestmark = pytest.mark.gpu


def _pair(W, grid=None, interp="cubic"):
    dski = need_gpu()
    m = grid or W.grid_m
    plan = dski.Plan(torch.tensor(W.X, device="cuda"), m, W.lo, W.hi, interp=interp, kernel="spline")
    plan.set_hypers(*W.hypers())
    op = spline.SplineDSKI(W.X, m, W.lo, W.hi, W.log_s, W.log_sigma_f, W.log_sigma_g, interp_kind=interp)
    return plan, op


CASES = {
    "terrain_40": (lambda: workloads.terrain(n=2000, grid=40), None),
    "terrain_ragged": (lambda: workloads.terrain(n=777, grid=23), [23, 31]),
    "torus_14": (lambda: workloads.torus(n=700, grid=14), None),
    "torus_17": (lambda: workloads.torus(n=1500, grid=17), None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_spline_mvm_matches_oracle(name):
    gen, grid = CASES[name]
    W = gen()
    plan, op = _pair(W, grid)
    say("spline mvm", name, W.n, grid or W.grid_m, "R", op.R)
    r = np.random.default_rng(2)
    for R in (1, 6, 17):
        V = r.standard_normal((op.N, R)).astype(np.float32).astype(np.float64)
        V[:, 0] = W.y.astype(np.float32)
        e2, emax = mvm_errors(from_gpu(plan.mvm(to_gpu(V))), op.matvec(V))
        say("  R", R, "FP32", e2, emax)
        assert e2 < 1e-5 and emax < 1e-5
    V = r.standard_normal((op.N, 3))
    Y = plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
    e2, emax = mvm_errors(Y, op.matvec(V))
    say("  FP64", e2, emax)
    assert e2 < 1e-11 and emax < 1e-10
    for which in range(op.d + 3):
        Yd = plan.mvm_dtheta(which, torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
        ref = op.matvec_dtheta(which, V)
        if which < op.d:
            assert np.abs(Yd).max() == 0.0
        else:
            assert rel_cols(Yd, ref).max() < 1e-11, which


def test_spline_1d_and_quintic():
    dski = need_gpu()
    say("spline 1-D and quintic 2-D")
    X1 = np.random.default_rng(4).random((200, 1))
    plan = dski.Plan(torch.tensor(X1, device="cuda"), [50], [0], [1], kernel="spline")
    plan.set_hypers([0.0], np.log(0.5), np.log(0.05), np.log(0.1))
    op = spline.SplineDSKI(X1, [50], [0], [1], np.log(0.5), np.log(0.05), np.log(0.1))
    V = np.random.default_rng(5).standard_normal((op.N, 4))
    assert rel_cols(plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T, op.matvec(V)).max() < 1e-11
    W = workloads.terrain(n=900, grid=30)
    plan, op = _pair(W, interp="quintic")
    V = np.random.default_rng(6).standard_normal((op.N, 5)).astype(np.float32).astype(np.float64)
    assert max(mvm_errors(from_gpu(plan.mvm(to_gpu(V))), op.matvec(V))) < 1e-5


def test_spline_pivchol_pcg_and_mll():
    W = workloads.torus(n=1500, grid=17)
    plan, op = _pair(W)
    say("spline pivchol / pcg / mll", W.n, W.grid_m)
    k, t = 30, 8
    pc = plan.pivchol(k)
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    err = np.linalg.norm(pc.factor().cpu().numpy().T - L) / np.linalg.norm(L)
    say("  near-tie gap", gaps.max(), "factor", err, "rank", pc.rank)
    assert gaps.max() <= 1e-4 and err < 1e-4
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, 3, op.N)], axis=1).astype(np.float32).astype(np.float64)
    X, iters, relres, st, _ = plan.pcg(to_gpu(B), pc, tol=1e-4, max_iter=20000)
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  pcg iters", iters, "oracle true relres", tr.max())
    assert st == 0 and tr.max() <= 1e-4
    y32 = W.y.astype(np.float32)
    res = plan.mll_and_grad(torch.tensor(y32, device="cuda")[None, :], pc, num_probes=t, seed=SEED, tol=1e-6,
                            max_iter=20000)
    orc = omll.stochastic(op, y32.astype(np.float64), L, t, SEED, 1e-6, max_iter=20000)
    g, go = np.asarray(res["grad"]), orc["grad"]
    eld = abs(res["logdet"] - orc["logdet"]) / abs(orc["logdet"])
    eg = np.linalg.norm(g - go) / np.linalg.norm(go)
    say("  log det", res["logdet"], orc["logdet"], "rel", eld, "grad rel", eg, "grad", g)
    assert eld < 1e-3 and eg < 1e-3
    assert np.all(g[:op.d] == 0.0)


def test_spline_predict_matches_oracle():
    W = workloads.terrain(n=1200, grid=30)
    plan, op = _pair(W)
    say("spline predict")
    alpha = np.random.default_rng(7).standard_normal(op.N)
    g = plan.predict_grid(torch.tensor(alpha, device="cuda"))
    g_ref = opred.grid_vector(op, alpha)
    Xs = np.random.default_rng(8).random((500, 2))
    mu = plan.predict(g, torch.tensor(Xs, device="cuda")).cpu().numpy()
    ref = opred.predict_mean(op, g_ref, Xs)
    e = np.abs(mu - ref).max() / np.abs(ref).max()
    say("  mean rel err", e)
    assert e < 1e-10


def test_spline_full_torus_sampled_rows():
    """The full torus (n = 30,000 on 48^3, the 128^3 embedding with the pruned
    axis passes): sampled rows of the FP64 MVM, each computed one by one from
    the oracle's interpolation matrix and the kernel function (the row's
    stencil nodes against every grid node), value and derivative rows."""
    from oracle import interp
    dski = need_gpu()
    W = workloads.torus()
    say("spline full torus", W.n, W.grid_m)
    plan = dski.Plan(torch.tensor(W.X, device="cuda"), W.grid_m, W.lo, W.hi, kernel="spline")
    plan.set_hypers(*W.hypers())
    r = np.random.default_rng(11)
    N = W.n * 4
    V = r.standard_normal((N, 2))
    Y = plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
    grid = interp.Grid(W.lo, W.hi, W.grid_m, "cubic")
    S = interp.interp_matrices(W.X, grid)
    G = S.T @ V
    nodes = np.stack(np.meshgrid(*[grid.nodes(p) for p in range(3)], indexing="ij"), -1).reshape(-1, 3)
    R = spline.grid_domain_size(grid)
    s2 = np.exp(2 * W.log_s)
    rows = np.concatenate([r.choice(W.n, 5, replace=False), W.n + r.choice(3 * W.n, 7, replace=False)])
    worst = 0.0
    for i in rows:
        idx = S.indices[S.indptr[i]:S.indptr[i + 1]]
        w = S.data[S.indptr[i]:S.indptr[i + 1]]
        dist = np.linalg.norm(nodes[idx][:, None, :] - nodes[None, :, :], axis=-1)
        ref = s2 * (w @ (spline.spline_k(dist, 3, R) @ G))
        ref += (np.exp(2 * W.log_sigma_f) if i < W.n else np.exp(2 * W.log_sigma_g)) * V[i]
        err = np.abs(Y[i] - ref).max() / np.abs(Y).max(axis=0).max()
        worst = max(worst, err)
    say("  sampled rows, worst error relative to max |Y|", worst)
    assert worst < 1e-10  # the element-wise FP64 bar of the small cases
    plan.close()
