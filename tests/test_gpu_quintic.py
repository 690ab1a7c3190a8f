"""GPU parity of quintic interpolation (Sec. 3.1; six nodes per axis) against
the FP64 oracle: the D-SKI MVM in 1-D, 2-D and 3-D (FP32 storage to 1e-5 as a
2-norm and element-wise, FP64 storage to 1e-12 as a 2-norm and element-wise,
1e-11 element-wise in 3-D), its hyper-parameter
derivatives, every scatter and gather variant giving the same bits, the
pivoted Cholesky and block PCG to an oracle true residual of 1e-4 (also at the
full terrain size), and the posterior mean at test points; also the plan's
refusal of a grid narrower than the stencil."""
import numpy as np
import pytest
import torch

import workloads
from oracle import krylov, pivchol, predict as opred, rng as orng
from tests.gpu_common import SEED, from_gpu, make, mvm_errors, need_gpu, rel_cols, say, to_gpu

pytestmark = pytest.mark.gpu

CASES = [
    ("small2d", lambda: workloads.small2d(), None),
    ("terrain_small", lambda: workloads.terrain(n=3000, grid=60), None),
    ("terrain_ragged", lambda: workloads.terrain(n=1111, grid=41), None),
    ("torus_small", lambda: workloads.torus(n=700, grid=14), None),
    ("torus_48", lambda: workloads.torus(n=4000), None),
]


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_quintic_mvm_matches_oracle(name):
    W = dict((c[0], c[1]) for c in CASES)[name]()
    say("quintic mvm", name, W.n, W.grid_m)
    plan, op = make(W, interp="quintic")
    r = np.random.default_rng(3)
    Vs = []
    for R in (1, 5, 17):
        V = r.standard_normal((op.N, R)).astype(np.float32).astype(np.float64)
        V[:, 0] = W.y.astype(np.float32)
        Vs.append(V)
    V64 = r.standard_normal((op.N, 3))
    # in 3-D the grouped scatter (variant 6) as well as the tiled one
    for sv in ((0, 6) if op.d == 3 else (0,)):
        plan.set_variants(sv, 0)
        for V in Vs:
            e2, emax = mvm_errors(from_gpu(plan.mvm(to_gpu(V))), op.matvec(V))
            say("  scatter", sv, "R", V.shape[1], "FP32", e2, emax)
            assert e2 < 1e-5 and emax < 1e-5
        Y = plan.mvm(torch.tensor(V64.T.copy(), device="cuda")).cpu().numpy().T
        e2, emax = mvm_errors(Y, op.matvec(V64))
        say("  scatter", sv, "FP64", e2, emax)
        # element-wise, a 3-D quintic output sums 216 stencil products per column
        # on each side (and the grid sums as many per node) in a different order
        # from the oracle's sparse products: 1e-11 of the column's largest entry
        assert e2 < 1e-12 and emax < (1e-11 if op.d == 3 else 1e-12)
    plan.set_variants(0, 0)
    V = V64
    for which in range(op.d + 3):
        Yd = plan.mvm_dtheta(which, torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
        assert rel_cols(Yd, op.matvec_dtheta(which, V)).max() < 1e-12, which


def test_quintic_1d_and_variants_agree():
    dski = need_gpu()
    from oracle import dski as odski
    say("quintic 1-D and variants")
    X1 = np.random.default_rng(2).random((300, 1))
    plan = dski.Plan(torch.tensor(X1, device="cuda"), [40], [0], [1], interp="quintic")
    plan.set_hypers([np.log(0.1)], 0.0, np.log(0.05), np.log(0.1))
    op = odski.DSKI(X1, [40], [0], [1], [np.log(0.1)], 0.0, np.log(0.05), np.log(0.1), interp_kind="quintic")
    V = np.random.default_rng(3).standard_normal((op.N, 4))
    assert rel_cols(plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T, op.matvec(V)).max() < 1e-12
    W = workloads.terrain(n=3000, grid=60)
    plan, op = make(W, interp="quintic")
    Vd = to_gpu(np.random.default_rng(4).standard_normal((op.N, 7)))
    outs = []
    for sv in range(6):
        plan.set_variants(sv, 0)
        outs.append(plan.mvm(Vd))
    for gv in range(3):
        plan.set_variants(0, gv)
        outs.append(plan.mvm(Vd))
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


def test_quintic_pivchol_and_pcg():
    W = workloads.terrain(n=3000, grid=60)
    say("quintic pivchol + pcg", W.n, W.grid_m)
    plan, op = make(W, interp="quintic")
    pc = plan.pivchol(W.rank)
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    err = np.linalg.norm(pc.factor().cpu().numpy().T - L) / np.linalg.norm(L)
    say("  near-tie gap", gaps.max(), "factor", err)
    assert gaps.max() <= 1e-4 and err < 1e-4
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, 4, op.N)], axis=1)
    B = B.astype(np.float32).astype(np.float64)
    X, iters, relres, st, _ = plan.pcg(to_gpu(B), pc, tol=1e-4, max_iter=20000)
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  iters", iters, "oracle true relres", tr.max())
    assert st == 0 and tr.max() <= 1e-4


def test_quintic_predict_matches_oracle():
    W = workloads.terrain(n=2000, grid=50)
    say("quintic predict", W.n)
    plan, op = make(W, interp="quintic")
    alpha = np.random.default_rng(5).standard_normal(op.N)
    g = plan.predict_grid(torch.tensor(alpha, device="cuda"))
    g_ref = opred.grid_vector(op, alpha)
    Xs = np.random.default_rng(6).random((999, 2))
    mu = plan.predict(g, torch.tensor(Xs, device="cuda")).cpu().numpy()
    ref = opred.predict_mean(op, g_ref, Xs)
    e = np.abs(mu - ref).max() / np.abs(ref).max()
    say("  mean rel err", e)
    assert e < 1e-11


def test_quintic_plan_needs_six_nodes_per_axis():
    dski = need_gpu()
    X = torch.tensor(np.random.default_rng(1).random((10, 2)), device="cuda")
    with pytest.raises(dski.DSKIError):
        dski.Plan(X, [5, 8], [0, 0], [1, 1], interp="quintic")
    with pytest.raises(ValueError):
        dski.Plan(X, [8, 8], [0, 0], [1, 1], interp="septic")
    dski.Plan(X, [6, 6], [0, 0], [1, 1], interp="quintic")


def test_quintic_full_terrain_mvm_and_pcg():
    """The terrain configuration with quintic weights (n = 20,000, 200^2, 17
    columns, rank 50, FP32 vectors): the MVM against the oracle (1e-5 as a
    2-norm and element-wise), and the block PCG to 1e-4 with every column's
    true residual by the oracle's FP64 operator."""
    W = workloads.terrain()
    say("quintic full terrain", W.n, W.grid_m)
    plan, op = make(W, interp="quintic")
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, 16, op.N)], axis=1)
    B = B.astype(np.float32).astype(np.float64)
    e2, emax = mvm_errors(from_gpu(plan.mvm(to_gpu(B))), op.matvec(B))
    say("  MVM", e2, emax)
    assert e2 < 1e-5 and emax < 1e-5
    pc = plan.pivchol(W.rank)
    X, iters, relres, st, _ = plan.pcg(to_gpu(B), pc, tol=W.tol, max_iter=20000)
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  iters", max(iters), "oracle true relres", tr.max())
    assert st == 0 and tr.max() <= 1e-4
    pc.close()
    plan.close()
