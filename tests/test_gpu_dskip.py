"""GPU parity of the D-SKIP operator (Sec. 3.2) against the FP64 oracle: same
points, same 1-D grids, same Lanczos start vectors (SplitMix64 Rademacher
columns), same tree.  Bars: MVM 1e-5 relative with FP32 storage, 1e-9 with
FP64 storage; untruncated D-SKIP equals D-SKI on the tensor grid; pivots as for
D-SKI (near-tie protocol, tau = 1e-4); PCG true relative residual <= 1e-4 with
the oracle's operator; converged SLQ log det 1e-3."""
import numpy as np
import pytest
import torch

import workloads
from oracle import dski as odski, dskip as odskip, pivchol, precond, rng as orng
from tests.gpu_common import SEED, from_gpu, need_gpu, rel_cols, say, to_gpu

pytestmark = pytest.mark.gpu

TAU = 1e-4


def make_skip(W, seed=SEED):
    dski = need_gpu()
    Xg = torch.tensor(W.X, dtype=torch.float64, device="cuda")
    plan = dski.DskipPlan(Xg, W.skip_m, W.skip_rank, seed, W.log_ell, W.lo, W.hi)
    plan.set_hypers(*W.hypers())
    op = odskip.DSKIP(W.X, W.skip_m, W.lo, W.hi, *W.hypers(), r=W.skip_rank, seed=seed)
    return plan, op


SMALL = {
    "d2": dict(n=150, d=2, skip_m=16, skip_rank=12),
    "d3": dict(n=200, d=3, skip_m=20, skip_rank=16),
    "d5": dict(n=120, d=5, skip_m=16, skip_rank=20),
    "d4_rank40": dict(n=160, d=4, skip_m=24, skip_rank=40),
    "d8": dict(n=300, d=8, skip_m=30, skip_rank=32),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_dskip_mvm_matches_oracle(name):
    W = workloads.ridge8d(**SMALL[name])
    say("dskip mvm", name, SMALL[name])
    plan, op = make_skip(W)
    ka, kb = plan.root_ranks
    assert (ka, kb) == (op.root[0][0].shape[1], op.root[1][0].shape[1])
    rng = np.random.default_rng(7)
    for R in (1, 5, 17):
        V = rng.standard_normal((op.N, R))
        ref = op.matvec(V)
        Vf = V.astype(np.float32).astype(np.float64)
        e32 = rel_cols(from_gpu(plan.mvm(to_gpu(Vf))), op.matvec(Vf)).max()
        Vd = torch.tensor(np.ascontiguousarray(V.T), device="cuda")
        e64 = rel_cols(plan.mvm(Vd).cpu().numpy().T, ref).max()
        say("  R", R, "fp32", e32, "fp64", e64)
        assert e32 < 1e-5
        assert e64 < 1e-9


@pytest.mark.parametrize("d", [2, 3])
def test_untruncated_dskip_equals_tensor_grid_dski(d):
    """With r >= N the Lanczos factors are exact and the Hadamard product is
    the D-SKI matrix on the tensor grid (checked with the oracle's D-SKI)."""
    dski = need_gpu()
    n, m = 5, 6
    rng = np.random.default_rng(d)
    X = rng.uniform(-1, 1, (n, d))
    lo, hi = -np.ones(d), np.ones(d)
    le = np.log(np.linspace(0.4, 0.7, d))
    N = n * (d + 1)
    say("untruncated dskip", d, N)
    plan = dski.DskipPlan(torch.tensor(X, device="cuda"), m, N, 7, le, lo, hi)
    plan.set_hypers(le, 0.3, np.log(0.05), np.log(0.1))
    K = plan.mvm(torch.eye(N, dtype=torch.float64, device="cuda")).cpu().numpy().T
    ref = odski.DSKI(X, [m] * d, lo, hi, le, 0.3, np.log(0.05), np.log(0.1)).dense()
    err = np.linalg.norm(K - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err < 1e-9


def test_dskip_hyper_change_rebuilds_factors():
    W = workloads.ridge8d(**SMALL["d3"])
    plan, _ = make_skip(W)
    le2 = W.log_ell + np.log(0.8)
    say("dskip set_hypers rebuild")
    plan.set_hypers(le2, 0.2, W.log_sigma_f, W.log_sigma_g)
    op2 = odskip.DSKIP(W.X, W.skip_m, W.lo, W.hi, le2, 0.2, W.log_sigma_f, W.log_sigma_g, r=W.skip_rank,
                       seed=SEED)
    V = np.random.default_rng(2).standard_normal((op2.N, 3))
    Vd = torch.tensor(np.ascontiguousarray(V.T), device="cuda")
    err = rel_cols(plan.mvm(Vd).cpu().numpy().T, op2.matvec(V)).max()
    say("  rel err", err)
    assert err < 1e-9


def test_dskip_derivatives_and_unsupported_calls():
    dski = need_gpu()
    W = workloads.ridge8d(**SMALL["d3"])
    plan, op = make_skip(W)
    d = W.d
    V = np.random.default_rng(4).standard_normal((op.N, 2))
    Vd = torch.tensor(np.ascontiguousarray(V.T), device="cuda")
    Ys = plan.mvm_dtheta(d, Vd).cpu().numpy().T
    assert rel_cols(Ys, 2.0 * op.matvec_K(V)).max() < 1e-9
    Yf = plan.mvm_dtheta(d + 1, Vd).cpu().numpy().T
    Dn = np.zeros(op.N)
    Dn[:W.n] = 2.0 * np.exp(2 * W.log_sigma_f)
    np.testing.assert_allclose(Yf, Dn[:, None] * V, rtol=1e-14, atol=0)
    with pytest.raises(dski.DSKIError, match="ENOTSUP"):
        plan.mvm_dtheta(0, Vd)
    pc = plan.pivchol(10)
    with pytest.raises(dski.DSKIError, match="ENOTSUP"):
        plan.mll_and_grad(to_gpu(W.y), pc, num_probes=2)
    with pytest.raises(dski.DSKIError, match="EINVAL"):
        dski.DskipPlan(torch.tensor(W.X[:, :1].copy(), device="cuda"), 10, 8, 1, [0.0])
    with pytest.raises(dski.DSKIError, match="EINVAL"):
        dski.DskipPlan(torch.tensor(W.X, device="cuda"), 10, 65, 1, W.log_ell)
    with pytest.raises(dski.DSKIError, match="EINVAL"):  # points outside the box
        dski.DskipPlan(torch.tensor(W.X, device="cuda"), 10, 8, 1, W.log_ell, W.lo * 0.5, W.hi * 0.5)


@pytest.mark.parametrize("name,k", [("d3", 40), ("d8", 60)])
def test_dskip_pivchol_matches_oracle(name, k):
    W = workloads.ridge8d(**SMALL[name])
    say("dskip pivchol", name, k)
    plan, op = make_skip(W)
    pc = plan.pivchol(k)
    piv = pc.pivots
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, len(piv), forced=piv)
    say("  rank", pc.rank, "max gap", gaps.max())
    assert gaps.max() <= TAU
    Lg = pc.factor().cpu().numpy().T
    err = np.linalg.norm(Lg - L) / np.linalg.norm(L)
    say("  factor rel err", err)
    assert err < 1e-4
    P = precond.Precond(L, op.Dn)
    assert pc.logdet() == pytest.approx(P.logdet(), rel=1e-5)


@pytest.mark.parametrize("name", ["d3", "d8"])
def test_dskip_pcg_true_residual(name):
    W = workloads.ridge8d(**SMALL[name])
    say("dskip pcg", name)
    plan, op = make_skip(W)
    pc = plan.pivchol(W.rank if W.rank < op.N // 2 else 40)
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, 4, op.N)], axis=1)
    Bf = B.astype(np.float32).astype(np.float64)
    X, iters, relres, st, _ = plan.pcg(to_gpu(Bf), pc, tol=1e-4, max_iter=5000)
    Xh = X.cpu().numpy().T
    true = rel_cols(op.matvec(Xh), Bf)  # |B - K~ X| / |B| per column
    say("  iters", iters, "true relres", true.max())
    assert st == 0
    assert true.max() <= 1e-4


def test_dskip_slq_converged_matches_oracle():
    from tests.test_gpu_solvers import _oracle_slq_pcg
    W = workloads.ridge8d(**SMALL["d3"])
    say("dskip slq")
    plan, op = make_skip(W)
    k = 30
    pc = plan.pivchol(k)
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    t = 8
    ld_gpu, se_gpu = plan.slq_logdet(pc, t, 0, tol=1e-6, max_iter=5000, seed=SEED)
    P = precond.Precond(L, op.Dn)
    Z = P.factor_apply(orng.rademacher(SEED, 0, t, op.N))
    ld_or, se_or = _oracle_slq_pcg(op, P, Z, tol=1e-6)
    exact = np.linalg.slogdet(op.matvec(np.eye(op.N)))[1]
    say("  gpu", ld_gpu, se_gpu, "oracle", ld_or, se_or, "exact", exact)
    assert ld_gpu == pytest.approx(ld_or, rel=1e-3)
    assert abs(ld_gpu - exact) < 4 * se_gpu + 1e-3 * abs(exact)


def test_dskip_full_ridge8d_mvm_and_pcg():
    """The full high-dimensional configuration: n = 4000, d = 8 (N = 36,000),
    1-D grids of 100 nodes, Lanczos rank 32; the 17-column block of the solver."""
    W = workloads.ridge8d()
    say("dskip full ridge8d", W.n, W.d, W.skip_m, W.skip_rank)
    plan, op = make_skip(W)
    R = 17
    V = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, R - 1, op.N)], axis=1)
    Vf = V.astype(np.float32).astype(np.float64)
    e32 = rel_cols(from_gpu(plan.mvm(to_gpu(Vf))), op.matvec(Vf)).max()
    say("  mvm fp32 rel err", e32)
    assert e32 < 1e-5
    pc = plan.pivchol(W.rank)
    X, iters, relres, st, _ = plan.pcg(to_gpu(Vf), pc, tol=W.tol, max_iter=20000)
    true = rel_cols(op.matvec(X.cpu().numpy().T), Vf)
    say("  pcg iters", max(iters), "true relres", true.max())
    assert st == 0
    assert true.max() <= W.tol
