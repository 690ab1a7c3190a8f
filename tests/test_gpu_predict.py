"""GPU parity of the posterior mean at test points (Sec. 1, O(1) prediction)
against the FP64 oracle: grid vector g = K_UU S^T alpha and the stencil means
[f, grad f] at test points, on the small 2-D and 3-D workloads (ragged grids
included), at the full terrain size on sampled test points, at the training
points (the identity mean = K alpha), and the out-of-box error."""
import numpy as np
import pytest
import torch

import workloads
from oracle import predict as opred
from tests.gpu_common import SEED, make, need_gpu, say, small_workloads

pytestmark = pytest.mark.gpu


def _alpha(N, seed):
    return np.random.default_rng(seed).standard_normal(N)


def _test_points(W, k, seed):
    r = np.random.default_rng(seed)
    lo, hi = np.asarray(W.lo, dtype=np.float64), np.asarray(W.hi, dtype=np.float64)
    return lo + (hi - lo) * r.uniform(0.0, 1.0, (k, len(lo)))


@pytest.mark.parametrize("name", [nm for nm, _ in small_workloads()])
def test_predict_matches_oracle(name):
    W = dict(small_workloads())[name]
    say("predict", name, W.n, W.grid_m)
    plan, op = make(W)
    alpha = _alpha(op.N, SEED)
    g = plan.predict_grid(torch.tensor(alpha, device="cuda"))
    g_ref = opred.grid_vector(op, alpha)
    eg = np.abs(g.cpu().numpy() - g_ref).max() / np.abs(g_ref).max()
    Xs = _test_points(W, 777, SEED + 1)
    mu = plan.predict(g, torch.tensor(Xs, device="cuda")).cpu().numpy()
    ref = opred.predict_mean(op, g_ref, Xs)
    em = np.abs(mu - ref).max() / np.abs(ref).max()
    # at the training points the mean is the noise-free K alpha
    mt = plan.predict(g, torch.tensor(W.X, device="cuda")).cpu().numpy()
    kt = op.matvec_K(alpha).reshape(W.d + 1, -1).T
    et = np.abs(mt - kt).max() / np.abs(kt).max()
    say("  grid vector", eg, "test means", em, "training means", et)
    assert eg < 1e-11 and em < 1e-11 and et < 1e-11


def test_predict_rejects_a_wrong_grid_vector():
    """The grid vector must be this plan's FP64 CUDA vector of prod(m) nodes:
    an FP32 copy, a host copy and the vector of a smaller grid are refused
    before any launch (the kernel reads 4^d nodes around each test point)."""
    W = workloads.small2d()
    plan, op = make(W)
    g = plan.predict_grid(torch.tensor(_alpha(op.N, SEED), device="cuda"))
    Xs = torch.tensor(_test_points(W, 10, SEED), device="cuda")
    small, _ = make(W, grid=[20, 20])
    g_small = small.predict_grid(torch.tensor(_alpha(op.N, SEED), device="cuda"))
    for bad, exc in ((g.float(), TypeError), (g.cpu(), TypeError), (g_small, ValueError), (g[:-1], ValueError)):
        with pytest.raises(exc):
            plan.predict(bad, Xs)
    assert plan.predict(g, Xs).shape == (10, W.d + 1)


def test_predict_full_terrain_sampled():
    """Terrain size (n = 20,000, 200 x 200 grid): 200,000 test points on the
    GPU, checked against the oracle on a sample of 2,000 of them."""
    W = workloads.terrain()
    say("predict terrain", W.n, W.grid_m)
    plan, op = make(W)
    alpha = _alpha(op.N, SEED + 2)
    g = plan.predict_grid(torch.tensor(alpha, device="cuda"))
    Xs = _test_points(W, 200000, SEED + 3)
    mu = plan.predict(g, torch.tensor(Xs, device="cuda")).cpu().numpy()
    idx = np.random.default_rng(4).choice(len(Xs), 2000, replace=False)
    ref = opred.predict_mean(op, opred.grid_vector(op, alpha), Xs[idx])
    e = np.abs(mu[idx] - ref).max() / np.abs(ref).max()
    say("  sampled rel err", e)
    assert e < 1e-11


def test_predict_rejects_points_outside_the_box():
    dski = need_gpu()
    W = workloads.small2d()
    plan, op = make(W)
    g = plan.predict_grid(torch.tensor(_alpha(op.N, 1), device="cuda"))
    Xs = _test_points(W, 10, 2)
    Xs[3, 0] = np.asarray(W.hi)[0] + 0.5
    with pytest.raises(dski.DSKIError) as e:
        plan.predict(g, torch.tensor(Xs, device="cuda"))
    assert e.value.status == -1  # DSKI_EINVAL
    assert plan.predict(g, torch.zeros((0, W.d), dtype=torch.float64, device="cuda")).shape == (0, W.d + 1)


def _var_case(W, k, n_test, seed, sample=None):
    """GPU predictive variance with a rank-k pivoted Cholesky against the oracle
    with the same pivots (near-ties may order them either way); relative to
    the larger of the two terms k(x, x) and K_{xX} M^{-1} K_{Xx} that v^ subtracts."""
    from oracle import pivchol
    plan, op = make(W)
    pc = plan.pivchol(k)
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    assert gaps.size == 0 or gaps.max() <= 1e-4
    Xs = _test_points(W, n_test, seed)
    v = plan.predict_var(pc, torch.tensor(Xs, device="cuda")).cpu().numpy()
    idx = np.arange(n_test) if sample is None else np.random.default_rng(seed).choice(n_test, sample, replace=False)
    ref = opred.predictive_variance(op, L, Xs[idx])
    kxx = opred.prior_cov(op, Xs[idx])[0]
    scale = np.maximum(kxx, np.abs(kxx - ref)).max()
    e = np.abs(v[idx] - ref).max() / scale
    say("  variance rel err", e, "rank", pc.rank, "min/max v", v.min(), v.max())
    return e


@pytest.mark.parametrize("name,k", [("small2d", 20), ("small2d_ragged", 0), ("terrain_small", 50),
                                    ("torus_small", 30)])
def test_predict_var_matches_oracle(name, k):
    """300 test points: two full batches of 128 grid columns and a ragged one."""
    W = dict(small_workloads())[name]
    say("predict_var", name, W.n, W.grid_m, k)
    assert _var_case(W, k, 300, SEED + 5) < 1e-7


def test_predict_var_full_terrain_sampled():
    """Terrain size (n = 20,000, 200 x 200 grid), rank 100: 2,000 test points on
    the GPU, 100 of them checked against the oracle."""
    W = workloads.terrain()
    say("predict_var terrain", W.n, W.grid_m)
    assert _var_case(W, 100, 2000, SEED + 6, sample=100) < 1e-7


def test_predict_var_rejects_points_outside_the_box():
    dski = need_gpu()
    W = workloads.small2d()
    plan, op = make(W)
    pc = plan.pivchol(10)
    Xs = _test_points(W, 40, 3)
    Xs[35, 1] = np.asarray(W.lo)[1] - 1.0
    with pytest.raises(dski.DSKIError) as e:
        plan.predict_var(pc, torch.tensor(Xs, device="cuda"))
    assert e.value.status == -1  # DSKI_EINVAL
    assert plan.predict_var(pc, torch.zeros((0, W.d), dtype=torch.float64, device="cuda")).shape == (0,)


@pytest.mark.parametrize("name,k,ns,R", [("small2d", 20, 40, 16), ("torus_small", 30, 24, 40),
                                         ("small2d_ragged", 10, 300, 8)])
def test_predict_var_probes_matches_oracle(name, k, ns, R):
    """Randomized variance with Rademacher probes (the same on both sides; R = 40
    runs a chunk of 32 probes and a ragged one) against the oracle's dense
    solves, relative to the size of the correction |v - v^|; PCG to 1e-10."""
    from oracle import pivchol
    W = dict(small_workloads())[name]
    say("predict_var_probes", name, k, ns, R)
    plan, op = make(W)
    pc = plan.pivchol(k)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    Xs = _test_points(W, ns, SEED + 7)
    Zp = np.random.default_rng(SEED + 8).choice([-1.0, 1.0], (R, ns))
    v, st = plan.predict_var_probes(pc, torch.tensor(Xs, device="cuda"), torch.tensor(Zp, device="cuda"),
                                    tol=1e-10, max_iter=20000)
    v = v.cpu().numpy()
    ref = opred.predictive_variance_probes(op, L, Xs, Zp)
    corr = np.abs(ref - opred.predictive_variance(op, L, Xs)).max()
    e = np.abs(v - ref).max() / corr
    say("  status", st, "rel err", e, "correction", corr)
    assert st == 0 and e < 1e-6


def test_predict_var_probes_with_unit_probes_is_the_exact_variance():
    """Probes sqrt(n*) e_j make the estimate exact: the GPU result equals the
    exact D-SKI posterior variance from the oracle's dense solve."""
    from oracle import pivchol
    W = workloads.small2d()
    plan, op = make(W)
    pc = plan.pivchol(20)
    ns = 12
    Xs = _test_points(W, ns, SEED + 9)
    Zp = np.sqrt(ns) * np.eye(ns)
    v, st = plan.predict_var_probes(pc, torch.tensor(Xs, device="cuda"), torch.tensor(Zp, device="cuda"),
                                    tol=1e-10, max_iter=20000)
    v = v.cpu().numpy()
    exact = opred.exact_variance(op, Xs)
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    corr = np.abs(exact - opred.predictive_variance(op, L, Xs)).max()
    e = np.abs(v - exact).max() / corr
    say("  unit probes: status", st, "rel err", e, "min v", v.min())
    assert st == 0 and e < 1e-6


def test_prediction_error_paths():
    """Forced from the host: a solve capped at one iteration reports
    DSKI_NOT_CONVERGED (1) with finite outputs; D-SKIP plans are refused by
    every prediction call (DSKI_ENOTSUP); a probe matrix of the wrong shape is
    refused by the binding."""
    dski = need_gpu()
    W = workloads.small2d()
    plan, op = make(W)
    pc = plan.pivchol(10)
    Xs = torch.tensor(_test_points(W, 20, 4), device="cuda")
    Zp = torch.tensor(np.random.default_rng(5).choice([-1.0, 1.0], (4, 20)), device="cuda")
    v, st = plan.predict_var_probes(pc, Xs, Zp, tol=1e-12, max_iter=1)
    assert st == 1 and torch.isfinite(v).all()
    with pytest.raises(TypeError):
        plan.predict_var_probes(pc, Xs, Zp[:, :10])
    Wk = workloads.ridge8d(n=300, skip_m=16, skip_rank=8)
    sp = dski.DskipPlan(torch.tensor(Wk.X, device="cuda"), Wk.skip_m, Wk.skip_rank, SEED, Wk.log_ell, Wk.lo, Wk.hi)
    sp.set_hypers(*Wk.hypers())
    spc = sp.pivchol(5)
    Xk = torch.tensor(_test_points(Wk, 5, 6), device="cuda")
    for call in (lambda: sp.predict_grid(torch.zeros(sp.N, dtype=torch.float64, device="cuda")),
                 lambda: sp.predict_var(spc, Xk),
                 lambda: sp.predict_var_probes(spc, Xk, torch.ones((2, 5), dtype=torch.float64, device="cuda"))):
        with pytest.raises(dski.DSKIError) as e:
            call()
        assert e.value.status == -5  # DSKI_ENOTSUP
