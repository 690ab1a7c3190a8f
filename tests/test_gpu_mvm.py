"""GPU parity of the D-SKI MVM (Sec. 3.1) against the FP64 oracle.

Bar: 1e-5 relative on the MVM, with inputs rounded to FP32 on both sides, both
as a 2-norm per column and element-wise (largest entry error over the
column's largest entry); bitwise reproducibility of reruns; bit-exact
probes."""
import numpy as np
import pytest
import torch

import workloads
from oracle import rng as orng
from tests.gpu_common import (SEED, from_gpu, make, mvm_errors, need_gpu, rel_cols, say, small_workloads,
                               to_gpu)

pytestmark = pytest.mark.gpu

TOL_MVM = 1e-5


@pytest.mark.parametrize("idx", range(4))
def test_mvm_matches_oracle(idx):
    name, W = small_workloads()[idx]
    say("mvm", name, W.n, W.grid_m)
    plan, op = make(W)
    r = np.random.default_rng(idx)
    for R in (1, 3, 17):
        V = r.standard_normal((op.N, R)).astype(np.float32).astype(np.float64)
        V[:, 0] = W.y.astype(np.float32)          # a smooth data column
        Y = from_gpu(plan.mvm(to_gpu(V)))
        ref = op.matvec(V)
        e2, emax = mvm_errors(Y, ref)
        say("  R", R, "max rel err", e2, "element-wise", emax)
        assert e2 < TOL_MVM and emax < TOL_MVM


@pytest.mark.parametrize("idx", [0, 3])
def test_mvm_fp64_matches_oracle(idx):
    name, W = small_workloads()[idx]
    say("mvm fp64", name)
    plan, op = make(W)
    V = np.random.default_rng(11).standard_normal((op.N, 5))
    Y = plan.mvm(torch.tensor(V.T.copy(), device="cuda"))
    err = rel_cols(Y.cpu().numpy().T, op.matvec(V))
    say("  max rel err", err.max())
    assert err.max() < 1e-12
    Yd = plan.mvm_dtheta(0, torch.tensor(V.T.copy(), device="cuda"))
    assert rel_cols(Yd.cpu().numpy().T, op.matvec_dtheta(0, V)).max() < 1e-12


def test_mvm_dtheta_matches_oracle():
    W = workloads.small2d(n=400, grid=40)
    say("mvm_dtheta", W.n)
    plan, op = make(W)
    V = np.random.default_rng(5).standard_normal((op.N, 2)).astype(np.float32).astype(np.float64)
    for which in range(op.d + 3):
        Y = from_gpu(plan.mvm_dtheta(which, to_gpu(V)))
        ref = op.matvec_dtheta(which, V)
        e2, emax = mvm_errors(Y, ref)
        say("  which", which, e2, emax)
        assert e2 < TOL_MVM and emax < TOL_MVM


def test_tiled_order_and_determinism():
    W = workloads.terrain(n=2000, grid=40)
    say("tiled", W.n)
    plan, op = make(W)
    V = to_gpu(np.random.default_rng(1).standard_normal((op.N, 5)))
    Y1 = plan.mvm(V)
    Y2 = plan.mvm(V)
    assert torch.equal(Y1, Y2)                      # fixed summation order, no atomics
    Vt = plan.permute(V, +1)
    Yt = plan.mvm_tiled(Vt)
    assert torch.equal(plan.permute(Yt, -1), Y1)
    perm = plan.tile_order()
    assert sorted(perm.tolist()) == list(range(W.n))
    # the back permutation inverts the forward one exactly
    assert torch.equal(plan.permute(Vt, -1), V)


def test_mvm_full_size_terrain():
    """The terrain workload at full size (n=20,000, 200x200 grid, 17 columns)."""
    W = workloads.terrain()
    say("mvm full terrain", W.n, W.grid_m)
    plan, op = make(W)
    r = np.random.default_rng(7)
    V = np.sign(r.standard_normal((op.N, 17))).astype(np.float64)
    V[:, 0] = W.y.astype(np.float32)
    Y = from_gpu(plan.mvm(to_gpu(V)))
    e2, emax = mvm_errors(Y, op.matvec(V))
    say("  max rel err", e2, "element-wise", emax)
    assert e2 < TOL_MVM and emax < TOL_MVM


def test_mvm_full_size_torus():
    """The implicit-surface workload at full size (n = 30,000 on the perturbed
    torus, 48^3 grid, N = 120,000, 17 columns): FP32 storage to 1e-5 (2-norm
    and element-wise), FP64 storage to 1e-12."""
    W = workloads.torus()
    say("mvm full torus", W.n, W.grid_m)
    plan, op = make(W)
    r = np.random.default_rng(8)
    V = np.sign(r.standard_normal((op.N, 17))).astype(np.float64)
    V[:, 0] = W.y.astype(np.float32)
    ref = op.matvec(V)
    for sv in (0, 6):  # the tiled and the grouped 3-D scatter
        plan.set_variants(sv, 0)
        e2, emax = mvm_errors(from_gpu(plan.mvm(to_gpu(V))), ref)
        say("  scatter", sv, "FP32 max rel err", e2, "element-wise", emax)
        assert e2 < TOL_MVM and emax < TOL_MVM
        Y64 = plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
        e2, emax = mvm_errors(Y64, ref)
        say("  scatter", sv, "FP64 max rel err", e2, "element-wise", emax)
        assert e2 < 1e-12 and emax < 1e-12


def test_mvm_edge_cases():
    dski = need_gpu()
    say("edge cases")
    # points exactly on the box corners, a 1-D problem and the smallest grid
    X = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.5, 0.25]])
    for m in ([4, 4], [5, 9]):
        plan = dski.Plan(torch.tensor(X, device="cuda"), m, [0, 0], [1, 1])
        plan.set_hypers(np.log([0.4, 0.3]), 0.1, np.log(0.05), np.log(0.1))
        from oracle import dski as odski
        op = odski.DSKI(X, m, [0, 0], [1, 1], np.log([0.4, 0.3]), 0.1, np.log(0.05), np.log(0.1))
        V = np.random.default_rng(0).standard_normal((op.N, 2)).astype(np.float32).astype(np.float64)
        assert max(mvm_errors(from_gpu(plan.mvm(to_gpu(V))), op.matvec(V))) < TOL_MVM
    X1 = np.random.default_rng(2).random((50, 1))
    plan = dski.Plan(torch.tensor(X1, device="cuda"), [25], [0], [1])
    plan.set_hypers([np.log(0.1)], 0.0, np.log(0.05), np.log(0.1))
    from oracle import dski as odski
    op = odski.DSKI(X1, [25], [0], [1], [np.log(0.1)], 0.0, np.log(0.05), np.log(0.1))
    V = np.random.default_rng(3).standard_normal((op.N, 3)).astype(np.float32).astype(np.float64)
    assert max(mvm_errors(from_gpu(plan.mvm(to_gpu(V))), op.matvec(V))) < TOL_MVM
    # a point outside the box is rejected
    with pytest.raises(dski.DSKIError):
        dski.Plan(torch.tensor([[0.0, 1.5]], device="cuda", dtype=torch.float64), [8, 8], [0, 0], [1, 1])
    # empty block of vectors
    plan = dski.Plan(torch.tensor(X, device="cuda"), [6, 6], [0, 0], [1, 1])
    out = plan.mvm(torch.zeros((0, 12), device="cuda"))
    assert out.shape == (0, 12)


def test_rademacher_matches_oracle_stream():
    dski = need_gpu()
    say("rademacher")
    for (seed, col0, nc, N) in ((SEED, 0, 3, 1000), (12345, 5, 2, 777)):
        g = dski.rademacher(seed, col0, nc, N).cpu().numpy().T.astype(np.float64)
        assert np.array_equal(g, orng.rademacher(seed, col0, nc, N))


@pytest.mark.parametrize("name", ["terrain_small", "torus_small"])
def test_kernel_variants_agree(name):
    """Scatter variants 0-5 give the same bits, and so does every gather
    variant.  Variant 6 is the grouped 3-D form (the same sums with the
    additions grouped by first-axis cell): in 3-D within FP32 rounding of the
    others (2-norm per column and element-wise, 1e-6), elsewhere variant 3's
    kernel, the same bits.  The autotuner's choice is one of them."""
    W = dict(small_workloads())[name]
    say("variants", name)
    plan, op = make(W)
    V = to_gpu(np.random.default_rng(4).standard_normal((op.N, 17)))
    outs = []
    for v in range(6):
        plan.set_variants(v, 0)
        outs.append(plan.mvm(V))
    for gv in range(3):
        plan.set_variants(0, gv)
        outs.append(plan.mvm(V))
    for o in outs[1:]:
        assert torch.equal(outs[0], o)
    plan.set_variants(6, 0)
    o6 = plan.mvm(V)
    if op.d == 3:
        e2, emax = mvm_errors(from_gpu(o6), from_gpu(outs[0]))
        say("  grouped form against the tiled one", e2, emax)
        assert e2 < 1e-6 and emax < 1e-6
    else:
        assert torch.equal(o6, outs[0])
    t = plan.autotune(17)
    say("  autotune us", t)
    assert t["scatter_us"][6] > 0 if op.d == 3 else t["scatter_us"][6] == -1
    y = plan.mvm(V)
    assert any(torch.equal(y, o) for o in outs + [o6])


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_dense_kuu_variant_matches_oracle(idx):
    """The dense Toeplitz product on the FP64 matrix cores, on every axis:
    FP64 MVM and all hyper-parameter derivatives to 1e-12 against the oracle,
    and agreement with the FFT variant."""
    name, W = small_workloads()[idx]
    say("dense K_UU", name, W.grid_m)
    plan, op = make(W)
    V = np.random.default_rng(13).standard_normal((op.N, 5))
    Vd = torch.tensor(V.T.copy(), device="cuda")
    Y_fft = plan.mvm(Vd).cpu().numpy().T
    for a in range(op.d):
        plan.set_kuu_variant(a, 1)
    Y = plan.mvm(Vd).cpu().numpy().T
    err = rel_cols(Y, op.matvec(V))
    say("  max rel err", err.max(), "vs FFT", rel_cols(Y, Y_fft).max())
    assert err.max() < 1e-12
    for which in range(op.d + 1):
        Yd = plan.mvm_dtheta(which, Vd).cpu().numpy().T
        e = rel_cols(Yd, op.matvec_dtheta(which, V)).max()
        say("  dtheta", which, e)
        assert e < 1e-12
    # FP32 storage path and the autotuner's choice
    Vf = V.astype(np.float32).astype(np.float64)
    assert max(mvm_errors(from_gpu(plan.mvm(to_gpu(Vf))), op.matvec(Vf))) < TOL_MVM
    times = plan.autotune(5)
    say("  tuner K_UU us", times["kuu_us"])
    assert rel_cols(plan.mvm(Vd).cpu().numpy().T, op.matvec(V)).max() < 1e-12


@pytest.mark.parametrize("m", [[600, 12], [12, 300], [1000]])
def test_mvm_long_axes_match_oracle(m):
    """Grid axes whose circulant length is 1024 or 2048 (the largest FFT), as the
    strided and as the contiguous axis, in FP64 to 1e-12 and FP32 storage to 1e-5."""
    dski = need_gpu()
    from oracle import dski as odski
    say("long axes", m)
    d = len(m)
    X = np.random.default_rng(21).random((300, d))
    ell = np.log(np.full(d, 0.05))
    plan = dski.Plan(torch.tensor(X, device="cuda"), m, [0] * d, [1] * d)
    plan.set_hypers(ell, 0.1, np.log(0.05), np.log(0.1))
    op = odski.DSKI(X, m, [0] * d, [1] * d, ell, 0.1, np.log(0.05), np.log(0.1))
    V = np.random.default_rng(22).standard_normal((op.N, 3))
    Y = plan.mvm(torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
    err = rel_cols(Y, op.matvec(V)).max()
    say("  fp64 max rel err", err)
    assert err < 1e-12
    Yd = plan.mvm_dtheta(0, torch.tensor(V.T.copy(), device="cuda")).cpu().numpy().T
    assert rel_cols(Yd, op.matvec_dtheta(0, V)).max() < 1e-12
    Vf = V.astype(np.float32).astype(np.float64)
    assert max(mvm_errors(from_gpu(plan.mvm(to_gpu(Vf))), op.matvec(Vf))) < TOL_MVM


def test_mvm_clustered_points_mix_both_scatter_paths():
    """A quarter of the points packed into a small disc: tiles there hold more
    than 256 region points (read through the cache), the others are staged in
    LDS; FP64 MVM to 1e-12 against the oracle and the same bits from every
    scatter and gather variant."""
    dski = need_gpu()
    from oracle import dski as odski
    say("clustered points")
    r = np.random.default_rng(31)
    Xu = r.random((3000, 2))
    ang, rad = r.uniform(0, 2 * np.pi, 1000), 0.04 * np.sqrt(r.random(1000))
    Xc = np.stack([0.5 + rad * np.cos(ang), 0.5 + rad * np.sin(ang)], axis=1)
    X = np.concatenate([Xu, Xc])
    m = [80, 80]
    ell = np.log([0.05, 0.05])
    plan = dski.Plan(torch.tensor(X, device="cuda"), m, [0, 0], [1, 1])
    plan.set_hypers(ell, 0.1, np.log(0.05), np.log(0.1))
    op = odski.DSKI(X, m, [0, 0], [1, 1], ell, 0.1, np.log(0.05), np.log(0.1))
    V = np.random.default_rng(32).standard_normal((op.N, 6))
    Vd = torch.tensor(V.T.copy(), device="cuda")
    outs = []
    for sv in range(6):
        plan.set_variants(sv, 0)
        outs.append(plan.mvm(Vd))
    for gv in range(3):
        plan.set_variants(0, gv)
        outs.append(plan.mvm(Vd))
    err = rel_cols(outs[0].cpu().numpy().T, op.matvec(V)).max()
    say("  fp64 max rel err", err)
    assert err < 1e-12
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


def test_autotune_cache_reuses_the_choice_per_shape(tmp_path):
    """The per-shape tuner cache: the first plan of a shape is timed and its
    choice appended; a second plan of the same shape reuses it without timing
    (and multiplies identically); another R or stencil width is a new shape."""
    W = workloads.terrain(n=3000, grid=60)
    say("autotune cache")
    cache = str(tmp_path / "tune.txt")
    plan, op = make(W)
    t1 = plan.autotune(17, cache=cache)
    # (scatter variant 6 is the grouped 3-D form: not timed on a 2-D plan)
    assert not t1["cached"] and min(t1["scatter_us"][:6]) > 0 and t1["scatter_us"][6] == -1
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and " R=17 : " in lines[0] and " S=4 " in lines[0]
    plan2, _ = make(W)
    t2 = plan2.autotune(17, cache=cache)
    assert t2["cached"] and all(v == -1 for v in t2["scatter_us"])
    V = to_gpu(np.random.default_rng(9).standard_normal((op.N, 17)))
    assert torch.equal(plan.mvm(V), plan2.mvm(V))
    assert not plan2.autotune(5, cache=cache)["cached"]
    plan3, _ = make(W, interp="quintic")
    assert not plan3.autotune(17, cache=cache)["cached"]
    assert len(open(cache).read().splitlines()) == 3
