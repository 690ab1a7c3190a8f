"""The allocation-free MVM entry point (dski_mvm_tiled_noalloc) against the
allocating one (dski_mvm_tiled) through the C ABI: two calls in a row on the
library's fixed grid workspace, the second with a smaller input (smaller
plan, fewer columns), each bitwise equal to dski_mvm_tiled (the same kernels)
and within 1e-5 of the FP64 oracle; sizes beyond the workspace are refused."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_common import from_gpu, make, mvm_errors, need_gpu, say, to_gpu

pytestmark = pytest.mark.gpu


def _case(W, R, seed):
    plan, op = make(W)
    V = np.sign(np.random.default_rng(seed).standard_normal((op.N, R)))
    V[:, 0] = W.y.astype(np.float32)
    Vt = plan.permute(to_gpu(V), +1)
    return plan, op, V, Vt


def test_noalloc_mvm_matches_allocating_entry_point():
    dski = need_gpu()
    for name, W, R in (("terrain", workloads.terrain(), 17), ("small2d", workloads.small2d(), 3)):
        say("noalloc mvm", name, W.n, W.grid_m, "R", R)
        plan, op, V, Vt = _case(W, R, 5)
        Y_ref = plan.mvm_tiled(Vt)
        Y = torch.full_like(Vt, float("nan"))
        plan.mvm_tiled_noalloc(Vt, Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_ref)
        e2, emax = mvm_errors(from_gpu(plan.permute(Y, -1)), op.matvec(V))
        say("  bitwise equal to dski_mvm_tiled; oracle rel err", e2, emax)
        assert e2 < 1e-5 and emax < 1e-5


def test_noalloc_mvm_refuses_what_does_not_fit():
    dski = need_gpu()
    W = workloads.terrain(n=2000, grid=200)
    say("noalloc limits", W.grid_m)
    plan, op = make(W)
    R = 2097152 // (200 * 200) + 1          # one column beyond the 16 MiB workspace
    V = torch.zeros((R, op.N), dtype=torch.float32, device="cuda")
    with pytest.raises(dski.DSKIError) as e:
        plan.mvm_tiled_noalloc(V, torch.empty_like(V))
    assert e.value.status == -1  # DSKI_EINVAL
    # the largest block that fits still runs
    Vf = V[:R - 1].normal_()
    Yf = torch.empty_like(Vf)
    plan.mvm_tiled_noalloc(Vf, Yf)
    assert torch.equal(Yf, plan.mvm_tiled(Vf))
