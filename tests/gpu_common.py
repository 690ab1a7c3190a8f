"""Shared helpers of the GPU parity tests (imported by tests/test_gpu_*.py)."""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import dski as odski

SEED = 0x181012283


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_12283_amd import dski
    import os
    if not os.path.exists(dski.LIB_PATH):
        raise RuntimeError("libdski.so is not built; the GPU path has no fallback")
    return dski


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make(W, grid=None, interp="cubic"):
    """(GPU plan, oracle operator) for a workload at its hyper-parameters."""
    dski = need_gpu()
    Xg = torch.tensor(W.X, dtype=torch.float64, device="cuda")
    m = grid or W.grid_m
    plan = dski.Plan(Xg, m, W.lo, W.hi, interp=interp)
    plan.set_hypers(*W.hypers())
    op = odski.DSKI(W.X, m, W.lo, W.hi, *W.hypers(), interp_kind=interp)
    return plan, op


def to_gpu(A):
    """(N, R) numpy -> (R, N) float32 cuda."""
    A = np.asarray(A)
    if A.ndim == 1:
        A = A[:, None]
    return torch.tensor(np.ascontiguousarray(A.T), dtype=torch.float32, device="cuda")


def from_gpu(T):
    """(R, N) cuda -> (N, R) float64 numpy."""
    return T.double().cpu().numpy().T.copy()


def rel_cols(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def rel_cols_max(a, b):
    """Element-wise bar: per column, the largest |a - b| over the largest |b|
    (catches an error at a few entries that a 2-norm over N entries hides)."""
    return np.abs(a - b).max(axis=0) / np.abs(b).max(axis=0)


def mvm_errors(Y, ref):
    """(2-norm error, element-wise error), each the worst over the columns."""
    return float(rel_cols(Y, ref).max()), float(rel_cols_max(Y, ref).max())


def small_workloads():
    return [
        ("small2d", workloads.small2d()),
        ("small2d_ragged", workloads.small2d(n=333, grid=37)),
        ("terrain_small", workloads.terrain(n=3000, grid=60)),
        ("torus_small", workloads.torus(n=700, grid=14)),
    ]
