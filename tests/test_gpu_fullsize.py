"""GPU parity at the full sizes of the terrain and implicit-surface workloads.

Terrain (n = 20,000 on [0,1]^2, 200 x 200 grid, N = 60,000, FP32 storage,
rank-50 pivoted Cholesky, one block PCG of the data vector and 16 probes to
1e-4; Sec. 2, Sec. 3.1, Sec. 3.3, eq. (1)):
* the GPU's pivots pass the near-tie protocol against the oracle forced to
  follow them, the factor is within 1e-4 and log det M within 1e-5;
* every column of the GPU's block PCG has an oracle FP64 true residual
  ||b - K~ x|| / ||b|| <= 1e-4 (one oracle MVM of all 17 columns);
* with the preconditioner built on the oracle's own pivots, the SLQ log det,
  the mll and its gradient agree with the oracle's same-probe estimator (one
  batched FP64 PCG to 1e-4, stored by tests/golden/make_oracle_golden.py)
  within 1e-3.

Implicit surface (the first 2,000 torus points on the 48^3 grid, N = 8,000):
the mll gradient against the oracle's same-probe estimator (1e-3), and against
central differences of the dense exact mll (stored) within four standard
errors of the probe average plus 1e-3 of the gradient's norm.
"""
import json
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import krylov, mll as omll, pivchol, precond, rng as orng
from tests.gpu_common import SEED, from_gpu, make, say, to_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TAU = 1e-4


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def terrain():
    W = workloads.terrain()
    say("terrain full size", W.n, W.grid_m)
    plan, op = make(W)
    return W, plan, op


def test_terrain_pivots_and_factor(terrain):
    W, plan, op = terrain
    pc = plan.pivchol(W.rank)
    assert pc.rank == W.rank
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    ref = _golden("terrain_full_oracle.json")
    same = int(np.sum(np.asarray(ref["pivots"]) == pc.pivots))
    say("  max near-tie gap", gaps.max(), "pivots equal to the oracle's own:", same, "of", W.rank)
    assert gaps.max() <= TAU
    Lg = pc.factor().cpu().numpy().T
    err = np.linalg.norm(Lg - L) / np.linalg.norm(L)
    P = precond.Precond(L, op.Dn)
    say("  factor rel err", err, "log det M", pc.logdet(), P.logdet())
    assert err < 1e-4
    assert pc.logdet() == pytest.approx(P.logdet(), rel=1e-5)


def test_terrain_block_pcg_oracle_true_residual(terrain):
    W, plan, op = terrain
    pc = plan.pivchol(W.rank)
    B = np.concatenate([W.y[:, None], orng.rademacher(SEED, 0, W.num_probes, op.N)], axis=1)
    B = B.astype(np.float32).astype(np.float64)
    X, iters, relres, st, _ = plan.pcg(to_gpu(B), pc, tol=W.tol, max_iter=20000)
    say("  GPU iters", max(iters), "status", st)
    assert st == 0
    tr = krylov.true_relres(op.matvec, B, from_gpu(X))
    say("  oracle FP64 true relres, worst column", tr.max())
    assert tr.max() <= W.tol


def test_terrain_slq_mll_and_gradient_match_oracle(terrain):
    W, plan, op = terrain
    ref = _golden("terrain_full_oracle.json")
    pc = plan.pivchol(W.rank, forced=ref["pivots"])
    assert pc.rank == W.rank and list(pc.pivots) == ref["pivots"]
    assert pc.logdet() == pytest.approx(ref["logdet_M"], rel=1e-5)
    y = torch.tensor(W.y.astype(np.float32), device="cuda")[None, :]
    res = plan.mll_and_grad(y, pc, num_probes=W.num_probes, seed=SEED, tol=W.tol, max_iter=20000)
    g, gr = np.asarray(res["grad"]), np.asarray(ref["grad"])
    eld = abs(res["logdet"] - ref["logdet"]) / abs(ref["logdet"])
    emll = abs(res["mll"] - ref["mll"]) / abs(ref["mll"])
    eg = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    say("  log det", res["logdet"], "oracle", ref["logdet"], "rel", eld)
    say("  mll rel", emll, "grad rel", eg, "GPU iters", max(res["iters"]), "oracle iters", max(ref["iters"]))
    assert res["status"] == 0
    assert eld <= 1e-3 and emll <= 1e-3 and eg <= 1e-3


def test_torus_2000_gradient_matches_oracle_and_central_differences():
    W = workloads.torus(n=2000)
    say("torus n=2000 on", W.grid_m)
    plan, op = make(W)
    k, t, tol = 50, 16, 1e-4
    pc = plan.pivchol(k)
    L, _, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, pc.rank, forced=pc.pivots)
    assert gaps.max() <= TAU
    y32 = W.y.astype(np.float32)
    res = plan.mll_and_grad(torch.tensor(y32, device="cuda")[None, :], pc, num_probes=t, seed=SEED, tol=tol,
                            max_iter=20000)
    orc = omll.stochastic(op, y32.astype(np.float64), L, t, SEED, tol, max_iter=20000)
    g, go = np.asarray(res["grad"]), orc["grad"]
    eg = np.linalg.norm(g - go) / np.linalg.norm(go)
    eld = abs(res["logdet"] - orc["logdet"]) / abs(orc["logdet"])
    say("  grad vs same-probe oracle", eg, "log det", eld)
    assert eg <= 1e-3 and eld <= 1e-3
    # the probe average's standard error per component (oracle's per-probe terms)
    P = orc["precond"]
    U = orc["pcg"]["x"][:, 1:]
    V = P.solve(P.factor_apply(orng.rademacher(SEED, 0, t, op.N)))
    se = np.empty(op.d + 3)
    for j in range(op.d + 3):
        terms = 0.5 * np.sum(U * op.matvec_dtheta(j, V), axis=0)
        se[j] = np.std(terms, ddof=1) / np.sqrt(t)
    gold = _golden("torus2000_oracle.json")
    fd = np.asarray(gold["fd_grad"])
    dev = np.abs(g - fd)
    say("  |grad - central differences|", dev, "4 se", 4 * se)
    assert np.all(dev <= 4 * se + 1e-3 * np.linalg.norm(fd))
    ld_se = orc["logdet_stderr"]
    say("  log det vs dense", res["logdet"], gold["logdet"], "4 se", 4 * ld_se)
    assert abs(res["logdet"] - gold["logdet"]) <= 4 * ld_se + 1e-3 * abs(gold["logdet"])
