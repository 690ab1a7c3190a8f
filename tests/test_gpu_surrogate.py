"""The learned log-det surrogate end to end on a reduced terrain problem
(n = 2,000, 60 x 60 grid, 64 training points within 0.5 log-units): training targets from the device SLQ, training with
the device Adam kernels, accuracy on fresh Sobol points, and an L-BFGS fit
with the surrogate (SLQ re-check every 10 evaluations, fall-back above 1e-3),
bounded to the trained region, against the same fit with plain SLQ: equal final marginal likelihood within
1e-3 relative, and what the surrogate saves per evaluation."""
import time

import numpy as np
import pytest
import torch

import workloads
from tests.gpu_common import SEED, need_gpu, say

pytestmark = pytest.mark.gpu


def test_surrogate_trains_and_drives_the_fit():
    dski = need_gpu()
    from paper_1810_12283_amd import surrogate as sg
    W = workloads.terrain(n=2000, grid=60)
    say("surrogate terrain", W.n, W.grid_m)
    plan = dski.Plan(torch.tensor(W.X, device="cuda"), W.grid_m, W.lo, W.hi)
    th_star = np.concatenate([W.log_ell, [W.log_s, W.log_sigma_f, W.log_sigma_g]])
    k, t, tol = 30, 16, 1e-4
    h = np.array(plan.h)
    thetas = sg.sobol_design(th_star, 64, 0.5, seed=4, ell_min=3.0 * h)
    t0 = time.perf_counter()
    T, G = sg.training_data(plan, thetas, k, t, SEED, tol,
                            progress=lambda i, v: say("  sample", i, v, round(time.perf_counter() - t0, 2)) if i % 8 == 0 else None)
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    S = sg.train(thetas, T, G, W.n, h, steps=3000, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    say("  data", round(t_data, 2), "s  train", round(t_train, 2), "s  loss", S.history[0][1], "->", S.history[-1][1])
    assert S.history[-1][1] < 0.05 * S.history[0][1]
    # accuracy on fresh points (different Sobol seed)
    test_th = sg.sobol_design(th_star, 8, 0.4, seed=99, ell_min=3.0 * h)
    errs = []
    for th in test_th:
        ld, _ = sg.logdet_and_grad(plan, th, k, t, SEED, tol)
        ls, _ = S(th)
        errs.append(abs(ls - ld) / abs(ld))
    say("  held-out relative log det error: median", np.median(errs), "max", max(errs))
    assert np.median(errs) < 2e-2
    # fits from the same start
    y = torch.tensor(W.y.astype(np.float32), device="cuda")[None, :].contiguous()
    theta0 = th_star + 0.2
    box = [(a - 0.45, a + 0.45) for a in th_star]  # inside the trained region
    plain = sg.fit(plan, y, theta0, k, t, SEED, tol, surrogate=None, max_evals=40, bounds=box)
    say("  plain fit done", round(plain.seconds, 2))
    withs = sg.fit(plan, y, theta0, k, t, SEED, tol, surrogate=S, max_evals=40, bounds=box)
    say("  plain: mll", plain.mll, "evals", plain.evals, "s", round(plain.seconds, 2))
    say("  surrogate: mll", withs.mll, "evals", withs.evals, "s", round(withs.seconds, 2), "fell back", withs.fell_back,
        "rechecks", withs.rechecks)
    assert withs.mll == pytest.approx(plain.mll, rel=1e-3)
    assert withs.rechecks, "the surrogate fit re-checks with SLQ"
    # the evaluation the surrogate replaces: SLQ (data + 16 probes) vs data-fit only
    th = th_star
    t0 = time.perf_counter()
    sg.logdet_and_grad(plan, th, k, t, SEED, tol)
    torch.cuda.synchronize()
    t_slq = time.perf_counter() - t0
    t0 = time.perf_counter()
    sg.data_fit_and_grad(plan, th, y, k, tol)
    S(th)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    say("  per evaluation: SLQ", round(t_slq, 4), "s, data fit + network", round(t_sur, 4), "s")
    assert t_sur < t_slq
