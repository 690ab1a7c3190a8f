"""Learned log-determinant surrogate and the hyper-parameter fit that uses it.

The network (``dski.Mlp``, FP32, trained and evaluated by the device kernels
behind ``mlp_*``) maps standardised features
    [log ell_1 .. log ell_d, log s, log sigma_f, log sigma_g, log n, log h_1 .. log h_d]
to the standardised value of log det(K~) / n, and its input tangents give the
gradient with respect to the d + 3 log hyper-parameters.  Training targets come
from the method itself: the SLQ log determinant and its stochastic trace
gradient (``mll_and_grad`` with a zero data vector, so only the log det terms
remain).  During a fit the data-fit part (one PCG column, ``mll_and_grad``
with zero probes) is exact and the log det comes from the network; every
``recheck`` evaluations SLQ re-computes the log det, and when the relative
error exceeds ``fallback_tol`` L-BFGS restarts from that point on plain SLQ.

This module only orchestrates device calls (and the 5-parameter L-BFGS on the
host); every numerical step of the method runs in the library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import dski

LOG2PI = math.log(2.0 * math.pi)


def logdet_and_grad(plan: dski.Plan, theta: np.ndarray, k: int, num_probes: int, seed: int, tol: float,
                    max_iter: int = 20000, info: Optional[dict] = None):
    """SLQ log det K~ and its gradient (d + 3 log hyper-parameters) at theta;
    `info` (a dict) receives the PCG iterations per column and the status."""
    d = plan.d
    plan.set_hypers(theta[:d], theta[d], theta[d + 1], theta[d + 2])
    zero = torch.zeros((1, plan.N), dtype=torch.float32, device="cuda")
    res = plan.mll_and_grad(zero, None, k=k, num_probes=num_probes, seed=seed, tol=tol, max_iter=max_iter)
    if info is not None:
        info["iters"] = res["iters"]
        info["status"] = res["status"]
    # with y = 0: mll = -(log det + N log 2 pi) / 2, grad = -(d log det) / 2
    return res["logdet"], -2.0 * np.asarray(res["grad"])


def _mll(plan: dski.Plan, y: torch.Tensor, k: int, num_probes: int, seed: int, tol: float, max_iter: int,
         warm: Optional[dict]):
    """mll_and_grad; with `warm` (a dict) the data solve starts from warm["alpha"]
    when present, and warm["alpha"] receives the new alpha (FP32 y only)."""
    if warm is None or y.dtype != torch.float32:
        return plan.mll_and_grad(y, None, k=k, num_probes=num_probes, seed=seed, tol=tol, max_iter=max_iter)
    res = plan.mll_and_grad(y, None, k=k, num_probes=num_probes, seed=seed, tol=tol, max_iter=max_iter,
                            x0=warm.get("alpha"), want_alpha=True)
    warm["alpha"] = res["alpha"]
    warm["iters"] = warm.get("iters", 0) + res["iters"][0]
    return res


def data_fit_and_grad(plan: dski.Plan, theta: np.ndarray, y: torch.Tensor, k: int, tol: float,
                      max_iter: int = 20000, warm: Optional[dict] = None):
    """-y^T K~^{-1} y / 2 - N log(2 pi) / 2 and its gradient (one PCG column),
    warm-started as in _mll when `warm` is given."""
    d = plan.d
    plan.set_hypers(theta[:d], theta[d], theta[d + 1], theta[d + 2])
    res = _mll(plan, y, k, 0, 0, tol, max_iter, warm)
    return res["mll"], np.asarray(res["grad"])


@dataclass
class Surrogate:
    net: dski.Mlp
    mu_x: np.ndarray
    sd_x: np.ndarray
    mu_t: float
    sd_t: float
    n: int
    const_feats: np.ndarray          # log n, log h_1 .. log h_d
    history: list = field(default_factory=list)

    def features(self, theta: np.ndarray) -> np.ndarray:
        return np.concatenate([np.asarray(theta, dtype=np.float64), self.const_feats])

    def __call__(self, theta: np.ndarray):
        """(log det, d log det / d theta) from the network."""
        x = (self.features(theta) - self.mu_x) / self.sd_x
        X = torch.tensor(x[None, :], dtype=torch.float32, device="cuda")
        y, dy = self.net.jvp(X)
        J = len(theta)
        val = self.n * (self.mu_t + self.sd_t * float(y[0]))
        grad = self.n * self.sd_t * dy[0, :J].double().cpu().numpy() / self.sd_x[:J]
        return val, grad


def sobol_design(theta_star: np.ndarray, m: int, radius: float, seed: int, ell_min: Optional[np.ndarray] = None):
    from scipy.stats import qmc
    u = qmc.Sobol(d=len(theta_star), scramble=True, seed=seed).random(m)
    th = theta_star[None, :] + radius * (2.0 * u - 1.0)
    if ell_min is not None:
        d = len(ell_min)
        th[:, :d] = np.maximum(th[:, :d], np.log(ell_min)[None, :])
    return th


def training_data(plan: dski.Plan, thetas: np.ndarray, k: int, num_probes: int, seed: int, tol: float,
                  max_iter: int = 20000, progress=None):
    T = np.empty(len(thetas))
    G = np.empty_like(thetas)
    for i, th in enumerate(thetas):
        T[i], G[i] = logdet_and_grad(plan, th, k, num_probes, seed, tol, max_iter)
        if progress:
            progress(i, T[i])
    return T, G


def train(thetas: np.ndarray, logdets: np.ndarray, grads: np.ndarray, n: int, h: np.ndarray, steps: int = 2000,
          lr: float = 2e-3, lam: float = 1.0, hidden: int = 128, seed: int = 0,
          lr_final: Optional[float] = None) -> Surrogate:
    """Fit the network to log det / n and its gradient with full-batch Adam on
    the device; the step size decays geometrically from lr to lr_final (if given)."""
    J = thetas.shape[1]
    const = np.concatenate([[math.log(n)], np.log(h)])
    Xf = np.concatenate([thetas, np.repeat(const[None, :], len(thetas), axis=0)], axis=1)
    F = Xf.shape[1]
    mu_x = Xf.mean(axis=0)
    sd_x = Xf.std(axis=0)
    sd_x[sd_x == 0] = 1.0
    t = logdets / n
    mu_t, sd_t = float(t.mean()), float(t.std() or 1.0)
    X = (Xf - mu_x) / sd_x
    ts = (t - mu_t) / sd_t
    gs = (grads / n) * sd_x[None, :J] / sd_t
    r = np.random.default_rng(seed)
    W1 = r.standard_normal((hidden, F)) * math.sqrt(2.0 / F)
    W2 = r.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden)
    w3 = r.standard_normal(hidden) * math.sqrt(1.0 / hidden)
    net = dski.Mlp(dski.Mlp.pack(W1, np.zeros(hidden), W2, np.zeros(hidden), w3, np.zeros(1)), F=F, H=hidden, J=J)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(ts, dtype=torch.float32, device="cuda")
    gd = torch.tensor(gs, dtype=torch.float32, device="cuda")
    hist = []
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1)) if lr_final else 1.0
    for s in range(steps):
        loss = net.backward(Xd, td, gd, lam)
        net.step(lr=lr * decay ** s)
        if s % 100 == 0 or s == steps - 1:
            hist.append((s, loss))
    return Surrogate(net, mu_x, sd_x, mu_t, sd_t, n, const, hist)


@dataclass
class FitResult:
    theta: np.ndarray
    mll: float
    evals: int
    seconds: float
    fell_back: bool
    rechecks: list
    data_iters: int = 0               # PCG iterations of the data column over all evaluations


def fit(plan: dski.Plan, y: torch.Tensor, theta0: np.ndarray, k: int, num_probes: int, seed: int, tol: float,
        surrogate: Optional[Surrogate] = None, recheck: int = 10, fallback_tol: float = 1e-3,
        max_evals: int = 60, gtol: float = 1e-5, bounds=None, warm: bool = True) -> FitResult:
    """Maximise the marginal likelihood over the log hyper-parameters with L-BFGS.

    With a surrogate: mll = data-fit part (exact) - log det (network) / 2, with
    SLQ re-checks every `recheck` evaluations and at the point where the search
    ends, and a fall-back to plain SLQ (L-BFGS restarted from that point) when
    the relative log det error exceeds `fallback_tol`.  `bounds` (a list of
    (lo, hi) per log hyper-parameter) keeps the search inside the region the
    surrogate was trained on.  `warm` starts each evaluation's data solve from
    the previous evaluation's alpha (FP32 y)."""
    from scipy.optimize import minimize

    state = {"evals": 0, "fallback": surrogate is None, "rechecks": []}
    wst = {} if warm else None
    t0 = time.perf_counter()
    d = plan.d
    # L-BFGS-B sees -mll / N: in nats the gradient is O(N) and the first
    # projected step would land on the bounds
    inv_n = 1.0 / plan.N

    class _FallBack(Exception):
        """Raised by a failed re-check: L-BFGS-B's curvature pairs and line
        search were built on the surrogate, so the search restarts from this
        point on plain SLQ instead of switching functions in mid-run."""

        def __init__(self, theta):
            super().__init__()
            self.theta = theta

    def slq_objective(theta):
        state["evals"] += 1
        plan.set_hypers(theta[:d], theta[d], theta[d + 1], theta[d + 2])
        res = _mll(plan, y, k, num_probes, seed, tol, 20000, wst)
        return -res["mll"] * inv_n, -np.asarray(res["grad"]) * inv_n

    def surrogate_objective(theta):
        state["evals"] += 1
        dfit, dgrad = data_fit_and_grad(plan, theta, y, k, tol, warm=wst)
        ld, ldg = surrogate(theta)
        if state["evals"] % recheck == 0:
            ld_slq, ldg_slq = logdet_and_grad(plan, theta, k, num_probes, seed, tol)
            err = abs(ld - ld_slq) / abs(ld_slq)
            state["rechecks"].append((state["evals"], ld, ld_slq, err))
            if err > fallback_tol:
                state["fallback"] = True
                raise _FallBack(np.array(theta, dtype=np.float64))
            # the re-check's own value and gradient are the better ones here
            ld, ldg = ld_slq, ldg_slq
        mll = dfit - 0.5 * ld
        grad = dgrad - 0.5 * ldg
        return -mll * inv_n, -grad * inv_n

    theta = np.asarray(theta0, dtype=np.float64)
    res = None
    if not state["fallback"]:
        try:
            res = minimize(surrogate_objective, theta, jac=True, method="L-BFGS-B", bounds=bounds,
                           options={"maxfun": max_evals, "gtol": gtol})
            # the search may end between re-checks: its end point is re-checked too
            ld_net, _ = surrogate(res.x)
            ld_slq, _ = logdet_and_grad(plan, res.x, k, num_probes, seed, tol)
            err = abs(ld_net - ld_slq) / abs(ld_slq)
            state["rechecks"].append((state["evals"], ld_net, ld_slq, err))
            if err > fallback_tol:
                state["fallback"] = True
                theta = np.array(res.x, dtype=np.float64)
                res = None
        except _FallBack as fb:
            theta = fb.theta
    if res is None:
        res = minimize(slq_objective, theta, jac=True, method="L-BFGS-B", bounds=bounds,
                       options={"maxfun": max(1, max_evals - state["evals"]), "gtol": gtol})
    # final value with the full method at the optimum
    th = res.x
    plan.set_hypers(th[:d], th[d], th[d + 1], th[d + 2])
    final = plan.mll_and_grad(y, None, k=k, num_probes=num_probes, seed=seed, tol=tol, max_iter=20000)
    torch.cuda.synchronize()
    return FitResult(th, final["mll"], state["evals"], time.perf_counter() - t0, state["fallback"],
                     state["rechecks"], (wst or {}).get("iters", 0))
