"""Bayesian optimisation with derivatives and active subspace learning
(Alg. 1, Sec. 3.4 and Sec. 4.4).

Each iteration of the loop:
  1. the active subspace of the gradients seen so far (dski_active_subspace):
     the k dominant eigenvectors of C = (1/n) sum g g^T, and P = k_dir random
     orthonormal directions inside it (the paper fixes d = 2 and picks two
     directions of the estimated subspace at random);
  2. the reduced data u_i = P^T x_i with values f_i and gradients P^T g_i
     (dski_active_project), and a D-SKI model on a grid over the reduced
     search box, its hyper-parameters refitted by a few L-BFGS-B steps on the
     marginal likelihood and its gradient (mll_and_grad);
  3. the expected improvement maximised over the reduced search space: EI of a
     seeded uniform candidate set (posterior mean by dski_predict, predictive
     variance by dski_predict_var with a full-rank pivoted-Cholesky
     preconditioner, EI by dski_expected_improvement), then refined by
     shrinking clouds of candidates around the best one;
  4. x = P u of the best candidate is sampled (value and gradient) and added
     to the data.

Readings of points the paper leaves open:
* The search box in x is the given domain box; a reduced candidate u is kept
  only if x = P u lies in that box (the reduced search space is the preimage
  of the box, sampled by rejection from its bounding box, which interval
  arithmetic gives exactly for each u_j = P_:j^T x).
* The GP grid covers the reduced search box and the reduced data with a
  margin of one cell; its hyper-parameters start from moment matching
  (s = std f, ell = s / rms(reduced gradient)) on the first iteration and
  from the previous fit afterwards.
* EI is maximised with the plain criterion (xi = 0 unless given); the
  refinement keeps the best point found (so it never loses EI).

This module orchestrates library calls and small host steps (the random
directions, the feasibility test of candidates, L-BFGS-B over the d + 3 log
hyper-parameters); every GP computation runs in the library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import torch

from . import dski


@dataclass
class BOStep:
    P: np.ndarray
    u: np.ndarray
    x: np.ndarray
    f: float
    ei: float
    theta: np.ndarray
    seconds: float


@dataclass
class BOResult:
    X: np.ndarray
    f: np.ndarray
    G: np.ndarray
    steps: List[BOStep] = field(default_factory=list)

    @property
    def best_f(self) -> float:
        return float(self.f.min())

    @property
    def best_x(self) -> np.ndarray:
        return self.X[int(np.argmin(self.f))]


def _reduced_box(P, lo, hi):
    """Exact range of u_j = P[:, j]^T x over the box lo <= x <= hi."""
    a = P * lo[:, None]
    b = P * hi[:, None]
    return np.minimum(a, b).sum(axis=0), np.maximum(a, b).sum(axis=0)


def _feasible(P, U, lo, hi, tol=1e-12):
    X = U @ P.T
    return np.all((X >= lo - tol) & (X <= hi + tol), axis=1)


def _candidates(rng, P, ulo, uhi, lo, hi, count, center=None, half=None, max_draws=64):
    """Up to `count` feasible reduced points, uniform in [ulo, uhi] (or in the
    box center +- half clipped to it)."""
    d = P.shape[1]
    if center is not None:
        blo = np.maximum(ulo, center - half)
        bhi = np.minimum(uhi, center + half)
    else:
        blo, bhi = ulo, uhi
    keep = []
    got = 0
    for _ in range(max_draws):
        U = blo + (bhi - blo) * rng.random((4 * count, d))
        U = U[_feasible(P, U, lo, hi)]
        keep.append(U)
        got += U.shape[0]
        if got >= count:
            break
    U = np.concatenate(keep)[:count] if keep else np.zeros((0, d))
    return U


def run_alg1(objective: Callable[[np.ndarray], tuple], X0: np.ndarray, lo, hi, iters: int, d: int = 2,
             k_active: Optional[int] = None, grid: int = 30, seed: int = 0, xi: float = 0.0, n_cand: int = 4096,
             n_local: int = 512, rounds: int = 3, fit_evals: int = 8, tol: float = 1e-8,
             probe_seed: int = 0x181012283) -> BOResult:
    """Run `iters` iterations of Alg. 1 from the initial design X0 (n0 x D).

    objective(x) -> (f, grad) for one point x (D,).  lo, hi: the domain box.
    d: dimension of the reduced space; k_active (>= d): dimension of the
    estimated active subspace the d directions are drawn from (default d)."""
    from scipy.optimize import minimize

    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    X = np.array(X0, dtype=np.float64)
    D = X.shape[1]
    vals = [objective(x) for x in X]
    f = np.array([v[0] for v in vals], dtype=np.float64)
    G = np.array([np.asarray(v[1], dtype=np.float64) for v in vals])
    k_active = d if k_active is None else int(k_active)
    rng = np.random.default_rng(seed)
    res = BOResult(X, f, G)
    theta = None
    for it in range(iters):
        t0 = time.perf_counter()
        n = X.shape[0]
        Xd = torch.tensor(X, device="cuda")
        Gd = torch.tensor(np.ascontiguousarray(G.T), device="cuda")
        # 1. active subspace and the d directions of this iteration
        Pa, _ = dski.active_subspace(Gd, k_active)
        if k_active > d:
            Qr, _ = np.linalg.qr(rng.standard_normal((k_active, d)))
            P = Pa @ Qr
        else:
            P = Pa
        # 2. reduced data and the D-SKI model over the reduced search box
        U, Gu = dski.active_project(Xd, Gd, P)
        ulo, uhi = _reduced_box(P, lo, hi)
        Uh = U.cpu().numpy()
        blo = np.minimum(ulo, Uh.min(axis=0))
        bhi = np.maximum(uhi, Uh.max(axis=0))
        h = (bhi - blo) / (grid - 3)
        blo, bhi = blo - h, bhi + h
        plan = dski.Plan(U.contiguous(), [grid] * d, blo, bhi)
        y = np.concatenate([f, Gu.cpu().numpy().reshape(-1)])
        yd = torch.tensor(y, device="cuda")[None, :]
        if theta is None:
            s0 = max(float(np.std(f)), 1e-3)
            gr = float(np.sqrt(np.mean(Gu.cpu().numpy() ** 2))) or 1.0
            ell0 = min(max(s0 / gr, 2.0 * float(h.max())), float((bhi - blo).max()))
            theta = np.concatenate([np.log(np.full(d, ell0)), [math.log(s0), math.log(1e-3 * s0),
                                                               math.log(1e-3 * gr)]])
        N = n * (d + 1)
        k = min(N, 256)
        s_log = theta[d]
        # noise levels at least 1e-4 of s: below that K~ is numerically singular
        # for smooth targets that the model can interpolate
        hlo = np.concatenate([np.log(np.full(d, 2.0 * float(h.max()))),
                              [s_log - 5.0, s_log + math.log(1e-4), s_log + math.log(1e-4)]])
        hhi = np.concatenate([np.log(np.full(d, 10.0 * float((bhi - blo).max()))), [s_log + 5.0,
                                                                                     s_log + 2.0, s_log + 2.0]])
        theta = np.clip(theta, hlo, hhi)

        def neg_mll(th):
            plan.set_hypers(th[:d], th[d], th[d + 1], th[d + 2])
            try:
                r = plan.mll_and_grad(yd, None, k=k, num_probes=8, seed=probe_seed, tol=tol, max_iter=20000)
            except dski.DSKIError as e:
                if e.status != -4:  # only a CG breakdown (numerically singular K~) is a rejected step
                    raise
                return 1e300, np.zeros_like(th)
            # scaled by 1/N: in nats the first L-BFGS-B step would land on the bounds
            return -r["mll"] / N, -np.asarray(r["grad"]) / N

        if fit_evals > 0:
            opt = minimize(neg_mll, theta, jac=True, method="L-BFGS-B", bounds=list(zip(hlo, hhi)),
                           options={"maxfun": fit_evals})
            theta = opt.x
        plan.set_hypers(theta[:d], theta[d], theta[d + 1], theta[d + 2])
        pc = plan.pivchol(k)
        alpha, _, _, _, _ = plan.pcg(yd, pc, tol=tol, max_iter=20000)
        g = plan.predict_grid(alpha[0].contiguous())
        f_best = float(f.min())

        def ei_of(Uc):
            Ut = torch.tensor(Uc, device="cuda")
            mu = plan.predict(g, Ut)
            var = plan.predict_var(pc, Ut)
            return dski.expected_improvement(mu, var, f_best, xi)

        # 3. EI over the reduced search space, then shrinking local clouds
        Uc = _candidates(rng, P, ulo, uhi, lo, hi, n_cand)
        if Uc.shape[0] == 0:
            raise RuntimeError("no feasible candidate in the reduced search space")
        _, j, best_ei = ei_of(Uc)
        u_best = Uc[j]
        half = 0.25 * (uhi - ulo)
        for _ in range(rounds):
            Ul = _candidates(rng, P, ulo, uhi, lo, hi, n_local, center=u_best, half=half)
            if Ul.shape[0] > 0:
                Ul = np.concatenate([u_best[None, :], Ul])
                _, j, e = ei_of(Ul)
                if e > best_ei:
                    best_ei, u_best = e, Ul[j]
            half = 0.5 * half
        # 4. sample x = P u and update the data
        x_new = P @ u_best
        f_new, g_new = objective(x_new)
        X = np.vstack([X, x_new])
        f = np.append(f, float(f_new))
        G = np.vstack([G, np.asarray(g_new, dtype=np.float64)])
        pc.close()
        plan.close()
        torch.cuda.synchronize()
        res.steps.append(BOStep(P, u_best, x_new, float(f_new), float(best_ei), theta.copy(),
                                time.perf_counter() - t0))
        res.X, res.f, res.G = X, f, G
    return res
