"""Seeded synthetic workloads for GP regression with derivatives.

This module only *draws inputs*: point sets, test functions with their exact
gradients, observation noise and the hyper-parameters a workload is run at.
It holds none of the method's arithmetic (no interpolation weights, no kernel
matrices, no solvers), so both the FP64 oracle and the GPU path can consume
the same inputs without sharing any code of the method.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) with a fixed
draw order, and returns a :class:`Workload` in FP64.  The GPU side casts to
FP32 itself.

Workloads (sizes follow the paper's experiment families, Sec. 4):

* ``small2d``   – n=500 on [0,1]^2, sum of 8 random sinusoids; 50x50 grid.
* ``terrain``   – n=20,000 on [0,1]^2, 64 random Fourier modes with a
                  |k|^-1.5 spectrum (stands in for the LiDAR terrain of
                  Sec. 4.2); 200x200 grid.
* ``torus``     – n=30,000 points on a perturbed torus with unit outward
                  normals as gradients and value 0 (stands in for the
                  implicit-surface experiment of Sec. 4.3); 48^3 grid.
* ``ridge8d``   – n=4,000 on [-1,1]^8, sum of 16 tanh ridge functions
                  (high-dimensional D-SKIP case of Sec. 3.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "Workload",
    "small2d",
    "terrain",
    "torus",
    "ridge8d",
    "by_name",
    "block_vector",
    "embedded_objective",
]


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray            # n x d, FP64, row-major
    f: np.ndarray            # n   noise-free values
    grad: np.ndarray         # n x d noise-free gradients
    y: np.ndarray            # N = n(d+1) observed block vector [f; d1 f; ...; dd f]
    log_ell: np.ndarray      # d natural-log length scales
    log_s: float             # natural-log signal scale
    log_sigma_f: float       # natural-log value-noise std
    log_sigma_g: float       # natural-log gradient-noise std
    grid_m: Optional[Sequence[int]]  # grid nodes per axis (None for grid-free operators)
    lo: np.ndarray           # data box lower corner (d,)
    hi: np.ndarray           # data box upper corner (d,)
    rank: int                # pivoted-Cholesky rank
    tol: float               # PCG relative residual tolerance
    num_probes: int          # Hutchinson probes
    lanczos_steps: int       # 0 = derive the quadrature from PCG to tolerance
    seed: int
    skip_m: int = 0          # D-SKIP: 1-D grid nodes per axis (0: not a D-SKIP workload)
    skip_rank: int = 0       # D-SKIP: Lanczos rank of every factor

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def N(self) -> int:
        return self.n * (self.d + 1)

    def hypers(self):
        return (np.array(self.log_ell, dtype=np.float64), float(self.log_s),
                float(self.log_sigma_f), float(self.log_sigma_g))


def block_vector(f: np.ndarray, grad: np.ndarray) -> np.ndarray:
    """Stack values and gradients as [f(x_1..x_n); d1 f(x_1..x_n); ...]."""
    n, d = grad.shape
    out = np.empty(n * (d + 1), dtype=np.float64)
    out[:n] = f
    for p in range(d):
        out[(p + 1) * n:(p + 2) * n] = grad[:, p]
    return out


def _noisy(rng, f, grad, sigma_f, sigma_g):
    n, d = grad.shape
    eps = rng.standard_normal(n * (d + 1))
    y = block_vector(f, grad)
    y[:n] += sigma_f * eps[:n]
    y[n:] += sigma_g * eps[n:]
    return y


def small2d(seed: int = 0, n: int = 500, grid: int = 50) -> Workload:
    """Sum of 8 sinusoids sin(w (cos(phi) x1 + sin(phi) x2) + psi), w~U[1,6]
    rad/unit, phi~U[0,2pi), psi~U[0,2pi); X~U[0,1]^2."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, 2))
    J = 8
    w = rng.uniform(1.0, 6.0, J)
    phi = rng.uniform(0.0, 2 * np.pi, J)
    psi = rng.uniform(0.0, 2 * np.pi, J)
    dirs = np.stack([np.cos(phi), np.sin(phi)], axis=1) * w[:, None]   # J x 2
    arg = X @ dirs.T + psi[None, :]
    f = np.sin(arg).sum(axis=1)
    grad = np.cos(arg) @ dirs
    sf, sg = 0.01, 0.05
    y = _noisy(rng, f, grad, sf, sg)
    return Workload("small2d", X, f, grad, y, np.log([0.2, 0.2]), 0.0,
                    math.log(sf), math.log(sg), [grid, grid], np.zeros(2),
                    np.ones(2), 20, 1e-6, 10, 30, seed)


def _terrain_modes(rng, J=64, kmax=30.0):
    kabs = rng.uniform(1.0, kmax, J)
    ang = rng.uniform(0.0, 2 * np.pi, J)
    psi = rng.uniform(0.0, 2 * np.pi, J)
    kvec = np.stack([np.cos(ang), np.sin(ang)], axis=1) * kabs[:, None]
    amp = kabs ** -1.5
    return kvec, psi, amp


def terrain_height(X, kvec, psi, amp):
    arg = 2 * np.pi * (X @ kvec.T) + psi[None, :]
    h = np.cos(arg) @ amp
    grad = -(np.sin(arg) * amp[None, :]) @ (2 * np.pi * kvec)
    return h, grad


def terrain(seed: int = 1, n: int = 20000, grid: int = 200,
            moment_match_n: Optional[int] = None) -> Workload:
    """Height = sum_j A_j cos(2 pi k_j.x + psi_j), |k_j|~U[1,30] cycles/unit,
    direction U[0,2pi), A_j=|k_j|^-1.5, 64 modes; X~U[0,1]^2.

    Hyper-parameters by moment matching on the noise-free field:
    s = std(h), ell = s / rms(dh/dx_p) (isotropic)."""
    rng = np.random.default_rng(seed)
    kvec, psi, amp = _terrain_modes(rng)
    X = rng.random((n, 2))
    f, grad = terrain_height(X, kvec, psi, amp)
    sf, sg = 0.05, 0.1
    y = _noisy(rng, f, grad, sf, sg)
    # moment matching on a fixed 20,000-point design so that the hyper-
    # parameters do not move with n in scaled-down variants
    mrng = np.random.default_rng(seed + 1000)
    Xm = mrng.random((moment_match_n or 20000, 2))
    fm, gm = terrain_height(Xm, kvec, psi, amp)
    s = float(np.std(fm))
    ell = s / float(np.sqrt(np.mean(gm ** 2)))
    return Workload("terrain", X, f, grad, y, np.log([ell, ell]), math.log(s),
                    math.log(sf), math.log(sg), [grid, grid], np.zeros(2),
                    np.ones(2), 50, 1e-4, 16, 0, seed)


def torus(seed: int = 2, n: int = 30000, grid: int = 48) -> Workload:
    """Perturbed torus R0=0.6, r0=0.25; radius rho(u,v) = r0 (1 + 0.15 sum_j
    a_j cos(m_j u + n_j v + psi_j)/sqrt(32)) with integer m_j, n_j in [0,4];
    value 0 and unit outward normal as gradient."""
    rng = np.random.default_rng(seed)
    J = 32
    mj = rng.integers(0, 5, J)
    nj = rng.integers(0, 5, J)
    aj = rng.standard_normal(J)
    pj = rng.uniform(0.0, 2 * np.pi, J)
    u = rng.uniform(0.0, 2 * np.pi, n)
    v = rng.uniform(0.0, 2 * np.pi, n)
    R0, r0 = 0.6, 0.25
    ph = mj[None, :] * u[:, None] + nj[None, :] * v[:, None] + pj[None, :]
    c = 0.15 / math.sqrt(J)
    rho = r0 * (1.0 + c * (np.cos(ph) @ aj))
    rho_u = r0 * c * (-(np.sin(ph) * mj[None, :]) @ aj)
    rho_v = r0 * c * (-(np.sin(ph) * nj[None, :]) @ aj)
    cu, su, cv, sv = np.cos(u), np.sin(u), np.cos(v), np.sin(v)
    Rr = R0 + rho * cv
    P = np.stack([Rr * cu, Rr * su, rho * sv], axis=1)
    # dP/du and dP/dv
    Pu = np.stack([(rho_u * cv) * cu - Rr * su, (rho_u * cv) * su + Rr * cu, rho_u * sv], axis=1)
    Pv = np.stack([(rho_v * cv - rho * sv) * cu, (rho_v * cv - rho * sv) * su,
                   rho_v * sv + rho * cv], axis=1)
    nrm = np.cross(Pu, Pv)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    # orient outward: away from the tube centre line
    centre = np.stack([R0 * cu, R0 * su, np.zeros(n)], axis=1)
    sgn = np.sign(np.sum(nrm * (P - centre), axis=1))
    sgn[sgn == 0] = 1.0
    nrm *= sgn[:, None]
    f = np.zeros(n)
    sf, sg = 0.01, 0.05
    y = _noisy(rng, f, nrm, sf, sg)
    lo = P.min(axis=0)
    hi = P.max(axis=0)
    return Workload("torus", P, f, nrm, y, np.log([0.2, 0.2, 0.2]), 0.0,
                    math.log(sf), math.log(sg), [grid, grid, grid], lo, hi,
                    50, 1e-4, 16, 0, seed)


def ridge8d(seed: int = 3, n: int = 4000, d: int = 8, skip_m: int = 100, skip_rank: int = 32) -> Workload:
    """f = sum_{j=1}^{16} tanh(a_j.x + b_j), |a_j|~U[0.5,2] along a uniform
    direction, b_j~U[-1,1]; X~U[-1,1]^d.  D-SKIP operator: 1-D grids of
    ``skip_m`` nodes, Lanczos rank ``skip_rank``; pivoted-Cholesky rank 100."""
    rng = np.random.default_rng(seed)
    J = 16
    dirs = rng.standard_normal((J, d))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    A = dirs * rng.uniform(0.5, 2.0, J)[:, None]
    b = rng.uniform(-1.0, 1.0, J)
    X = rng.uniform(-1.0, 1.0, (n, d))
    th = np.tanh(X @ A.T + b[None, :])
    f = th.sum(axis=1)
    grad = (1.0 - th ** 2) @ A
    sf, sg = 0.05, 0.1
    y = _noisy(rng, f, grad, sf, sg)
    return Workload("ridge8d", X, f, grad, y, np.log(np.full(d, 0.5)), 0.0,
                    math.log(sf), math.log(sg), None, -np.ones(d), np.ones(d),
                    100, 1e-4, 16, 0, seed, skip_m, skip_rank)


def by_name(name: str, **kw) -> Workload:
    return {"small2d": small2d, "terrain": terrain, "torus": torus,
            "ridge8d": ridge8d}[name](**kw)



def embedded_objective(kind: str, D: int, d_eff: int, seed: int):
    """A test function of d_eff variables embedded in D dimensions, as the
    Bayesian-optimisation experiment of Sec. 4.4 does (5-D Ackley and
    Rastrigin in [-10, 15]^50 and [-4, 5]^50): f(x) = g(Q^T x) with Q a seeded
    D x d_eff matrix with orthonormal columns.  Returns (objective, lo, hi,
    Q) where objective(x) -> (f, grad f) and [lo, hi] is the domain box.
    kind: "quadratic" (|z - c|^2, c seeded in [-0.3, 0.3]^d_eff, box [-1, 1]^D),
    "ackley" (box [-10, 15]^D) or "rastrigin" (box [-4, 5]^D)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((D, d_eff)))
    if kind == "quadratic":
        c = rng.uniform(-0.3, 0.3, d_eff)
        lo, hi = -np.ones(D), np.ones(D)

        def g(z):
            r = z - c
            return float(r @ r), 2.0 * r
    elif kind == "ackley":
        lo, hi = np.full(D, -10.0), np.full(D, 15.0)

        def g(z):
            k = z.size
            a = math.sqrt(float(z @ z) / k)
            b = float(np.cos(2 * math.pi * z).sum()) / k
            e1, e2 = math.exp(-0.2 * a), math.exp(b)
            val = -20.0 * e1 - e2 + 20.0 + math.e
            ga = (z / (k * a)) if a > 0 else np.zeros_like(z)
            grad = 20.0 * 0.2 * e1 * ga + e2 * (2 * math.pi / k) * np.sin(2 * math.pi * z)
            return val, grad
    elif kind == "rastrigin":
        lo, hi = np.full(D, -4.0), np.full(D, 5.0)

        def g(z):
            val = 10.0 * z.size + float((z * z - 10.0 * np.cos(2 * math.pi * z)).sum())
            grad = 2.0 * z + 20.0 * math.pi * np.sin(2 * math.pi * z)
            return val, grad
    else:
        raise ValueError(kind)

    def objective(x):
        z = Q.T @ np.asarray(x, dtype=np.float64)
        v, gz = g(z)
        return v, Q @ gz

    return objective, lo, hi, Q
