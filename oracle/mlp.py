"""FP64 reference of the learned log-determinant surrogate (TEST INFRASTRUCTURE).

The network maps standardised hyper-parameter features x (F = 8) to the
standardised value of log det(K~)/n:
    a1 = W1 x + b1,  h1 = gelu(a1)            (H1 = 128)
    a2 = W2 h1 + b2, h2 = gelu(a2)            (H2 = 128)
    y  = w3 . h2 + b3
with the exact GELU, gelu(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2.

Its derivative with respect to the first J inputs (the log hyper-parameters)
comes from forward-mode tangent propagation along the unit directions e_j:
    da1_j = W1 e_j,  dh1_j = gelu'(a1) * da1_j,  da2_j = W2 dh1_j,
    dh2_j = gelu'(a2) * da2_j,  dy_j = w3 . dh2_j.
Training loss over a batch of B samples (value and gradient matching, weight
lam on the gradient term):
    loss = (1/B) sum_b [(y_b - t_b)^2 + lam sum_j (dy_bj - g_bj)^2],
whose weight gradient needs gelu'' through the tangent path (`backward`).

The paper does not describe this component; the design (architecture, loss,
GELU form) is this project's and is pinned here by central differences.
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / SQRT2))


def gelu_d1(a):
    """d/da [a Phi(a)] = Phi(a) + a phi(a)."""
    return 0.5 * (1.0 + erf(a / SQRT2)) + a * INV_SQRT_2PI * np.exp(-0.5 * a * a)


def gelu_d2(a):
    """d^2/da^2 [a Phi(a)] = phi(a) (2 - a^2)."""
    return INV_SQRT_2PI * np.exp(-0.5 * a * a) * (2.0 - a * a)


def init(F=8, H1=128, H2=128, seed=0):
    """He-style normal initialisation (FP64); b = 0."""
    r = np.random.default_rng(seed)
    return {
        "W1": r.standard_normal((H1, F)) * math.sqrt(2.0 / F),
        "b1": np.zeros(H1),
        "W2": r.standard_normal((H2, H1)) * math.sqrt(2.0 / H1),
        "b2": np.zeros(H2),
        "w3": r.standard_normal(H2) * math.sqrt(1.0 / H2),
        "b3": np.zeros(1),
    }


def forward(P, X, J=5):
    """X: B x F.  Returns (y (B,), dy (B, J), cache)."""
    a1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(a2)
    y = h2 @ P["w3"] + P["b3"][0]
    g1, g2 = gelu_d1(a1), gelu_d1(a2)
    da1 = P["W1"][:, :J].T[None, :, :]               # 1 x J x H1 (W1 e_j)
    dh1 = g1[:, None, :] * da1                        # B x J x H1
    da2 = dh1 @ P["W2"].T                             # B x J x H2
    dh2 = g2[:, None, :] * da2
    dy = dh2 @ P["w3"]                                # B x J
    cache = dict(X=X, a1=a1, h1=h1, a2=a2, h2=h2, g1=g1, g2=g2, da1=np.broadcast_to(da1, dh1.shape),
                 dh1=dh1, da2=da2, dh2=dh2)
    return y, dy, cache


def loss(P, X, t, g, lam=1.0):
    y, dy, _ = forward(P, X, g.shape[1])
    B = X.shape[0]
    return (np.sum((y - t) ** 2) + lam * np.sum((dy - g) ** 2)) / B


def backward(P, X, t, g, lam=1.0):
    """Gradient of `loss` with respect to every parameter (same keys as P)."""
    J = g.shape[1]
    y, dy, c = forward(P, X, J)
    B = X.shape[0]
    ey = 2.0 * (y - t) / B                            # B
    eg = 2.0 * lam * (dy - g) / B                     # B x J
    G = {}
    # output layer
    G["w3"] = ey @ c["h2"] + np.einsum("bj,bjh->h", eg, c["dh2"])
    G["b3"] = np.array([ey.sum()])
    dh2 = ey[:, None] * P["w3"][None, :]              # B x H2
    ddh2 = eg[:, :, None] * P["w3"][None, None, :]     # B x J x H2
    # second layer
    dda2 = ddh2 * c["g2"][:, None, :]
    da2 = dh2 * c["g2"] + np.sum(ddh2 * gelu_d2(c["a2"])[:, None, :] * c["da2"], axis=1)
    G["W2"] = da2.T @ c["h1"] + np.einsum("bjh,bjl->hl", dda2, c["dh1"])
    G["b2"] = da2.sum(axis=0)
    dh1 = da2 @ P["W2"]
    ddh1 = dda2 @ P["W2"]                             # B x J x H1
    # first layer
    dda1 = ddh1 * c["g1"][:, None, :]
    da1 = dh1 * c["g1"] + np.sum(ddh1 * gelu_d2(c["a1"])[:, None, :] * c["da1"], axis=1)
    G["W1"] = da1.T @ X
    G["W1"][:, :J] += np.sum(dda1, axis=0).T
    G["b1"] = da1.sum(axis=0)
    return G


def adam_step(P, G, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in place; state holds m, v and t."""
    state["t"] = state.get("t", 0) + 1
    tt = state["t"]
    for key in P:
        m = state.setdefault("m_" + key, np.zeros_like(P[key]))
        v = state.setdefault("v_" + key, np.zeros_like(P[key]))
        m *= beta1
        m += (1.0 - beta1) * G[key]
        v *= beta2
        v += (1.0 - beta2) * G[key] ** 2
        mh = m / (1.0 - beta1 ** tt)
        vh = v / (1.0 - beta2 ** tt)
        P[key] -= lr * mh / (np.sqrt(vh) + eps)
