"""Pins of the FP64 surrogate network (oracle/mlp.py): GELU against its
definition and central differences, the tangent outputs against central
differences of the forward pass, and the weight gradient of the
value-and-gradient loss against central differences on every parameter."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_definition_and_derivatives():
    a = np.linspace(-6, 6, 241)
    ref = np.array([0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))) for v in a])
    np.testing.assert_allclose(mlp.gelu(a), ref, rtol=1e-15, atol=1e-300)
    h = 1e-5
    np.testing.assert_allclose(mlp.gelu_d1(a), (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h), atol=1e-9)
    np.testing.assert_allclose(mlp.gelu_d2(a), (mlp.gelu_d1(a + h) - mlp.gelu_d1(a - h)) / (2 * h), atol=1e-9)
    # special values: gelu(0) = 0, gelu'(0) = 1/2, gelu''(0) = 2 phi(0)
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert mlp.gelu_d1(np.array(0.0)) == 0.5
    assert mlp.gelu_d2(np.array(0.0)) == pytest.approx(2.0 / math.sqrt(2 * math.pi), rel=1e-15)


def test_tangents_are_input_derivatives():
    P = mlp.init(seed=1)
    X = np.random.default_rng(2).standard_normal((6, 8))
    y, dy, _ = mlp.forward(P, X, J=5)
    h = 1e-5
    for j in range(5):
        E = np.zeros(8)
        E[j] = h
        yp, _, _ = mlp.forward(P, X + E, J=5)
        ym, _, _ = mlp.forward(P, X - E, J=5)
        np.testing.assert_allclose(dy[:, j], (yp - ym) / (2 * h), rtol=1e-7, atol=1e-9)


def test_backward_matches_central_differences_on_every_weight():
    r = np.random.default_rng(3)
    P = mlp.init(seed=4)
    for k in P:  # non-zero biases so that every term is exercised
        P[k] = P[k] + 0.1 * r.standard_normal(P[k].shape)
    X = r.standard_normal((4, 8))
    t = r.standard_normal(4)
    g = r.standard_normal((4, 5))
    G = mlp.backward(P, X, t, g, lam=0.7)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        fd = np.empty_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(P, X, t, g, lam=0.7)
            flat[i] = old - h
            lm = mlp.loss(P, X, t, g, lam=0.7)
            flat[i] = old
            fd[i] = (lp - lm) / (2 * h)
        err = np.abs(G[k].reshape(-1) - fd).max() / max(np.abs(fd).max(), 1e-12)
        assert err < 1e-6, (k, err)


def test_adam_first_step_moves_by_lr():
    P = {"w": np.array([1.0, -2.0])}
    G = {"w": np.array([0.3, -5.0])}
    mlp.adam_step(P, G, {}, lr=0.01)
    # with bias correction the first step is lr * sign(g) (up to eps)
    np.testing.assert_allclose(P["w"], [1.0 - 0.01, -2.0 + 0.01], rtol=1e-7)


def test_adam_two_steps_hand_computed():
    """Two Adam steps worked out by hand with beta1 = 0.5, beta2 = 0.75,
    eps = 0 (Kingma & Ba 2015, Alg. 1), where a wrong decay or bias-correction
    exponent changes the second step (the first is lr * sign(g) whatever the
    betas):
      t = 1: m = 0.25, v = 0.0625, m^ = 0.5, v^ = 0.25, step 0.1  -> 0.9
      t = 2: m = -0.375, v = 0.296875, m^ = -0.5, v^ = 19/28,
             step -0.1 * 0.5 / sqrt(19/28) = -0.0606976979 -> 0.9606976979"""
    P = {"w": np.array([1.0])}
    state = {}
    mlp.adam_step(P, {"w": np.array([0.5])}, state, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    np.testing.assert_allclose(P["w"], [0.9], rtol=1e-15)
    mlp.adam_step(P, {"w": np.array([-1.0])}, state, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    np.testing.assert_allclose(P["w"], [0.9606976978666885], rtol=1e-14)
    np.testing.assert_allclose(state["m_w"], [-0.375], rtol=1e-15)
    np.testing.assert_allclose(state["v_w"], [0.296875], rtol=1e-15)
