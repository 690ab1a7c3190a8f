"""Pins of the oracle's active subspace (Sec. 3.4): a ridge function whose
gradients span a known plane, the trace identity of C, and the reduced
gradients against finite differences of u -> f(P u)."""
import numpy as np

from oracle import active


def _ridge(D=12, n=400, seed=3):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((D, 2)))
    a, b = Q[:, 0], Q[:, 1]
    X = r.uniform(-1.0, 1.0, (n, D))
    f = lambda x: np.sin(2.0 * x @ a) + 0.5 * (x @ b) ** 2
    G = 2.0 * np.cos(2.0 * X @ a)[:, None] * a[None, :] + (X @ b)[:, None] * b[None, :]
    return X, G, f, a, b


def test_ridge_function_subspace_is_the_span_of_its_directions():
    X, G, f, a, b = _ridge()
    P, lam = active.active_subspace(G, 2)
    Q = np.stack([a, b], axis=1)
    assert np.abs(P @ P.T - Q @ Q.T).max() < 1e-12
    assert np.abs(P.T @ P - np.eye(2)).max() < 1e-12
    assert lam[1] > 1e-3 and np.abs(lam[2:]).max() < 1e-13 * lam[0]
    assert (np.diff(lam) <= 1e-15).all()


def test_trace_of_c_is_mean_squared_gradient_norm():
    r = np.random.default_rng(4)
    G = r.standard_normal((300, 7))
    _, lam = active.active_subspace(G, 3)
    assert abs(lam.sum() - np.mean(np.sum(G * G, axis=1))) < 1e-12 * lam.sum()


def test_reduced_gradients_are_derivatives_of_the_reduced_function():
    X, G, f, a, b = _ridge(n=50)
    P, _ = active.active_subspace(G, 2)
    U, Gu = active.project(X, G, P)
    # f(x) = f(P P^T x) for a ridge function in span(P): the reduced function is u -> f(P u)
    assert np.abs(f(X) - f(U @ P.T)).max() < 1e-12
    h = 1e-6
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        fd = (f((U + e) @ P.T) - f((U - e) @ P.T)) / (2 * h)
        assert np.abs(fd - Gu[:, j]).max() < 1e-7


def test_sign_convention_makes_the_largest_entry_positive():
    r = np.random.default_rng(5)
    G = r.standard_normal((200, 6)) * np.array([3.0, 2.0, 1.5, 1.0, 0.5, 0.2])
    P, _ = active.active_subspace(G, 6)
    for j in range(6):
        assert P[np.argmax(np.abs(P[:, j])), j] > 0
    P2, _ = active.active_subspace(-G, 6)
    assert np.abs(P - P2).max() < 1e-12
