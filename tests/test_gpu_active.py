"""GPU parity of the active-subspace reduction (Sec. 3.4) against the FP64
oracle: eigenvalues of C = (1/n) sum g g^T, the signed dominant eigenvectors,
and the reduced points and gradients, on a ridge function in 20 dimensions
(n = 20,000) and on anisotropic random gradients at the dimension limit (64)
with a ragged sample count; the dimension limit and empty input."""
import numpy as np
import pytest
import torch

from oracle import active as oact
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _ridge(D, n, seed):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((D, 3)))
    a, b, c = Q.T
    X = r.uniform(-1.0, 1.0, (n, D))
    G = (2.0 * np.cos(2.0 * X @ a)[:, None] * a + (X @ b)[:, None] * b
         + 0.05 * np.tanh(X @ c)[:, None] * c)
    return X, G


def _aniso(D, n, seed):
    r = np.random.default_rng(seed)
    X = r.uniform(-1.0, 1.0, (n, D))
    G = r.standard_normal((n, D)) * np.linspace(3.0, 0.1, D)
    return X, G


@pytest.mark.parametrize("name,D,n,d", [("ridge20", 20, 20000, 2), ("aniso64", 64, 1017, 3),
                                        ("ridge3_tiny", 3, 5, 1)])
def test_active_subspace_matches_oracle(name, D, n, d):
    dski = need_gpu()
    X, G = (_ridge if name.startswith("ridge") else _aniso)(D, n, 7)
    say("active subspace", name, D, n, d)
    Gd = torch.tensor(np.ascontiguousarray(G.T), device="cuda")
    P, lam = dski.active_subspace(Gd, d)
    P_ref, lam_ref = oact.active_subspace(G, d)
    el = np.abs(lam - lam_ref).max() / lam_ref[0]
    ep = np.abs(P - P_ref).max()
    U, Gu = dski.active_project(torch.tensor(X, device="cuda"), Gd, P)
    U_ref, Gu_ref = oact.project(X, G, P_ref)
    eu = np.abs(U.cpu().numpy() - U_ref).max() / np.abs(U_ref).max()
    eg = np.abs(Gu.cpu().numpy().T - Gu_ref).max() / np.abs(Gu_ref).max()
    gap = (lam_ref[d - 1] - lam_ref[d]) / lam_ref[0]
    say("  eigenvalues", el, "P", ep, "U", eu, "Gu", eg, "relative gap", gap)
    assert el < 1e-12 and ep < 1e-10 and eu < 1e-10 and eg < 1e-10


def test_active_subspace_limits():
    dski = need_gpu()
    r = np.random.default_rng(1)
    with pytest.raises(dski.DSKIError) as e:
        dski.active_subspace(torch.tensor(r.standard_normal((65, 100)), device="cuda"), 2)
    assert e.value.status == -5  # DSKI_ENOTSUP
    P = np.eye(4)[:, :2]
    U, Gu = dski.active_project(torch.zeros((0, 4), dtype=torch.float64, device="cuda"), None, P)
    assert U.shape == (0, 2) and Gu is None


def test_active_project_rejects_wrong_shapes():
    """P must be (D, d) and G (D, n): the oracle's n x D gradient layout and a
    transposed P are refused before any launch."""
    dski = need_gpu()
    r = np.random.default_rng(2)
    X = torch.tensor(r.uniform(-1, 1, (50, 6)), device="cuda")
    P = np.linalg.qr(r.standard_normal((6, 2)))[0]
    G = torch.tensor(r.standard_normal((6, 50)), device="cuda")
    with pytest.raises(ValueError):
        dski.active_project(X, G, P.T)
    with pytest.raises(ValueError):
        dski.active_project(X, G.T.contiguous(), P)
    with pytest.raises(ValueError):
        dski.active_project(X, G.float(), P)
    U, Gu = dski.active_project(X, G, P)
    assert U.shape == (50, 2) and Gu.shape == (2, 50)
