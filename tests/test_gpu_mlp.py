"""GPU surrogate-network kernels against the FP64 oracle network (same FP32
parameters and inputs): outputs, tangents, loss, weight gradient and one Adam
step, to 1e-5 relative (FP32 arithmetic over 128-term dot products)."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _net(seed=0, F=8, H=128):
    P = omlp.init(F, H, H, seed=seed)
    r = np.random.default_rng(seed + 100)
    for k in P:
        P[k] = (P[k] + 0.05 * r.standard_normal(P[k].shape)).astype(np.float32).astype(np.float64)
    return P


def _pack(P):
    from paper_1810_12283_amd.dski import Mlp
    return Mlp.pack(P["W1"], P["b1"], P["W2"], P["b2"], P["w3"], P["b3"])


def _unpack(v, F=8, H=128):
    v = v.astype(np.float64)
    o = 0
    out = {}
    for k, shp in (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))):
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


@pytest.mark.parametrize("B", [1, 37, 2000])
def test_mlp_forward_and_tangents(B):
    dski = need_gpu()
    say("mlp forward/jvp", B)
    P = _net(1)
    X = np.random.default_rng(2).standard_normal((B, 8)).astype(np.float32)
    net = dski.Mlp(_pack(P))
    y, dy = net.jvp(torch.tensor(X, device="cuda"))
    yr, dyr, _ = omlp.forward(P, X.astype(np.float64), J=5)
    ey = np.abs(y.cpu().numpy() - yr).max() / np.abs(yr).max()
    ed = np.abs(dy.cpu().numpy() - dyr).max() / np.abs(dyr).max()
    say("  rel err y", ey, "dy", ed)
    assert ey < 1e-5 and ed < 1e-5
    y2 = net.forward(torch.tensor(X, device="cuda"))
    np.testing.assert_array_equal(y2.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("B", [3, 500])
def test_mlp_backward_and_adam(B):
    dski = need_gpu()
    say("mlp backward", B)
    P = _net(3)
    r = np.random.default_rng(4)
    X = r.standard_normal((B, 8)).astype(np.float32)
    t = r.standard_normal(B).astype(np.float32)
    g = r.standard_normal((B, 5)).astype(np.float32)
    lam = 0.7
    net = dski.Mlp(_pack(P))
    Xd, td, gd = (torch.tensor(a, device="cuda") for a in (X, t, g))
    loss = net.backward(Xd, td, gd, lam)
    X64, t64, g64 = X.astype(np.float64), t.astype(np.float64), g.astype(np.float64)
    lref = omlp.loss(P, X64, t64, g64, lam)
    Gr = omlp.backward(P, X64, t64, g64, lam)
    Gg = _unpack(net.grad())
    say("  loss", loss, lref)
    assert loss == pytest.approx(lref, rel=1e-5)
    for k in Gr:
        err = np.abs(Gg[k] - Gr[k]).max() / max(np.abs(Gr[k]).max(), 1e-30)
        say("  grad", k, err)
        assert err < 1e-5, k
    # five Adam steps from zero moments, each on the gradient at the current
    # parameters (beyond the first step the bias corrections and both decay
    # rates matter)
    state = {}
    Pn = {k: v.copy() for k, v in P.items()}
    for step in range(5):
        if step > 0:
            net.backward(Xd, td, gd, lam)
            Gr = omlp.backward(Pn, X64, t64, g64, lam)
        net.step(lr=1e-3, beta1=0.8, beta2=0.95)
        omlp.adam_step(Pn, Gr, state, lr=1e-3, beta1=0.8, beta2=0.95)
        Pg = _unpack(net.params())
        dev = max(np.abs(Pg[k] - Pn[k]).max() for k in Pn)
        say("  Adam step", step + 1, "max parameter deviation", dev)
        assert dev < 2e-6 * (step + 1)


def test_mlp_training_reduces_the_loss_on_a_smooth_target():
    """A few hundred full-batch Adam steps on values and gradients of a smooth
    function of the first five inputs cut the loss by two orders of magnitude."""
    dski = need_gpu()
    say("mlp training")
    r = np.random.default_rng(5)
    B = 512
    X = r.uniform(-1.5, 1.5, (B, 8)).astype(np.float32)
    a = np.array([0.7, -0.4, 0.3, 0.2, -0.5])
    t = (np.sin(X[:, :5] @ a) + 0.1 * (X[:, :5] ** 2).sum(1)).astype(np.float32)
    g = (np.cos(X[:, :5] @ a)[:, None] * a[None, :] + 0.2 * X[:, :5]).astype(np.float32)
    net = dski.Mlp(_pack(_net(6)))
    Xd, td, gd = (torch.tensor(v, device="cuda") for v in (X, t, g))
    l0 = net.backward(Xd, td, gd, 1.0)
    for _ in range(400):
        net.backward(Xd, td, gd, 1.0)
        net.step(lr=3e-3)
    l1 = net.backward(Xd, td, gd, 1.0)
    say("  loss", l0, "->", l1)
    assert l1 < 1e-2 * l0
