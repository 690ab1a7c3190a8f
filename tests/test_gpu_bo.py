"""GPU parity of the expected-improvement acquisition (Sec. 4.4) against the
FP64 oracle: EI of 100,003 candidates (several hundred work-groups and a ragged
tail; zero and negative variances included), the best candidate with a planted
tie (the first index wins), the value column of a predict-shaped mean, and the
error when no EI is finite."""
import numpy as np
import pytest
import torch

from oracle import bo
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _cands(n, seed):
    r = np.random.default_rng(seed)
    mu = r.normal(0.0, 1.0, n)
    var = r.uniform(0.0, 2.0, n)
    var[::97] = 0.0
    var[5::89] = -r.uniform(0.0, 1.0, var[5::89].size)
    return mu, var


def test_ei_matches_oracle_and_first_index_on_ties():
    dski = need_gpu()
    n = 100003
    mu, var = _cands(n, 11)
    f_best, xi = -0.5, 0.01
    ref = bo.expected_improvement(mu, var, f_best, xi)
    j = int(np.argmax(ref))
    # plant a tie of the maximum at a later and an earlier position
    for k in (n - 1, j // 2):
        mu[k], var[k] = mu[j], var[j]
    ref = bo.expected_improvement(mu, var, f_best, xi)
    jr, vr = bo.best_candidate(mu, var, f_best, xi)
    say("ei", n, "best", jr, vr)
    ei, idx, best = dski.expected_improvement(torch.tensor(mu, device="cuda"), torch.tensor(var, device="cuda"),
                                              f_best, xi)
    e = np.abs(ei.cpu().numpy() - ref).max() / ref.max()
    say("  rel err", e, "gpu best", idx, best)
    assert e < 1e-13
    assert idx == jr == j // 2 and abs(best - vr) <= 1e-13 * vr


def test_ei_reads_the_value_column_of_a_predict_output():
    dski = need_gpu()
    mu, var = _cands(1000, 12)
    M = np.stack([mu, np.ones_like(mu) * 7.0, -np.ones_like(mu)], axis=1)  # [f, df/dx1, df/dx2]
    ei, idx, best = dski.expected_improvement(torch.tensor(M, device="cuda"), torch.tensor(var, device="cuda"), 0.0)
    ref = bo.expected_improvement(mu, var, 0.0)
    assert np.abs(ei.cpu().numpy() - ref).max() <= 1e-13 * ref.max()
    assert idx == int(np.argmax(ref))


def test_ei_rejects_all_non_finite():
    dski = need_gpu()
    mu = torch.full((10,), float("nan"), dtype=torch.float64, device="cuda")
    var = torch.ones(10, dtype=torch.float64, device="cuda")
    with pytest.raises(dski.DSKIError) as e:
        dski.expected_improvement(mu, var, 0.0)
    assert e.value.status == -1
