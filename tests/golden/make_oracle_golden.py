"""Write the oracle's reference values for the full-size GPU parity tests.

    python tests/golden/make_oracle_golden.py terrain   # ~10 min on 8 cores
    python tests/golden/make_oracle_golden.py torus2000

Calls only the FP64 oracle (``oracle/``) and the seeded input generators
(``workloads/``); nothing here touches the GPU library.  Outputs
(``tests/golden/*.json``):

* ``terrain_full_oracle.json`` -- the terrain workload at its full size
  (n = 20,000, 200 x 200 grid, 17 columns = data + 16 probes): the oracle's
  greedy pivots at rank 50 (Sec. 3.3), log det M, and the stochastic log det,
  mll and gradient of eq. (1) from one batched FP64 PCG to 1e-4 on the data
  vector (rounded to FP32, as the GPU receives it) and the 16 probes of the
  shared SplitMix64 stream mapped through the preconditioner's square-root
  factor (Sec. 2, Sec. 3.3).
* ``torus2000_oracle.json`` -- the first 2,000 torus points on the 48^3 grid:
  the exact D-SKI mll and gradient from a dense Cholesky of the 8,000 x 8,000
  matrix, and central differences (h = 1e-3 in the log hyper-parameters) of
  the dense mll, which pin the dense gradient.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import dski as odski, mll as omll, pivchol, precond  # noqa: E402

SEED = 0x181012283


def terrain():
    W = workloads.terrain()
    t0 = time.time()
    op = odski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    L, piv, gaps = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, W.rank)
    P = precond.Precond(L, op.Dn)
    y = W.y.astype(np.float32).astype(np.float64)
    res = omll.stochastic(op, y, L, W.num_probes, SEED, W.tol, max_iter=20000)
    out = dict(workload="terrain", n=W.n, grid=list(W.grid_m), k=W.rank, num_probes=W.num_probes, tol=W.tol,
               seed=SEED, pivots=[int(v) for v in piv], logdet_M=P.logdet(), logdet=res["logdet"],
               logdet_stderr=res["logdet_stderr"], mll=res["mll"], grad=[float(v) for v in res["grad"]],
               iters=[int(v) for v in res["pcg"]["iters"]], relres=[float(v) for v in res["pcg"]["relres"]],
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "terrain_full_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k not in ("pivots", "relres")}))


def torus2000():
    W = workloads.torus(n=2000)
    t0 = time.time()
    op = odski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    y = W.y.astype(np.float32).astype(np.float64)
    ex = omll.exact(op, y)
    theta = np.concatenate([np.asarray(W.log_ell, dtype=np.float64),
                            [W.log_s, W.log_sigma_f, W.log_sigma_g]])
    h = 1e-3
    fd = []
    for j in range(op.d + 3):
        vals = []
        for sgn in (+1, -1):
            th = theta.copy()
            th[j] += sgn * h
            op.set_hypers(th[:op.d], th[op.d], th[op.d + 1], th[op.d + 2])
            A = op.dense()
            import scipy.linalg as sla
            cf = sla.cho_factor(A, lower=True)
            alpha = sla.cho_solve(cf, y)
            ld = 2.0 * np.sum(np.log(np.diag(cf[0])))
            vals.append(-0.5 * (y @ alpha + ld + op.N * math.log(2 * math.pi)))
        fd.append((vals[0] - vals[1]) / (2 * h))
    out = dict(workload="torus", n=W.n, grid=list(W.grid_m), mll=ex["mll"], logdet=ex["logdet"],
               grad=[float(v) for v in ex["grad"]], fd_grad=[float(v) for v in fd], fd_h=h,
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "torus2000_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    {"terrain": terrain, "torus2000": torus2000}[sys.argv[1]]()
