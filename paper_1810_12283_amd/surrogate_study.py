"""The learned log-det surrogate on the 2-D terrain data (n = 20,000, 200 x 200
grid, rank-50 preconditioner, 16 probes, tol 1e-4): training data from the
method's own SLQ at Sobol points within +-2 log-units of the generating
hyper-parameters, training with the device MLP kernels, held-out accuracy, and
L-BFGS fits with and without the surrogate at equal final marginal likelihood.

Phases (each prints one line per step and writes JSON):
  cost      SLQ log det + gradient at the first `--count` points of a second
            Sobol design (seconds, PCG iterations, status per point)
  data      samples [start, start + count) of the training design, appended
            one JSON line each to --out, stopping early after --seconds
  evaluate  train on the samples in --data (the last --holdout converged ones
            held out), report the held-out error, then fit from --starts
            starting points with plain SLQ and with the surrogate

python -m paper_1810_12283_amd.surrogate_study cost --count 32 --out c.json
python -m paper_1810_12283_amd.surrogate_study data --start 0 --count 500 --out d.jsonl
python -m paper_1810_12283_amd.surrogate_study evaluate --data d.jsonl --out e.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

RADIUS = 2.0           # half-width of the training box in log-units
DESIGN = 2048          # Sobol design size (a power of two); the first 2,000 are used
DESIGN_SEED = 17
COST_SEED = 29
PROBE_SEED = 0x181012283


def _say(*a):
    print(*a, flush=True)


def _setup():
    import workloads
    from . import dski
    W = workloads.terrain()
    plan = dski.Plan(torch.tensor(W.X, dtype=torch.float64, device="cuda"), W.grid_m, W.lo, W.hi)
    plan.set_hypers(*W.hypers())
    plan.autotune(1 + W.num_probes)
    theta_star = np.concatenate([W.log_ell, [W.log_s, W.log_sigma_f, W.log_sigma_g]])
    return W, plan, theta_star


def _sample(plan, W, th):
    from . import surrogate as sg
    info = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ld, g = sg.logdet_and_grad(plan, th, W.rank, W.num_probes, PROBE_SEED, W.tol, max_iter=20000, info=info)
    torch.cuda.synchronize()
    return dict(theta=[float(v) for v in th], logdet=float(ld), grad=[float(v) for v in g],
                seconds=time.perf_counter() - t0, iters=int(max(info["iters"])), status=int(info["status"]))


def phase_cost(a):
    from . import surrogate as sg
    W, plan, th_star = _setup()
    pts = sg.sobol_design(th_star, 32 if a.count <= 32 else DESIGN, RADIUS, seed=COST_SEED)[:a.count]
    out = []
    for i, th in enumerate(pts):
        r = _sample(plan, W, th)
        out.append(r)
        _say(f"cost {i} theta {np.round(th, 3).tolist()} s {r['seconds']:.3f} iters {r['iters']} "
             f"status {r['status']} logdet {r['logdet']:.6g}")
    sec = np.array([r["seconds"] for r in out])
    summ = dict(workload=f"terrain n={W.n} grid={W.grid_m[0]}x{W.grid_m[1]} rank={W.rank} probes={W.num_probes}"
                         f" tol={W.tol}", radius=RADIUS, points=len(out), mean_s=float(sec.mean()),
                median_s=float(np.median(sec)), max_s=float(sec.max()),
                not_converged=int(sum(r["status"] != 0 for r in out)),
                projected_2000_min=float(sec.mean() * 2000 / 60.0), samples=out)
    with open(a.out, "w") as f:
        json.dump(summ, f)
    _say("cost summary", json.dumps({k: v for k, v in summ.items() if k != "samples"}))
    plan.close()


def phase_data(a):
    from . import surrogate as sg
    W, plan, th_star = _setup()
    pts = sg.sobol_design(th_star, DESIGN, RADIUS, seed=DESIGN_SEED)
    t_start = time.perf_counter()
    done = 0
    with open(a.out, "a") as f:
        for i in range(a.start, min(a.start + a.count, 2000)):
            if time.perf_counter() - t_start > a.seconds:
                _say(f"data: time budget reached after {done} samples")
                break
            r = _sample(plan, W, pts[i])
            r["index"] = i
            f.write(json.dumps(r) + "\n")
            f.flush()
            done += 1
            _say(f"data {i} s {r['seconds']:.3f} iters {r['iters']} status {r['status']}")
    plan.close()
    _say(f"data: {done} samples in {time.perf_counter() - t_start:.1f} s")


def _load(paths):
    rows = {}
    for p in paths:
        with open(p) as f:
            for line in f:
                line = line.strip()
                if line:
                    r = json.loads(line)
                    rows[r["index"]] = r
    return [rows[i] for i in sorted(rows)]


def phase_evaluate(a):
    from . import surrogate as sg
    rows = _load(a.data)
    ok = [r for r in rows if r["status"] == 0 or a.include_capped]
    _say(f"evaluate: {len(rows)} samples, {sum(r['status'] == 0 for r in rows)} converged, "
         f"{len(ok)} used")
    hold = ok[-a.holdout:]
    tr = ok[:-a.holdout]
    W, plan, th_star = _setup()
    h = np.array(plan.h)
    th = np.array([r["theta"] for r in tr])
    T = np.array([r["logdet"] for r in tr])
    G = np.array([r["grad"] for r in tr])
    t_data = float(sum(r["seconds"] for r in rows))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = sg.train(th, T, G, W.n, h, steps=a.steps, lr=a.lr, lr_final=a.lr_final, lam=a.lam)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    errs = []
    for r in hold:
        ls, _ = S(np.array(r["theta"]))
        errs.append(abs(ls - r["logdet"]) / abs(r["logdet"]))
    errs = np.array(errs)
    _say(f"train {len(tr)} samples, {a.steps} steps in {t_train:.2f} s, loss {S.history[0][1]:.4g} -> "
         f"{S.history[-1][1]:.4g}; held-out relative log det error median {np.median(errs):.3g} "
         f"p90 {np.quantile(errs, 0.9):.3g} max {errs.max():.3g}")
    y = torch.tensor(W.y.astype(np.float32), device="cuda")[None, :].contiguous()
    box = [(c - RADIUS, c + RADIUS) for c in th_star]
    # a centre (the moment-matched hyper-parameters plus --start-offset), then
    # Sobol points around it
    c0 = th_star + np.array([float(v) for v in a.start_offset.split(",")]) if a.start_offset else th_star
    starts = np.vstack([c0[None, :], sg.sobol_design(c0, 8, a.start_radius, seed=43)])[:a.starts]
    fits = []
    for j, t0v in enumerate(starts):
        plain = sg.fit(plan, y, t0v, W.rank, W.num_probes, PROBE_SEED, W.tol, surrogate=None,
                       max_evals=a.max_evals, bounds=box)
        _say(f"fit {j} plain: mll {plain.mll:.8g} evals {plain.evals} s {plain.seconds:.2f} "
             f"theta {np.round(plain.theta, 4).tolist()}")
        withs = sg.fit(plan, y, t0v, W.rank, W.num_probes, PROBE_SEED, W.tol, surrogate=S,
                       max_evals=a.max_evals, bounds=box, recheck=10, fallback_tol=1e-3)
        _say(f"fit {j} surrogate: mll {withs.mll:.8g} evals {withs.evals} s {withs.seconds:.2f} "
             f"fell back {withs.fell_back} rechecks {[(e, round(x, 6)) for e, _, _, x in withs.rechecks]} "
             f"theta {np.round(withs.theta, 4).tolist()}")
        fits.append(dict(start=[float(v) for v in t0v], plain=dict(mll=plain.mll, evals=plain.evals,
                                                                    seconds=plain.seconds,
                                                                    theta=plain.theta.tolist()),
                         surrogate=dict(mll=withs.mll, evals=withs.evals, seconds=withs.seconds,
                                        fell_back=withs.fell_back, theta=withs.theta.tolist(),
                                        rechecks=[list(map(float, r)) for r in withs.rechecks]),
                         rel_mll=abs(withs.mll - plain.mll) / abs(plain.mll)))
    tp = np.array([f["plain"]["seconds"] for f in fits])
    ts = np.array([f["surrogate"]["seconds"] for f in fits])
    gain = float(tp.mean() - ts.mean())
    summ = dict(workload=f"terrain n={W.n} grid={W.grid_m[0]}x{W.grid_m[1]}", train_samples=len(tr),
                holdout=len(hold), data_s=t_data, train_s=t_train,
                holdout_err=dict(median=float(np.median(errs)), p90=float(np.quantile(errs, 0.9)),
                                 max=float(errs.max())),
                include_capped=bool(a.include_capped), fits=fits, plain_fit_s=float(tp.mean()), surrogate_fit_s=float(ts.mean()),
                fit_speedup=float(tp.mean() / ts.mean()),
                equal_mll=bool(all(f["rel_mll"] <= 1e-3 for f in fits)),
                break_even_fits=(float((t_data + t_train) / gain) if gain > 0 else None))
    with open(a.out, "w") as f:
        json.dump(summ, f)
    _say("evaluate summary", json.dumps({k: v for k, v in summ.items() if k != "fits"}))
    plan.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("phase", choices=["cost", "data", "evaluate"])
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--seconds", type=float, default=1e9)
    ap.add_argument("--out", required=True)
    ap.add_argument("--data", nargs="*", default=[])
    ap.add_argument("--holdout", type=int, default=100)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--starts", type=int, default=3)
    ap.add_argument("--start-radius", type=float, default=0.5)
    ap.add_argument("--start-offset", default="",
                    help="comma-separated offsets (log-units) of the starts' centre from the moment-matched values")
    ap.add_argument("--include-capped", action="store_true",
                    help="train on samples whose PCG reached max_iter too (their log det is the method's "
                         "output at that cap)")
    ap.add_argument("--max-evals", type=int, default=60)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the surrogate study needs a GPU")
    {"cost": phase_cost, "data": phase_data, "evaluate": phase_evaluate}[a.phase](a)


if __name__ == "__main__":
    main()
