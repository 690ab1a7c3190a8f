"""Benchmark of the D-SKI hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the synthetic terrain problem (n = 20,000 points on [0,1]^2, values
and gradients, N = 60,000; 200 x 200 grid; SE kernel with moment-matched
hyper-parameters; 17 right-hand sides = the data vector + 16 preconditioned
Rademacher probes; pivoted-Cholesky rank 50; PCG tolerance 1e-4).

One step = one pass of the whole hot path on resident inputs:
  plan set-up (cells, tile order, region tables) and spectra, the tuner,
  23 block MVMs with the 17 columns (3 untimed, 20 timed one by one) and the
  per-stage timings,
  pivoted Cholesky (rank 50) and the preconditioner,
  block PCG of the 17 columns to 1e-4,
  mll and its gradient (its own block PCG, SLQ log det, adjoint products),
  the same block PCG and mll with FP64 vectors (`f64_vectors`).

Printed: one JSON line.  `value` is the D-SKI MVM throughput in GB/s of
algorithmic bytes B = 4 (3 N R + 4 m R + 2 n (d + 1)) per product over the
median product time (`mvm_ms_p10_p90` the spread); `copy_gbs_same_size` the
rate of a device copy of B bytes; `pcg_s` the block-PCG seconds to 1e-4.
`roofline` is that of the dominant MVM stage, timed live with events on the
stream the kernels run on, with the measured traffic of the tuned variant;
`dskip` a D-SKIP block MVM and block PCG (8-D ridge workload); `surrogate`
the learned log det surrogate's evaluation and training costs at this size;
`predict` the posterior mean at 1,000,000 test points;
`cpu_baseline` the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_MARKER_SEED = 0x504D43
SEED = 0x181012283
PMC_SUMMARY = os.path.join(ROOT, "profiles", "terrain_mvm_pmc.md")
MVM_SOURCE = os.path.join(ROOT, "paper_1810_12283_amd", "csrc", "mvm.hip")


def source_digest(path=MVM_SOURCE):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def _fastest(times):
    """Index of the smallest time; -1 marks a variant that was not timed."""
    return min(range(len(times)), key=lambda i: times[i] if times[i] >= 0 else float("inf"))


def tuned_variants(tune):
    """The variants the tuner keeps: the first fastest scatter and gather form, and
    per axis the FFT unless the dense form (timed, not -1) is strictly faster."""
    return {"scatter": _fastest(tune["scatter_us"]), "gather": _fastest(tune["gather_us"]),
            "kuu": [0 if (t[1] < 0 or t[0] <= t[1]) else 1 for t in tune["kuu_us"]]}


def measured_traffic():
    """HBM bytes per launch of each MVM kernel variant (scatter_v0.., gather_v0..,
    kuu_fft, kuu_dense: one launch, one axis for K_UU) from the committed PMC
    summary (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of known size), or
    None when the summary is missing or was taken on a different mvm.hip."""
    try:
        with open(PMC_SUMMARY) as f:
            for line in f:
                if line.startswith("traffic-bytes-per-launch:"):
                    fields = dict(kv.split("=") for kv in line.split(":", 1)[1].split())
                    if fields.pop("source", None) != source_digest():
                        return None
                    return {k: float(v) for k, v in fields.items()}
    except OSError:
        return None
    return None


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stats_table(csv_path, top=40):
    """Markdown rows (kernel, calls, total ms, avg us, %) of a rocprofv3
    --kernel-trace --stats kernel_stats.csv, largest total first."""
    import csv
    rows = []
    with open(csv_path, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["Percentage"])))
    rows.sort(key=lambda r: -r[2])
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows[:top]:
        out.append(f"| `{_short_kernel(name)}` | {calls} | {tot / 1e6:.1f} | {avg / 1e3:.2f} | {pct:.1f} |")
    out.append("")
    out.append(f"Total kernel time {sum(r[2] for r in rows) / 1e6:.1f} ms over {len(rows)} kernels "
               f"({min(top, len(rows))} largest shown).")
    return "\n".join(out)


def _pmc_dispatches(folder):
    """{dispatch id: (kernel name, grid size, {counter: value})} from the
    counter-collection CSV files rocprofv3 wrote under `folder`."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *counter_collection.csv under {folder}")
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                did = int(row["Dispatch_Id"])
                name = row.get("Kernel_Name", "")
                grid = int(float(row.get("Grid_Size", 0) or 0))
                ent = out.setdefault(did, (name, grid, {}))
                c = row["Counter_Name"]
                ent[2][c] = ent[2].get(c, 0.0) + float(row["Counter_Value"])
    return out


def _pmc_groups(disp, labels):
    """Dispatches split at the marker dispatches (the 64-entry Rademacher column)
    into {label: [(name, counters), ...]} in dispatch order."""
    groups, cur = {}, None
    marks = 0
    for did in sorted(disp):
        name, grid, ctr = disp[did]
        if "k_rademacher" in name and 0 < grid <= 1024:
            if marks >= len(labels):
                raise ValueError("more marker dispatches than labels")
            cur = labels[marks]
            marks += 1
            groups[cur] = []
            continue
        if cur is not None:
            groups[cur].append((name, ctr))
    if marks != len(labels):
        raise ValueError(f"{marks} marker dispatches for {len(labels)} labels")
    return groups


def _short_kernel(name):
    name = name.split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def pmc_summary(fetch_dir, write_dir, log_path, sq_dir=None, out_path=PMC_SUMMARY, commands=None):
    """Write the PMC summary of `bench.py --pmc-mvm` (one rocprofv3 run per counter
    group) with per-variant HBM bytes per launch keyed to the mvm.hip digest."""
    import numpy as np
    info = None
    with open(log_path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"pmc_mvm"' in line:
                info = json.loads(line)
    if info is None:
        raise ValueError(f"no pmc_mvm line in {log_path}")
    labels = info["labels"]
    gf = _pmc_groups(_pmc_dispatches(fetch_dir), labels)
    gw = _pmc_groups(_pmc_dispatches(write_dir), labels)
    gs = _pmc_groups(_pmc_dispatches(sq_dir), labels) if sq_dir else None

    family = {"scatter": "k_scatter", "gather": "k_gather", "kuu": "k_toeplitz"}

    def main_kernel(lab, group):
        # the most frequent kernel of the stage's family in the group
        fam = family.get(lab.split("_")[0], "")
        names = {}
        for name, _ in group:
            if fam in name:
                names[name] = names.get(name, 0) + 1
        return max(names, key=names.get)

    def med(group, name, counter):
        v = [c.get(counter) for n, c in group if n == name and counter in c]
        return float(np.median(v)) if v else float("nan")

    # calibration on the copy group: the runtime copy and the multiply each move
    # copy_bytes in and copy_bytes out
    cb = info["copy_bytes"]
    copy_f = [c["FETCH_SIZE"] for _, c in gf["copy"] if c.get("FETCH_SIZE", 0) * 1024 > 0.25 * cb]
    copy_w = [c["WRITE_SIZE"] for _, c in gw["copy"] if c.get("WRITE_SIZE", 0) * 1024 > 0.25 * cb]
    kf = cb / (float(np.median(copy_f)) * 1024)
    kw = cb / (float(np.median(copy_w)) * 1024)
    rows, traffic = [], {}
    for lab in labels:
        if lab == "copy":
            continue
        multi = lab in ("pcg", "pivchol")
        names = sorted({n for n, _ in gf[lab]}) if multi else [main_kernel(lab, gf[lab])]
        for name in names:
            fk = med(gf[lab], name, "FETCH_SIZE")
            wk = med(gw[lab], name, "WRITE_SIZE")
            byts = fk * 1024 * kf + wk * 1024 * kw
            extra = ""
            if gs is not None:
                waves = med(gs[lab], name, "SQ_WAVES")
                vals = [med(gs[lab], name, c) for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT",
                                                        "SQ_WAIT_INST_ANY")]
                extra = f" | {waves:.0f} | " + " | ".join(f"{v / waves:.0f}" if waves else "-" for v in vals)
            rows.append(f"| {lab} | `{_short_kernel(name)}` | {fk:.0f} | {wk:.0f} | {byts / 1e6:.2f} MB{extra} |")
            if not multi:
                traffic[lab] = byts
    cmd = "\n".join(commands or [])
    head = ("| label | kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes / launch"
            + (" | waves | VALU instr / wave | LDS instr / wave | LDS bank-conflict cycles / wave | "
               "wait-any instr cycles / wave |" if gs is not None else " |"))
    sep = "|---|---|---:|---:|---:" + ("|---:|---:|---:|---:|---:|" if gs is not None else "|")
    text = [
        "# PMC counters of the terrain MVM stages and PCG kernels "
        "(n = 20,000, d = 2, 200 x 200 grid, 17 columns, rank 50)",
        "",
        "Commands (from the repository root on one MI355X; one counter group per run), then "
        "`python bench.py --pmc-summary` on their output folders:",
        "",
        "```",
        cmd,
        "```",
        "",
        "`bench.py --pmc-mvm` builds the plan and runs the tuner, then launches every scatter, gather and "
        "K_UU variant three times, a 20-iteration block PCG with direct launches and the rank-50 "
        "preconditioner, and three 256 MiB copies through the runtime's copy kernel and an elementwise "
        "multiply; a 64-entry Rademacher column before each group marks where it starts. Figures are "
        "medians over the launches of a group's kernel.",
        "",
        f"Calibration on the copies ({cb / 2**20:.0f} MiB read and written per launch): FETCH_SIZE reads "
        f"{np.median(copy_f):.0f} KiB, WRITE_SIZE {np.median(copy_w):.0f} KiB, so fetched bytes = FETCH_SIZE x "
        f"1024 x {kf:.3f} and written bytes = WRITE_SIZE x 1024 x {kw:.3f}. FETCH_SIZE counts what the L2s of "
        "all 8 XCDs fetch from the fabric, part of which the Infinity Cache serves, so the fetch figures "
        "bound HBM reads from above.",
        "",
        head,
        sep,
        *rows,
        "",
        "traffic-bytes-per-launch: " + " ".join(f"{k}={v:.0f}" for k, v in traffic.items())
        + f" source={info['source']}",
        "",
    ]
    with open(out_path, "w") as f:
        f.write("\n".join(text))
    return traffic


def _events_ms(fn, reps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def _events_stats(fn, reps, stream, warm=3):
    """Median, 10th and 90th percentile (ms) of `reps` launches of fn, each
    bracketed by its own pair of events on `stream`, after `warm` untimed ones."""
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    ev[-1][1].synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return float(np.median(t)), float(np.percentile(t, 10)), float(np.percentile(t, 90))


def dskip_block(R, stream, reps=20):
    """D-SKIP block MVM on the 8-D ridge workload (n = 4,000, 1-D grids of 100,
    Lanczos rank 32): build seconds, MVM time and the root products' flop rate
    (4 N r^2 R flops per block MVM with r padded to 32, against the FP32
    matrix-core peak the two root products run on), then the configuration's block PCG (data vector and 16
    probes, rank-100 pivoted-Cholesky preconditioner, tolerance 1e-4)."""
    import torch
    import workloads
    from paper_1810_12283_amd import dski
    W = workloads.ridge8d()
    X = torch.tensor(W.X, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = dski.DskipPlan(X, W.skip_m, W.skip_rank, 7, W.log_ell, W.lo, W.hi)
    plan.set_hypers(W.log_ell, W.log_s, W.log_sigma_f, W.log_sigma_g)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    V = dski.rademacher(99, 0, R, W.N, device="cuda")
    Y = torch.empty_like(V)
    med, p10, p90 = _events_stats(lambda: plan.mvm_tiled(V, out=Y), reps, stream)
    flops = 4.0 * W.N * 32 * 32 * R
    # the block PCG of the configuration: data vector + 16 probes, rank-100 preconditioner
    import numpy as np
    B = V.clone()
    B[0] = torch.tensor(W.y.astype(np.float32), device="cuda")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pc = plan.pivchol(W.rank)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, iters, _, st, _ = plan.pcg(B, pc, tol=W.tol, max_iter=20000)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    pc.close()
    plan.close()
    return {"workload": f"ridge n={W.n} d={W.d} m_1d={W.skip_m} rank={W.skip_rank} R={R}",
            "build_s": round(build_s, 4), "mvm_ms": round(med, 4), "mvm_ms_p10_p90": [round(p10, 4), round(p90, 4)],
            "gflops": round(flops / (med * 1e-3) / 1e9, 1),
            "frac_fp32_mfma_peak": round(flops / (med * 1e-3) / 157.3e12, 4),
            "pivchol_s": round(t2 - t1, 4), "pcg_s": round(t3 - t2, 4), "pcg_iters": int(max(iters)),
            "pcg_status": int(st), "rank": W.rank, "tol": W.tol}


def surrogate_block(W, y, rank, stream, reps=20):
    """The learned log-det surrogate on the terrain data: one SLQ log det +
    gradient evaluation (16 probes) against one data-fit evaluation (a single
    PCG column) at the true hyper-parameters, and the network's kernels at the
    sizes of the configuration (8 -> 128 -> 128 -> 1, 2,000 training points):
    one full-batch value + gradient training step (backward and Adam) and one
    inference (value and 5 input tangents, batch 1)."""
    import numpy as np
    import torch
    from paper_1810_12283_amd import dski, surrogate
    plan = dski.Plan(torch.tensor(W.X, dtype=torch.float64, device="cuda"), W.grid_m, W.lo, W.hi)
    theta = np.concatenate([W.log_ell, [W.log_s, W.log_sigma_f, W.log_sigma_g]])
    plan.set_hypers(W.log_ell, W.log_s, W.log_sigma_f, W.log_sigma_g)
    plan.autotune(1 + W.num_probes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    surrogate.logdet_and_grad(plan, theta, rank, W.num_probes, 7, W.tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    surrogate.data_fit_and_grad(plan, theta, y, rank, W.tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plan.close()
    F, H, J, B = 8, 128, 5, 2000
    r = np.random.default_rng(0)
    net = dski.Mlp(dski.Mlp.pack(r.standard_normal((H, F)) * 0.5, np.zeros(H), r.standard_normal((H, H)) * 0.1,
                                 np.zeros(H), r.standard_normal(H) * 0.1, np.zeros(1)), F=F, H=H, J=J)
    X = torch.tensor(r.standard_normal((B, F)), dtype=torch.float32, device="cuda")
    t = torch.tensor(r.standard_normal(B), dtype=torch.float32, device="cuda")
    g = torch.tensor(r.standard_normal((B, J)), dtype=torch.float32, device="cuda")
    x1 = X[:1].contiguous()

    def train_step():
        net.backward(X, t, g, 1.0)
        net.step(lr=1e-4)
    train_ms = _events_stats(train_step, reps, stream)[0]
    infer_ms = _events_stats(lambda: net.jvp(x1), reps, stream)[0]
    net.close()
    return {"workload": f"terrain n={W.n} d={W.d} grid={W.grid_m[0]}x{W.grid_m[1]}, network {F}-{H}-{H}-1, "
                        f"{B} training points",
            "slq_logdet_grad_s": round(t1 - t0, 4), "data_fit_grad_s": round(t2 - t1, 4),
            "mlp_train_step_ms": round(train_ms, 4), "mlp_infer_ms": round(infer_ms, 4),
            "eval_speedup": round((t1 - t0) / (t2 - t1 + infer_ms * 1e-3), 3)}


def predict_block(W, stream, npts=1_000_000, reps=20):
    """Posterior mean at test points on the terrain workload: the grid vector
    g = K_UU S^T alpha (one scatter and the K_UU factors) and the stencil means
    [f, grad f] of 1,000,000 uniform test points (16 grid reads each); the
    pivoted-Cholesky predictive variance (rank 100) of 4,096 of them, 128 per
    batch (one grid column each: stencil, K_UU, gather, preconditioner
    projection); the randomized variance of 1,024 of them with 16 probes; the
    EI acquisition over all 1,000,000 and its best candidate."""
    import numpy as np
    import torch
    from paper_1810_12283_amd import dski
    plan = dski.Plan(torch.tensor(W.X, dtype=torch.float64, device="cuda"), W.grid_m, W.lo, W.hi)
    plan.set_hypers(*W.hypers())
    alpha = torch.tensor(np.random.default_rng(5).standard_normal(W.N), device="cuda")
    r = np.random.default_rng(6)
    Xs = torch.tensor(r.uniform(0.0, 1.0, (npts, W.d)), device="cuda")
    g_ms = _events_stats(lambda: plan.predict_grid(alpha), reps, stream)[0]
    g = plan.predict_grid(alpha)
    p_ms = _events_stats(lambda: plan.predict(g, Xs), reps, stream)[0]
    # EI acquisition over the same 1,000,000 candidates (value column of the
    # means, synthetic variances)
    mu_all = plan.predict(g, Xs)
    var_all = torch.tensor(r.uniform(0.0, 1.0, npts), device="cuda")
    ei_ms = _events_stats(lambda: dski.expected_improvement(mu_all, var_all, 0.0), reps, stream)[0]
    nvar = 4096
    pc = plan.pivchol(100)
    Xv = Xs[:nvar].contiguous()
    v_ms = _events_stats(lambda: plan.predict_var(pc, Xv), 5, stream)[0]
    # randomized variance with that estimate as control variate: 16 Rademacher
    # probes over 1,024 test points, block PCG to the workload's tolerance
    nprb, npv = 16, 1024
    Zp = torch.tensor(r.choice([-1.0, 1.0], (nprb, npv)), device="cuda")
    Xp = Xs[:npv].contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, pst = plan.predict_var_probes(pc, Xp, Zp, tol=W.tol, max_iter=20000)
    torch.cuda.synchronize()
    pr_s = time.perf_counter() - t0
    pc.close()
    plan.close()
    return {"workload": f"terrain n={W.n} grid={W.grid_m[0]}x{W.grid_m[1]}, {npts} test points",
            "grid_vector_ms": round(g_ms, 4), "predict_ms": round(p_ms, 4),
            "test_points_per_s": round(npts / (p_ms * 1e-3), 1),
            "ei_ms": round(ei_ms, 4), "ei_candidates_per_s": round(npts / (ei_ms * 1e-3), 1),
            "variance_rank": 100, "variance_points": nvar, "variance_ms": round(v_ms, 3),
            "variance_points_per_s": round(nvar / (v_ms * 1e-3), 1),
            "randomized_variance": {"points": npv, "probes": nprb, "tol": W.tol, "s": round(pr_s, 3),
                                    "status": int(pst)}}


def active_block(D=20, n=20000, reps=10):
    """Active subspace of a ridge function in D = 20 dimensions from n = 20,000
    gradient samples (C on the GPU, Jacobi on the host) and the projection of
    the points and gradients onto its 2 dominant directions."""
    import numpy as np
    import torch
    from paper_1810_12283_amd import dski
    r = np.random.default_rng(8)
    Q, _ = np.linalg.qr(r.standard_normal((D, 2)))
    X = r.uniform(-1.0, 1.0, (n, D))
    G = 2.0 * np.cos(2.0 * X @ Q[:, 0])[:, None] * Q[:, 0] + (X @ Q[:, 1])[:, None] * Q[:, 1]
    Gd = torch.tensor(np.ascontiguousarray(G.T), device="cuda")
    Xd = torch.tensor(X, device="cuda")
    dski.active_subspace(Gd, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P, lam = dski.active_subspace(Gd, 2)
    s_ms = (time.perf_counter() - t0) / reps * 1e3
    dski.active_project(Xd, Gd, P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dski.active_project(Xd, Gd, P)
    torch.cuda.synchronize()
    p_ms = (time.perf_counter() - t0) / reps * 1e3
    return {"workload": f"ridge function D={D}, n={n}, d=2", "subspace_ms": round(s_ms, 3),
            "project_ms": round(p_ms, 3), "eigenvalue_ratio_3_1": float(lam[2] / lam[0])}


def grid_block(W, R, stream, interp="cubic", reps=20, solve=True, max_iter=20000, kernel="se"):
    """One D-SKI workload on its own (tuner, block MVM of R columns with its
    per-stage times and the roofline of the dominant stage), then, with solve,
    the rank-k pivoted Cholesky and mll_and_grad with 16 probes to the
    workload's tolerance: used for the implicit-surface workload (torus,
    n = 30,000 on 48^3) and for the terrain workload with quintic weights."""
    import numpy as np
    import torch
    from paper_1810_12283_amd import dski
    t0 = time.perf_counter()
    plan = dski.Plan(torch.tensor(W.X, dtype=torch.float64, device="cuda"), W.grid_m, W.lo, W.hi, interp=interp,
                     kernel=kernel)
    plan.set_hypers(*W.hypers())
    tune = plan.autotune(R)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    N, n, d, M = W.N, W.n, W.d, plan.grid_nodes
    V = torch.sign(torch.randn((R, N), device="cuda", dtype=torch.float32))
    Vt = plan.permute(V, +1)
    Yt = torch.empty_like(Vt)
    med, p10, p90 = _events_stats(lambda: plan.mvm_tiled(Vt, out=Yt), reps, stream)
    stage = {"scatter": _events_ms(lambda: plan.mvm_stage(0, Vt), reps, stream),
             "kuu": _events_ms(lambda: plan.mvm_stage(1, Vt), reps, stream)}
    plan.mvm_stage(0, Vt)
    stage["gather"] = _events_ms(lambda: plan.mvm_stage(2, Vt, Yt), reps, stream)
    Bm = mvm_bytes(N, M, n, d, R)
    sb = stage_bytes(N, M, n, d, R)
    dom = max(stage, key=stage.get)
    ach = sb[dom] / (stage[dom] * 1e-3) / 1e9
    out = {"workload": f"{W.name} n={n} d={d} grid={'x'.join(map(str, W.grid_m))} R={R} interp={interp} "
                       f"kernel={kernel}",
           "setup_and_tune_s": round(t_setup, 3), "mvm_ms": round(med, 4), "mvm_ms_p10_p90": [round(p10, 4),
                                                                                            round(p90, 4)],
           "mvm_algorithmic_bytes": Bm, "mvm_gbs": round(Bm / (med * 1e-3) / 1e9, 1),
           "stage_ms": {k: round(v, 4) for k, v in stage.items()}, "variants": tuned_variants(tune),
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}}
    if solve:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pc = plan.pivchol(W.rank)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        y = torch.tensor(W.y, dtype=torch.float32, device="cuda")[None, :]
        res = plan.mll_and_grad(y, pc, num_probes=W.num_probes, seed=SEED, tol=W.tol, max_iter=max_iter)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out.update({"rank": W.rank, "tol": W.tol, "pivchol_s": round(t2 - t1, 4),
                    "mll_and_grad_s": round(t3 - t2, 4), "mll_pcg_iters": int(max(res["iters"])),
                    "mll_status": int(res["status"]), "mll": res["mll"], "logdet": res["logdet"],
                    "grad": [float(v) for v in res["grad"]]})
        pc.close()
    plan.close()
    return out


def bo_block(iters=10, n0=60, seed=11):
    """Alg. 1 (Sec. 4.4) on the paper's setting: 5-D Ackley embedded in
    [-10, 15]^50, d = 2 random directions inside the 5-D estimated active
    subspace, D-SKI on a 30 x 30 reduced grid, EI; n0 initial samples (the
    reduced system stays within the full-rank pivoted Cholesky, N <= 256)."""
    import numpy as np
    import workloads
    from paper_1810_12283_amd import bo
    obj, lo, hi, _ = workloads.embedded_objective("ackley", 50, 5, seed)
    X0 = lo + (hi - lo) * np.random.default_rng(seed + 1).random((n0, 50))
    f0 = min(obj(x)[0] for x in X0)
    r = bo.run_alg1(obj, X0, lo, hi, iters=iters, d=2, k_active=5, grid=30, seed=seed + 2)
    return {"workload": f"ackley 5-D in 50-D, n0={n0}, {iters} iterations, d=2 of a 5-D active subspace",
            "s_per_iter": round(float(np.mean([s.seconds for s in r.steps])), 4),
            "initial_best": round(float(f0), 4), "best": round(r.best_f, 4),
            "trace": [round(s.f, 4) for s in r.steps]}


def mvm_bytes(N, M, n, d, R):
    """Algorithmic bytes of one block MVM (FP32 vectors and grid):
    V read by the scatter and again for the noise term, Y written (3 N R);
    grid written by the scatter, read + written by K_UU, read by the gather
    (4 m R); point records (cell id + d offsets) read by scatter and gather."""
    return 4 * (3 * N * R + 4 * M * R + 2 * n * (d + 1))


def stage_bytes(N, M, n, d, R):
    return {
        "scatter": 4 * (N * R + M * R + n * (d + 1)),
        "kuu": 4 * (2 * M * R),
        "gather": 4 * (M * R + 2 * N * R + n * (d + 1)),
    }


def cpu_baseline(W, R, X_gpu=None, B=None, budget_s=12.0, pcg_iters=20):
    """The FP64 oracle on the same workload, timed on the host cores: its MVM
    of the R-column block (repeated for about budget_s), and its block PCG with
    the oracle's rank-k pivoted-Cholesky preconditioner, of which `pcg_iters`
    iterations are timed and the seconds to 1e-4 extrapolated from that
    per-iteration time and the oracle's iteration count (stored by
    tests/golden/make_oracle_golden.py from a full oracle run).  With the GPU's
    block-PCG solution X_gpu of B (host arrays, N x R), also the oracle's FP64
    true relative residual ||b - K~ x|| / ||b|| of every column (worst one)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import dski as odski, krylov, pivchol, precond
    op = odski.DSKI(W.X, W.grid_m, W.lo, W.hi, *W.hypers())
    V = np.random.default_rng(0).standard_normal((op.N, R))
    op.matvec(V)  # warm
    t0 = time.perf_counter()
    reps = 0
    while True:
        op.matvec(V)
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 50:
            break
    dt = (time.perf_counter() - t0) / reps
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    Bm = mvm_bytes(op.N, op.grid.size, op.n, op.d, R)
    out = {"value": round(Bm / dt / 1e9, 4), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{reps} FP64 oracle MVMs (scipy CSR + dense Kronecker K_UU) of the {R}-column "
                     f"terrain block, {dt * 1e3:.1f} ms each; {pcg_iters} oracle block-PCG iterations"}
    # block PCG: per-iteration time of the oracle's own loop on the same columns
    L, _, _ = pivchol.pivoted_cholesky(op.diag_K(), op.row_K, W.rank)
    P = precond.Precond(L, op.Dn)
    Bo = B if B is not None else V
    t1 = time.perf_counter()
    krylov.pcg(op.matvec, Bo, precond=P.solve, fixed_iters=pcg_iters)
    per_iter = (time.perf_counter() - t1) / pcg_iters
    gold = os.path.join(ROOT, "tests", "golden", "terrain_full_oracle.json")
    iters = None
    if os.path.exists(gold):
        with open(gold) as f:
            iters = int(max(json.load(f)["iters"]))
    out["pcg_s_per_iter"] = round(per_iter, 5)
    out["pcg_oracle_iters"] = iters
    out["pcg_s"] = round(per_iter * iters, 2) if iters else None
    out["pcg_s_kind"] = ("extrapolated: measured per-iteration time x the iteration count of a full oracle run "
                         "to 1e-4 (stored)")
    if X_gpu is not None and B is not None:
        out["gpu_pcg_true_relres_oracle"] = float(krylov.true_relres(op.matvec, B, X_gpu).max())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mvm-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--grid", type=int, default=200)
    ap.add_argument("--sweep", action="store_true",
                    help="MVM throughput at n = 20k, 200k, 500k (grids 200^2, 632^2, 1000^2; working set above "
                         "the Infinity Cache at the largest) instead of the full step; one JSON line per size")
    ap.add_argument("--variants", default=None,
                    help="S,G,K0,K1: pin the scatter, gather and per-axis K_UU variants after the tuner has run "
                         "(for profiled runs, whose per-dispatch overhead distorts the tuner's timings)")
    ap.add_argument("--dskip-only", action="store_true",
                    help="only the D-SKIP block of the 8-D ridge workload (build, block MVMs, block PCG)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate block of the terrain workload (SLQ and data-fit evaluations, "
                         "training step and inference of the network)")
    ap.add_argument("--predict-only", action="store_true",
                    help="only the prediction block of the terrain workload (grid vector, means of 1,000,000 "
                         "test points, pivoted-Cholesky and randomized variance) and the active-subspace block")
    ap.add_argument("--pcg-only", action="store_true",
                    help="only the terrain block PCG (tuner, pivoted Cholesky, one solve with FP32 and one with "
                         "FP64 vectors): per-kernel profiles of the solver's iteration")
    ap.add_argument("--pmc-summary", nargs="+", metavar="PATH", default=None,
                    help="FETCH_DIR WRITE_DIR LOG [SQ_DIR]: write the PMC summary from rocprofv3 --pmc runs of "
                         "--pmc-mvm (counter folders and the run's stdout), no GPU needed")
    ap.add_argument("--stats-table", default=None, metavar="CSV",
                    help="print the markdown table of a rocprofv3 --stats kernel_stats.csv (no GPU needed)")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="a command line to record in the PMC summary (repeatable)")
    ap.add_argument("--pmc-mvm", action="store_true",
                    help="run only the MVM stages (and a 256 MiB device copy for calibration) for rocprofv3 --pmc")
    a = ap.parse_args(argv)
    if a.stats_table:
        print(stats_table(a.stats_table))
        return 0
    if a.pmc_summary:
        p = a.pmc_summary
        if len(p) not in (3, 4):
            print("--pmc-summary takes FETCH_DIR WRITE_DIR LOG [SQ_DIR]", file=sys.stderr)
            return 2
        t = pmc_summary(p[0], p[1], p[2], p[3] if len(p) == 4 else None, commands=a.pmc_command)
        print(json.dumps({"pmc_summary": PMC_SUMMARY, "traffic": t}))
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the block PCG would shard "
              f"its right-hand sides across GPUs, which is not implemented.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads
    from paper_1810_12283_amd import dski

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    W = workloads.terrain(n=a.n, grid=a.grid)
    pinned = None
    if a.variants:
        pinned = [int(v) for v in a.variants.split(",")]
        if len(pinned) != 2 + len(W.grid_m):
            print(f"--variants needs {2 + len(W.grid_m)} integers (scatter, gather, one K_UU form per axis)",
                  file=sys.stderr)
            return 2
    t_probes = W.num_probes
    R = 1 + t_probes
    X = torch.tensor(W.X, dtype=torch.float64, device=dev)
    y = torch.tensor(W.y.astype(np.float32), device=dev)[None, :].contiguous()
    N, n, d = W.N, W.n, W.d
    M = int(np.prod(W.grid_m))
    Vblk = dski.rademacher(12345, 0, R, N, device=dev)
    Vblk[0] = y[0]

    if a.dskip_only:
        print(json.dumps({"dskip": dskip_block(R, stream)}), flush=True)
        return 0
    if a.surrogate_only:
        print(json.dumps({"surrogate": surrogate_block(W, y, W.rank, stream)}), flush=True)
        return 0
    if a.predict_only:
        print(json.dumps({"predict": predict_block(W, stream), "active_subspace": active_block()}), flush=True)
        return 0

    if a.pcg_only:
        plan = dski.Plan(X, W.grid_m, W.lo, W.hi)
        plan.set_hypers(*W.hypers())
        tune = plan.autotune(R)
        variants = tuned_variants(tune)
        if pinned is not None:
            variants = {"scatter": pinned[0], "gather": pinned[1], "kuu": pinned[2:2 + d]}
            plan.set_variants(variants["scatter"], variants["gather"])
            for ax, v in enumerate(variants["kuu"]):
                plan.set_kuu_variant(ax, v)
        pc = plan.pivchol(W.rank)
        B = torch.empty((R, N), dtype=torch.float32, device=dev)
        B[0] = y[0]
        B[1:] = dski.rademacher(SEED, 0, t_probes, N, device=dev)
        out = {"workload": f"terrain n={n} d={d} grid={W.grid_m[0]}x{W.grid_m[1]} R={R} rank={W.rank}",
               "variants": variants}
        for name, Bv in (("f32", B), ("f64", B.double())):
            _progress(f"pcg {name}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, iters, _, st, _ = plan.pcg(Bv, pc, tol=W.tol, max_iter=20000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            it = int(max(iters))
            out[name] = {"pcg_s": round(dt, 4), "iters": it, "us_per_iter": round(dt / it * 1e6, 2),
                         "status": int(st)}
        print(json.dumps({"pcg_only": out}), flush=True)
        plan.close()
        return 0

    if a.sweep:
        for n_s, g_s in ((20000, 200), (200000, 632), (500000, 1000)):
            Ws = workloads.terrain(n=n_s, grid=g_s)
            Xs = torch.tensor(Ws.X, dtype=torch.float64, device=dev)
            t0 = time.perf_counter()
            plan = dski.Plan(Xs, Ws.grid_m, Ws.lo, Ws.hi)
            plan.set_hypers(*Ws.hypers())
            tune = plan.autotune(R)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            V = dski.rademacher(12345, 0, R, Ws.N, device=dev)
            Vt = plan.permute(V, +1)
            Yt = torch.empty_like(Vt)
            med, p10, p90 = _events_stats(lambda: plan.mvm_tiled(Vt, out=Yt), a.mvm_reps, stream)
            Ms = int(np.prod(Ws.grid_m))
            Bs = mvm_bytes(Ws.N, Ms, Ws.n, Ws.d, R)
            src = torch.ones(Bs // 8, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            ms_copy = _events_stats(lambda: dst.copy_(src), a.mvm_reps, stream)[0]
            del src, dst
            stage = {"scatter": _events_stats(lambda: plan.mvm_stage(0, Vt), a.mvm_reps, stream)[0],
                     "kuu": _events_stats(lambda: plan.mvm_stage(1, Vt), a.mvm_reps, stream)[0]}
            plan.mvm_stage(0, Vt)
            stage["gather"] = _events_stats(lambda: plan.mvm_stage(2, Vt, Yt), a.mvm_reps, stream)[0]
            gbs = Bs / (med * 1e-3) / 1e9
            print(json.dumps({"sweep": f"terrain n={n_s} grid={g_s}x{g_s} R={R}", "N": Ws.N, "grid_nodes": Ms,
                              "algorithmic_bytes": Bs, "mvm_ms": round(med, 4),
                              "mvm_ms_p10_p90": [round(p10, 4), round(p90, 4)], "gbs": round(gbs, 1),
                              "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
                              "copy_gbs_same_size": round(2 * (Bs // 8) * 4 / (ms_copy * 1e-3) / 1e9, 1),
                              "stage_ms": {k: round(v, 4) for k, v in stage.items()},
                              "setup_and_tune_s": round(t_setup, 3),
                              "tuned": {"scatter": _fastest(tune["scatter_us"]),
                                        "gather": _fastest(tune["gather_us"]),
                                        "kuu": ["fft" if t[1] < 0 or t[0] <= t[1] else "dense"
                                                for t in tune["kuu_us"]]}}),
                  flush=True)
            plan.close()
            del Xs, V, Vt, Yt
            torch.cuda.empty_cache()
        return 0

    if a.pmc_mvm:
        plan = dski.Plan(X, W.grid_m, W.lo, W.hi)
        plan.set_hypers(*W.hypers())
        tuned_first = plan.autotune(R)
        Vt = plan.permute(Vblk, +1)
        Yt = torch.empty_like(Vt)
        labels = []

        def mark(label):
            # a 64-entry Rademacher column: a dispatch the summary recognises by name and
            # size, so every dispatch after it (up to the next marker) belongs to `label`
            dski.rademacher(PMC_MARKER_SEED, 0, 1, 64, device=dev)
            labels.append(label)

        # every scatter, gather and K_UU variant a few times (the tuner's pick is not
        # stable while counters are collected; the summary keys traffic by variant)
        for sv in range(len(tuned_first["scatter_us"])):
            if tuned_first["scatter_us"][sv] < 0:  # not a form of this plan
                continue
            plan.set_variants(sv, 0)
            mark(f"scatter_v{sv}")
            for _ in range(3):
                plan.mvm_stage(0, Vt)
        for gv in range(len(tuned_first["gather_us"])):
            plan.set_variants(0, gv)
            plan.mvm_stage(0, Vt)
            mark(f"gather_v{gv}")
            for _ in range(3):
                plan.mvm_stage(2, Vt, Yt)
        for v, name in ((1, "kuu_dense"), (0, "kuu_fft")):
            for ax in range(d):
                plan.set_kuu_variant(ax, v)
            mark(name)
            for _ in range(3):
                plan.mvm_stage(1, Vt)
        # a short direct-launch block PCG with the rank-k preconditioner (per-dispatch counters)
        plan.set_graph(False)
        mark("pivchol")
        pc = plan.pivchol(W.rank)
        mark("pcg")
        plan.pcg(Vblk, pc, tol=1e-30, max_iter=20)
        plan.set_graph(True)
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        mark("copy")
        for _ in range(3):
            dst.copy_(src)                   # runtime copy kernel: 256 MiB read, 256 MiB written
            torch.mul(src, 1.0, out=dst)     # elementwise kernel: the same bytes
        torch.cuda.synchronize()
        print(json.dumps({"pmc_mvm": "done", "copy_bytes": src.numel() * 4, "source": source_digest(),
                          "labels": labels}), flush=True)
        return 0

    def step(record):
        t0 = time.perf_counter()
        plan = dski.Plan(X, W.grid_m, W.lo, W.hi)
        plan.set_hypers(*W.hypers())
        tune = plan.autotune(R)
        variants = tuned_variants(tune)
        if pinned is not None:
            variants = {"scatter": pinned[0], "gather": pinned[1], "kuu": pinned[2:2 + d]}
            plan.set_variants(variants["scatter"], variants["gather"])
            for ax, v in enumerate(variants["kuu"]):
                plan.set_kuu_variant(ax, v)
        Vt = plan.permute(Vblk, +1)
        Yt = torch.empty_like(Vt)
        ms_mvm, ms_p10, ms_p90 = _events_stats(lambda: plan.mvm_tiled(Vt, out=Yt), a.mvm_reps, stream)
        # per stage (each stage's kernels alone between events)
        ms_stage = {"scatter": _events_ms(lambda: plan.mvm_stage(0, Vt), a.mvm_reps, stream)}
        ms_stage["kuu"] = _events_ms(lambda: plan.mvm_stage(1, Vt), a.mvm_reps, stream)
        plan.mvm_stage(0, Vt)  # fresh grid for the gather (K_UU was applied repeatedly)
        ms_stage["gather"] = _events_ms(lambda: plan.mvm_stage(2, Vt, Yt), a.mvm_reps, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pc = plan.pivchol(W.rank)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # block PCG: data vector + 16 probes z = C w (covariance M)
        Wr = dski.rademacher(SEED, 0, t_probes, N, device=dev)
        B = torch.empty((R, N), dtype=torch.float32, device=dev)
        B[0] = y[0]
        B[1:] = Wr  # plain Rademacher probes for the timing solve
        Xs, iters, relres, st, _ = plan.pcg(B, pc, tol=W.tol, max_iter=20000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        res = plan.mll_and_grad(y, pc, num_probes=t_probes, seed=SEED, tol=W.tol, max_iter=20000)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        # the same solve and mll with FP64 vectors (the solver's storage precision
        # above the configuration's FP32: fewer iterations to the same tolerance)
        B64 = B.double()
        Xs64, iters64, _, _, _ = plan.pcg(B64, pc, tol=W.tol, max_iter=20000)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        res64 = plan.mll_and_grad(y.double(), pc, num_probes=t_probes, seed=SEED, tol=W.tol, max_iter=20000)
        torch.cuda.synchronize()
        t6 = time.perf_counter()
        out = None
        if record:
            # true relative residual of the FP64 solutions with the FP64-storage operator
            Bd = B.double()
            Rt = Bd - plan.mvm(Xs)
            true_rel = (Rt.norm(dim=1) / Bd.norm(dim=1)).max().item()
            Rt64 = Bd - plan.mvm(Xs64)
            true_rel64 = (Rt64.norm(dim=1) / Bd.norm(dim=1)).max().item()
            out = dict(X_host=Xs.cpu().numpy().T.copy(), B_host=B.double().cpu().numpy().T.copy(),
                       tune=tune, variants=variants, ms_mvm=ms_mvm, ms_p10=ms_p10, ms_p90=ms_p90, ms_stage=ms_stage,
                       setup_s=t1 - t0, pivchol_s=t2 - t1,
                       pcg_s=t3 - t2, mll_s=t4 - t3, iters=iters, relres=max(relres), status=st,
                       true_rel=true_rel, mll=res["mll"], logdet=res["logdet"],
                       mll_iters=max(res["iters"]), grad=res["grad"].tolist(),
                       pcg64_s=t5 - t4, iters64=iters64, true_rel64=true_rel64, mll64_s=t6 - t5,
                       mll64_iters=max(res64["iters"]), mll64=res64["mll"], logdet64=res64["logdet"])
        pc.close()
        plan.close()
        return out

    for i in range(a.warmup):
        step(False)
        _progress(f"warm-up step {i + 1}/{a.warmup}")
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        recs.append(step(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _progress(f"{a.steps} timed steps in {wall:.1f} s")

    ms_mvm = float(np.mean([r["ms_mvm"] for r in recs]))
    Bm = mvm_bytes(N, M, n, d, R)
    # a device copy of the same number of bytes as one MVM moves (half read, half
    # written): the rate that memory traffic of this size reaches on this GPU
    src = torch.ones(Bm // 8, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms_copy = _events_stats(lambda: dst.copy_(src), a.mvm_reps, stream)[0]
    copy_gbs = round(2 * src.numel() * 4 / (ms_copy * 1e-3) / 1e9, 1)
    del src, dst
    gbs = Bm / (ms_mvm * 1e-3) / 1e9
    sb = stage_bytes(N, M, n, d, R)
    stage_ms = {k: float(np.mean([r["ms_stage"][k] for r in recs])) for k in sb}
    dom = max(stage_ms, key=stage_ms.get)
    ach = sb[dom] / (stage_ms[dom] * 1e-3) / 1e9
    # measured HBM bytes of the dominant stage for the variant the tuner picked
    var = recs[-1]["variants"]
    pick = {"scatter": f"scatter_v{var['scatter']}", "gather": f"gather_v{var['gather']}",
            "kuu": "kuu_" + ("fft" if all(v == 0 for v in var["kuu"]) else "dense")}[dom]
    traffic = (measured_traffic() or {}).get(pick)
    if traffic is not None and dom == "kuu":
        traffic *= d  # one launch per axis
    line = {
        "metric": "D-SKI grad-kernel MVM GB/s; block-PCG s to 1e-4 resid (n=20k,d=2,17 RHS)",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage_dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"terrain n={n} d={d} grid={W.grid_m[0]}x{W.grid_m[1]} R={R} "
                               f"(1 data + {t_probes} probes) k={W.rank} tol={W.tol}",
                   "n": n, "d": d, "N": N, "grid": list(W.grid_m), "rhs": R, "rank": W.rank,
                   "tol": W.tol},
        "mvm_ms": round(ms_mvm, 4),
        "mvm_ms_p10_p90": [round(float(np.mean([r["ms_p10"] for r in recs])), 4),
                           round(float(np.mean([r["ms_p90"] for r in recs])), 4)],
        "copy_gbs_same_size": copy_gbs,
        "mvm_algorithmic_bytes": Bm,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "pcg_s": round(float(np.mean([r["pcg_s"] for r in recs])), 4),
        "pcg_iters": int(max(max(r["iters"]) for r in recs)),
        "pcg_true_relres": float(max(r["true_rel"] for r in recs)),
        "pivchol_s": round(float(np.mean([r["pivchol_s"] for r in recs])), 4),
        "mll_and_grad_s": round(float(np.mean([r["mll_s"] for r in recs])), 4),
        "mll_pcg_iters": int(max(r["mll_iters"] for r in recs)),
        "f64_vectors": {"pcg_s": round(float(np.mean([r["pcg64_s"] for r in recs])), 4),
                        "pcg_iters": int(max(max(r["iters64"]) for r in recs)),
                        "pcg_true_relres": float(max(r["true_rel64"] for r in recs)),
                        "mll_and_grad_s": round(float(np.mean([r["mll64_s"] for r in recs])), 4),
                        "mll_pcg_iters": int(max(r["mll64_iters"] for r in recs)),
                        "mll": recs[-1]["mll64"], "logdet": recs[-1]["logdet64"]},
        "autotune_us": recs[-1]["tune"],
        "variants": recs[-1]["variants"],
        "variants_pinned": pinned is not None,
        "mll": recs[-1]["mll"],
        "logdet": recs[-1]["logdet"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
    }
    blocks = (("torus", lambda: grid_block(workloads.torus(), R, stream)),
              ("terrain_quintic", lambda: grid_block(W, R, stream, interp="quintic")),
              ("torus_spline", lambda: grid_block(workloads.torus(), R, stream, kernel="spline")),
              ("dskip", lambda: dskip_block(R, stream)),
              ("surrogate", lambda: surrogate_block(W, y, W.rank, stream)),
              ("predict", lambda: predict_block(W, stream)),
              ("active_subspace", active_block),
              ("bo_alg1", bo_block))
    for name, fn in blocks:
        tb = time.perf_counter()
        line[name] = fn()
        _progress(f"{name} block {time.perf_counter() - tb:.1f} s")
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, R, recs[-1]["X_host"], recs[-1]["B_host"])
        # the headline solve's residual as the oracle's FP64 operator sees it
        line["pcg_true_relres_oracle"] = line["cpu_baseline"].get("gpu_pcg_true_relres_oracle")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
