"""Benchmark of the covariance apply and of time-to-k eigenpairs on one MI355X.

A step is one covariance apply (Algorithm 1) of a 32-vector block: forward Kronecker
stages, the stage-5 covariance-times-block kernel in the workload's precision, backward
Kronecker stages.  value = pair evaluations per second = Ntilde^2 per step / step time.
The same run also times the eigensolve to k pairs at relative residual 1e-6 (FP32 form
with FP64 refinement, and the plain FP64 form), reports the stage-5 kernel against its
roofline (HIP events around every stage-5 launch in the timed region), and times the
CPU oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c5|c1]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
# HBM bytes per stage-5 launch from the FETCH_SIZE / WRITE_SIZE counter passes (scaled by a
# plain 256 MiB copy), keyed by (workload, precision, rb, nsplit); see
# profiles/stage5_f32_c2_hbm_traffic.md.  Only reported for the setting it was measured on.
MEASURED_TRAFFIC = {("c2", "f32", 2, 6): 8453 * 1024, ("c2", "f32", 2, 7): 9029 * 1024,
                    ("c2", "f32", 8, 6): 8428 * 1024, ("c2", "f32", 8, 7): 9003 * 1024}
WORKLOADS = {
    "c2": ("2D quarter annulus (r in [1,2], NURBS map) 64x64 cubic, Ntilde = N = 4489, "
           "squared exponential L = 0.5, k = 40"),
    "c3": ("3D sine-perturbed unit cube 24^3 quadratic, Ntilde = N = 17576, exponential L = 0.5, "
           "k = 50"),
    "c5": "2D quarter annulus 48x48 cubic, Ntilde = N = 2601, squared exponential L = 0.5, k = 16",
    "c1": "2D unit square 16x16 quadratic, Ntilde = N = 324, exponential L = 1, k = 20",
}


def cpu_baseline(desc, b, budget_s=12.0):
    """Oracle (literal Algorithm 1 with the C/OpenMP stage 5, FP64) applied to 32-vector
    blocks of the same workload until about budget_s seconds have passed."""
    import numpy as np

    import workloads
    from oracle import cstage5, operator
    P = operator.Problem(desc)
    V = workloads.random_block(P.N, b, seed=0)
    s5 = lambda Y: cstage5.stage5(P, Y)   # noqa: E731
    P.apply(V[:, :1], stage5=s5)          # load the shared object
    n = 0
    t0 = time.perf_counter()
    while True:
        P.apply(V, stage5=s5)
        n += 1
        dt = time.perf_counter() - t0
        if dt > budget_s or n >= 50:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": P.Nt ** 2 * n / dt, "unit": "pair evals/s", "cores": threads, "kind": "oracle",
            "sample": "%d oracle applies (FP64, %d-vector block) of the same workload in %.1f s"
                      % (n, b, dt)}, float(np.float64(dt / n))


def warm_start_section(n_train, epochs, n_eval, solves=3):
    """Config 5: the network is trained on n_train method-generated FP64 solves (tol 1e-10)
    of the 48x48 cubic quarter annulus (training draws seed 2000), then the held-out draws
    (seed 2001) are solved to 1e-6 four ways: plain FP64 from a random block, FP32 with
    FP64 refinement from a random block, the same from the predicted block, and plain FP64
    from the predicted block (network inference included in the timed warm solves).  Times
    are medians over the held-out draws."""
    import numpy as np
    import torch

    import paper_2011_13861_amd as kl
    import workloads
    from paper_2011_13861_amd import warmstart
    K = 16

    def covs(L, a, flag):
        out = []
        for Li, ai, fi in zip(L, a, flag):
            d = workloads.mlp_problem(Li, ai, fi)
            out.append((d["cov"]["kind"], d["cov"]["sigma2"], d["cov"]["corr_len"]))
        return out

    G = kl.Problem(workloads.mlp_problem(1.0, 1.0, 0))
    L, a, flag = workloads.mlp_parameters(2000, n_train)
    t = time.perf_counter()
    T, _, _ = warmstart.generate(G, covs(L, a, flag), K, block=16, tol=1e-10)
    gen_s = time.perf_counter() - t
    ws = warmstart.WarmStart(G.N, K, seed=0)
    t = time.perf_counter()
    losses = ws.fit(warmstart.features(L, a, flag), T, epochs=epochs, batch=64, lr0=1e-3, lr1=3e-5)
    train_s = time.perf_counter() - t
    del T
    Le, ae, fe = workloads.mlp_parameters(2001, n_eval)
    rec = {"f64": [], "f32_random": [], "f32_warm": [], "f64_warm": []}
    app = {k: [] for k in rec}
    for i, cov in enumerate(covs(Le, ae, fe)):
        G.set_cov(*cov)
        f = warmstart.features(Le[i], ae[i], fe[i])[0]
        runs = {"f64": lambda: G.eigs(K, precision="f64", block=16, tol=1e-6),
                "f32_random": lambda: G.eigs(K, precision="f32", block=16, tol=1e-6),
                "f32_warm": lambda: warmstart.solve(G, K, ws, f, precision="f32", block=16, tol=1e-6),
                "f64_warm": lambda: warmstart.solve(G, K, ws, f, precision="f64", block=16, tol=1e-6)}
        for name, fn in runs.items():
            best = None
            for _ in range(solves):
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, _, rep = fn()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            rec[name].append(best)
            app[name].append(sum(rep["n_applies"]))
    med = {k: float(np.median(v)) * 1e3 for k, v in rec.items()}
    return {"workload": "c5: 2D quarter annulus 48x48 cubic, N = 2601, k = 16, block 16; "
                        "L ~ logU[0.1,2], a ~ logU[0.5,2], flag ~ B(1/2)",
            "n_train": n_train, "epochs": epochs, "generate_s": gen_s, "train_s": train_s,
            "loss_first_last": [float(losses[0]), float(losses[-1])], "n_eval": n_eval,
            "median_ms": med, "mean_applies": {k: float(np.mean(v)) for k, v in app.items()},
            "f32_warm_speedup_vs_f64": med["f64"] / med["f32_warm"],
            "f64_warm_speedup_vs_f64": med["f64"] / med["f64_warm"]}


def batch_section(reps=20):
    """Config 4: 64 uneven 2D problems (seed 1127).  The batched apply (one graph replay
    of 32 columns per problem, autotuned tiles) against the same 64 applies issued one
    problem after the other; then 20 eigenpairs of every problem at 1e-6, batched
    (FP32 with FP64 refinement, median of three runs: the solve is bound by host threads
    and varies from run to run) against 64 sequential kl_eigs calls."""
    import numpy as np
    import torch

    import paper_2011_13861_amd as kl
    import workloads
    from paper_2011_13861_amd import autotune
    descs = workloads.batch_problems(1127)
    kinds = [d["cov"]["kind"] for d in descs]
    B = kl.Batch(descs)
    pairs = float(sum(nt * nt for nt in B.Nt))
    out = {"workload": "c4: 64 unit-square problems, nelem ~ U{16..96}^2, p ~ U{2,3,4}, exp/sqexp, "
                       "L ~ logU[0.1,2] (seed 1127), 32 vectors each",
           "pairs_per_apply": pairs}
    x = torch.randn(B.Ntot * 32, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    singles = [kl.Problem(d) for d in descs]
    for prec in ("f32", "f64"):
        rb, lc, _ = autotune.tune_batch(B, kinds, prec, reps=5)
        for _ in range(3):
            B.apply(x, y, 32, prec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            B.apply(x, y, 32, prec)
        e1.record()
        torch.cuda.synchronize()
        t_b = e0.elapsed_time(e1) / reps * 1e-3
        xs = [B.block(x, i, 32) for i in range(B.n)]
        ys = [kl.new_block(G.N, 32) for G in singles]
        for G, xi, yi in zip(singles, xs, ys):
            G.apply(xi, yi, prec)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(max(1, reps // 4)):
            for G, xi, yi in zip(singles, xs, ys):
                G.apply(xi, yi, prec)
        e1.record()
        torch.cuda.synchronize()
        t_s = e0.elapsed_time(e1) / max(1, reps // 4) * 1e-3
        out["apply_" + prec] = {"batched_ms": t_b * 1e3, "pair_evals_per_s": pairs / t_b, "rb": rb, "lchunk": lc,
                                "sequential_ms": t_s * 1e3, "speedup": t_s / t_b}
    B.eigs(20, precision="f32", block=32, tol=1e-6)          # warm (solver buffers, handles)
    t_ebs = []                                               # host-thread bound: median of three
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ev, _, reps_b = B.eigs(20, precision="f32", block=32, tol=1e-6)
        torch.cuda.synchronize()
        t_ebs.append(time.perf_counter() - t)
    t_eb = float(np.median(t_ebs))
    seq = {}
    for prec in ("f32", "f64"):
        for G in singles[:2]:
            G.eigs(20, precision=prec, block=32, tol=1e-6)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for G in singles:
            G.eigs(20, precision=prec, block=32, tol=1e-6)
        torch.cuda.synchronize()
        seq[prec] = (time.perf_counter() - t) * 1e3
    out["eigs_k20"] = {"batched_f32_refined_ms": t_eb * 1e3, "batched_runs_ms": [t * 1e3 for t in t_ebs],
                       "all_converged": all(r["converged"] == 20 for r in reps_b),
                       "sequential_f32_refined_ms": seq["f32"], "sequential_f64_ms": seq["f64"],
                       "speedup_vs_sequential_f64": seq["f64"] / (t_eb * 1e3)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["f32", "f64"])
    ap.add_argument("--solves", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mlp-train", type=int, default=2000,
                    help="training solves for the warm-start section (0 = skip the section)")
    ap.add_argument("--mlp-epochs", type=int, default=1000)
    ap.add_argument("--mlp-eval", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true", help="skip the config-4 batch section")
    ap.add_argument("--no-tune", action="store_true", help="keep the automatic stage-5 split")
    ap.add_argument("--tune-objective", default="apply", choices=["apply", "stage5"],
                    help="what the stage-5 tile search minimises: the whole apply (default) or the kernel alone")
    ap.add_argument("--tiles", default=None, metavar="RB,NSPLIT",
                    help="force the stage-5 tiles instead of tuning (e.g. 2,6), for profiler runs")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MB",
                    help="also run one plain device-to-device copy of MB MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (it has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2011_13861_amd as kl
    import workloads

    torch.cuda.set_device(0)
    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    desc, k, b = workloads.config(args.workload)
    prec = args.precision or "f32"
    G = kl.Problem(desc)
    if args.tiles:
        rb_, ns_ = (int(v) for v in args.tiles.split(","))
        G.stage5_config(prec, rb=rb_, nsplit=ns_)
    elif not args.no_tune:
        from paper_2011_13861_amd import autotune
        autotune.tune_problem(G, desc["cov"]["kind"], precisions=(prec,), reps=10, objective=args.tune_objective)
    x = kl.to_device_block(workloads.random_block(G.N, b, seed=1))
    y = kl.new_block(G.N, b)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        G.apply(x, y, prec)
    torch.cuda.synchronize()
    G.profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        G.apply(x, y, prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = G.profile_read()
    G.profile_enable(False)
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    pairs = float(G.Nt) ** 2
    value = pairs / (ms_per_step * 1e-3)
    cnt, kms = prof[prec]
    k_avg_s = kms / max(cnt, 1) * 1e-3
    flops = 2.0 * b * pairs                    # MFMA contraction flops per stage-5 launch
    achieved = flops / k_avg_s / 1e12
    tiles = G.stage5_config(prec)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[prec],
                "traffic": MEASURED_TRAFFIC.get((args.workload, prec) + tuple(tiles)),
                "kernel": "stage5_%s_kernel" % prec, "kernel_avg_us": k_avg_s * 1e6,
                "kernel_pairs_per_s": pairs / k_avg_s, "launches": cnt,
                "stage5_tiles": {"rb": tiles[0], "nsplit": tiles[1]}}

    # time to k eigenpairs at relative residual 1e-6 (criterion under the FP64 operator)
    def solve(p):
        G.eigs(k, precision=p, tol=1e-6)          # warm (allocations, handles)
        times, reps = [], []
        for _ in range(args.solves):
            torch.cuda.synchronize()
            t = time.perf_counter()
            w, V, rep = G.eigs(k, precision=p, tol=1e-6)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            reps.append(rep)
        i = int(np.argsort(times)[len(times) // 2])
        return times[i], reps[i]
    if args.solves > 0:
        t_lo, rep_lo = solve("f32")
        t_64, rep_64 = solve("f64")
    else:
        t_lo = t_64 = float("nan")
        rep_lo = rep_64 = None

    # truncated KL expansion from the k eigenpairs: m field samples and the variance at the
    # Greville points (kl_kle_field); inputs resident, HIP events on the default stream
    kle_out = None
    if args.solves > 0:
        w, V, _ = G.eigs(k, precision="f64", tol=1e-6)
        m = 1024
        xi = kl.to_device_block(np.random.default_rng(5).standard_normal((k, m)))
        for _ in range(3):
            G.kle_field(w, V, xi)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            G.kle_field(w, V, xi)
        e1.record()
        torch.cuda.synchronize()
        t_kle = e0.elapsed_time(e1) / reps * 1e-3
        kle_bytes = 8 * (G.N * k + k * m + G.Nt * m + G.Nt)
        kle_out = {"M": k, "samples": m, "ms": t_kle * 1e3, "samples_per_s": m / t_kle,
                   "algorithmic_bytes": kle_bytes, "achieved_GBps": kle_bytes / t_kle / 1e9,
                   "hbm_frac": kle_bytes / t_kle / 8e12}

    out = {
        "metric": "covariance-apply pair evals/s (% peak); time to k eigenpairs at 1e-6 err",
        "value": value, "unit": "pair evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "block": b, "k": k, "stage5_precision": prec},
        "roofline": roofline,
        "time_to_k": {"f32_refined_fp64_ms": t_lo * 1e3, "f64_ms": t_64 * 1e3,
                      "f32_report": rep_lo, "f64_report": rep_64},
        "wall_s_timed_region": wall,
        "kle_field": kle_out,
    }
    if not args.no_batch:
        out["batch"] = batch_section()
    if args.mlp_train > 0:
        out["warm_start"] = warm_start_section(args.mlp_train, args.mlp_epochs, args.mlp_eval)
    if not args.no_cpu:
        cb, _ = cpu_baseline(desc, b)
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
