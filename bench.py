"""Benchmark of the covariance apply and of time-to-k eigenpairs on one MI355X.

A step is one covariance apply (Algorithm 1) of a 32-vector block: forward Kronecker
stages, the stage-5 covariance-times-block kernel, backward Kronecker stages.  The
headline is the 3D workload (24^3 quadratic sine-perturbed cube, 17,576 dofs, exponential
kernel) with stage 5 in FP64, the paper's arithmetic.  value = pair evaluations per second
= Ntilde^2 per step / step time.  The same run reports the stage-5 kernel against its
roofline (HIP events around every stage-5 launch in the timed region), times the FP32,
BF16x3 and BF16 stage-5 kernels on the same block, times the eigensolve to k pairs at
relative residual 1e-6 in every form, and times the CPU oracle on the same workload (all
host cores, and one core on a bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube24|annulus64|annulus48|square16]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
# vector-ALU lane operations per second: 256 compute units x 64 lanes x 2.4 GHz
VALU_LANE_OPS = 256 * 64 * 2.4e9
# HBM bytes per stage-5 launch from the FETCH_SIZE / WRITE_SIZE counter passes (scaled by a
# plain 256 MiB copy), keyed by (workload, precision, rb, nsplit), or (workload, "f64",
# "symmetric") for the symmetric form with its automatic work split (covariance kernel
# and ordered reduction); see profiles/stage5_f64_cube24_hbm_traffic.md,
# profiles/stage5_f64sym_cube24_hbm_traffic.md and profiles/stage5_f32_annulus64_hbm_traffic.md.
# Only reported for the setting it was measured on.
MEASURED_TRAFFIC = {("cube24", "f64", 4, 10): 82960 * 1024, ("annulus64", "f32", 8, 6): 8434 * 1024,
                    ("cube24", "f64", "symmetric"): 517741 * 1024}
WORKLOADS = {
    "annulus64": ("2D quarter annulus (r in [1,2], NURBS map) 64x64 cubic, Ntilde = N = 4489, "
                  "squared exponential L = 0.5, k = 40"),
    "cube24": ("3D sine-perturbed unit cube 24^3 quadratic, Ntilde = N = 17576, exponential L = 0.5, "
               "k = 50"),
    "annulus48": "2D quarter annulus 48x48 cubic, Ntilde = N = 2601, squared exponential L = 0.5, k = 16",
    "square16": "2D unit square 16x16 quadratic, Ntilde = N = 324, exponential L = 1, k = 20",
}


def cpu_baseline(desc, b, budget_s=12.0):
    """Oracle (literal Algorithm 1 with the C/OpenMP FP64 stage 5) applied to 32-vector
    blocks of the same workload on every host core until about budget_s seconds have passed
    (at least one whole apply)."""
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
            "sample": "%d whole oracle applies (FP64, %d-vector block) of the same workload in %.1f s"
                      % (n, b, dt)}, float(np.float64(dt / n))


def cpu_baseline_one_core(desc, b, budget_s=8.0):
    """The same oracle apply on one core (one OpenMP thread, one BLAS thread), for the
    like-for-like comparison with the paper's single-core runs: the Kronecker stages on the
    whole block, stage 5 on a bounded sample of rows (all columns, all vectors), its time
    scaled to all rows."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import cstage5, operator
    P = operator.Problem(desc)
    V = workloads.random_block(P.N, b, seed=0)
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        Y = P.forward(V)
        P.backward(Y)
        t_kron = time.perf_counter() - t
        rows = 64
        while True:
            t = time.perf_counter()
            cstage5.stage5(P, Y, rows=(0, rows), threads=1)
            dt = time.perf_counter() - t
            if dt > budget_s / 4 or rows >= P.Nt:
                break
            rows = min(P.Nt, rows * 4)
    t_apply = t_kron + dt * P.Nt / rows
    return {"value": P.Nt ** 2 / t_apply, "unit": "pair evals/s", "cores": 1, "kind": "oracle",
            "sample": "one oracle apply (FP64, %d-vector block): Kronecker stages in full (%.2f s), stage 5 "
                      "on %d of %d rows (%.1f s), scaled to all rows" % (b, t_kron, rows, P.Nt, dt)}


def oracle_time_to_k(desc, k):
    """The oracle's eigenpairs by ARPACK (the paper's implicitly restarted Lanczos family,
    one vector per apply, C/OpenMP stage 5 on every host core) to relative accuracy 1e-6."""
    from oracle import cstage5, operator
    from oracle import eigs as oeigs
    P = operator.Problem(desc)
    count = [0]

    def s5(Y):
        count[0] += 1 if Y.ndim == 1 else Y.shape[1]
        return cstage5.stage5(P, Y)
    t = time.perf_counter()
    oeigs.iterative_eigs(P, k, tol=1e-6, stage5=s5)
    return {"seconds": time.perf_counter() - t, "applies": count[0], "k": k,
            "cores": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()}


def measured_rates():
    """Issue rates measured by the library's rate microbenchmark (lib/klrates), or None."""
    exe = os.path.join(ROOT, "paper_2011_13861_amd", "lib", "klrates")
    if not os.path.exists(exe):
        return None
    import subprocess
    r = subprocess.run([exe, "2048"], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return None
    out = {}
    for line in r.stdout.splitlines():
        rec = json.loads(line)
        out[rec.pop("test")] = rec
    return out


def valu_slots_per_pair(kind, d, precision, rates):
    """Algorithmic vector-ALU issue slots per pair of the exp2-based kernels (FP32 kernel
    evaluation): d subtractions and d multiply-adds for the squared distance (d for the L1
    form), a square root for the exponential kernel, one base-2 exponential, and the
    rounding of the value to the matrix operand (BF16: one conversion; BF16x3: the hi part,
    the remainder and its conversion).  The square root and exponential cost their measured
    issue time relative to an FMA."""
    fma_ns = rates["fma_f32"]["ns_per_wave_instr_per_simd"]
    c_exp = rates["exp_f32"]["ns_per_wave_instr_per_simd"] / fma_ns
    c_sqrt = rates["sqrt_f32"]["ns_per_wave_instr_per_simd"] / fma_ns
    s = 2 * d + c_exp
    if kind == "exp":
        s += c_sqrt
    s += {"f32": 0, "bf16": 1, "bf16x3": 3}[precision]
    return s, c_exp, c_sqrt


def warm_start_section(n_train, epochs, n_eval, solves=3, subspace=3.0):
    """Warm-start section: the network is trained on n_train method-generated FP64 solves (tol 1e-10)
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
    losses = ws.fit(warmstart.features(L, a, flag), T, epochs=epochs, batch=64, lr0=1e-3, lr1=3e-5,
                    subspace=subspace)
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
    return {"workload": "annulus48: 2D quarter annulus 48x48 cubic, N = 2601, k = 16, block 16; "
                        "L ~ logU[0.1,2], a ~ logU[0.5,2], flag ~ B(1/2)",
            "n_train": n_train, "epochs": epochs, "subspace_weight": subspace, "generate_s": gen_s, "train_s": train_s,
            "loss_first_last": [float(losses[0]), float(losses[-1])], "n_eval": n_eval,
            "median_ms": med, "mean_applies": {k: float(np.mean(v)) for k, v in app.items()},
            "f32_warm_speedup_vs_f64": med["f64"] / med["f32_warm"],
            "f64_warm_speedup_vs_f64": med["f64"] / med["f64_warm"]}


def batch_section(reps=20, eigs=True):
    """Batch section: 64 uneven 2D problems (seed 1127).  The batched apply (one graph replay
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
    out = {"workload": "batch64: 64 unit-square problems, nelem ~ U{16..96}^2, p ~ U{2,3,4}, exp/sqexp, "
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
    if not eigs:
        return out
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


def stage5_runs(G, kind, prec, x, y, steps, warmup, tune, objective, tiles=None, symmetric="auto"):
    """Times `steps` applies of the 32-vector block in one precision (stage-5 tiles tuned or
    forced; FP64 stage 5 in its symmetric form as tuned, or forced on / off); returns (ms
    per apply, stage-5 launches, stage-5 ms in total, tiles)."""
    import torch
    if tiles:
        G.stage5_config(prec, rb=tiles[0], nsplit=tiles[1])
    elif tune:
        from paper_2011_13861_amd import autotune
        autotune.tune_problem(G, kind, precisions=(prec,), reps=10, objective=objective)
    if prec in ("f64", "bf16", "bf16x3") and symmetric != "auto":
        G.stage5_symmetric(symmetric == "on", precision=prec)
    for _ in range(warmup):
        G.apply(x, y, prec)
    torch.cuda.synchronize()
    G.profile_enable(True)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        G.apply(x, y, prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    cnt, kms = G.profile_read()[prec]
    G.profile_enable(False)
    return ev0.elapsed_time(ev1) / steps, cnt, kms, G.stage5_config(prec)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cube24", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "bf16x3", "bf16"],
                    help="stage-5 precision of the headline (default FP64, the paper's arithmetic)")
    ap.add_argument("--other-precisions", default="f32,bf16x3,bf16",
                    help="stage-5 precisions timed beside the headline ('' = none)")
    ap.add_argument("--eig-precisions", default="f64,f32,bf16x3,bf16",
                    help="forms timed to k eigenpairs at 1e-6 (low precisions with FP64 refinement)")
    ap.add_argument("--solves", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-eigs", action="store_true",
                    help="also time the oracle's ARPACK eigenpairs on the host cores (about a minute on the 24^3 cube)")
    ap.add_argument("--symmetric", choices=("auto", "on", "off"), default="auto",
                    help="stage 5 of the headline precision (FP64, BF16, BF16x3) in its symmetric form: "
                         "as the tuner finds faster (auto), or forced")
    ap.add_argument("--mlp-train", type=int, default=2000,
                    help="training solves for the warm-start section (0 = skip the section)")
    ap.add_argument("--mlp-epochs", type=int, default=1000)
    ap.add_argument("--mlp-subspace", type=float, default=3.0,
                    help="weight of the subspace term of the warm-start loss (0 = per-eigenvector term only)")
    ap.add_argument("--mlp-eval", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch section")
    ap.add_argument("--no-batch-eigs", action="store_true",
                    help="in the batch section, time the batched applies only (no eigensolves)")
    ap.add_argument("--no-tune", action="store_true", help="keep the automatic stage-5 split")
    ap.add_argument("--tune-objective", default="apply", choices=["apply", "stage5"],
                    help="what the stage-5 tile search minimises: the whole apply (default) or the kernel alone")
    ap.add_argument("--tiles", default=None, metavar="RB,NSPLIT",
                    help="force the headline's stage-5 tiles instead of tuning (e.g. 2,6), for profiler runs")
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
    kind = desc["cov"]["kind"]
    prec = args.precision
    G = kl.Problem(desc)
    x = kl.to_device_block(workloads.random_block(G.N, b, seed=1))
    y = kl.new_block(G.N, b)
    tiles = tuple(int(v) for v in args.tiles.split(",")) if args.tiles else None
    t0 = time.perf_counter()
    ms_per_step, cnt, kms, tiles = stage5_runs(G, kind, prec, x, y, args.steps, args.warmup,
                                               not args.no_tune, args.tune_objective, tiles, args.symmetric)
    sym = prec in G.symmetric
    # kernel values the symmetric form evaluates per launch: the 2 NB (NB + 1) tiles of 64 x
    # 256 (NB 256-point blocks of the padded grid) at or below the diagonal blocks
    nb = (G.Nt + 255) // 256
    evaluated = 2.0 * nb * (nb + 1) * 64 * 256
    wall = time.perf_counter() - t0
    pairs = float(G.Nt) ** 2
    value = pairs / (ms_per_step * 1e-3)
    k_avg_s = kms / max(cnt, 1) * 1e-3
    flops = 2.0 * b * pairs                    # matrix-core contraction flops per stage-5 launch
    if prec == "f64":
        # FP64: the kernel evaluation (vector ALU) and the contraction (matrix cores) share
        # the FP64 arithmetic rate (they were measured not to overlap on this chip), so the
        # bound is FP64 arithmetic with the paper-style flops of a pair: per coordinate a
        # subtraction and a square (3d - 1 with the sum), the scaling, one exponential, one
        # square root for the exponential kernel, and 2b for the contraction
        d = desc["dim"]
        per_pair = (3 * d - 1) + 1 + 1 + (1 if kind == "exp" else 0) + 2 * b
        achieved = per_pair * pairs / k_avg_s / 1e12
        bound = "alu"
        if sym:
            # symmetric form: every evaluated kernel value serves two pairs; the algorithmic
            # flops are those of the evaluated values plus the full contraction
            achieved = ((per_pair - 2 * b) * evaluated + 2 * b * pairs) / k_avg_s / 1e12
    else:
        per_pair = 2 * b
        achieved = flops / k_avg_s / 1e12
        bound = "mfma"
    roofline = {"bound": bound, "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[prec],
                "traffic": MEASURED_TRAFFIC.get((args.workload, prec) + tuple(tiles)),
                "flops_per_pair": per_pair,
                "contraction_only_frac": flops / k_avg_s / 1e12 / PEAK_TFLOPS[prec],
                "kernel": "stage5_%s_kernel" % prec, "kernel_avg_us": k_avg_s * 1e6,
                "kernel_pairs_per_s": pairs / k_avg_s, "launches": cnt,
                "stage5_tiles": {"rb": tiles[0], "nsplit": tiles[1]},
                "stage5_form": "symmetric" if sym else "plain"}
    if sym:
        roofline["kernel"] = "stage5_%s_sym_kernel + sym_reduce_kernel" % ("f64" if prec == "f64" else "bf16")
        roofline["evaluated_pairs"] = evaluated
        roofline["logical_pairs"] = pairs
        roofline["traffic"] = MEASURED_TRAFFIC.get((args.workload, prec, "symmetric"))
    rates = measured_rates()

    # the other stage-5 precisions on the same block (matrix-core and vector-ALU bounds)
    others = {}
    for p in [q for q in args.other_precisions.split(",") if q and q != prec]:
        ms_p, cnt_p, kms_p, tiles_p = stage5_runs(G, kind, p, x, y, args.steps, args.warmup,
                                                  not args.no_tune, args.tune_objective)
        ks = kms_p / max(cnt_p, 1) * 1e-3
        ach = flops / ks / 1e12
        rec = {"apply_ms": ms_p, "apply_pair_evals_per_s": pairs / (ms_p * 1e-3), "kernel_avg_us": ks * 1e6,
               "kernel_pairs_per_s": pairs / ks, "mfma_achieved_TFLOPs": ach,
               "mfma_frac": ach / PEAK_TFLOPS[p], "stage5_tiles": {"rb": tiles_p[0], "nsplit": tiles_p[1]},
               "stage5_form": "symmetric" if p in G.symmetric else "plain"}
        if rates is not None:
            # the vector-ALU bound counts the kernel values the form evaluates
            slots, c_exp, c_sqrt = valu_slots_per_pair(kind, desc["dim"], p, rates)
            values = evaluated if p in G.symmetric else pairs
            rec["valu_bound"] = {"slots_per_value": slots, "exp_cost_fma": c_exp, "sqrt_cost_fma": c_sqrt,
                                 "evaluated_values": values, "peak_values_per_s": VALU_LANE_OPS / slots,
                                 "frac": (values / ks) / (VALU_LANE_OPS / slots)}
        others[p] = rec

    # time to k eigenpairs at relative residual 1e-6 (criterion under the FP64 operator)
    def solve(p):
        G.eigs(k, precision=p, block=b, tol=1e-6)          # warm (allocations, handles)
        times, reps = [], []
        for _ in range(args.solves):
            torch.cuda.synchronize()
            t = time.perf_counter()
            w, V, rep = G.eigs(k, precision=p, block=b, tol=1e-6)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            reps.append(rep)
        i = int(np.argsort(times)[len(times) // 2])
        return times[i], reps[i]
    time_to_k = {}
    if args.solves > 0:
        for p in [q for q in args.eig_precisions.split(",") if q]:
            t_p, rep_p = solve(p)
            time_to_k[p + ("_refined_fp64" if p != "f64" else "") + "_ms"] = t_p * 1e3
            time_to_k[p + "_report"] = rep_p

    # truncated KL expansion from the k eigenpairs: m field samples and the variance at the
    # Greville points (kl_kle_field); inputs resident, HIP events on the default stream
    kle_out = None
    if args.solves > 0:
        w, V, _ = G.eigs(k, precision="f64", block=b, tol=1e-6)
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
        "stage5_other_precisions": others,
        "measured_rates": rates,
        "time_to_k": time_to_k,
        "wall_s_timed_region": wall,
        "kle_field": kle_out,
    }
    if not args.no_batch:
        out["batch"] = batch_section(eigs=not args.no_batch_eigs)
    if args.mlp_train > 0:
        out["warm_start"] = warm_start_section(args.mlp_train, args.mlp_epochs, args.mlp_eval,
                                               subspace=args.mlp_subspace)
    if not args.no_cpu:
        cb, _ = cpu_baseline(desc, b)
        out["cpu_baseline"] = cb
        out["cpu_baseline_1core"] = cpu_baseline_one_core(desc, b)
        if args.oracle_eigs:
            out["oracle_time_to_k"] = oracle_time_to_k(desc, k)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
