#!/usr/bin/env python3
"""Benchmark of the MHAR step on one MI355X.

Workload (single-GPU configuration of the headline metric): random
full-dimensional polytope, n = 100, m = 2000 unit-norm Gaussian rows, b = 1
(contains the unit ball), z = 1024 walks started at the origin, exact FP64
slack recompute every 50 steps, A*D on the matrix cores in FP32 and in the
BF16x3 split (the faster of the two is reported, the other is listed).

A "step" is one MHAR iteration of all z walks (directions, screening
product, exact chords, update).  value = z * steps / seconds (chain-steps/s,
the paper's samples per second with no thinning).  Inputs are resident in
HBM before timing starts.  Also reported:
  * roofline of the step kernel from HIP events around every launch;
  * min-marginal ESS/s from a bitwise-identical recorded replay of 64 walks;
  * the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chain-steps/sec and min-marginal ESS/sec at 1 GPU, learned vs plain MHAR"
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "fp64": 78.6}
MFMA_PER_FLOP = {"fp32": 1, "bf16x3": 3, "fp64": 1}   # matrix-core products per algorithmic product


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(p, precision, steps, warmup, launch_steps, seed=0):
    import torch
    from paper_2104_07097_amd import mhar
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(a, device=dev, dtype=torch.float64)
    prob = mhar.Problem(t(p.A), t(p.b), precision=precision, recompute_every=50,
                        steps_per_launch=launch_steps)
    ch = mhar.Chains(prob, t(p.X0), seed=seed)
    ch.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    nlaunch = steps // launch_steps
    events = [torch.cuda.Event(enable_timing=True) for _ in range(nlaunch + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    events[0].record(stream)
    for i in range(nlaunch):
        ch.step(launch_steps)
        events[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch = [events[i].elapsed_time(events[i + 1]) / 1e3 for i in range(nlaunch)]
    gpu_time = sum(per_launch)
    flags = ch.sync()
    stats = ch.stats()
    X, _ = ch.state()
    X = X.cpu().numpy()
    ch.close()
    prob.close()
    return dict(wall=wall, gpu_time=gpu_time, per_launch=per_launch, flags=flags, stats=stats, X=X)


def record_ess(p, precision, steps, warmup, launch_steps, chains=64, seed=0):
    """Replay the same trajectories (same seed) recording `chains` walks every step."""
    import numpy as np
    import torch
    from paper_2104_07097_amd import mhar
    from paper_2104_07097_amd.stats import min_marginal_ess
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(a, device=dev, dtype=torch.float64)
    prob = mhar.Problem(t(p.A), t(p.b), precision=precision, recompute_every=50,
                        steps_per_launch=launch_steps)
    ch = mhar.Chains(prob, t(p.X0), seed=seed)
    ch.step(warmup)
    rec = ch.record(steps, 1, chains)
    torch.cuda.synchronize()
    samples = rec.cpu().numpy()
    X, _ = ch.state()
    X = X.cpu().numpy()
    ch.close()
    prob.close()
    ess_min, per = min_marginal_ess(samples)
    return ess_min * (p.z / chains), X, float(np.median(per)) * (p.z / chains)


def cpu_baseline(p, seconds):
    import numpy as np
    import oracle
    orc = oracle.Oracle()
    threads = min(16, os.cpu_count() or 1)
    # calibrate on 1 step, then run a bounded sample of ~`seconds` of CPU work
    t0 = time.perf_counter()
    X, _, _ = orc.run(p.A, p.b, p.X0, 1, seed=0, threads=threads)
    one = time.perf_counter() - t0
    k = int(max(1, min(200, seconds / max(one, 1e-6))))
    t0 = time.perf_counter()
    orc.run(p.A, p.b, X, k, seed=0, step0=1, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": p.z * k / dt, "unit": "chain-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"all {p.z} walks, steps 1..{k} of the same workload (FP64, slack "
                      f"recomputed every step), {dt:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", choices=["auto", "fp32", "bf16x3", "fp64"], default="auto")
    ap.add_argument("--launch-steps", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ess", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            "(walks shard across GPUs with no communication; see DESIGN.md).")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2104_07097_amd import instances as inst

    if not torch.cuda.is_available():
        log("bench.py needs a HIP device")
        sys.exit(1)
    launch_steps = max(1, min(args.launch_steps, args.steps))
    steps = (args.steps // launch_steps) * launch_steps
    p = inst.randpoly()  # n=100, m=2000, z=1024
    precs = ["fp32", "bf16x3"] if args.precision == "auto" else [args.precision]
    results = {}
    for prec in precs:
        log(f"[bench] {prec}: warmup {args.warmup}, {steps} timed steps in launches of {launch_steps}")
        r = run_gpu(p, prec, steps, args.warmup, launch_steps)
        feasible = bool(np.all(r["X"] @ p.A.T <= p.b + 1e-12))
        r["feasible"] = feasible
        results[prec] = r
        log(f"[bench] {prec}: {r['gpu_time'] * 1e3 / steps:.4f} ms/step, "
            f"{p.z * steps / r['gpu_time'] / 1e6:.2f} M chain-steps/s, flags={r['flags']}, "
            f"feasible={feasible}, exact rows/chain-step="
            f"{r['stats']['exact_rows'] / max(1, r['stats']['chain_steps']):.2f}")
    best = max(precs, key=lambda k: p.z * steps / results[k]["gpu_time"])
    r = results[best]
    value = p.z * steps / r["gpu_time"]
    avg_launch = float(np.mean(r["per_launch"]))
    flops_per_launch = 2.0 * p.m * p.n * p.z * launch_steps * MFMA_PER_FLOP[best]
    achieved = flops_per_launch / avg_launch / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["gpu_time"] * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": best,
        "data": "synthetic",
        "config": {"workload": "random polytope n=100 m=2000 (unit-norm Gaussian rows, b=1), "
                               "z=1024 walks from the origin, plain MHAR, exact FP64 slack "
                               "recompute every 50 steps",
                   "n": p.n, "m": p.m, "z": p.z, "precision": best, "recompute_every": 50,
                   "steps_per_launch": launch_steps},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[best],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[best], "traffic": None,
                     "kernel": f"mhar_steps_kernel<{best}>",
                     "avg_launch_ms": avg_launch * 1e3,
                     "flops_per_launch": flops_per_launch},
        "wall_s": sum(results[k]["wall"] for k in precs),
        "feasible": all(results[k]["feasible"] for k in precs),
        "flags": {k: results[k]["flags"] for k in precs},
        "exact_rows_per_chain_step": {k: results[k]["stats"]["exact_rows"] /
                                      max(1, results[k]["stats"]["chain_steps"]) for k in precs},
        "variants": {k: {"value": p.z * steps / results[k]["gpu_time"],
                         "ms_per_step": results[k]["gpu_time"] * 1e3 / steps} for k in precs},
    }
    if not args.no_ess:
        log("[bench] ESS replay (64 recorded walks, same seed)")
        ess, Xr, ess_med = record_ess(p, best, steps, args.warmup, launch_steps)
        identical = bool(np.array_equal(Xr, r["X"]))
        line["ess"] = {"min_marginal_ess": ess, "median_marginal_ess": ess_med,
                       "min_marginal_ess_per_sec": ess / r["gpu_time"],
                       "walks_recorded": 64, "scaled_to_z": p.z,
                       "replay_bitwise_identical": identical,
                       "window": f"steps {args.warmup}..{args.warmup + steps}"}
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
