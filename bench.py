#!/usr/bin/env python3
"""Throughput of the fused k-means Lloyd iteration on one MI355X.

One step = one Lloyd iteration over the whole input: the per-sample pass
(distances to every centroid, argmin label, per-label FP64 sums and counts,
objective) and the finalize (fixed-order combine, mean, empty-cluster rule),
all inside one kmeans_lloyd call of STEPS iterations with the input already
resident in HBM.  Default workload: n = 2^20 samples, d = 64, k = 64, 64
Gaussian blobs (sigma 1, centres uniform in [-10, 10]^d, seed 1), k initial
centroids sampled without replacement, 20 iterations, FP32 distances.

Prints ONE JSON line on stdout (diagnostics go to stderr).  Besides the timed
throughput it carries:
  roofline      the per-sample pass (dominant kernel): algorithmic VALU work
                per launch / its mean duration from HIP events recorded on the
                launch stream during the timed region;
  cpu_baseline  the FP64 oracle timed on this host's cores on a bounded sample
                of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 FP32 lanes at 2.4 GHz, one non-packed FP32
# VALU operation per lane per clock (packed FP32 is not used by this build).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "plain_pass_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1109_0778_amd", "csrc", "km_plain.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_sha256(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(n_launch_units):
    """HBM bytes per launch from committed rocprofv3 PMC counts, valid only
    while the kernel source is unchanged since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != src_sha256(KERNEL_SRC) or t.get("workload") != n_launch_units:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(X, C0, iters, budget_s):
    import numpy as np
    import oracle
    C = C0.astype(np.float64)
    done = 0
    t0 = time.perf_counter()
    while done < iters:
        r = oracle.lloyd(X, C, 1)
        C = r["C"]
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "Lloyd iters/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} full Lloyd iteration(s) of the same input from the same initial centroids "
                      f"(n={X.shape[0]}, d={X.shape[1]}, k={C0.shape[0]}), FP64, OpenMP over samples; "
                      f"{el:.1f} s",
            "host_cpus": len(os.sched_getaffinity(0))}


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE counts to bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed Lloyd iterations (default: workload's 20)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain", choices=["plain", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (PMC calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    from paper_1109_0778_amd import binding as B
    from paper_1109_0778_amd import datagen

    w = datagen.WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else w.iters
    log(f"workload {w.name}: n={w.n} d={w.d} k={w.k}, {steps} timed iterations, {args.warmup} warmup")
    X, C0 = datagen.workload(w.name)
    dev = torch.device("cuda", 0)
    Xg = torch.from_numpy(X).to(dev)
    C0g = torch.from_numpy(C0).to(dev)
    plan = B.Plan(w.n, w.d, w.k, "fp32")
    labels = torch.empty(w.n, dtype=torch.int32, device=dev)
    counts = torch.empty(w.k, dtype=torch.int64, device=dev)
    hist = torch.empty(max(steps, args.warmup, 1), dtype=torch.float64, device=dev)

    if args.warmup > 0:
        Cw = C0g.clone()
        B.kmeans_lloyd(plan, Xg, Cw, labels, counts, hist, args.warmup, -1.0)
        torch.cuda.synchronize()

    C = C0g.clone()
    plan.enable_timing(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.kmeans_lloyd(plan, Xg, C, labels, counts, hist, steps, -1.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = plan.kernel_times(steps)
    plan.enable_timing(0)

    J = hist[:steps].cpu().numpy()
    kmean_ms = float(np.mean(kt)) if kt else float("nan")
    ops = 2.0 * w.n * w.k * w.d                # one subtract + one FMA per (sample, centroid, feature)
    achieved = ops / (kmean_ms * 1e-3) / 1e12
    algo_bytes = w.n * w.d * 4 + 2 * w.n * 4   # X once, labels read + written
    traffic = measured_traffic(f"{w.name}:{w.n}x{w.d}x{w.k}")
    log(f"timed {steps} iterations in {el * 1e3:.2f} ms; per-sample pass mean {kmean_ms * 1e3:.1f} us "
        f"over {len(kt)} launches; J[0]={J[0]:.6e} J[-1]={J[-1]:.6e}")

    out = {
        "metric": "Lloyd iters/s and point-centroid dist evals/s; mixed vs FP32 at equal labels",
        "value": steps / el,
        "unit": "Lloyd iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: FP32 Lloyd, n={w.n}, d={w.d}, k={w.k}, {w.blobs} Gaussian blobs "
                               f"sigma={w.sigma}, centres U[-10,10]^d, seed {w.seed}, init={w.init}, "
                               f"{w.iters} iterations",
                   "n": w.n, "d": w.d, "k": w.k, "iters": steps, "precision": "fp32"},
        "dist_evals_per_s": w.n * w.k * steps / el,
        "hbm_gbps_algorithmic": algo_bytes * steps / el / 1e9,
        "roofline": {
            "kernel": "plain_pass (fused assign + per-label reduce)",
            "bound": "alu",
            "achieved": achieved,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS,
            "traffic": traffic,
            "ops_per_launch": ops,
            "mean_launch_ms": kmean_ms,
            "launches": len(kt),
            "hbm_gbps_algorithmic_kernel": algo_bytes / (kmean_ms * 1e-3) / 1e9,
        },
        "objective_first_last": [float(J[0]), float(J[-1])],
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(X, C0, w.iters, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
