#!/usr/bin/env python3
"""Throughput of the fused k-means Lloyd iteration on one MI355X.

One step = one Lloyd iteration over the whole input: the distance pass
(distances to every centroid, argmin label), the per-label FP64 sums and
counts, the objective and the finalize (fixed-order combine, mean, empty
rule), inside one kmeans_lloyd call of STEPS iterations with the input
already resident in HBM.

Headline workload (default ``--workload bf16``): n = 2^22 samples, d = 128,
k = 1024, 1024 Gaussian blobs (sigma 2, centres uniform in [-10, 10]^d,
seed 2), k initial centroids sampled without replacement, 20 iterations;
distances as a BF16 MFMA contraction with FP32 accumulation, an exact FP32
recheck of every sample inside the proven band, FP64 sums; the same call on
the plain FP32 path beside it, and the labels and centroids of the two
compared bit for bit ("mixed vs FP32 at equal labels").

Timing (the paper's method, section 4.2): RUNS timed runs of the whole call
(default 10) from the same initial centroids, launched directly with HIP
events around every distance pass, the reported time the mean of the last
five; the same call captured as one graph is timed beside them.

Prints ONE JSON line on stdout (diagnostics go to stderr).  Besides the
throughput it carries:
  roofline        the dominant kernel (the BF16 screen: every sample against
                  every centroid) at 2 n k d FLOP per launch over its mean
                  duration from HIP events on its launch stream;
  error_vs_oracle the last iteration against the FP64 oracle (stepwise: the
                  GPU's C_{T-1} fed to the oracle's assign on a 2^16-sample
                  subsample, the GPU's labels to its full update and
                  objective);
  plain_workload  n = 2^20, d = 64, k = 64 in FP32 and BF16;
  fp8_workload    n = 2^24, d = 32, k = 256 in FP8, BF16 and FP32;
  batched_workload  512 independent instances, BF16 and FP32 batches;
  spade_workload  SPADE's density step (section 4.1) at n = 235,000, d = 32;
  nb_workload, gda_workload  naive Bayes and GDA training, n = 2^20, d = 64;
  metric_layout   the assign step under L1 / squared Euclidean distances with
                  row-major / feature-major samples;
  cpu_baseline    the FP64 oracle on this host's cores, one Lloyd iteration
                  over a bounded subsample of the headline input, scaled to
                  the whole input.
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

# MI355X published peaks.  FP32 vector: 256 CUs x 128 FP32 FMA lanes per
# clock x 2 FLOP x 2.4 GHz = 157.3 TFLOP/s (reached only with packed FP32
# operations, which this library does not emit).  Dense MFMA (no sparsity).
VALU_PEAK_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_1109_0778_amd", "csrc")
NEAR_TIE = 1e-6
LAST = 5          # runs averaged (the last LAST of RUNS)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_sha256(name):
    with open(os.path.join(CSRC, name), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of a kernel on a workload, from committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counts, valid only while the kernel's source file
    is unchanged since they were taken (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entries = json.load(fh)["entries"]
    except (OSError, ValueError, KeyError):
        return None
    for e in entries:
        if e.get("key") != key:
            continue
        srcs = e.get("sources", {e.get("source"): e.get("source_sha256")})
        if all(src_sha256(f) == h for f, h in srcs.items()):
            return e.get("bytes_per_launch")
    return None


def lloyd_runs(B, torch, Xg, C0g, precision, iters, warmup, runs, graph_runs=2):
    """`runs` timed direct-launch calls from C0, with HIP events around every
    distance-pass launch inside each timed call; then the same call captured
    as one graph and replayed `graph_runs` times (its time and results are
    reported beside the direct runs')."""
    import numpy as np
    n, d = Xg.shape
    k = C0g.shape[0]
    plan = B.Plan(n, d, k, precision)
    dev = Xg.device
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    counts = torch.empty(k, dtype=torch.int64, device=dev)
    hist = torch.empty(max(iters, warmup, 1), dtype=torch.float64, device=dev)
    C = C0g.clone()
    if warmup > 0:
        B.kmeans_lloyd(plan, Xg, C, labels, counts, hist, warmup, -1.0)
        torch.cuda.synchronize()
    cap = 3 * iters
    run_s, kts = [], []
    for _ in range(runs):
        plan.enable_timing(cap)           # fresh events; recording restarts
        C.copy_(C0g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.kmeans_lloyd(plan, Xg, C, labels, counts, hist, iters, -1.0)
        torch.cuda.synchronize()
        run_s.append(time.perf_counter() - t0)
        kts.append(plan.kernel_times(cap))
    plan.enable_timing(0)
    res = {"run_s": run_s, "el": float(np.mean(run_s[-LAST:])),
           "C": C.cpu().numpy(), "labels": labels.cpu().numpy(), "J": hist[:iters].cpu().numpy(),
           "counts": counts.cpu().numpy()}
    # per-iteration launches of the distance passes (1 FP32 / short BF16 sweep; 2 BF16 cascade; 3 FP8)
    per = max(1, len(kts[-1]) // iters)
    res["passes"] = per
    res["pass_ms"] = [float(np.mean([kt[p::per] for kt in kts[-LAST:]])) for p in range(per)]
    res["launches_timed"] = sum(len(kt[0::per]) for kt in kts[-LAST:])
    if precision != "fp32":
        res["recheck"], res["full_scans"] = plan.recheck_count()
    if graph_runs > 0:
        plan.use_graphs(True)
        C.copy_(C0g)
        B.kmeans_lloyd(plan, Xg, C, labels, counts, hist, iters, -1.0)   # capture + run
        torch.cuda.synchronize()
        gs = []
        for _ in range(graph_runs):
            C.copy_(C0g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.kmeans_lloyd(plan, Xg, C, labels, counts, hist, iters, -1.0)
            torch.cuda.synchronize()
            gs.append(time.perf_counter() - t0)
        res["el_graph"] = float(np.mean(gs))
        res["graph_equals_direct"] = bool(np.array_equal(C.cpu().numpy(), res["C"])
                                          and np.array_equal(labels.cpu().numpy(), res["labels"]))
    plan.close()
    return res


def c_prev(B, torch, Xg, C0g, precision, iters):
    """C_{T-1}: the first T-1 iterations of the same deterministic call."""
    if iters <= 1:
        return C0g.cpu().numpy()
    n, d = Xg.shape
    k = C0g.shape[0]
    plan = B.Plan(n, d, k, precision)
    C = C0g.clone()
    lab = torch.empty(n, dtype=torch.int32, device=Xg.device)
    B.kmeans_lloyd(plan, Xg, C, lab, None, None, iters - 1, -1.0)
    torch.cuda.synchronize()
    plan.close()
    return C.cpu().numpy()


def error_vs_oracle(X, Cprev, res, sample=1 << 16, seed=0):
    """The last iteration against the FP64 oracle (stepwise protocol): labels
    of a seeded subsample against the oracle's assign with the GPU's C_{T-1}
    (mismatches outside and inside the 1e-6 near-tie band), C_T against the
    oracle's update of the GPU's labels (per-centroid relative L2 error),
    J_{T-1} against the oracle's objective of those labels."""
    import numpy as np
    import oracle
    n, d = X.shape
    t0 = time.perf_counter()
    C64 = Cprev.astype(np.float64)
    idx = np.sort(np.random.default_rng(seed).choice(n, min(sample, n), replace=False))
    lab_o, dmin, d2, _ = oracle.assign(X[idx], C64)
    m = oracle.near_tie_margin(dmin, d2)
    mism = res["labels"][idx] != lab_o
    C_o, cnt_o = oracle.update(X, res["labels"], C64)
    nrm = np.linalg.norm(C_o, axis=1)
    floor = float(np.sqrt(np.mean(X[idx].astype(np.float64) ** 2)))
    cerr = np.linalg.norm(res["C"].astype(np.float64) - C_o, axis=1) / np.maximum(nrm, floor)
    J_o = oracle.objective(X, C64, res["labels"])
    J_g = float(res["J"][-1])
    return {"assign_sample": int(idx.size),
            "label_mismatches_outside_near_ties": int((mism & (m >= NEAR_TIE)).sum()),
            "label_mismatches_in_near_ties": int((mism & (m < NEAR_TIE)).sum()),
            "near_ties_in_sample": int((m < NEAR_TIE).sum()),
            "counts_equal": bool(np.array_equal(res["counts"], cnt_o)),
            "centroid_max_rel_err": float(cerr.max()),
            "objective_rel_err": abs(J_g - J_o) / J_o,
            "bars": "labels exact outside near-ties; centroids and objective within 1e-5",
            "within_bars": bool(not (mism & (m >= NEAR_TIE)).any() and cerr.max() <= 1e-5
                                and abs(J_g - J_o) <= 1e-5 * J_o and np.array_equal(res["counts"], cnt_o)),
            "seconds": time.perf_counter() - t0}


def pass_bytes(w, precision, stage):
    """HBM bytes one distance pass must move: its copy of X (FP32 rows for the
    plain pass; the BF16 copy with 4-byte |x| bounds for BF16 passes; the
    e4m3 copy with 8 bytes of band inputs for the FP8 screen) plus labels
    read (changed count) and written."""
    dp = (w.d + 15) // 16 * 16
    if precision == "fp32":
        return w.n * w.d * 4 + 8 * w.n
    if precision == "fp8" and stage == "screen":
        return w.n * (dp + 8) + 8 * w.n
    return w.n * (2 * dp + 4) + 8 * w.n


def roof(kind, amount, ms, peak, unit, **extra):
    achieved = amount / (ms * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
    r = {"bound": kind, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak}
    r.update(extra)
    return r


def workload_report(B, torch, w, X, C0, precision, iters, warmup, runs, fp=None, oracle_check=True):
    """One precision on one workload: throughput (mean of the last runs),
    the distance passes on their rooflines, equality with the FP32 run, and
    the error against the oracle."""
    dev = torch.device("cuda", 0)
    Xg = torch.from_numpy(X).to(dev)
    C0g = torch.from_numpy(C0).to(dev)
    r = lloyd_runs(B, torch, Xg, C0g, precision, iters, warmup, runs)
    ms_step = r["el"] * 1e3 / iters
    flops = 2.0 * w.n * w.k * w.d
    out = {"precision": precision, "value": iters / r["el"], "unit": "Lloyd iters/s", "ms_per_step": ms_step,
           "dist_evals_per_s": w.n * w.k * iters / r["el"],
           "runs_ms": [s * 1e3 for s in r["run_s"]], "reported": f"mean of the last {min(LAST, runs)} of {runs} runs",
           "ms_per_step_graph": r["el_graph"] * 1e3 / iters, "graph_equals_direct": r["graph_equals_direct"],
           "iteration_hbm_frac": (w.n * w.d * 4) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    if precision == "fp32":
        km = r["pass_ms"][0]
        out["roofline"] = roof("alu", flops, km, VALU_PEAK_TFLOPS, "TFLOP/s",
                               kernel="plain_pass (distances + argmin, fused with the per-label reduce when the record fits)",
                               traffic=measured_traffic(f"plain_pass:{w.name}"), flops_per_launch=flops,
                               bytes_per_launch=pass_bytes(w, "fp32", "pass"), mean_launch_ms=km,
                               launches=r["launches_timed"])
        out["iteration_valu_frac"] = flops / (ms_step * 1e-3) / 1e12 / VALU_PEAK_TFLOPS
    else:
        peak = MFMA_PEAK_TFLOPS[precision]
        names = (["screen"] if r["passes"] == 1 else ["screen", "refine"] if r["passes"] == 2
                 else ["screen", "bf16_screen", "refine"])
        km = r["pass_ms"][0]
        nb = pass_bytes(w, precision, "screen")
        ai = flops / nb
        bound = "mfma" if ai > peak * 1e12 / (HBM_PEAK_GBPS * 1e9) else "hbm"
        kern = f"mfma_assign<{precision}> {'screen (two smallest keys)' if r['passes'] > 1 else 'one sweep with candidate lists'}"
        extra = dict(kernel=kern, traffic=measured_traffic(f"mfma_screen_{precision}:{w.name}"),
                     flops_per_launch=flops, bytes_per_launch=nb, mean_launch_ms=km, launches=r["launches_timed"],
                     mfma_tflops=flops / (km * 1e-3) / 1e12, hbm_gbps=nb / (km * 1e-3) / 1e9)
        if bound == "mfma":
            out["roofline"] = roof("mfma", flops, km, peak, "TFLOP/s", **extra)
        else:
            out["roofline"] = roof("hbm", nb, km, HBM_PEAK_GBPS, "GB/s", **extra)
        out["pass_ms"] = dict(zip(names, r["pass_ms"]))
        out["iteration_mfma_frac"] = flops / (ms_step * 1e-3) / 1e12 / peak
        out["recheck_fraction_last_iter"] = r["recheck"] / w.n
        out["full_scan_fraction_last_iter"] = r["full_scans"] / w.n
    if fp is not None:
        import numpy as np
        out["fp32_value"] = iters / fp["el"]
        out["speedup_vs_fp32"] = fp["el"] / r["el"]
        out["labels_equal_fp32"] = bool(np.array_equal(r["labels"], fp["labels"]))
        out["centroids_equal_fp32"] = bool(np.array_equal(r["C"], fp["C"]))
        out["objective_rel_diff_vs_fp32"] = float(np.max(np.abs(r["J"] - fp["J"]) / fp["J"]))
    if oracle_check:
        Cp = c_prev(B, torch, Xg, C0g, precision, iters)
        out["error_vs_oracle"] = error_vs_oracle(X, Cp, r)
    log(f"{w.name} {precision}: {ms_step:.3f} ms/iteration ({out['reported']}); passes {r['pass_ms']} ms; "
        f"roofline {out['roofline']['bound']} frac {out['roofline']['frac']:.3f}"
        + (f"; vs fp32 {out['speedup_vs_fp32']:.2f}x, labels equal {out['labels_equal_fp32']}" if fp else "")
        + (f"; oracle {out['error_vs_oracle']}" if oracle_check else ""))
    del Xg, C0g
    torch.cuda.empty_cache()
    return out, r


def workload_desc(w):
    shape = "anisotropic blobs (per-blob per-feature sigma U[0.5,3])" if w.aniso else f"Gaussian blobs sigma={w.sigma}"
    return (f"{w.name}: Lloyd k-means, n={w.n}, d={w.d}, k={w.k}, {w.blobs} {shape}, centres U[-10,10]^d, "
            f"seed {w.seed}, init={w.init}, {w.iters} iterations")


PERSIST_SCHEDULE = (32, 1, [])


def _batched_run(B, torch, inst, C0, iters, precision, schedule=None, persistent=False):
    """Autotune (or set) the schedule, capture the iterations as one graph,
    reset the centroids and time one graph launch (with `persistent`, the
    persistent launch at the given schedule)."""
    from paper_1109_0778_amd import autotune
    batch = B.Batch(inst, precision=precision)
    if schedule is None:
        choice, tune_ms = autotune.tune_batch(batch, use_cache=False)
    else:
        autotune._apply(batch, *schedule)
        choice, tune_ms = tuple(schedule), {}
    if persistent:
        batch.use_persistent(True)
    batch.use_graphs(True)
    B.kmeans_lloyd_batched(batch, iters)            # capture + warm-up
    torch.cuda.synchronize()
    for t, c in zip(inst, C0):
        t["C"].copy_(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.kmeans_lloyd_batched(batch, iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = [(t["labels"].clone(), t["C"].clone()) for t in inst]
    for t, c in zip(inst, C0):
        t["C"].copy_(c)
    del batch
    torch.cuda.synchronize()
    return el, choice, tune_ms, out


def batched_instances(torch, iters):
    from paper_1109_0778_amd import datagen
    dev = torch.device("cuda", 0)
    inst, shapes = [], []
    for s_ in range(datagen.BATCH_COUNT):
        shp, X, C = datagen.batch_instance(s_)
        shapes.append(shp)
        inst.append({"X": torch.from_numpy(X).to(dev), "C": torch.from_numpy(C).to(dev),
                     "labels": torch.empty(shp.n, dtype=torch.int32, device=dev),
                     "counts": torch.empty(shp.k, dtype=torch.int64, device=dev),
                     "obj_hist": torch.zeros(iters, dtype=torch.float64, device=dev)})
    return inst, shapes


def batched_fixed(B, torch, iters, schedule):
    """The BF16 batch alone at a given (tiles per block, order): one graph
    launch to capture and warm up, one timed (for counter runs: every batch
    kernel is dispatched 2 x iters times, the run-level prep twice)."""
    inst, _ = batched_instances(torch, iters)
    C0 = [t["C"].clone() for t in inst]
    el, ch, _, _ = _batched_run(B, torch, inst, C0, iters, "bf16", schedule=schedule)
    return {"precision": "bf16", "schedule": list(ch), "iterations": iters, "ms_per_round": el * 1e3 / iters}


def batched_report(B, torch, iters, per_instance_sample=32):
    """The 512-instance workload with BF16 MFMA distances (and the FP32 batch
    beside it): autotuned schedule, one graph launch for all iterations of all
    instances, timed; the FP32 batch re-run at the BF16 schedule must give the
    same labels and centroids; next to them the same instances through
    single-instance FP32 kmeans_lloyd calls (a sample, extrapolated)."""
    import numpy as np
    inst, shapes = batched_instances(torch, iters)
    C0 = [t["C"].clone() for t in inst]
    el32, ch32, tm32, _ = _batched_run(B, torch, inst, C0, iters, "fp32")
    # the persistent launch at its best measured schedule (32 tiles per block),
    # beside the per-class launches at that same schedule (identical results)
    el32p, _, _, res32p = _batched_run(B, torch, inst, C0, iters, "fp32", schedule=PERSIST_SCHEDULE, persistent=True)
    el32c, _, _, res32c = _batched_run(B, torch, inst, C0, iters, "fp32", schedule=PERSIST_SCHEDULE)
    same_p = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(res32c, res32p))
    el16, ch16, tm16, res16 = _batched_run(B, torch, inst, C0, iters, "bf16")
    _, _, _, res32s = _batched_run(B, torch, inst, C0, iters, "fp32", schedule=ch16)
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(res16, res32s))
    pts = sum(s_.n for s_ in shapes)
    evals = sum(s_.n * s_.k for s_ in shapes)
    flops = sum(2.0 * s_.n * s_.k * s_.d for s_ in shapes)
    nbytes = sum(s_.n * s_.d * 4 + 8 * s_.n for s_ in shapes)
    idx = np.random.default_rng(0).choice(len(inst), per_instance_sample, replace=False)
    el_single = 0.0
    for i in idx:
        t = inst[i]
        n, d = t["X"].shape
        k = t["C"].shape[0]
        plan = B.Plan(n, d, k)
        C = C0[i].clone()
        B.kmeans_lloyd(plan, t["X"], C, t["labels"], None, None, 1)
        torch.cuda.synchronize()
        C = C0[i].clone()
        t1 = time.perf_counter()
        B.kmeans_lloyd(plan, t["X"], C, t["labels"], None, None, iters)
        torch.cuda.synchronize()
        el_single += time.perf_counter() - t1
    el_single *= len(inst) / per_instance_sample
    ms_round = el16 * 1e3 / iters
    log(f"batched: {len(inst)} instances x {iters} iterations: BF16 {el16 * 1e3:.1f} ms (schedule {ch16}), "
        f"FP32 {el32 * 1e3:.1f} ms (schedule {ch32}), FP32 persistent launch {el32p * 1e3:.1f} ms (identical: "
        f"{same_p}); BF16 identical to FP32 at the same schedule: {same}; "
        f"per-instance FP32 launches, extrapolated: {el_single * 1e3:.1f} ms")
    return {"workload": f"batched: {len(inst)} instances, n log-uniform [1e3, 2e5] (total {pts}), d in {{16,32,64}}, "
                        f"k uniform [4,128], blobs = k, sigma 1, seeds 0..{len(inst) - 1}, {iters} iterations",
            "precision": "bf16", "value": len(inst) * iters / el16, "unit": "instance-iterations/s",
            "ms_per_round": ms_round,
            "dist_evals_per_s": evals * iters / el16,
            "roofline": roof("hbm", nbytes, ms_round, HBM_PEAK_GBPS, "GB/s",
                             kernel="one round of every instance (all launches of one iteration)",
                             traffic=measured_traffic("batched_round:bf16"), bytes_per_round=nbytes,
                             flops_per_round=flops,
                             mfma_frac_of_round=flops / (ms_round * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16"]),
            "fp32_batched_value": len(inst) * iters / el32,
            "fp32_persistent": {"value": len(inst) * iters / el32p, "ms_per_round": el32p * 1e3 / iters,
                                "schedule": list(PERSIST_SCHEDULE[:2]),
                                "class_schedule_ms_per_round_same_schedule": el32c * 1e3 / iters,
                                "vs_best_class_schedule": el32 / el32p,
                                "identical_to_class_schedule": bool(same_p),
                                "launch": "one persistent kernel per 32 iterations: device queue, per-instance "
                                          "completion tickets, graph-captured"},
            "speedup_vs_fp32_batched": el32 / el16,
            "labels_and_centroids_equal_fp32_batched": bool(same),
            "per_instance_launches_value": len(inst) * iters / el_single,
            "speedup_vs_per_instance_launches": el_single / el16,
            "schedule": {"tiles_per_block": ch16[0], "order": ch16[1], "class_tiles_per_block": ch16[2],
                         "candidates_ms": tm16},
            "schedule_fp32": {"tiles_per_block": ch32[0], "order": ch32[1], "class_tiles_per_block": ch32[2],
                              "candidates_ms": tm32},
            "graph": True}


# MI355X FP64: one FP64 add (or FMA) per lane per clock, 256 CUs x 64 lanes
# x 2.4 GHz = 39.3 T lane-operations/s (the published 78.6 TFLOP/s counts an
# FMA as two); the dense FP64 matrix peak is 78.6 TFLOP/s.
FP64_LANE_OPS = 256 * 64 * 2.4e9
FP64_MFMA_PEAK_TFLOPS = 78.6


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def spade_report(B, torch, runs):
    """SPADE's density step (section 4.1) on the synthetic cytometry matrix:
    n = 235,000 rows, d = 32, the section's two widths, L1 distances in FP64.
    Algorithmic work: the rows the sequential loop visits, each against every
    sample, 2 d FP64 operations per pair (subtract, add of the magnitude)."""
    import numpy as np
    from paper_1109_0778_amd import datagen
    X, _ = datagen.cytometry()
    n, d = X.shape
    Xg = torch.from_numpy(X).cuda()
    dens, nvis, ws = B.spade_densities(Xg, datagen.SPADE_APPRX_WIDTH, datagen.SPADE_KERNEL_WIDTH, "l1")
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        e0, e1 = _events(torch)
        e0.record()
        dens, nvis, ws = B.spade_densities(Xg, datagen.SPADE_APPRX_WIDTH, datagen.SPADE_KERNEL_WIDTH, "l1",
                                           densities=dens, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    batches, cands = B.spade_stats(ws, n, d)
    ms = float(np.mean(times[-LAST:]))
    ops = float(nvis) * n * 2 * d
    log(f"spade: n={n} d={d}: {ms:.2f} ms, visited {nvis}, {batches} batches, {cands} candidate rows")
    return {"workload": f"SPADE density step (section 4.1): synthetic cytometry matrix n={n}, d={d} "
                        f"({datagen.SPADE_POPS} populations, seed {datagen.SPADE_SEED}), L1 distance, widths "
                        f"{datagen.SPADE_APPRX_WIDTH} / {datagen.SPADE_KERNEL_WIDTH}, FP64",
            "ms": ms, "runs_ms": times, "visited_rows": nvis, "batches": batches, "candidate_rows": cands,
            "speculation_efficiency": nvis / max(cands, 1),
            "row_evals_per_s": float(nvis) * n / (ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e12, "peak": FP64_LANE_OPS / 1e12,
                         "unit": "T FP64 op/s", "frac": ops / (ms * 1e-3) / FP64_LANE_OPS,
                         "kernel": "spade_densities, whole call (one launch per batch: claims, rows, resolve and selection)",
                         "ops_per_call": ops, "formed_ops_per_call": float(cands) * n * 2 * d, "traffic": None}}


def nb_gda_report(B, torch, runs, n=1 << 20, d=64, k=16):
    """Naive Bayes (count features) and GDA training on n = 2^20 labelled
    samples, d = 64, k = 16 classes."""
    import numpy as np
    from paper_1109_0778_amd import datagen
    out = {}
    X, y = datagen.nb_counts(n, d, k, seed=11)
    Xg, yg = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    plan = B.Plan(n, d, k)
    prior = torch.empty(k, dtype=torch.float64, device="cuda")
    phi = torch.empty((k, d), dtype=torch.float64, device="cuda")
    B.nb_train(plan, Xg, yg, prior, phi)
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        e0, e1 = _events(torch)
        e0.record()
        B.nb_train(plan, Xg, yg, prior, phi)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times[-LAST:]))
    nbytes = n * d * 4 + n * 4
    out["nb_workload"] = {"workload": f"multinomial naive Bayes training: n={n} Poisson count samples, d={d}, "
                                      f"k={k} classes, seed 11", "ms": ms, "runs_ms": times,
                          "samples_per_s": n / (ms * 1e-3),
                          "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                                       "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                       "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                       "kernel": "nb_train, whole call (class reduce + combine + finalize)",
                                       "bytes_per_call": nbytes, "traffic": None}}
    X, y = datagen.gda_classes(n, d, k, seed=12)
    Xg, yg = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    mu = torch.empty((k, d), dtype=torch.float64, device="cuda")
    sigma = torch.empty((d, d), dtype=torch.float64, device="cuda")
    ws = B.gda_train(plan, Xg, yg, prior, mu, sigma)
    torch.cuda.synchronize()
    times, kts = [], []
    for _ in range(runs):
        plan.enable_timing(1)
        e0, e1 = _events(torch)
        e0.record()
        B.gda_train(plan, Xg, yg, prior, mu, sigma, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        kts.append(plan.kernel_times(1)[0])
    plan.enable_timing(0)
    ms = float(np.mean(times[-LAST:]))
    kms = float(np.mean(kts[-LAST:]))
    flops = 2.0 * n * d * d
    out["gda_workload"] = {"workload": f"GDA training: n={n} samples of {k} Gaussian classes with one shared "
                                       f"covariance, d={d}, seed 12", "ms": ms, "runs_ms": times,
                           "samples_per_s": n / (ms * 1e-3),
                           "roofline": {"bound": "mfma", "achieved": flops / (kms * 1e-3) / 1e12,
                                        "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                        "frac": flops / (kms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                                        "kernel": "gda_cov_kernel (FP64 MFMA sum of outer products)",
                                        "flops_per_launch": flops, "mean_launch_ms": kms,
                                        "launches": len(kts[-LAST:]), "traffic": None}}
    log(f"nb: {out['nb_workload']['ms']:.3f} ms; gda: {ms:.3f} ms (covariance {kms:.3f} ms)")
    plan.close()
    return out


def metric_layout_report(B, torch, runs, n=1 << 22, k=64):
    """Assign step under L1 and squared Euclidean distances with row-major and
    feature-major samples, d = 8, 16, 32: one kmeans_assign_metric call each
    (2 n k d FP32 operations: subtract, then add of the magnitude or FMA)."""
    import numpy as np
    from paper_1109_0778_amd import datagen
    rows = []
    for d in (8, 16, 32):
        X, C = datagen.blobs(n, d, k, k, 1.0, seed=40 + d)
        plan = B.Plan(n, d, k)
        Cg = torch.from_numpy(C).cuda()
        lab = torch.empty(n, dtype=torch.int32, device="cuda")
        for layout in ("row", "feature"):
            Xg = torch.from_numpy(X if layout == "row" else np.ascontiguousarray(X.T)).cuda()
            for metric in ("l1", "sqeuclidean"):
                B.kmeans_assign_metric(plan, Xg, Cg, lab, metric, layout)
                times = []
                for _ in range(runs):
                    e0, e1 = _events(torch)
                    e0.record()
                    B.kmeans_assign_metric(plan, Xg, Cg, lab, metric, layout)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                ms = float(np.mean(times[-LAST:]))
                flops = 2.0 * n * k * d
                rows.append({"d": d, "layout": layout, "metric": metric, "ms": ms,
                             "dist_evals_per_s": n * k / (ms * 1e-3),
                             "valu_frac": flops / (ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS})
            del Xg
        plan.close()
    log("metric/layout: " + ", ".join(f"d{r['d']} {r['layout']} {r['metric']} {r['ms']:.3f}ms" for r in rows))
    return {"workload": f"assign step, n={n}, k={k}, blobs sigma 1, d in 8/16/32, L1 and squared Euclidean, "
                        f"row-major and feature-major samples", "results": rows}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, X, C0, rows):
    """The FP64 oracle as it stands: one Lloyd iteration (assign against all k
    centroids, update) over the first `rows` samples of the input, on every
    host core; both steps are linear in n, so the whole input's rate is the
    sample's scaled by rows / n."""
    import oracle
    rows = min(rows, X.shape[0])
    Xs = X[:rows]
    t0 = time.perf_counter()
    oracle.lloyd(Xs, C0.astype("float64"), 1)
    el = time.perf_counter() - t0
    full = el * X.shape[0] / rows
    return {"value": 1.0 / full, "unit": "Lloyd iters/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one FP64 Lloyd iteration (assign over all k={w.k} centroids + update) of the first {rows} "
                      f"of the {X.shape[0]} samples (d={w.d}), {el:.1f} s, scaled by n/{rows} to the whole input",
            "dist_evals_per_s": rows * w.k / el, "cpu_model": cpu_model(),
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


HEADLINE_PRECISION = {"small": "fp32", "plain": "fp32", "bf16": "bf16", "fp8": "fp8"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="Lloyd iterations per timed run (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed Lloyd iterations before the runs")
    ap.add_argument("--runs", type=int, default=10, help="timed runs; the mean of the last five is reported")
    ap.add_argument("--workload", default="bf16", choices=["bf16", "plain", "fp8", "small", "batched", "spade"],
                    help="headline workload (batched, spade: only that workload, for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true", help="skip the error-vs-oracle reports")
    ap.add_argument("--no-plain-workload", action="store_true", help="skip n=2^20, d=64, k=64")
    ap.add_argument("--no-fp8-workload", action="store_true", help="skip n=2^24, d=32, k=256")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-instance batched workload")
    ap.add_argument("--no-apps", action="store_true",
                    help="skip SPADE, naive Bayes, GDA and the metric / layout comparison")
    ap.add_argument("--cpu-rows", type=int, default=1 << 22,
                    help="samples in the oracle's timed iteration (default: all 2^22 of the headline input)")
    ap.add_argument("--batched-schedule", default=None, metavar="T,O",
                    help="with --workload batched: only the BF16 batch at tiles per block T and order O "
                         "(no autotuning, no FP32 batch; for counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (PMC calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.runs < 1:
        print("--runs must be >= 1", file=sys.stderr)
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

    if args.workload == "spade":
        rep = spade_report(B, torch, args.runs)
        rep.update({"metric": "SPADE density step, ms per call", "n_gpus": 1, "higher_is_better": False,
                    "data": "synthetic"})
        print(json.dumps(rep), flush=True)
        return
    if args.workload == "batched" and args.batched_schedule:
        t_, o_ = (int(v) for v in args.batched_schedule.split(","))
        print(json.dumps(batched_fixed(B, torch, datagen.BATCH_ITERS, (t_, o_, []))), flush=True)
        return
    if args.workload == "batched":
        rep = batched_report(B, torch, datagen.BATCH_ITERS)
        rep.update({"metric": "instance-iterations/s of the batched workload", "n_gpus": 1,
                    "higher_is_better": True, "data": "synthetic"})
        print(json.dumps(rep), flush=True)
        return
    w = datagen.WORKLOADS[args.workload]
    prec = HEADLINE_PRECISION[args.workload]
    steps = args.steps if args.steps is not None else w.iters
    check = not args.no_oracle_check
    log(f"headline workload {w.name}: n={w.n} d={w.d} k={w.k}, {prec}, {args.runs} runs x {steps} iterations, "
        f"{args.warmup} warmup")
    X, C0 = datagen.workload(w.name)
    fp_rep, fp = workload_report(B, torch, w, X, C0, "fp32", steps, args.warmup, args.runs,
                                 oracle_check=check and prec == "fp32")
    if prec == "fp32":
        head, hr = fp_rep, fp
    else:
        head, hr = workload_report(B, torch, w, X, C0, prec, steps, args.warmup, args.runs, fp=fp, oracle_check=check)
    out = {
        "metric": "Lloyd iters/s and point-centroid dist evals/s; mixed vs FP32 at equal labels",
        "value": head["value"],
        "unit": "Lloyd iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8-e4m3"}[prec],
        "data": "synthetic",
        "config": {"workload": workload_desc(w) + (
                       "; distances as a BF16 MFMA contraction with FP32 accumulation, exact FP32 recheck inside "
                       "the proven band, FP64 sums" if prec == "bf16" else
                       "; distances as an FP8 e4m3 MFMA contraction (per-feature power-of-two scales), exact FP32 "
                       "recheck, FP64 sums" if prec == "fp8" else "; FP32 direct-form distances, FP64 sums"),
                   "n": w.n, "d": w.d, "k": w.k, "iters": steps, "precision": prec},
        "launch": "direct (HIP events around the distance passes inside the timed calls; the graph-launched "
                  "call's time is ms_per_step_graph)",
        "runs": args.runs,
        "reported": head["reported"],
        "dist_evals_per_s": head["dist_evals_per_s"],
        "roofline": head["roofline"],
    }
    for key in ("fp32_value", "speedup_vs_fp32", "labels_equal_fp32", "centroids_equal_fp32",
                "objective_rel_diff_vs_fp32", "pass_ms", "iteration_mfma_frac", "iteration_hbm_frac",
                "recheck_fraction_last_iter", "full_scan_fraction_last_iter", "error_vs_oracle", "runs_ms",
                "ms_per_step_graph", "graph_equals_direct"):
        if key in head:
            out[key] = head[key]
    if prec != "fp32":
        out["fp32"] = fp_rep
    objective = [float(hr["J"][0]), float(hr["J"][-1])]
    out["objective_first_last"] = objective
    del fp, hr

    if args.workload == "bf16" and not args.no_plain_workload:
        wp = datagen.WORKLOADS["plain"]
        Xp, Cp = datagen.workload("plain")
        rep32, fpp = workload_report(B, torch, wp, Xp, Cp, "fp32", wp.iters, args.warmup, args.runs, oracle_check=check)
        rep16, _ = workload_report(B, torch, wp, Xp, Cp, "bf16", wp.iters, args.warmup, args.runs, fp=fpp,
                                   oracle_check=False)
        out["plain_workload"] = {"workload": workload_desc(wp), "fp32": rep32, "bf16": rep16}
        del Xp, Cp, fpp
    if args.workload == "bf16" and not args.no_fp8_workload:
        w8 = datagen.WORKLOADS["fp8"]
        X8, C8 = datagen.workload("fp8")
        rep32, fp8 = workload_report(B, torch, w8, X8, C8, "fp32", w8.iters, 1, min(args.runs, 3), oracle_check=False)
        rep = {"workload": workload_desc(w8), "fp32": rep32}
        for p_ in ("fp8", "bf16"):
            rep[p_], _ = workload_report(B, torch, w8, X8, C8, p_, w8.iters, 1, args.runs, fp=fp8,
                                         oracle_check=check and p_ == "fp8")
        out["fp8_workload"] = rep
        del X8, C8, fp8
    if args.workload == "bf16" and not args.no_batched:
        out["batched_workload"] = batched_report(B, torch, datagen.BATCH_ITERS)
    if args.workload == "bf16" and not args.no_apps:
        out["spade_workload"] = spade_report(B, torch, args.runs)
        out.update(nb_gda_report(B, torch, args.runs))
        out["metric_layout"] = metric_layout_report(B, torch, args.runs)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(w, X, C0, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
