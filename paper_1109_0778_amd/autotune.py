"""Autotuner for the batched Lloyd schedule.

A batch's per-iteration cost depends on how each instance's tiles (256
samples) are cut into blocks (tiles per block: fewer, longer blocks mean fewer
partial records to merge; more, shorter blocks fill the 256 CUs better) and on
the order blocks are launched in (largest work first evens out the tail).  The
tuner times one Lloyd iteration of every candidate on the batch itself, with
HIP events, and keeps the fastest; results are cached in a JSON file keyed by
the GPU architecture, the distance precision and a signature of the batch's
shapes.
"""
from __future__ import annotations

import hashlib
import json
import os

CANDIDATES = [(tpb, order) for tpb in (1, 2, 4, 8, 16, 32) for order in (1, 0)]


def cache_path() -> str:
    return os.environ.get("KM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1109_0778_amd", "tune.json"))


def signature(instances) -> str:
    """Shape signature: sorted (n rounded to 2 significant digits, d, k)."""
    def r2(n):
        s = f"{n:.1e}"
        return s
    shapes = sorted((r2(t["X"].shape[0]), int(t["X"].shape[1]), int(t["C"].shape[0])) for t in instances)
    return hashlib.sha1(json.dumps(shapes).encode()).hexdigest()[:16]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_batch(batch, reps: int = 2, use_cache: bool = True, verbose: bool = False):
    """Pick (tiles_per_block, order) for `batch` and apply it.  The instances'
    centroids are restored afterwards.  Returns (choice, {candidate: ms})."""
    import torch
    from . import binding as B

    key = f"{_arch()}:{getattr(batch, 'precision', 'fp32')}:{signature(batch.instances)}"
    db = _load() if use_cache else {}
    if key in db:
        tpb, order = db[key]["choice"]
        batch.set_schedule(tpb, order)
        return (tpb, order), db[key].get("ms", {})
    saved = [t["C"].clone() for t in batch.instances]
    times = {}
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for tpb, order in CANDIDATES:
        batch.set_schedule(tpb, order)
        B.kmeans_lloyd_batched(batch, 1)          # warm-up
        torch.cuda.synchronize()
        start.record()
        for _ in range(reps):
            B.kmeans_lloyd_batched(batch, 1)
        end.record()
        torch.cuda.synchronize()
        times[f"{tpb},{order}"] = start.elapsed_time(end) / reps
        if verbose:
            print(f"tiles_per_block={tpb} order={order}: {times[f'{tpb},{order}']:.3f} ms", flush=True)
    for t, c in zip(batch.instances, saved):
        t["C"].copy_(c)
    best = min(times, key=times.get)
    tpb, order = (int(v) for v in best.split(","))
    batch.set_schedule(tpb, order)
    db[key] = {"choice": [tpb, order], "ms": times}
    if use_cache:
        _store(db)
    return (tpb, order), times
