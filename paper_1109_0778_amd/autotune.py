"""Autotuner for the batched Lloyd schedule.

A batch's per-iteration cost depends on how each instance's tiles (256
samples) are cut into blocks (tiles per block: fewer, longer blocks mean fewer
partial records to merge; more, shorter blocks fill the 256 CUs better) and on
the order blocks are launched in (largest work first evens out the tail).  The
tuner times one Lloyd iteration of every candidate on the batch itself, with
HIP events, and keeps the fastest.  Instances of different shape classes
(8-feature chunks of d, LDS size of the per-label record) favour different
block lengths, so after the batch-wide choice each class with more than one
instance is tuned on its own, the others held fixed (one sweep of coordinate
descent).  Results are cached in a JSON file keyed by the GPU architecture,
the distance precision and a signature of the batch's shapes.
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


def _time(batch, reps, start, end) -> float:
    import torch
    from . import binding as B
    B.kmeans_lloyd_batched(batch, 1)          # warm-up
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        B.kmeans_lloyd_batched(batch, 1)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def _apply(batch, tpb, order, class_tpb):
    batch.set_schedule(tpb, order)
    for c, v in enumerate(class_tpb or []):
        if v:
            batch.set_class_schedule(c, v)


def tune_batch(batch, reps: int = 2, use_cache: bool = True, verbose: bool = False,
               per_class: bool = True, timer=None, arch: str | None = None):
    """Pick (tiles_per_block, order), then per-class tiles per block, for
    `batch` and apply them.  The instances' centroids are restored afterwards.
    `timer(batch) -> ms` times the batch's current schedule (default: one
    Lloyd iteration, HIP events, `reps` repetitions after a warm-up).
    Returns ((tiles_per_block, order, [per-class tiles per block]), {candidate: ms})."""
    key = f"{arch or _arch()}:{getattr(batch, 'precision', 'fp32')}:{signature(batch.instances)}"
    db = _load() if use_cache else {}
    if key in db and ("class_tpb" in db[key] or not per_class):
        tpb, order = db[key]["choice"]
        ctpb = db[key].get("class_tpb", []) if per_class else []
        _apply(batch, tpb, order, ctpb)
        return (tpb, order, ctpb), db[key].get("ms", {})
    if timer is None:
        import torch
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        timer = lambda b: _time(b, reps, start, end)   # noqa: E731
    saved = [t["C"].clone() for t in batch.instances]
    times = {}
    for tpb, order in CANDIDATES:
        batch.set_schedule(tpb, order)
        times[f"{tpb},{order}"] = timer(batch)
        if verbose:
            print(f"tiles_per_block={tpb} order={order}: {times[f'{tpb},{order}']:.3f} ms", flush=True)
    best = min(times, key=times.get)
    tpb, order = (int(v) for v in best.split(","))
    batch.set_schedule(tpb, order)
    ctpb = [0] * len(batch.classes())
    if per_class and len(ctpb) > 1:
        cur = times[best]
        for c, (d8, lds, cnt, _) in enumerate(batch.classes()):
            if cnt < 2:
                continue
            for v in (1, 2, 4, 8, 16, 32, 64):
                if v == tpb:
                    continue
                batch.set_class_schedule(c, v)
                t = timer(batch)
                times[f"class{c}:{v}"] = t
                if verbose:
                    print(f"class {c} (D8={d8}, lds={lds}, {cnt} instances) tiles_per_block={v}: {t:.3f} ms",
                          flush=True)
                if t < cur * 0.98:                # keep only clear gains
                    cur, ctpb[c] = t, v
            batch.set_class_schedule(c, ctpb[c])
    for t, c in zip(batch.instances, saved):
        t["C"].copy_(c)
    db[key] = {"choice": [tpb, order], "class_tpb": ctpb, "ms": times}
    if use_cache:
        _store(db)
    return (tpb, order, ctpb), times
