"""Seeded random shapes across the whole boundary (1 <= d <= 1024, ragged n
and k, FP32 / BF16 / FP8 plans), two Lloyd iterations each, checked stepwise
against the FP64 oracle (needs an MI355X).  Bar, as in the other parity
suites: labels equal the oracle's outside documented near-ties (top-2 margin
below 1e-6), counts exact, centroids within 1e-5 relative; the mixed plans'
labels and centroids equal the FP32 plan's on the same centroids.  Shapes are
drawn log-uniformly (d in [1, 1024], k in [1, 3000], n in [k, 60000]) with
n k d <= 1.5e8 so that the oracle finishes quickly."""
import math

import numpy as np
import pytest

import oracle
from paper_1109_0778_amd import datagen
from test_gpu_plain import _bind, _torch, check_centroids, check_labels, say

pytestmark = pytest.mark.gpu


def _shapes(count=24, large_k=9, seed=2024):
    """`count` shapes drawn over the whole range, then `large_k` with k in
    [256, 3000] (the screen-and-refine sweeps of the mixed plans)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count + large_k:
        lk = len(out) >= count
        d = int(round(math.exp(rng.uniform(0.0, math.log(1024.0 if not lk else 256.0)))))
        k = int(round(math.exp(rng.uniform(math.log(256.0) if lk else 0.0, math.log(3000.0)))))
        n = max(k, int(round(math.exp(rng.uniform(math.log(k), math.log(60000.0))))))
        if n * k * d > 1.5e8:
            continue
        prec = ("fp32", "bf16", "fp8")[len(out) % 3]
        out.append((n, d, k, prec, int(rng.integers(0, 1 << 30))))
    return out


SHAPES = _shapes()


@pytest.mark.parametrize("n,d,k,prec,seed", SHAPES)
def test_random_shape_stepwise(n, d, k, prec, seed):
    torch, B = _torch(), _bind()
    say(f"random shape n={n} d={d} k={k} {prec} seed={seed}")
    X, C0 = datagen.blobs(n, d, k, max(1, min(k, 64)), 1.0, seed)
    dev = torch.device("cuda")
    Xg = torch.from_numpy(X).to(dev)
    plan = B.Plan(n, d, k, prec)
    ref = B.Plan(n, d, k, "fp32") if prec != "fp32" else None
    Cg = torch.from_numpy(C0).to(dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(k, dtype=torch.int64, device=dev)
    C = C0.copy()
    for t in range(2):
        if ref is not None:
            Cr = Cg.clone()
            labr = torch.empty_like(lab)
            B.kmeans_lloyd(ref, Xg, Cr, labr, None, None, 1)
        B.kmeans_lloyd(plan, Xg, Cg, lab, cnt, None, 1)
        torch.cuda.synchronize()
        L = lab.cpu().numpy()
        check_labels(L, C, X, f"{prec} n={n} d={d} k={k} t={t}")
        Co, cnto = oracle.update(X, L, C.astype(np.float64))
        assert np.array_equal(cnt.cpu().numpy(), cnto), f"counts t={t}"
        Cn = Cg.cpu().numpy()
        check_centroids(Cn, Co, X, f"{prec} n={n} d={d} k={k} t={t}")
        if ref is not None:
            assert torch.equal(labr, lab), f"{prec} labels differ from the FP32 plan's, t={t}"
            assert torch.equal(Cr, Cg), f"{prec} centroids differ from the FP32 plan's, t={t}"
        C = Cn


def _batch_shapes(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        d = int(round(math.exp(rng.uniform(0.0, math.log(300.0)))))
        k = int(round(math.exp(rng.uniform(0.0, math.log(200.0)))))
        n = max(k, int(round(math.exp(rng.uniform(math.log(max(k, 2)), math.log(20000.0))))))
        if n * k * d > 4e7 or k * min(d, 128) * 8 > 80 * 1024:
            continue
        out.append((n, d, k))
    return out


@pytest.mark.parametrize("prec,persistent", [("fp32", False), ("bf16", False), ("fp8", False), ("fp32", True)])
def test_random_batch_stepwise(prec, persistent):
    """A seeded random mix of instances (d up to 300: narrow shape classes and
    wide instances; FP8 batches through per-instance plans; the persistent
    FP32 launch over instances of d <= 64), two iterations, every instance
    checked against the oracle after each."""
    torch, B = _torch(), _bind()
    shapes = _batch_shapes(20, 31 + len(prec) + persistent)
    if persistent:
        shapes = [s_ for s_ in shapes if s_[1] <= 64] or [(1000, 16, 5)]
    say(f"random batch {prec} persistent={persistent}: {shapes}")
    dev = torch.device("cuda")
    inst, host = [], []
    for i, (n, d, k) in enumerate(shapes):
        X, C = datagen.blobs(n, d, k, max(1, min(k, 32)), 1.0, 5000 + i)
        host.append((X, C))
        inst.append({"X": torch.from_numpy(X).to(dev), "C": torch.from_numpy(C).to(dev),
                     "labels": torch.empty(n, dtype=torch.int32, device=dev),
                     "counts": torch.empty(k, dtype=torch.int64, device=dev)})
    batch = B.Batch(inst, precision=prec)
    if persistent:
        batch.use_persistent(True)
    Cs = [C.copy() for _, C in host]
    for t in range(2):
        B.kmeans_lloyd_batched(batch, 1)
        torch.cuda.synchronize()
        if persistent:
            assert not batch.persistent_aborted()
        for i, ((X, _), ti) in enumerate(zip(host, inst)):
            lab = ti["labels"].cpu().numpy()
            check_labels(lab, Cs[i], X, f"{prec} batch instance {i} {X.shape} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto), f"instance {i} counts t={t}"
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"{prec} batch instance {i} t={t}")
            Cs[i] = Cg
