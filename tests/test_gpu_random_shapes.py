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
