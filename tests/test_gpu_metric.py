"""Assign under the L1 or squared Euclidean metric, samples row-major or
feature-major (kmeans_assign_metric), against the FP64 oracle (needs an
MI355X).

Bar:
  - labels equal the oracle's (lowest index on ties) except where the
    oracle's top-2 margin (d2 - d1) / (d1 + d2) is below 1e-6: the canonical
    forms' error is at most (2 + 8 + ceil(log2 P)) 2^-24 < 1e-6 relative for
    d <= 128 (P = ceil(d / 8) chunks), so a label can only flip inside that
    band;
  - each chosen distance within that bound of the oracle's;
  - the objective within 1e-5 relative;
  - both layouts bit-identical; the squared form bit-identical to
    kmeans_assign.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ml
from paper_1109_0778_amd import datagen

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bound(d):
    P = (d + 7) // 8
    return (2 + 8 + (math.ceil(math.log2(P)) if P > 1 else 0)) * 2.0 ** -24


def run(torch, B, plan, X, C, metric, layout):
    n, d = X.shape
    Xl = X if layout == "row" else np.ascontiguousarray(X.T)
    Xg = torch.from_numpy(np.ascontiguousarray(Xl)).cuda()
    Cg = torch.from_numpy(C).cuda()
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    md = torch.empty(n, dtype=torch.float32, device="cuda")
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    B.kmeans_assign_metric(plan, Xg, Cg, lab, metric, layout, md, obj)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), md.cpu().numpy(), float(obj.item())


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (1000, 3, 7), (4097, 8, 16), (30000, 16, 64), (20001, 33, 100),
                                   (5000, 64, 300), (3000, 128, 1024), (9000, 20, 2)])
def test_assign_metric_matches_oracle(n, d, k):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"assign metric n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, k, 1.0, seed=d + k)
    plan = B.Plan(n, d, k)
    for metric in ("l1", "sqeuclidean"):
        lab, md, J = run(torch, B, plan, X, C, metric, "row")
        lab_f, md_f, J_f = run(torch, B, plan, X, C, metric, "feature")
        assert np.array_equal(lab, lab_f) and np.array_equal(md, md_f) and J == J_f, f"{metric}: layouts differ"
        lo, d1, d2 = ml.assign_metric(X, C.astype(np.float64), metric)
        with np.errstate(invalid="ignore", divide="ignore"):
            m = np.where(d1 + d2 == 0, 0.0, (d2 - d1) / (d1 + d2))
        m = np.where(np.isinf(d2), np.inf, m)
        bad = (lab != lo) & (m >= 1e-6)
        assert not bad.any(), f"{metric}: {bad.sum()} label mismatches outside near-ties"
        same = lab == lo
        err = np.abs(md[same].astype(np.float64) - d1[same])
        assert np.all(err <= bound(d) * d1[same] + 1e-30), f"{metric}: distance error {err.max():.3e}"
        Jo = float(d1.sum())
        assert abs(J - Jo) <= 1e-5 * max(Jo, 1e-30), (metric, J, Jo)
        say(f"  {metric}: near-ties {(m < 1e-6).sum()}, mismatches inside them {(lab != lo).sum()}")
    # the squared form is the plain path's assign, bit for bit
    lab, md, _ = run(torch, B, plan, X, C, "sqeuclidean", "row")
    lab2 = torch.empty(n, dtype=torch.int32, device="cuda")
    md2 = torch.empty(n, dtype=torch.float32, device="cuda")
    B.kmeans_assign(plan, torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(), lab2, md2)
    torch.cuda.synchronize()
    assert np.array_equal(lab, lab2.cpu().numpy()) and np.array_equal(md, md2.cpu().numpy())


def test_assign_metric_ties_and_errors():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    rng = np.random.default_rng(2)
    X = rng.integers(-3, 4, (2000, 6)).astype(np.float32)
    C = rng.integers(-3, 4, (12, 6)).astype(np.float32)
    C[5] = C[2]                         # duplicate centroid: the lower index wins
    plan = B.Plan(2000, 6, 12)
    for metric in ("l1", "sqeuclidean"):
        lab, md, _ = run(torch, B, plan, X, C, metric, "feature")
        lo, d1, _ = ml.assign_metric(X, C.astype(np.float64), metric)
        assert np.array_equal(lab, lo)              # integer data: every distance is exact
        assert np.array_equal(md.astype(np.float64), d1)
        assert not (lab == 5).any()
    mixed = B.Plan(2000, 6, 12, "bf16")
    with pytest.raises(B.KMeansError):
        run(torch, B, mixed, X, C, "l1", "row")
