"""Rows of more than 128 features (up to the interface's 1024) on the FP32
path: the streaming assign and the reduce over 128-feature slices, against
the FP64 oracle (needs an MI355X).

Bar (BF16 and FP8 plans: labels and centroids equal the FP32 path's, as
at d <= 128): as for the narrow rows, with the canonical form's bound
gamma = (2 + 8 + ceil(log2 P)) 2^-24 (P = ceil(d / 8) chunks): a label can
differ from the oracle's only where the top-2 margin (d2 - d1) / (d1 + d2)
is below gamma (1.01e-6 at d = 1024, so the band is max(1e-6, gamma));
distances within gamma relative; centroids within 1e-5 relative and at most
one FP32 ulp from the oracle's mean; counts exact; tolerance-mode runs equal
the oracle's stop iteration, labels and centroids.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import ml
from paper_1109_0778_amd import datagen

from test_gpu_plain import check_centroids, run_assign, run_lloyd, run_update

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gamma(d):
    P = (d + 7) // 8
    return (2 + 8 + math.ceil(math.log2(P))) * 2.0 ** -24


def check_labels_wide(lab, C, X):
    lab_o, dmin, d2, J = oracle.assign(X, C.astype(np.float64))
    m = oracle.near_tie_margin(dmin, d2)
    band = max(1e-6, gamma(X.shape[1]))
    bad = (lab != lab_o) & (m >= band)
    assert not bad.any(), f"{bad.sum()} label mismatches outside the band"
    return lab_o, dmin, J


WIDE = [(3000, 129, 7), (5001, 256, 40), (2000, 1000, 25), (1500, 1024, 300), (4097, 200, 1), (2500, 640, 2000)]


@pytest.mark.parametrize("n,d,k", WIDE)
def test_wide_assign_and_update(n, d, k):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"wide n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, max(2, k // 2), 1.5, seed=n + d + k)
    plan = B.Plan(n, d, k)
    lab, md, obj = run_assign(torch, B, X, C, plan=plan)
    lab_o, dmin, J = check_labels_wide(lab, C, X)
    ok = lab == lab_o
    rel = np.abs(md[ok].astype(np.float64) - dmin[ok]) / np.maximum(dmin[ok], 1e-300)
    assert np.all((rel <= gamma(d)) | (dmin[ok] == 0)), rel.max()
    assert abs(obj - J) <= 1e-5 * J
    labels = np.random.default_rng(n).integers(0, k, n).astype(np.int32)
    if k > 2:
        labels[labels == 1] = 0
    Cn, cnt = run_update(torch, B, X, labels, C, plan=plan)
    Co, cnto = oracle.update(X, labels, C.astype(np.float64))
    assert np.array_equal(cnt, cnto)
    check_centroids(Cn, Co, X, "wide update")
    ulp = np.spacing(np.abs(Co).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Cn.astype(np.float64) - Co) <= ulp + 1e-300)
    if k > 2:
        assert np.array_equal(Cn[1], C[1])


@pytest.mark.parametrize("n,d,k,iters", [(4000, 300, 12, 4), (3000, 1024, 30, 3), (6000, 136, 500, 3)])
def test_wide_lloyd_stepwise(n, d, k, iters):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"wide stepwise n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, k, 2.0, seed=5 * n + d)
    plan = B.Plan(n, d, k)
    Ct = C.copy()
    for t in range(iters):
        g = run_lloyd(torch, B, X, Ct, 1, plan=plan)
        _, _, J = check_labels_wide(g["labels"], Ct, X)
        assert abs(g["J"][0] - J) <= 1e-5 * J
        Co, cnto = oracle.update(X, g["labels"], Ct.astype(np.float64))
        assert np.array_equal(g["counts"], cnto)
        check_centroids(g["C"], Co, X, f"t={t}")
        Ct = g["C"]
    # the same iterations in one call give the same result (deterministic slices)
    g1 = run_lloyd(torch, B, X, C, iters, plan=plan)
    assert np.array_equal(g1["C"], Ct)


def test_wide_tolerance_mode_matches_oracle():
    """Well-separated blobs (no near-ties): the stop iteration, labels and
    centroids of a tolerance run equal the oracle's."""
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    n, d, k = 6000, 512, 10
    X, C0 = datagen.blobs(n, d, k, k, 0.5, seed=77)
    for tol in (0.0, 1e-3):
        g = run_lloyd(torch, B, X, C0, 40, tol)
        o = oracle.lloyd(X, C0.astype(np.float64), 40, tol)
        assert g["iters"] == o["iters"], (tol, g["iters"], o["iters"])
        assert np.array_equal(g["labels"], o["labels"])
        check_centroids(g["C"], o["C"], X, f"tol={tol}")


def test_wide_class_sums_and_gda():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    n, d, k = 3000, 300, 6
    X, y = datagen.gda_classes(n, d, k, seed=9)
    plan = B.Plan(n, d, k)
    S = torch.empty((k, d), dtype=torch.float64, device="cuda")
    cnt = torch.empty(k, dtype=torch.int64, device="cuda")
    B.km_class_sums(plan, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), S, cnt)
    torch.cuda.synchronize()
    S_o, c_o = ml.class_sums(X, y, k)
    assert np.array_equal(cnt.cpu().numpy(), c_o)
    absum = np.zeros((k, d))
    np.add.at(absum, y, np.abs(X.astype(np.float64)))
    assert np.all(np.abs(S.cpu().numpy() - S_o) <= 2.0 * (c_o[:, None] - 1) * 2.0 ** -53 * absum)


@pytest.mark.parametrize("n,d,k,prec", [(3000, 129, 50, "bf16"), (4001, 256, 200, "bf16"), (2500, 1000, 20, "bf16"),
                                         (2000, 1024, 130, "bf16"), (3000, 136, 40, "fp8"), (2500, 1024, 150, "fp8"),
                                         (1500, 520, 300, "fp8")])
def test_wide_mixed_equals_fp32(n, d, k, prec):
    """BF16 / FP8 MFMA distances with the exact recheck at d > 128: labels and
    centroids equal the FP32 path's every iteration, and the FP32 path is
    held to the oracle stepwise."""
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"wide mixed n={n} d={d} k={k} {prec}")
    X, C = datagen.blobs(n, d, k, max(2, k // 3), 1.5, seed=n + 3 * d + k)
    p32 = B.Plan(n, d, k)
    pm = B.Plan(n, d, k, prec)
    Ct = C.copy()
    for t in range(3):
        g32 = run_lloyd(torch, B, X, Ct, 1, plan=p32)
        gm = run_lloyd(torch, B, X, Ct, 1, plan=pm)
        assert np.array_equal(gm["labels"], g32["labels"]), f"t={t}: labels differ from FP32"
        assert np.array_equal(gm["C"], g32["C"]) and np.array_equal(gm["counts"], g32["counts"])
        _, _, J = check_labels_wide(g32["labels"], Ct, X)
        # the mixed objective comes from the FP64 identity (within 1e-9 of the
        # oracle's), the FP32 path's from FP32 distances (within 1e-6)
        assert abs(gm["J"][0] - J) <= 1e-9 * J
        assert abs(g32["J"][0] - J) <= 1e-6 * J
        Co, _ = oracle.update(X, g32["labels"], Ct.astype(np.float64))
        check_centroids(g32["C"], Co, X, f"t={t}")
        Ct = g32["C"]
    rc, full = pm.recheck_count()
    say(f"  last iteration: {rc} rechecks, {full} full scans")
