"""BF16- and FP8-MFMA paths with FP32 recheck (needs an MI355X).

Bar: the mixed path's labels equal the FP32 path's labels bit for bit (the
recheck band is a proven bound), so whole Lloyd trajectories coincide: same
labels and bit-identical centroids every iteration.  Against the FP64 oracle
the labels follow the near-tie rule, centroids and objective are within 1e-5
(the objective comes from the exact identity J = sum|x|^2 + sum_j (cnt_j
|c_j|^2 - 2 c_j . S_j) on the FP64 sums, so it is much closer than that).
"""
import numpy as np
import pytest

import oracle
from paper_1109_0778_amd import datagen
from test_gpu_plain import (REL_TOL, _bind, _torch, check_centroids, check_labels, check_tolerance_run,
                            no_near_ties, robust_tolerances, run_assign, run_lloyd, run_update, say)

pytestmark = pytest.mark.gpu


PRECS = ["bf16", "fp8"]


def mixed_assign(torch, B, X, C, plan=None, prec="bf16"):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C.shape[0]
    plan = plan or B.Plan(n, d, k, prec)
    Xg = torch.from_numpy(X).to(dev)
    Cg = torch.from_numpy(np.ascontiguousarray(C, np.float32)).to(dev)
    lab = torch.full((n,), -7, dtype=torch.int32, device=dev)
    B.kmeans_assign(plan, Xg, Cg, lab)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


SHAPES = [(3000, 8, 8), (5000, 3, 5), (4099, 17, 13), (2500, 64, 64), (1200, 128, 9),
          (257, 33, 40), (700, 1, 4), (20000, 24, 100), (999, 96, 3), (64, 5, 64),
          (20000, 128, 200), (9001, 100, 150), (5000, 24, 600), (40000, 64, 64),
          (20000, 8, 16384), (3000, 40, 1500)]   # the largest k the mixed path takes; k above the row-block size


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,d,k", SHAPES)
def test_mixed_assign_equals_fp32(n, d, k, prec):
    torch, B = _torch(), _bind()
    say(f"mixed assign {prec} n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, max(2, k // 2), 1.5, seed=n + d + k)
    lab_m = mixed_assign(torch, B, X, C, prec=prec)
    lab_p, _, _ = run_assign(torch, B, X, C)
    diff = np.flatnonzero(lab_m != lab_p)
    assert diff.size == 0, f"{diff.size} labels differ from the FP32 path, first {diff[:5]}"
    check_labels(lab_m, C, X, "mixed assign")


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_exact_ties_and_duplicates(prec):
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(6000, 12, 5, 5, 1.0, seed=4)
    C2 = np.concatenate([C, C, C[:2]], 0)      # exact duplicates: every sample has a tie
    lab_m = mixed_assign(torch, B, X, C2, prec=prec)
    lab_p, _, _ = run_assign(torch, B, X, C2)
    assert np.array_equal(lab_m, lab_p)
    assert lab_m.max() < 5                      # the lowest index of each duplicate set wins


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["separated", "all_tied"])
def test_mixed_cascade_extremes(prec, case):
    """Sweeps of more than two 64-centroid chunks screen first (FP8 plans
    screen their open samples again in BF16) and refine the rest inside the
    screen's band.  Tight, well separated blobs leave almost nothing open;
    every centroid duplicated leaves every sample open down to the recheck.
    Both give the FP32 path's labels."""
    torch, B = _torch(), _bind()
    if case == "separated":
        X, C = datagen.blobs(20000, 48, 300, 300, 0.01, seed=31)
    else:
        X, C0 = datagen.blobs(20000, 48, 150, 150, 1.0, seed=32)
        C = np.concatenate([C0, C0], 0)
    say(f"cascade {case} {prec}")
    lab_m = mixed_assign(torch, B, X, C, prec=prec)
    lab_p, _, _ = run_assign(torch, B, X, C)
    diff = np.flatnonzero(lab_m != lab_p)
    assert diff.size == 0, f"{diff.size} labels differ from the FP32 path, first {diff[:5]}"
    check_labels(lab_m, C, X, f"cascade {case}")
    if case == "all_tied":
        assert lab_m.max() < 150                # the lower index of each duplicate pair wins


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,d,k,iters", [(30000, 32, 48, 6), (12000, 128, 180, 4), (5000, 7, 11, 5)])
def test_mixed_lloyd_equals_fp32(n, d, k, iters, prec):
    torch, B = _torch(), _bind()
    say(f"mixed lloyd {prec} n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, k, 2.0, seed=5 * n + k)
    m = run_lloyd(torch, B, X, C, iters, plan=B.Plan(n, d, k, prec))
    p = run_lloyd(torch, B, X, C, iters, plan=B.Plan(n, d, k, "fp32"))
    assert np.array_equal(m["labels"], p["labels"])
    assert np.array_equal(m["C"], p["C"])
    assert np.array_equal(m["counts"], p["counts"])
    np.testing.assert_allclose(m["J"], p["J"], rtol=1e-6)
    o = oracle.lloyd(X, C.astype(np.float64), 1)
    assert abs(m["J"][0] - o["J"][0]) <= 1e-9 * o["J"][0]


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_stepwise_against_oracle(prec):
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(15000, 48, 30, 30, 1.5, seed=9)
    plan = B.Plan(15000, 48, 30, prec)
    Ct = C.copy()
    for t in range(4):
        g = run_lloyd(torch, B, X, Ct, 1, plan=plan)
        lab_o, dmin, J, _, _ = check_labels(g["labels"], Ct, X, f"t={t}")
        assert abs(g["J"][0] - J) <= 1e-9 * J
        Co, cnto = oracle.update(X, g["labels"], Ct.astype(np.float64))
        assert np.array_equal(g["counts"], cnto)
        check_centroids(g["C"], Co, X, f"t={t}")
        Ct = g["C"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,d,k,seed", [(8000, 8, 6, 8), (6000, 16, 200, 7)])   # one-pass sweep; screen + refine
def test_mixed_tolerance_mode_against_oracle(prec, n, d, k, seed):
    """Tolerance mode of the mixed paths against oracle.lloyd(X, C0, 40, tol):
    the changed-label counts of every pass (screen, refine, recheck) add up to
    the stop decision, so stop iteration, labels, counts, objective history
    and centroids follow the oracle's run; and they equal the FP32 path's."""
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(n, d, k, k, 1.0, seed=seed)
    full = oracle.lloyd(X, C.astype(np.float64), 40)
    assert no_near_ties(X, C, full["iters"]) > 1e-5, "input has near-ties: pick another seed"
    for tol in [0.0] + robust_tolerances(full["J"])[:2]:
        say(f"mixed tolerance {prec} n={n} d={d} k={k} tol={tol:.6g}")
        o = oracle.lloyd(X, C.astype(np.float64), 40, tol=tol)
        m = run_lloyd(torch, B, X, C, 40, tol=tol, plan=B.Plan(n, d, k, prec))
        check_tolerance_run(m, o, X, f"{prec} tol={tol}")
        p = run_lloyd(torch, B, X, C, 40, tol=tol, plan=B.Plan(n, d, k, "fp32"))
        assert m["iters"] == p["iters"]
        assert np.array_equal(m["C"], p["C"]) and np.array_equal(m["labels"], p["labels"])


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_rejects_distance_outputs(prec):
    torch, B = _torch(), _bind()
    plan = B.Plan(100, 4, 3, prec)
    X = torch.zeros(400, dtype=torch.float32, device="cuda")
    C = torch.zeros(12, dtype=torch.float32, device="cuda")
    lab = torch.zeros(100, dtype=torch.int32, device="cuda")
    md = torch.zeros(100, dtype=torch.float32, device="cuda")
    with pytest.raises(B.KMeansError) as e:
        B.kmeans_assign(plan, X, C, lab, md)
    assert e.value.status == B.KM_ENOTSUP


@pytest.mark.slow
@pytest.mark.parametrize("name,prec", [("plain", "bf16"), ("bf16", "bf16"), ("fp8", "fp8"), ("fp8", "bf16")])
def test_mixed_full_size_equals_fp32(name, prec):
    """Full-size workloads, launched as the benchmark launches them: the
    mixed path's whole trajectory (labels, centroids every iteration) equals
    the FP32 path's; the last iteration is checked against the oracle on a
    fixed 2^16-sample subset (assign) and over all samples (update)."""
    torch, B = _torch(), _bind()
    w = datagen.WORKLOADS[name]
    iters = 5
    say(f"full size {name} ({prec}): n={w.n} d={w.d} k={w.k}, {iters} iterations")
    X, C0 = datagen.workload(name)
    pm = B.Plan(w.n, w.d, w.k, prec)
    pp = B.Plan(w.n, w.d, w.k, "fp32")
    a = run_lloyd(torch, B, X, C0, iters - 1, plan=pm)
    m = run_lloyd(torch, B, X, a["C"], 1, plan=pm)
    p4 = run_lloyd(torch, B, X, C0, iters - 1, plan=pp)
    assert np.array_equal(p4["C"], a["C"]) and np.array_equal(p4["labels"], a["labels"])
    p = run_lloyd(torch, B, X, p4["C"], 1, plan=pp)
    assert np.array_equal(p["labels"], m["labels"]) and np.array_equal(p["C"], m["C"])
    idx = np.sort(np.random.default_rng(0).choice(w.n, 1 << 16, replace=False))
    check_labels(m["labels"][idx], a["C"], X[idx], f"{name} sampled")
    Co, cnto = oracle.update(X, m["labels"], a["C"].astype(np.float64))
    assert np.array_equal(m["counts"], cnto)
    check_centroids(m["C"], Co, X, f"{name} full update")
    np.testing.assert_allclose(m["J"][0], p["J"][0], rtol=1e-6)


def test_fp8_extreme_feature_scales():
    """Features whose ranges differ by many binades (per-feature scales), a
    constant-zero feature (scale guard), and values that land on e4m3
    subnormals after scaling: labels still equal the FP32 path's."""
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(20000, 20, 40, 40, 1.0, seed=17)
    scale = np.float32(2.0) ** np.arange(-12, 8, dtype=np.float32)
    X = (X * scale).astype(np.float32)
    C = (C * scale).astype(np.float32)
    X[:, 3] = 0.0
    C[:, 3] = 0.0
    X[:50, 5] = np.float32(1e-30)
    lab_m = mixed_assign(torch, B, X, C, prec="fp8")
    lab_p, _, _ = run_assign(torch, B, X, C)
    assert np.array_equal(lab_m, lab_p)
    check_labels(lab_m, C, X, "fp8 scales")


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_recheck_counters(prec):
    """The recheck counters are plausible: every sample is either decided by
    the MFMA pass or queued, never more than n per iteration."""
    torch, B = _torch(), _bind()
    n, d, k = 30000, 32, 64
    X, C = datagen.blobs(n, d, k, k, 1.0, seed=23)
    plan = B.Plan(n, d, k, prec)
    run_lloyd(torch, B, X, C, 2, plan=plan)
    cnt, full = plan.recheck_count()
    say(f"{prec}: {cnt} rechecks, {full} full scans over 2 iterations")
    assert 0 <= full <= cnt <= 2 * n
