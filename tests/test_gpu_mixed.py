"""BF16-MFMA path with FP32 recheck (needs an MI355X).

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
from test_gpu_plain import (REL_TOL, _bind, _torch, check_centroids, check_labels, run_assign,
                            run_lloyd, run_update, say)

pytestmark = pytest.mark.gpu


def mixed_assign(torch, B, X, C, plan=None):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C.shape[0]
    plan = plan or B.Plan(n, d, k, "bf16")
    Xg = torch.from_numpy(X).to(dev)
    Cg = torch.from_numpy(np.ascontiguousarray(C, np.float32)).to(dev)
    lab = torch.full((n,), -7, dtype=torch.int32, device=dev)
    B.kmeans_assign(plan, Xg, Cg, lab)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


SHAPES = [(3000, 8, 8), (5000, 3, 5), (4099, 17, 13), (2500, 64, 64), (1200, 128, 9),
          (257, 33, 40), (700, 1, 4), (20000, 24, 100), (999, 96, 3), (64, 5, 64),
          (20000, 128, 200), (9001, 100, 150), (5000, 24, 600), (40000, 64, 64)]


@pytest.mark.parametrize("n,d,k", SHAPES)
def test_mixed_assign_equals_fp32(n, d, k):
    torch, B = _torch(), _bind()
    say(f"mixed assign n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, max(2, k // 2), 1.5, seed=n + d + k)
    lab_m = mixed_assign(torch, B, X, C)
    lab_p, _, _ = run_assign(torch, B, X, C)
    diff = np.flatnonzero(lab_m != lab_p)
    assert diff.size == 0, f"{diff.size} labels differ from the FP32 path, first {diff[:5]}"
    check_labels(lab_m, C, X, "mixed assign")


def test_mixed_exact_ties_and_duplicates():
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(6000, 12, 5, 5, 1.0, seed=4)
    C2 = np.concatenate([C, C, C[:2]], 0)      # exact duplicates: every sample has a tie
    lab_m = mixed_assign(torch, B, X, C2)
    lab_p, _, _ = run_assign(torch, B, X, C2)
    assert np.array_equal(lab_m, lab_p)
    assert lab_m.max() < 5                      # the lowest index of each duplicate set wins


@pytest.mark.parametrize("n,d,k,iters", [(30000, 32, 48, 6), (12000, 128, 180, 4), (5000, 7, 11, 5)])
def test_mixed_lloyd_equals_fp32(n, d, k, iters):
    torch, B = _torch(), _bind()
    say(f"mixed lloyd n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, k, 2.0, seed=5 * n + k)
    m = run_lloyd(torch, B, X, C, iters, plan=B.Plan(n, d, k, "bf16"))
    p = run_lloyd(torch, B, X, C, iters, plan=B.Plan(n, d, k, "fp32"))
    assert np.array_equal(m["labels"], p["labels"])
    assert np.array_equal(m["C"], p["C"])
    assert np.array_equal(m["counts"], p["counts"])
    np.testing.assert_allclose(m["J"], p["J"], rtol=1e-6)
    o = oracle.lloyd(X, C.astype(np.float64), 1)
    assert abs(m["J"][0] - o["J"][0]) <= 1e-9 * o["J"][0]


def test_mixed_stepwise_against_oracle():
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(15000, 48, 30, 30, 1.5, seed=9)
    plan = B.Plan(15000, 48, 30, "bf16")
    Ct = C.copy()
    for t in range(4):
        g = run_lloyd(torch, B, X, Ct, 1, plan=plan)
        lab_o, dmin, J, _, _ = check_labels(g["labels"], Ct, X, f"t={t}")
        assert abs(g["J"][0] - J) <= 1e-9 * J
        Co, cnto = oracle.update(X, g["labels"], Ct.astype(np.float64))
        assert np.array_equal(g["counts"], cnto)
        check_centroids(g["C"], Co, X, f"t={t}")
        Ct = g["C"]


def test_mixed_tolerance_mode_matches_fp32():
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(8000, 8, 6, 6, 1.0, seed=5)
    for tol in (0.0, 1e-3):
        m = run_lloyd(torch, B, X, C, 40, tol=tol, plan=B.Plan(8000, 8, 6, "bf16"))
        p = run_lloyd(torch, B, X, C, 40, tol=tol, plan=B.Plan(8000, 8, 6, "fp32"))
        assert m["iters"] == p["iters"]
        assert np.array_equal(m["C"], p["C"]) and np.array_equal(m["labels"], p["labels"])


def test_mixed_rejects_distance_outputs():
    torch, B = _torch(), _bind()
    plan = B.Plan(100, 4, 3, "bf16")
    X = torch.zeros(400, dtype=torch.float32, device="cuda")
    C = torch.zeros(12, dtype=torch.float32, device="cuda")
    lab = torch.zeros(100, dtype=torch.int32, device="cuda")
    md = torch.zeros(100, dtype=torch.float32, device="cuda")
    with pytest.raises(B.KMeansError) as e:
        B.kmeans_assign(plan, X, C, lab, md)
    assert e.value.status == B.KM_ENOTSUP


@pytest.mark.slow
@pytest.mark.parametrize("name", ["plain", "bf16"])
def test_mixed_full_size_equals_fp32(name):
    """Full-size workloads, launched as the benchmark launches them: the BF16
    path's whole trajectory (labels, centroids every iteration) equals the
    FP32 path's; the last iteration is checked against the oracle on a fixed
    2^16-sample subset (assign) and over all samples (update)."""
    torch, B = _torch(), _bind()
    w = datagen.WORKLOADS[name]
    iters = 5
    say(f"full size {name}: n={w.n} d={w.d} k={w.k}, {iters} iterations")
    X, C0 = datagen.workload(name)
    pm = B.Plan(w.n, w.d, w.k, "bf16")
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
