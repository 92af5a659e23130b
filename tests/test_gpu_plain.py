"""Parity of the FP32 GPU path with the FP64 oracle (needs an MI355X).

Bar (stated per check):
  - labels equal the oracle's except where the oracle's own top-2 margin
    (d2 - d1) / (d1 + d2) is below 1e-6 (documented near-ties);
  - per-point distances within the canonical form's proven bound
    (2 + 8 + ceil(log2(ceil(d / 8)))) * 2^-24 relative;
  - centroids within 1e-5 relative (per centroid, L2), objective within 1e-5;
  - counts exact.
Trajectories are compared stepwise: each GPU iterate is fed to the oracle
(assign with the GPU's C_t, update with the GPU's L_t).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1109_0778_amd import datagen

pytestmark = pytest.mark.gpu

NEAR_TIE = 1e-6
REL_TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bind():
    from paper_1109_0778_amd import binding
    return binding


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dist_bound(d):
    P = (d + 7) // 8
    return (2 + 8 + math.ceil(math.log2(P)) if P > 1 else 10) * 2.0 ** -24


def check_labels(lab_gpu, C32, X, where=""):
    """GPU labels vs oracle assign with the same FP32 centroids."""
    lab_o, dmin, d2, J = oracle.assign(X, C32.astype(np.float64))
    m = oracle.near_tie_margin(dmin, d2)
    bad = (lab_gpu != lab_o) & (m >= NEAR_TIE)
    assert not bad.any(), f"{where}: {bad.sum()} label mismatches outside near-ties, first {np.flatnonzero(bad)[:5]}"
    return lab_o, dmin, J, int((m < NEAR_TIE).sum()), int((lab_gpu != lab_o).sum())


def check_centroids(C_gpu, C_ref, X, where=""):
    C_gpu = C_gpu.astype(np.float64)
    err = np.linalg.norm(C_gpu - C_ref, axis=1)
    floor = REL_TOL * math.sqrt(float((X.astype(np.float64) ** 2).mean()))
    lim = np.maximum(REL_TOL * np.linalg.norm(C_ref, axis=1), floor)
    assert np.all(err <= lim), f"{where}: centroid error {err.max():.3e} > {lim[err.argmax()]:.3e}"


def run_assign(torch, B, X, C, plan=None):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C.shape[0]
    plan = plan or B.Plan(n, d, k)
    Xg = torch.from_numpy(X).to(dev)
    Cg = torch.from_numpy(np.ascontiguousarray(C, np.float32)).to(dev)
    lab = torch.empty(n, dtype=torch.int32, device=dev)
    md = torch.empty(n, dtype=torch.float32, device=dev)
    obj = torch.empty(1, dtype=torch.float64, device=dev)
    B.kmeans_assign(plan, Xg, Cg, lab, md, obj)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), md.cpu().numpy(), float(obj.item())


def run_update(torch, B, X, labels, C_old, plan=None):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C_old.shape[0]
    plan = plan or B.Plan(n, d, k)
    Xg = torch.from_numpy(X).to(dev)
    Lg = torch.from_numpy(np.ascontiguousarray(labels, np.int32)).to(dev)
    Co = torch.from_numpy(np.ascontiguousarray(C_old, np.float32)).to(dev)
    Cn = torch.empty_like(Co)
    cnt = torch.empty(k, dtype=torch.int64, device=dev)
    B.kmeans_update(plan, Xg, Lg, Co, Cn, cnt)
    torch.cuda.synchronize()
    return Cn.cpu().numpy(), cnt.cpu().numpy()


def run_lloyd(torch, B, X, C0, iters, tol=-1.0, plan=None):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C0.shape[0]
    plan = plan or B.Plan(n, d, k)
    Xg = torch.from_numpy(X).to(dev)
    Cg = torch.from_numpy(np.ascontiguousarray(C0, np.float32)).to(dev)
    lab = torch.full((n,), -1, dtype=torch.int32, device=dev)
    cnt = torch.empty(k, dtype=torch.int64, device=dev)
    hist = torch.zeros(iters, dtype=torch.float64, device=dev)
    it = B.kmeans_lloyd(plan, Xg, Cg, lab, cnt, hist, iters, tol)
    torch.cuda.synchronize()
    return {"C": Cg.cpu().numpy(), "labels": lab.cpu().numpy(), "counts": cnt.cpu().numpy(),
            "J": hist.cpu().numpy()[:it], "iters": it}


SHAPES = [  # (n, d, k): several tiles, ragged tails, odd d, d not a multiple of 8
    (3000, 8, 8), (5000, 3, 5), (4099, 17, 13), (2500, 64, 64), (1200, 128, 9),
    (257, 33, 40), (700, 1, 4), (20000, 24, 100), (999, 96, 3), (64, 5, 64),
    # per-label record beyond one block's LDS: assign + label-chunked update
    (20000, 128, 200), (9001, 96, 150), (5000, 24, 600), (12001, 128, 2000),
    # record too large for the fused pass but within one update block: update over 2 label chunks
    (30000, 64, 120), (20000, 32, 256),
]


@pytest.mark.parametrize("n,d,k", SHAPES)
def test_assign_parity(n, d, k):
    torch, B = _torch(), _bind()
    say(f"assign n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, max(2, k // 2), 1.5, seed=n + d + k)
    lab, md, obj = run_assign(torch, B, X, C)
    lab_o, dmin, J, nties, nmis = check_labels(lab, C, X, "assign")
    ok = lab == lab_o
    rel = np.abs(md[ok].astype(np.float64) - dmin[ok]) / np.maximum(dmin[ok], 1e-300)
    assert np.all((rel <= dist_bound(d)) | (dmin[ok] == 0)), rel.max()
    assert abs(obj - J) <= REL_TOL * J + 1e-30
    say(f"  near-ties {nties}, mismatches {nmis}")


@pytest.mark.parametrize("n,d,k", SHAPES)
def test_update_parity(n, d, k):
    torch, B = _torch(), _bind()
    say(f"update n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, max(2, k // 2), 1.5, seed=7 * n + d + k)
    labels = np.random.default_rng(n).integers(0, k, n).astype(np.int32)
    if k > 2:
        labels[labels == 1] = 0     # leave cluster 1 empty
    Cn, cnt = run_update(torch, B, X, labels, C)
    Co, cnto = oracle.update(X, labels, C.astype(np.float64))
    assert np.array_equal(cnt, cnto)
    check_centroids(Cn, Co, X, "update")
    if k > 2:
        assert np.array_equal(Cn[1], C[1])          # empty cluster keeps its centroid
    # FP64 sums then one rounding: at most 1 FP32 ulp from the oracle's mean
    ulp = np.spacing(np.abs(Co).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Cn.astype(np.float64) - Co) <= ulp + 1e-300)


@pytest.mark.parametrize("k", [176128, 180000])
def test_update_many_label_chunks(k):
    """Records far above LDS size: the update partitions each 4096-sample
    sub-range by label chunk (43 labels of d = 128 per chunk).  k = 176128
    gives 4096 chunks, the most the four-wave partition's per-wave counts
    fit in 64 KiB; k = 180000 gives 4187 chunks, which take the one-wave
    partition.  Random labels leave about a third of the clusters empty."""
    torch, B = _torch(), _bind()
    n, d = 200000, 128
    nch = -(-k // ((44 * 1024) // (8 * d + 4)))
    assert (nch <= 4096) == (k == 176128)
    say(f"update n={n} d={d} k={k} ({nch} label chunks)")
    rng = np.random.default_rng(k)
    X = (3.0 * rng.standard_normal((n, d))).astype(np.float32)
    C = rng.standard_normal((k, d)).astype(np.float32)
    labels = rng.integers(0, k, n).astype(np.int32)
    Cn, cnt = run_update(torch, B, X, labels, C)
    Co, cnto = oracle.update(X, labels, C.astype(np.float64))
    assert np.array_equal(cnt, cnto)
    empty = cnto == 0
    assert empty.sum() > k // 4
    assert np.array_equal(Cn[empty], C[empty])
    ulp = np.spacing(np.abs(Co).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Cn.astype(np.float64) - Co) <= ulp + 1e-300)


def test_small_workload_end_to_end():
    """The small workload (n=4096, d=8, k=8, 10 iterations, init = first k
    points) end to end against the oracle's own trajectory."""
    torch, B = _torch(), _bind()
    w = datagen.WORKLOADS["small"]
    X, C0 = datagen.workload("small")
    say("small workload end-to-end")
    g = run_lloyd(torch, B, X, C0, w.iters)
    o = oracle.lloyd(X, C0.astype(np.float64), w.iters)
    assert g["iters"] == w.iters
    assert np.array_equal(g["labels"], o["labels"])
    assert np.array_equal(g["counts"], o["counts"])
    check_centroids(g["C"], o["C"], X, "small")
    np.testing.assert_allclose(g["J"], o["J"], rtol=REL_TOL)


@pytest.mark.parametrize("n,d,k,iters", [(20000, 16, 20, 6), (6001, 64, 64, 4), (3001, 7, 11, 5),
                                          (12000, 128, 180, 3)])
def test_lloyd_stepwise(n, d, k, iters):
    """Each iteration of the GPU run checked against the oracle fed with the
    GPU's own iterate; the fused pass equals assign-then-update bit for bit."""
    torch, B = _torch(), _bind()
    say(f"stepwise n={n} d={d} k={k}")
    X, C = datagen.blobs(n, d, k, k, 2.0, seed=3 * n + k)
    plan = B.Plan(n, d, k)
    Ct = C.copy()
    J_prev = None
    for t in range(iters):
        g = run_lloyd(torch, B, X, Ct, 1, plan=plan)
        lab_o, dmin, J, _, _ = check_labels(g["labels"], Ct, X, f"t={t}")
        assert abs(g["J"][0] - J) <= REL_TOL * J
        Co, cnto = oracle.update(X, g["labels"], Ct.astype(np.float64))
        assert np.array_equal(g["counts"], cnto)
        check_centroids(g["C"], Co, X, f"t={t}")
        lab_u, _, _ = run_assign(torch, B, X, Ct, plan=plan)
        assert np.array_equal(lab_u, g["labels"])
        Cu, cntu = run_update(torch, B, X, lab_u, Ct, plan=plan)
        assert np.array_equal(Cu, g["C"]) and np.array_equal(cntu, g["counts"])
        if J_prev is not None:
            assert g["J"][0] <= J_prev * (1 + 1e-6)
        J_prev = g["J"][0]
        Ct = g["C"]


def test_multi_iteration_equals_stepwise_and_is_deterministic():
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(30000, 32, 48, 48, 1.0, seed=11)
    plan = B.Plan(30000, 32, 48)
    a = run_lloyd(torch, B, X, C, 7, plan=plan)
    b = run_lloyd(torch, B, X, C, 7, plan=plan)
    assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["labels"], b["labels"])
    assert np.array_equal(a["J"], b["J"])
    Ct = C.copy()
    for t in range(7):
        s = run_lloyd(torch, B, X, Ct, 1, plan=plan)
        assert s["J"][0] == a["J"][t]
        Ct = s["C"]
    assert np.array_equal(Ct, a["C"])
    r1 = run_lloyd(torch, B, X, C, 3, plan=plan)   # resume: 3 + 4 == 7
    r2 = run_lloyd(torch, B, X, r1["C"], 4, plan=plan)
    assert np.array_equal(r2["C"], a["C"]) and np.array_equal(r2["labels"], a["labels"])


def robust_tolerances(J, fixed=(1e-3, 1e-1), gap=1e-4):
    """Tolerances whose stop iteration cannot depend on rounding: every
    relative decrease r_t = (J_{t-1} - J_t) / J_{t-1} of the oracle's
    trajectory lies at least `gap` away from the tolerance (the GPU's J agrees
    with the oracle's to about 1e-7 relative).  The fixed values are kept
    when they qualify; midpoints between neighbouring r_t are added."""
    r = np.sort((J[:-1] - J[1:]) / J[:-1])
    ok = lambda tol: bool(np.all(np.abs(r - tol) >= gap))   # noqa: E731
    tols = [t for t in fixed if ok(t)]
    for a, b in zip(r[:-1], r[1:]):
        if b - a > 2 * gap and len(tols) < len(fixed) + 3:
            tols.append(float(0.5 * (a + b)))
    return sorted(set(tols))


def no_near_ties(X, C0, iters):
    """Oracle trajectory with its smallest top-2 margin over all iterations."""
    Ct = C0.astype(np.float64)
    worst = np.inf
    for _ in range(iters):
        lab, dmin, d2, _ = oracle.assign(X, Ct)
        worst = min(worst, float(oracle.near_tie_margin(dmin, d2).min()))
        Ct, _ = oracle.update(X, lab, Ct)
    return worst


def check_tolerance_run(g, o, X, where):
    """A GPU tolerance-mode run against the oracle's: same stop iteration,
    labels, counts, objective history within 1e-5, centroids within 1e-5."""
    assert g["iters"] == o["iters"], f"{where}: GPU stopped after {g['iters']}, oracle after {o['iters']}"
    assert np.array_equal(g["labels"], o["labels"]), where
    assert np.array_equal(g["counts"], o["counts"]), where
    np.testing.assert_allclose(g["J"], o["J"], rtol=REL_TOL, atol=0, err_msg=where)
    check_centroids(g["C"], o["C"], X, where)


TOL_CASES = [(8000, 8, 6, 8), (12000, 16, 40, 5)]   # seeds whose oracle trajectory has no top-2 margin below 1e-5


@pytest.mark.parametrize("n,d,k,seed", TOL_CASES)
def test_tolerance_mode(n, d, k, seed):
    """Tolerance mode against oracle.lloyd(X, C0, 40, tol): tol = 0 (stable
    labels) and tolerances where the relative-decrease rule decides, placed
    so that no iteration's decrease is within 1e-4 of them."""
    torch, B = _torch(), _bind()
    X, C = datagen.blobs(n, d, k, k, 1.0, seed=seed)
    full = oracle.lloyd(X, C.astype(np.float64), 40)
    assert no_near_ties(X, C, full["iters"]) > 1e-5, "input has near-ties: pick another seed"
    tols = [0.0] + robust_tolerances(full["J"])
    j_rule_stops = 0
    for tol in tols:
        say(f"tolerance n={n} d={d} k={k} tol={tol:.6g}")
        o = oracle.lloyd(X, C.astype(np.float64), 40, tol=tol)
        g = run_lloyd(torch, B, X, C, 40, tol=tol)
        check_tolerance_run(g, o, X, f"fp32 tol={tol}")
        j_rule_stops += int(o["iters"] < 40 and o["changed"][o["iters"] - 1] > 0)
    # at least one stop decided by the relative-decrease rule, labels still changing
    assert j_rule_stops >= 1, tols


def test_edge_cases():
    torch, B = _torch(), _bind()
    # n = 1, k = 1
    X = np.array([[1.5, -2.0, 3.0]], np.float32)
    g = run_lloyd(torch, B, X, X.copy(), 2)
    assert g["labels"].tolist() == [0] and np.array_equal(g["C"], X) and g["J"].tolist() == [0.0, 0.0]
    # k = n with distinct samples: identity labels, J = 0
    X, _ = datagen.blobs(300, 5, 1, 3, 4.0, seed=2)
    g = run_lloyd(torch, B, X, X.copy(), 2)
    assert g["labels"].tolist() == list(range(300)) and np.all(g["J"] == 0)
    # duplicate centroids: the lowest index wins every exact tie
    X, C = datagen.blobs(5000, 12, 4, 4, 1.0, seed=3)
    C2 = np.concatenate([C, C], 0)
    lab, _, _ = run_assign(torch, B, X, C2)
    lab1, _, _ = run_assign(torch, B, X, C)
    assert np.array_equal(lab, lab1)
    # a far centroid stays empty and keeps its position
    C3 = np.concatenate([C, np.full((1, 12), 1e4, np.float32)], 0)
    g = run_lloyd(torch, B, X, C3, 3)
    assert g["counts"][4] == 0 and np.array_equal(g["C"][4], C3[4])
    # labels outside [0, k) are ignored by the update
    labels = np.random.default_rng(0).integers(0, 4, 5000).astype(np.int32)
    bad = labels.copy()
    bad[::7] = 99
    bad[1::11] = -3
    Cn, cnt = run_update(torch, B, X, bad, C)
    keep = (bad >= 0) & (bad < 4)
    Co, cnto = oracle.update(X[keep], bad[keep], C.astype(np.float64))
    assert np.array_equal(cnt, cnto)
    check_centroids(Cn, Co, X, "bad labels")


def test_misaligned_and_wrong_shapes_rejected():
    torch, B = _torch(), _bind()
    plan = B.Plan(100, 4, 3)
    X = torch.zeros(401, dtype=torch.float32, device="cuda")[1:]
    C = torch.zeros(12, dtype=torch.float32, device="cuda")
    lab = torch.zeros(100, dtype=torch.int32, device="cuda")
    with pytest.raises(B.KMeansError) as e:
        B.kmeans_assign(plan, X, C, lab)
    assert e.value.status == B.KM_EINVAL
    with pytest.raises(ValueError):
        B.kmeans_assign(plan, torch.zeros(404, dtype=torch.float32, device="cuda"), C, lab)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert B.lib().km_plan_set_workspace(plan.handle, small.data_ptr(), 16) == B.KM_EWORKSPACE


@pytest.mark.slow
def test_plain_workload_full_size_sampled():
    """n = 2^20, d = 64, k = 64, launched exactly as the benchmark launches it:
    20 Lloyd iterations; the last iteration is checked against the oracle
    (assign on a fixed 2^16-sample subset with the GPU's C_19, update over all
    samples with the GPU's L_19, and the full objective J_19)."""
    torch, B = _torch(), _bind()
    w = datagen.WORKLOADS["plain"]
    say("plain workload full size")
    X, C0 = datagen.workload("plain")
    plan = B.Plan(w.n, w.d, w.k)
    a = run_lloyd(torch, B, X, C0, w.iters - 1, plan=plan)
    g = run_lloyd(torch, B, X, a["C"], 1, plan=plan)
    full = run_lloyd(torch, B, X, C0, w.iters, plan=plan)
    assert np.array_equal(full["C"], g["C"]) and np.array_equal(full["labels"], g["labels"])
    assert np.array_equal(full["J"][:-1], a["J"]) and full["J"][-1] == g["J"][0]
    idx = np.sort(np.random.default_rng(0).choice(w.n, 1 << 16, replace=False))
    check_labels(g["labels"][idx], a["C"], X[idx], "plain sampled")
    Co, cnto = oracle.update(X, g["labels"], a["C"].astype(np.float64))
    assert np.array_equal(g["counts"], cnto)
    check_centroids(g["C"], Co, X, "plain full update")
    _, _, _, J = oracle.assign(X, a["C"].astype(np.float64))
    assert abs(g["J"][0] - J) <= REL_TOL * J
    assert np.all(np.diff(full["J"]) <= 1e-6 * full["J"][:-1])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_replays_match_direct_launches(precision):
    """kmeans_lloyd captured into a HIP graph: several replays, with direct
    work and synchronisations in between, each equal to a direct call."""
    torch, B = _torch(), _bind()
    dev = torch.device("cuda")
    X, C0 = datagen.blobs(20000, 24, 30, 30, 1.5, seed=21)
    n, d = X.shape
    k = C0.shape[0]
    Xg = torch.from_numpy(X).to(dev)
    ref = B.Plan(n, d, k, precision)
    gp = B.Plan(n, d, k, precision)
    gp.use_graphs(True)
    C_ref = torch.from_numpy(C0).to(dev)
    C_g = torch.from_numpy(C0).to(dev)
    lab_r = torch.empty(n, dtype=torch.int32, device=dev)
    lab_g = torch.empty(n, dtype=torch.int32, device=dev)
    cnt_r = torch.empty(k, dtype=torch.int64, device=dev)
    cnt_g = torch.empty(k, dtype=torch.int64, device=dev)
    h_r = torch.empty(3, dtype=torch.float64, device=dev)
    h_g = torch.empty(3, dtype=torch.float64, device=dev)
    for rep in range(4):
        B.kmeans_lloyd(ref, Xg, C_ref, lab_r, cnt_r, h_r, 3, -1.0)
        torch.cuda.synchronize()
        B.kmeans_lloyd(gp, Xg, C_g, lab_g, cnt_g, h_g, 3, -1.0)   # capture on rep 0, replay after
        torch.cuda.synchronize()
        _ = (Xg[:100] * 2).sum().item()                           # unrelated direct work in between
        assert torch.equal(C_g, C_ref) and torch.equal(lab_g, lab_r), f"replay {rep}"
        assert torch.equal(cnt_g, cnt_r) and torch.equal(h_g, h_r), f"replay {rep}"
    # tolerance mode through the graph: iterations done come back each replay
    C_a = torch.from_numpy(C0).to(dev)
    C_b = torch.from_numpy(C0).to(dev)
    it_a = B.kmeans_lloyd(ref, Xg, C_a, lab_r, None, None, 50, 0.0)
    it_b = B.kmeans_lloyd(gp, Xg, C_b, lab_g, None, None, 50, 0.0)
    assert it_a == it_b and torch.equal(C_a, C_b)


def test_validate_mode_rejects_out_of_range_labels():
    """Debug-validate mode: kmeans_update returns KM_EINVAL for labels outside
    [0, k), enqueues nothing (outputs untouched), and with valid labels gives
    the same result as without the check."""
    torch, B = _torch(), _bind()
    dev = torch.device("cuda")
    X, C = datagen.blobs(5000, 12, 4, 4, 1.0, seed=3)
    plan = B.Plan(5000, 12, 4)
    plan.set_validate(True)
    labels = np.random.default_rng(0).integers(0, 4, 5000).astype(np.int32)
    Cn, cnt = run_update(torch, B, X, labels, C, plan=plan)
    Co, cnto = oracle.update(X, labels, C.astype(np.float64))
    assert np.array_equal(cnt, cnto)
    check_centroids(Cn, Co, X, "validate, valid labels")
    for bad_value in (4, -1, 1 << 30):
        bad = labels.copy()
        bad[1234] = bad_value
        Xg = torch.from_numpy(X).to(dev)
        Lg = torch.from_numpy(bad).to(dev)
        Cg = torch.from_numpy(C).to(dev)
        out = torch.full_like(Cg, 7.0)
        counts = torch.full((4,), -5, dtype=torch.int64, device=dev)
        with pytest.raises(B.KMeansError) as e:
            B.kmeans_update(plan, Xg, Lg, Cg, out, counts)
        assert e.value.status == B.KM_EINVAL and "outside" in str(e.value)
        torch.cuda.synchronize()
        assert torch.all(out == 7.0) and torch.all(counts == -5)
    plan.set_validate(False)
    bad = labels.copy()
    bad[::9] = 17
    Cn, cnt = run_update(torch, B, X, bad, C, plan=plan)
    keep = bad < 4
    Co, cnto = oracle.update(X[keep], bad[keep], C.astype(np.float64))
    assert np.array_equal(cnt, cnto)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_after_workspace_rebind(precision):
    """A plan that captured kmeans_lloyd into a graph, then bound a fresh
    workspace (the old one freed): the next call must not replay kernels that
    point at the old workspace; results equal a direct call's."""
    torch, B = _torch(), _bind()
    dev = torch.device("cuda")
    X, C0 = datagen.blobs(20000, 24, 30, 30, 1.5, seed=22)
    n, d = X.shape
    k = C0.shape[0]
    Xg = torch.from_numpy(X).to(dev)
    ref = B.Plan(n, d, k, precision)
    gp = B.Plan(n, d, k, precision)
    gp.use_graphs(True)
    lab_r = torch.empty(n, dtype=torch.int32, device=dev)
    lab_g = torch.empty(n, dtype=torch.int32, device=dev)
    h_r = torch.empty(3, dtype=torch.float64, device=dev)
    h_g = torch.empty(3, dtype=torch.float64, device=dev)
    C_g = torch.from_numpy(C0).to(dev)
    B.kmeans_lloyd(gp, Xg, C_g, lab_g, None, h_g, 3, -1.0)    # capture + run
    torch.cuda.synchronize()
    gp.rebind_workspace()                                     # the old workspace tensor is released
    torch.cuda.empty_cache()
    junk = torch.full((gp.workspace_bytes // 4 + 64,), -1.0, device=dev)   # reuse of freed memory
    for rep in range(2):
        C_r = torch.from_numpy(C0).to(dev)
        C_g.copy_(C_r)
        B.kmeans_lloyd(ref, Xg, C_r, lab_r, None, h_r, 3, -1.0)
        B.kmeans_lloyd(gp, Xg, C_g, lab_g, None, h_g, 3, -1.0)
        torch.cuda.synchronize()
        assert torch.equal(C_g, C_r) and torch.equal(lab_g, lab_r) and torch.equal(h_g, h_r), f"rep {rep}"
    del junk
