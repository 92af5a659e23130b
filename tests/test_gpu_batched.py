"""Batched Lloyd: many instances of different n, d, k in the same launches
(needs an MI355X).  Each instance is checked stepwise against the FP64 oracle
(labels under the near-tie rule, centroids from the oracle's update of the
GPU's labels, counts exact, objective within 1e-5), and graph replays against
direct launches."""
import numpy as np
import pytest

import oracle
from paper_1109_0778_amd import datagen
from test_gpu_plain import REL_TOL, _bind, _torch, check_centroids, check_labels, say

pytestmark = pytest.mark.gpu


def make_batch(torch, B, shapes, seed0=0, iters=4):
    dev = torch.device("cuda")
    inst, host = [], []
    for i, (n, d, k) in enumerate(shapes):
        X, C = datagen.blobs(n, d, k, k, 1.0, seed=seed0 + i)
        host.append((X, C))
        inst.append({"X": torch.from_numpy(X).to(dev), "C": torch.from_numpy(C).to(dev),
                     "labels": torch.full((n,), -1, dtype=torch.int32, device=dev),
                     "counts": torch.empty(k, dtype=torch.int64, device=dev),
                     "obj_hist": torch.zeros(iters, dtype=torch.float64, device=dev)})
    return inst, host


SHAPES = [(1000, 16, 4), (257, 32, 7), (5000, 64, 128), (12345, 16, 60), (3000, 33, 17), (700, 8, 9),
          (40000, 64, 100), (2048, 128, 20), (1, 5, 1), (999, 1, 3), (65536, 32, 64), (300, 64, 128)]


def test_batched_stepwise_against_oracle():
    torch, B = _torch(), _bind()
    inst, host = make_batch(torch, B, SHAPES)
    batch = B.Batch(inst)
    Cs = [C.copy() for _, C in host]
    for t in range(3):
        B.kmeans_lloyd_batched(batch, 1)
        torch.cuda.synchronize()
        for i, ((X, _), ti) in enumerate(zip(host, inst)):
            say(f"t={t} instance {i} shape {X.shape} k={Cs[i].shape[0]}")
            lab = ti["labels"].cpu().numpy()
            _, _, J, _, _ = check_labels(lab, Cs[i], X, f"instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto)
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"instance {i} t={t}")
            assert abs(ti["obj_hist"][0].item() - J) <= REL_TOL * J + 1e-30
            Cs[i] = Cg


@pytest.mark.parametrize("tpb,order", [(1, 0), (3, 1), (64, 1)])
def test_batched_schedules_and_graphs(tpb, order):
    """Any schedule gives oracle-valid results; with a fixed schedule the graph
    replays equal direct launches bit for bit, replay after replay."""
    torch, B = _torch(), _bind()
    inst, host = make_batch(torch, B, SHAPES[:8], seed0=50, iters=3)
    inst2, _ = make_batch(torch, B, SHAPES[:8], seed0=50, iters=3)
    b1 = B.Batch(inst)
    b2 = B.Batch(inst2)
    b1.set_schedule(tpb, order)
    b2.set_schedule(tpb, order)
    b2.use_graphs(True)
    for rep in range(3):
        B.kmeans_lloyd_batched(b1, 3)
        torch.cuda.synchronize()
        B.kmeans_lloyd_batched(b2, 3)
        torch.cuda.synchronize()
        for a, b in zip(inst, inst2):
            assert torch.equal(a["C"], b["C"]) and torch.equal(a["labels"], b["labels"]), f"replay {rep}"
            assert torch.equal(a["counts"], b["counts"]) and torch.equal(a["obj_hist"], b["obj_hist"])


def test_batched_equals_single_instance_path():
    """The same instance alone (kmeans_lloyd) and inside a batch.  From the
    same C_0 both compute the canonical FP32 distances, so the first
    iteration's labels are identical; centroids agree within one FP32 ulp (the
    two group samples into different FP64 partial sums).  The second
    iteration's labels are identical wherever the oracle's top-2 margin for
    the batch's C_1 is at least 1e-5 (the two runs' C_1 differ by up to one
    ulp, which moves a distance by up to about 2u |c| / |x - c| relative)."""
    torch, B = _torch(), _bind()
    inst, host = make_batch(torch, B, SHAPES[:6], seed0=80, iters=2)
    batch = B.Batch(inst)
    single = []
    for (X, C0), ti in zip(host, inst):
        n, d = X.shape
        k = C0.shape[0]
        single.append((B.Plan(n, d, k), torch.from_numpy(C0).cuda(), torch.from_numpy(X).cuda(),
                       torch.empty(n, dtype=torch.int32, device="cuda")))
    ti_prev = None
    for t in range(2):
        B.kmeans_lloyd_batched(batch, 1)
        for i, ((X, _), ti, (plan, Cg, Xg, lab)) in enumerate(zip(host, inst, single)):
            B.kmeans_lloyd(plan, Xg, Cg, lab, None, None, 1)
            torch.cuda.synchronize()
            say(f"t={t} instance {i} shape {X.shape}")
            lb, ls = ti["labels"].cpu().numpy(), lab.cpu().numpy()
            if t == 0:
                assert np.array_equal(lb, ls), f"instance {i}: labels differ"
            else:
                lab_o, dmin, d2, _ = oracle.assign(X, ti_prev[i].astype(np.float64))
                m = oracle.near_tie_margin(dmin, d2)
                bad = (lb != ls) & (m >= 1e-5)
                assert not bad.any(), f"instance {i}: {bad.sum()} labels differ outside near-ties"
            a, b = Cg.cpu().numpy(), ti["C"].cpu().numpy()
            if t == 0:
                ulp = np.spacing(np.abs(a)).astype(np.float32)
                assert np.all(np.abs(a - b) <= ulp), f"instance {i}: centroids differ by more than one ulp"
        ti_prev = [ti["C"].cpu().numpy() for ti in inst]


def test_batched_bf16_stepwise_against_oracle():
    """BF16 MFMA distances + exact recheck in the batched launches: each
    instance checked against the oracle every iteration, like the FP32 batch."""
    torch, B = _torch(), _bind()
    inst, host = make_batch(torch, B, SHAPES, seed0=200)
    batch = B.Batch(inst, precision="bf16")
    Cs = [C.copy() for _, C in host]
    for t in range(3):
        B.kmeans_lloyd_batched(batch, 1)
        torch.cuda.synchronize()
        for i, ((X, _), ti) in enumerate(zip(host, inst)):
            say(f"bf16 t={t} instance {i} shape {X.shape} k={Cs[i].shape[0]}")
            lab = ti["labels"].cpu().numpy()
            _, _, J, _, _ = check_labels(lab, Cs[i], X, f"bf16 instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto)
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"bf16 instance {i} t={t}")
            assert abs(ti["obj_hist"][0].item() - J) <= 1e-9 * J + 1e-30
            Cs[i] = Cg


@pytest.mark.parametrize("tpb,order", [(1, 0), (4, 1), (16, 0)])
def test_batched_bf16_equals_fp32_batch(tpb, order):
    """At a common schedule the BF16 batch's labels, counts and centroids equal
    the FP32 batch's bit for bit (same labels, same reduction order), iteration
    after iteration, with and without graph launch."""
    torch, B = _torch(), _bind()
    inst32, host = make_batch(torch, B, SHAPES, seed0=300, iters=4)
    inst16, _ = make_batch(torch, B, SHAPES, seed0=300, iters=4)
    b32 = B.Batch(inst32)
    b16 = B.Batch(inst16, precision="bf16")
    b32.set_schedule(tpb, order)
    b16.set_schedule(tpb, order)
    b16.use_graphs(True)
    for rep in range(2):
        B.kmeans_lloyd_batched(b32, 4)
        B.kmeans_lloyd_batched(b16, 4)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(inst32, inst16)):
            assert torch.equal(a["labels"], b["labels"]), f"instance {i} rep {rep}"
            assert torch.equal(a["C"], b["C"]) and torch.equal(a["counts"], b["counts"]), f"instance {i} rep {rep}"
            np.testing.assert_allclose(b["obj_hist"].cpu().numpy(), a["obj_hist"].cpu().numpy(), rtol=1e-6)


def test_batched_per_class_schedules():
    """Per-class tiles per block: the classes cover every instance, the values
    are applied, BF16 and FP32 batches given the same per-class schedule agree
    bit for bit, and the results stay oracle-valid (stepwise, one iteration)."""
    torch, B = _torch(), _bind()
    inst32, host = make_batch(torch, B, SHAPES, seed0=400, iters=2)
    inst16, _ = make_batch(torch, B, SHAPES, seed0=400, iters=2)
    b32 = B.Batch(inst32)
    b16 = B.Batch(inst16, precision="bf16")
    cl = b32.classes()
    assert cl == b16.classes() and len(cl) > 1
    assert sum(c[2] for c in cl) == len(SHAPES)
    assert [c[0] for c in cl] == sorted(c[0] for c in cl)
    for b in (b32, b16):
        b.set_schedule(4, 1)
        for c in range(len(cl)):
            b.set_class_schedule(c, (1, 64, 3, 0, 16)[c % 5])
    got = b32.classes()
    assert [g[3] for g in got] == [(1, 64, 3, 4, 16)[c % 5] for c in range(len(cl))]
    b16.use_graphs(True)
    Cs = [C.copy() for _, C in host]
    for t in range(2):
        B.kmeans_lloyd_batched(b32, 1)
        B.kmeans_lloyd_batched(b16, 1)
        torch.cuda.synchronize()
        for i, ((X, _), a, b) in enumerate(zip(host, inst32, inst16)):
            assert torch.equal(a["labels"], b["labels"]), f"instance {i} t={t}"
            assert torch.equal(a["C"], b["C"]) and torch.equal(a["counts"], b["counts"]), f"instance {i} t={t}"
            lab = a["labels"].cpu().numpy()
            check_labels(lab, Cs[i], X, f"class schedule instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(a["counts"].cpu().numpy(), cnto)
            Cg = a["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"class schedule instance {i} t={t}")
            Cs[i] = Cg
    with pytest.raises(B.KMeansError):
        b32.set_class_schedule(len(cl), 2)
    with pytest.raises(B.KMeansError):
        b32.set_class_schedule(0, -1)
    with pytest.raises(B.KMeansError):
        b32.set_class_schedule(0, (1 << 20) + 1)
    with pytest.raises(B.KMeansError):
        b32.set_schedule((1 << 20) + 1, 0)
    # a schedule far longer than any instance: one block and one queue region each
    b16.set_schedule(1 << 20, 1)
    for c in range(len(cl)):
        b16.set_class_schedule(c, 0)
    B.kmeans_lloyd_batched(b16, 1)
    torch.cuda.synchronize()
    for i, ((X, _), t) in enumerate(zip(host, inst16)):
        check_labels(t["labels"].cpu().numpy(), Cs[i], X, f"long schedule instance {i}")


WIDE_SHAPES = [(3000, 16, 20), (2500, 129, 17), (4000, 300, 40), (700, 64, 9), (1500, 1024, 12)]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_wide_instances(prec):
    """Instances of more than 128 features in a batch run the single-instance
    path inside the call: stepwise against the oracle (every instance, two
    iterations), the wide ones equal to kmeans_lloyd on their own bit for bit,
    graph replays equal to direct launches, and a batch of wide instances only."""
    torch, B = _torch(), _bind()
    inst, host = make_batch(torch, B, WIDE_SHAPES, seed0=600, iters=2)
    inst2, _ = make_batch(torch, B, WIDE_SHAPES, seed0=600, iters=2)
    batch = B.Batch(inst, precision=prec)
    b2 = B.Batch(inst2, precision=prec)
    b2.use_graphs(True)
    Cs = [C.copy() for _, C in host]
    for t in range(2):
        B.kmeans_lloyd_batched(batch, 1)
        B.kmeans_lloyd_batched(b2, 1)
        torch.cuda.synchronize()
        for i, ((X, _), ti, tj) in enumerate(zip(host, inst, inst2)):
            say(f"{prec} t={t} instance {i} shape {X.shape} k={Cs[i].shape[0]}")
            lab = ti["labels"].cpu().numpy()
            check_labels(lab, Cs[i], X, f"{prec} wide batch instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto)
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"{prec} wide batch instance {i} t={t}")
            assert torch.equal(ti["C"], tj["C"]) and torch.equal(ti["labels"], tj["labels"]), f"graph, instance {i}"
            Cs[i] = Cg
    # the wide instances alone, through kmeans_lloyd from the same C_0
    for i, (n, d, k) in enumerate(WIDE_SHAPES):
        if d <= 128:
            continue
        X, C0 = host[i]
        plan = B.Plan(n, d, k, prec)
        Xg, Cg = torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda()
        lab = torch.empty(n, dtype=torch.int32, device="cuda")
        B.kmeans_lloyd(plan, Xg, Cg, lab, None, None, 2)
        torch.cuda.synchronize()
        assert torch.equal(Cg, inst[i]["C"]) and torch.equal(lab, inst[i]["labels"]), f"instance {i} alone"
    # wide instances only
    only, ohost = make_batch(torch, B, [s_ for s_ in WIDE_SHAPES if s_[1] > 128], seed0=700, iters=1)
    ob = B.Batch(only, precision=prec)
    assert ob.classes() == []
    B.kmeans_lloyd_batched(ob, 1)
    torch.cuda.synchronize()
    for i, ((X, C0), ti) in enumerate(zip(ohost, only)):
        check_labels(ti["labels"].cpu().numpy(), C0, X, f"{prec} wide-only instance {i}")


def test_batched_optional_outputs():
    """counts and obj_hist are optional for every kind of instance (class
    schedule, wide, FP8 through plans): labels and centroids are unchanged
    by leaving them out."""
    torch, B = _torch(), _bind()
    shapes = [(2000, 16, 10), (1500, 200, 8)]
    for prec in ("fp32", "bf16", "fp8"):
        full, host = make_batch(torch, B, shapes, seed0=900, iters=2)
        bare, _ = make_batch(torch, B, shapes, seed0=900, iters=2)
        for t in bare:
            del t["counts"], t["obj_hist"]
        bf, bb = B.Batch(full, precision=prec), B.Batch(bare, precision=prec)
        B.kmeans_lloyd_batched(bf, 2)
        B.kmeans_lloyd_batched(bb, 2)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(full, bare)):
            assert torch.equal(a["labels"], b["labels"]) and torch.equal(a["C"], b["C"]), f"{prec} instance {i}"
            assert int(a["counts"].sum()) == shapes[i][0]


def test_batched_persistent_launch():
    """The persistent FP32 launch (device queue, per-instance completion
    tickets): labels, centroids, counts and objectives equal the per-class
    launches' at the same schedule, iteration after iteration, over more
    iterations than one launch holds and with graph replay; stepwise valid
    against the oracle; no wait ever reaches its bound."""
    torch, B = _torch(), _bind()
    shapes = [s_ for s_ in SHAPES if s_[1] <= 64]
    iters = 40
    inst, host = make_batch(torch, B, shapes, seed0=1000, iters=iters)
    inst2, _ = make_batch(torch, B, shapes, seed0=1000, iters=iters)
    ref, per = B.Batch(inst), B.Batch(inst2)
    ref.set_schedule(4, 1)
    per.set_schedule(4, 1)
    per.use_persistent(True)
    B.kmeans_lloyd_batched(ref, iters)
    B.kmeans_lloyd_batched(per, iters)
    torch.cuda.synchronize()
    assert not per.persistent_aborted()
    for i, (a, b) in enumerate(zip(inst, inst2)):
        assert torch.equal(a["labels"], b["labels"]) and torch.equal(a["C"], b["C"]), f"instance {i}"
        assert torch.equal(a["counts"], b["counts"]) and torch.equal(a["obj_hist"], b["obj_hist"]), f"instance {i}"
    # stepwise against the oracle, graph-launched
    per.use_graphs(True)
    Cs = [t["C"].cpu().numpy() for t in inst2]
    for t in range(2):
        B.kmeans_lloyd_batched(per, 1)
        torch.cuda.synchronize()
        assert not per.persistent_aborted()
        for i, ((X, _), ti) in enumerate(zip(host, inst2)):
            lab = ti["labels"].cpu().numpy()
            check_labels(lab, Cs[i], X, f"persistent instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto)
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"persistent instance {i} t={t}")
            Cs[i] = Cg
    with pytest.raises(B.KMeansError) as e:
        B.Batch(make_batch(torch, B, [(500, 16, 4)], seed0=1)[0], precision="bf16").use_persistent(True)
    assert e.value.status == B.KM_ENOTSUP
    with pytest.raises(B.KMeansError) as e:
        B.Batch(make_batch(torch, B, [(500, 100, 4)], seed0=1)[0]).use_persistent(True)
    assert e.value.status == B.KM_ENOTSUP


def test_batched_rejects_bad_instances():
    torch, B = _torch(), _bind()
    dev = torch.device("cuda")
    good = {"X": torch.zeros(100, 4, device=dev), "C": torch.zeros(3, 4, device=dev),
            "labels": torch.zeros(100, dtype=torch.int32, device=dev)}
    bad = {"X": torch.zeros(10, 4, device=dev), "C": torch.zeros(11, 4, device=dev),
           "labels": torch.zeros(10, dtype=torch.int32, device=dev)}
    with pytest.raises(B.KMeansError) as e:
        B.Batch([good, bad])
    assert e.value.status == B.KM_EINVAL
    big = {"X": torch.zeros(300, 64, device=dev), "C": torch.zeros(200, 64, device=dev),
           "labels": torch.zeros(300, dtype=torch.int32, device=dev)}
    with pytest.raises(B.KMeansError) as e:          # a 200 x 64 FP64 record does not fit 80 KiB
        B.Batch([good, big])
    assert e.value.status == B.KM_ENOTSUP
    with pytest.raises(B.KMeansError) as e:
        B.Batch([good, bad], precision="fp8")
    assert e.value.status == B.KM_EINVAL


def test_batched_fp8_through_plans():
    """FP8 batches: every instance through its own FP8 plan in the call; stepwise
    against the oracle and equal to kmeans_lloyd with the same plan bit for bit."""
    torch, B = _torch(), _bind()
    shapes = [(3000, 32, 20), (2500, 64, 70), (1500, 200, 12)]
    inst, host = make_batch(torch, B, shapes, seed0=800, iters=2)
    batch = B.Batch(inst, precision="fp8")
    assert batch.classes() == []
    Cs = [C.copy() for _, C in host]
    for t in range(2):
        B.kmeans_lloyd_batched(batch, 1)
        torch.cuda.synchronize()
        for i, ((X, _), ti) in enumerate(zip(host, inst)):
            lab = ti["labels"].cpu().numpy()
            check_labels(lab, Cs[i], X, f"fp8 batch instance {i} t={t}")
            Co, cnto = oracle.update(X, lab, Cs[i].astype(np.float64))
            assert np.array_equal(ti["counts"].cpu().numpy(), cnto)
            Cg = ti["C"].cpu().numpy()
            check_centroids(Cg, Co, X, f"fp8 batch instance {i} t={t}")
            Cs[i] = Cg
    for i, (n, d, k) in enumerate(shapes):
        X, C0 = host[i]
        plan = B.Plan(n, d, k, "fp8")
        Xg, Cg = torch.from_numpy(X).cuda(), torch.from_numpy(C0).cuda()
        lab = torch.empty(n, dtype=torch.int32, device="cuda")
        B.kmeans_lloyd(plan, Xg, Cg, lab, None, None, 2)
        torch.cuda.synchronize()
        assert torch.equal(Cg, inst[i]["C"]) and torch.equal(lab, inst[i]["labels"]), f"instance {i} alone"


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_workload_sampled(prec):
    """The 512-instance workload (n log-uniform in [1e3, 2e5], d in {16, 32,
    64}, k uniform in [4, 128], seeds 0..511), autotuned and graph-launched as
    the benchmark runs it: 24 iterations, then iteration 25 checked against the
    oracle on a fixed sample of 24 instances."""
    torch, B = _torch(), _bind()
    from paper_1109_0778_amd import autotune
    dev = torch.device("cuda")
    inst, host = [], []
    for s in range(datagen.BATCH_COUNT):
        shp, X, C = datagen.batch_instance(s)
        host.append((X, C))
        inst.append({"X": torch.from_numpy(X).to(dev), "C": torch.from_numpy(C).to(dev),
                     "labels": torch.empty(shp.n, dtype=torch.int32, device=dev),
                     "counts": torch.empty(shp.k, dtype=torch.int64, device=dev),
                     "obj_hist": torch.zeros(datagen.BATCH_ITERS, dtype=torch.float64, device=dev)})
    batch = B.Batch(inst, precision=prec)
    choice, _ = autotune.tune_batch(batch, use_cache=False)
    say(f"autotuned schedule {choice}")
    batch.use_graphs(True)
    B.kmeans_lloyd_batched(batch, datagen.BATCH_ITERS - 1)
    torch.cuda.synchronize()
    C24 = [t["C"].cpu().numpy() for t in inst]
    B.kmeans_lloyd_batched(batch, 1)
    torch.cuda.synchronize()
    for i in np.random.default_rng(0).choice(len(inst), 24, replace=False):
        X = host[i][0]
        lab = inst[i]["labels"].cpu().numpy()
        check_labels(lab, C24[i], X, f"instance {i}")
        Co, cnto = oracle.update(X, lab, C24[i].astype(np.float64))
        assert np.array_equal(inst[i]["counts"].cpu().numpy(), cnto)
        check_centroids(inst[i]["C"].cpu().numpy(), Co, X, f"instance {i}")
