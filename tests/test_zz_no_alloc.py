"""kmeans_lloyd_static (no workspace: the library's static device scratch)
against kmeans_lloyd on a bound workspace (needs an MI355X).

Bar: both entry points run the same kernels in the same order on the same
inputs, so labels, counts, centroids, the objective history and iters_done
must agree bit for bit; the first call is also held to the FP64 oracle
(labels outside documented near-ties exact, centroids within 1e-5 relative).
Calls come in a row on the one scratch array, each later one on a smaller
input than the one before, so a result that leaned on stale scratch contents
would show.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
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


def _run(torch, B, X, C0, iters, tol, static, precision="fp32"):
    dev = torch.device("cuda")
    n, d = X.shape
    k = C0.shape[0]
    plan = B.Plan(n, d, k, precision, bind_workspace=not static)
    Xg = torch.from_numpy(X).to(dev)
    C = torch.from_numpy(np.ascontiguousarray(C0, np.float32)).to(dev)
    lab = torch.full((n,), -7, dtype=torch.int32, device=dev)
    cnt = torch.full((k,), -7, dtype=torch.int64, device=dev)
    hist = torch.full((iters,), -1.0, dtype=torch.float64, device=dev)
    fn = B.kmeans_lloyd_static if static else B.kmeans_lloyd
    done = fn(plan, Xg, C, lab, cnt, hist, iters, tol)
    torch.cuda.synchronize()
    out = {"C": C.cpu().numpy(), "labels": lab.cpu().numpy(), "counts": cnt.cpu().numpy(),
           "J": hist.cpu().numpy()[:done], "iters": done}
    plan.close()
    return out


def _same(a, b, where):
    assert a["iters"] == b["iters"], f"{where}: iters {a['iters']} vs {b['iters']}"
    for key in ("labels", "counts", "C", "J"):
        assert np.array_equal(a[key], b[key]), f"{where}: {key} differ"


def _blobs(n, d, k, seed):
    return datagen.blobs(n, d, k, k, 1.0, seed, init="sample")


def test_static_scratch_matches_workspace_calls():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    cases = [
        # (n, d, k, iters, tol, precision): each call smaller than the one before
        (300_001, 64, 64, 4, -1.0, "fp32"),
        (40_000, 40, 300, 30, 0.0, "fp32"),      # split passes, tolerance stop
        (12_289, 32, 200, 3, -1.0, "bf16"),      # mixed path (BF16 copy of X in the scratch)
        (5_000, 16, 10, 25, 1e-4, "fp32"),
    ]
    for i, (n, d, k, iters, tol, prec) in enumerate(cases):
        say(f"case {i}: n={n} d={d} k={k} iters={iters} tol={tol} {prec}")
        X, C0 = _blobs(n, d, k, 100 + i)
        plan = B.Plan(n, d, k, prec, bind_workspace=False)
        assert plan.workspace_bytes <= B.STATIC_SCRATCH_BYTES, plan.workspace_bytes
        plan.close()
        ref = _run(torch, B, X, C0, iters, tol, static=False, precision=prec)
        got = _run(torch, B, X, C0, iters, tol, static=True, precision=prec)
        _same(got, ref, f"case {i}")
        if i == 0:
            # the static call against the oracle: C_T is the FP64 mean of the
            # members L_{T-1} gives it, rounded once (counts exact) ...
            # (an empty cluster keeps C_{T-1}, which this call does not return:
            # the oracle is handed the GPU's C_T there, so only members count)
            C_o, cnt_o = oracle.update(X, got["labels"], got["C"].astype(np.float64))
            assert np.array_equal(got["counts"], cnt_o)
            err = np.linalg.norm(got["C"].astype(np.float64) - C_o, axis=1)
            assert np.all(err <= 1e-5 * np.linalg.norm(C_o, axis=1)), err.max()
            # ... and one iteration's labels equal the oracle's assign outside near-ties
            one = _run(torch, B, X, C0, 1, -1.0, static=True)
            lab_o, dmin, d2, J_o = oracle.assign(X, C0.astype(np.float64))
            m = oracle.near_tie_margin(dmin, d2)
            assert not ((one["labels"] != lab_o) & (m >= 1e-6)).any()
            assert abs(one["J"][0] - J_o) <= 1e-5 * J_o
    say("static scratch reused across shrinking calls: all identical")


def test_static_scratch_rejects_large_plans():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    dev = torch.device("cuda")
    # a BF16 plan at n = 2^22, d = 128, k = 1024 keeps a 1 GiB BF16 copy of X
    plan = B.Plan(1 << 22, 128, 1024, "bf16", bind_workspace=False)
    assert plan.workspace_bytes > B.STATIC_SCRATCH_BYTES
    X = torch.zeros(1024, dtype=torch.float32, device=dev)
    C = torch.zeros(1024, dtype=torch.float32, device=dev)
    lab = torch.zeros(1024, dtype=torch.int32, device=dev)
    it = ctypes.c_int32(0)
    # rejected on the host before anything is enqueued (nothing reads X, C or labels)
    st = B.lib().kmeans_lloyd_static(plan.handle, X.data_ptr(), C.data_ptr(), lab.data_ptr(), None, None, 1,
                                     -1.0, ctypes.byref(it), torch.cuda.current_stream().cuda_stream)
    assert st == B.KM_EWORKSPACE, st
    assert b"static scratch" in B.lib().km_last_error()
    plan.close()
