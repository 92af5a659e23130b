"""SPADE density step (paper section 4.1) on the GPU against the FP64 oracle
(needs an MI355X).

Bar: densities and visited flags are integers decided by FP64 threshold
tests that both sides evaluate with the same operations in the same order,
so they must be equal element by element (bit-exact).  At the section's full
row length (n = 235,000), where the sequential oracle takes minutes, sampled
rows are checked against the definition one by one: a visited row's density
is its own count, no visited row before it lies within the approximation
width, and a skipped row holds the count of the first visited row that lies
within that width of it.
"""
import sys

import numpy as np
import pytest

from oracle import ml
from paper_1109_0778_amd import datagen

pytestmark = pytest.mark.gpu

APPRX = datagen.SPADE_APPRX_WIDTH
KERNEL = datagen.SPADE_KERNEL_WIDTH


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_spade(X, apprx, kern, metric="l1"):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    n = X.shape[0]
    Xg = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    vis = torch.full((n,), 7, dtype=torch.int8, device="cuda")
    dens, nvis, ws = B.spade_densities(Xg, apprx, kern, metric, visited=vis)
    torch.cuda.synchronize()
    stats = B.spade_stats(ws, n, X.shape[1])
    return dens.cpu().numpy(), vis.cpu().numpy().astype(bool), nvis, stats


def check_equal(X, apprx, kern, metric, where):
    d_o, v_o = ml.spade_densities(X, apprx, kern, metric)
    d_g, v_g, nvis, (batches, cands) = gpu_spade(X, apprx, kern, metric)
    assert np.array_equal(v_g, v_o), f"{where}: visited rows differ at {np.flatnonzero(v_g != v_o)[:5]}"
    assert np.array_equal(d_g, d_o), f"{where}: densities differ at {np.flatnonzero(d_g != d_o)[:5]}"
    assert nvis == int(v_o.sum())
    assert cands >= nvis and batches >= 1
    return nvis, batches, cands


@pytest.mark.parametrize("n,d,metric", [
    (1, 1, "l1"), (2, 3, "l1"), (37, 8, "l1"), (1000, 13, "l1"), (3001, 32, "l1"),
    (3001, 32, "sqeuclidean"), (2000, 64, "l1"), (1500, 65, "l1"), (1200, 100, "sqeuclidean"),
    (5003, 7, "sqeuclidean"),
])
def test_spade_matches_oracle(n, d, metric):
    say(f"spade n={n} d={d} {metric}")
    X, _ = datagen.cytometry(n, d, seed=11 + d)
    # widths scaled with the dimension so that both tests fire
    scale = d / datagen.SPADE_D
    a, k = APPRX * scale, KERNEL * scale
    if metric == "sqeuclidean":
        a, k = a * 0.5, k * 2.0
    nvis, batches, cands = check_equal(X, a, k, metric, f"n={n} d={d}")
    say(f"  visited {nvis} of {n}, {batches} batches, {cands} candidate rows")


def test_spade_section_widths_20k():
    """The section's widths on 20,000 rows of the synthetic cytometry data."""
    X, _ = datagen.cytometry(20_000)
    nvis, batches, cands = check_equal(X, APPRX, KERNEL, "l1", "20k")
    say(f"20k: visited {nvis}, {batches} batches, {cands} candidate rows")


def test_spade_degenerate_widths():
    X, _ = datagen.cytometry(2000, 5, seed=3)
    # no approximation width: every row is visited, densities are the counts
    check_equal(X, 0.0, 3.0, "l1", "apprx 0")
    check_equal(X, -1.0, 3.0, "l1", "apprx < 0")
    # both widths empty: every row visited, every density 0
    d_g, v_g, nvis, _ = gpu_spade(X, 0.0, 0.0)
    assert v_g.all() and nvis == 2000 and not d_g.any()
    check_equal(X, 0.0, 0.0, "l1", "both 0")
    # an approximation width larger than the kernel width, and one that covers everything
    check_equal(X, 5.0, 2.0, "l1", "apprx > kernel")
    check_equal(X, 1e9, 1e9, "l1", "all within")


def test_spade_ties_and_duplicates():
    """Duplicate rows (distance 0) and distances exactly on a width (strict <)."""
    rng = np.random.default_rng(5)
    G = rng.integers(0, 4, (1500, 6)).astype(np.float32)      # integer grid: many exact distances
    check_equal(G, 2.0, 4.0, "l1", "grid 2/4")
    check_equal(G, 3.0, 3.0, "l1", "grid 3/3")
    check_equal(G, 1.0, 5.0, "sqeuclidean", "grid sq 1/5")
    dup = np.repeat(G[:300], 3, axis=0)
    check_equal(dup, 0.5, 2.0, "l1", "duplicates")


def test_spade_rejects_bad_arguments():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(B.KMeansError):
        B.spade_densities(X, float("nan"), 1.0)
    ws = B._workspace(64, X.device)
    with pytest.raises(B.KMeansError):
        B.spade_densities(X, 1.0, 2.0, workspace=ws)       # workspace too small


def _row_dist(X64, i, idx):
    """FP64 L1 distances of row i to rows idx, features summed in increasing order."""
    acc = np.zeros(len(idx))
    for f in range(X64.shape[1]):
        acc = acc + np.abs(X64[i, f] - X64[idx, f])
    return acc


@pytest.mark.slow
def test_spade_full_size_properties():
    """n = 235,000, d = 32 with the section's widths: sampled rows against the definition."""
    X, _ = datagen.cytometry()
    n = X.shape[0]
    dens, vis, nvis, (batches, cands) = gpu_spade(X, APPRX, KERNEL)
    say(f"full size: visited {nvis} of {n}, {batches} batches, {cands} candidate rows")
    X64 = X.astype(np.float64)
    V = np.flatnonzero(vis)
    rng = np.random.default_rng(0)
    alln = np.arange(n)
    for i in rng.choice(V, 40, replace=False):
        dist = _row_dist(X64, i, alln)
        assert dens[i] == int(((dist < APPRX) | (dist < KERNEL)).sum()), f"visited row {i}: count"
        earlier = V[V < i]
        assert not (_row_dist(X64, i, earlier) < APPRX).any(), f"visited row {i} lies near an earlier visited row"
    for j in rng.choice(np.flatnonzero(~vis), 200, replace=False):
        earlier = V[V < j]
        near = earlier[_row_dist(X64, j, earlier) < APPRX]
        assert near.size > 0, f"skipped row {j} has no earlier visited row within the width"
        assert dens[j] == dens[near[0]], f"skipped row {j}: density of row {near[0]} expected"
