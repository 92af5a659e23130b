"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each ``pin_*`` function raises AssertionError when the oracle (the shared
library at ``lib``) disagrees with:
  - hand-worked values (``tests/golden``),
  - an independent library routine for a special case (scipy's pairwise
    squared-Euclidean distances; scikit-learn's Lloyd k-means),
  - brute force over every labeling of a tiny input,
  - closed forms (k = 1: global mean and total variance; k = n: identity),
  - invariants (exact power-of-two scaling, permutation equivariance,
    non-increasing objective, centroid = mean of members, counts sum to n).

The same pins run against deliberately broken copies of the oracle
(``test_oracle_mutants.py``) to show that each plausible mistake is caught.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _rand_case(seed, n, d, k, spread=3.0):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, spread, (n, d)).astype(np.float32)
    C = X[rng.choice(n, k, replace=False)].astype(np.float64)
    return X, C


# ---------------------------------------------------------------- golden values
def pin_golden_assign(lib):
    g = _golden("assign_pythagorean.json")
    X = np.array(g["X"], np.float32)
    C = np.array(g["C"], np.float64)
    lab, dmin, d2, J = oracle.assign(X, C, lib=lib)
    assert lab.tolist() == g["labels"], (lab, g["labels"])
    assert np.array_equal(dmin, np.array(g["dmin"], np.float64)), dmin
    assert np.array_equal(d2, np.array(g["d2nd"], np.float64)), d2
    assert J == g["J"], J
    Cn, cnt = oracle.update(X, lab, C, lib=lib)
    assert np.array_equal(Cn, np.array(g["C_new"], np.float64)), Cn
    assert cnt.tolist() == g["counts"]


def pin_golden_lloyd(lib):
    g = _golden("lloyd_1d.json")
    X = np.array(g["X"], np.float32)
    C0 = np.array(g["C0"], np.float64)
    r = oracle.lloyd(X, C0, 3, lib=lib)
    assert r["iters"] == 3
    np.testing.assert_allclose(r["J"], g["J"], rtol=1e-13, atol=0)
    assert r["changed"].tolist() == g["changed"]
    assert r["labels"].tolist() == g["labels_final"]
    assert np.array_equal(r["C"], np.array(g["C_final"], np.float64))
    assert r["counts"].tolist() == g["counts_final"]
    r0 = oracle.lloyd(X, C0, 50, tol=0.0, lib=lib)
    assert r0["iters"] == g["iters_tol0"], r0["iters"]


def pin_golden_tolerance(lib):
    """Tolerance mode: the relative-decrease rule (not only unchanged labels)
    decides the stop, with equality counting as a stop."""
    g = _golden("lloyd_tol.json")
    X = np.array(g["X"], np.float32)
    C0 = np.array(g["C0"], np.float64)
    r = oracle.lloyd(X, C0, 3, lib=lib)
    assert r["J"].tolist() == g["J"], r["J"]
    assert r["changed"].tolist() == g["changed"], r["changed"]
    for tol, iters in g["stops"]:
        rt = oracle.lloyd(X, C0, 10, tol=tol, lib=lib)
        assert rt["iters"] == iters, (tol, rt["iters"], iters)
        assert rt["J"].tolist() == g["J"][:iters]
        if iters == 2:
            assert rt["labels"].tolist() == g["labels_after_t1"]
            assert np.array_equal(rt["C"], np.array(g["C_after_t1"], np.float64))
            assert rt["counts"].tolist() == g["counts_after_t1"]


def pin_near_tie_margin(lib, margin_fn=None):
    """The near-tie margin against hand-worked values (exact ties, a shared
    zero distance, no second centroid, and both sides of the 1e-6 band)."""
    fn = margin_fn or oracle.near_tie_margin
    g = _golden("near_tie_margin.json")
    f = lambda v: np.array([float(x) for x in v], np.float64)   # noqa: E731  ("inf" -> inf)
    m = np.asarray(fn(f(g["d1"]), f(g["d2"])), np.float64)
    want = f(g["margin"])
    assert m.shape == want.shape
    assert not np.isnan(m).any(), m
    exact = np.isinf(want) | (want == 0.0)
    assert np.array_equal(m[exact], want[exact]), (m, want)
    np.testing.assert_allclose(m[~exact], want[~exact], rtol=1e-8, atol=0)
    assert ((m < 1e-6) == np.array(g["near_tie_1e-6"])).all(), m


def pin_golden_empty(lib):
    g = _golden("empty_cluster.json")
    X = np.array(g["X"], np.float32)
    C0 = np.array(g["C0"], np.float64)
    lab, dmin, _, J = oracle.assign(X, C0, lib=lib)
    assert lab.tolist() == g["labels"]
    assert J == g["J"]
    Cn, cnt = oracle.update(X, lab, C0, lib=lib)
    assert np.array_equal(Cn, np.array(g["C_new"], np.float64))
    assert cnt.tolist() == g["counts"]


# ------------------------------------------------------- independent routines
def pin_assign_vs_scipy(lib):
    """Distances equal scipy's pairwise squared Euclidean distances."""
    from scipy.spatial.distance import cdist
    for seed, (n, d, k) in enumerate([(400, 7, 9), (300, 1, 5), (257, 33, 17), (64, 128, 3)]):
        X, C = _rand_case(seed, n, d, k)
        lab, dmin, d2, J = oracle.assign(X, C, lib=lib)
        D = cdist(X.astype(np.float64), C, "sqeuclidean")
        np.testing.assert_allclose(dmin, D.min(1), rtol=1e-12, atol=1e-12)
        Ds = np.sort(D, 1)
        if k > 1:
            np.testing.assert_allclose(d2, Ds[:, 1], rtol=1e-12, atol=1e-12)
        m = oracle.near_tie_margin(dmin, d2)
        clear = m > 1e-9
        assert np.array_equal(lab[clear], D.argmin(1)[clear])
        np.testing.assert_allclose(J, D.min(1).sum(), rtol=1e-12)


def pin_lloyd_vs_sklearn(lib):
    """C_T equals scikit-learn's Lloyd k-means run for T iterations from the
    same initial centroids (no empty clusters occur on these inputs)."""
    from sklearn.cluster import KMeans
    for seed, (n, d, k, T) in enumerate([(2000, 4, 6, 7), (1500, 16, 10, 12)]):
        rng = np.random.default_rng(100 + seed)
        centers = rng.uniform(-10, 10, (k, d))
        X = (centers[rng.integers(0, k, n)] + rng.normal(0, 2.0, (n, d))).astype(np.float32)
        C0 = X[rng.choice(n, k, replace=False)].astype(np.float64)
        r = oracle.lloyd(X, C0, T, lib=lib)
        km = KMeans(k, init=C0, n_init=1, max_iter=T, tol=0.0, algorithm="lloyd")
        km.fit(X.astype(np.float64))
        assert (r["counts"] > 0).all()
        np.testing.assert_allclose(r["C"], km.cluster_centers_, rtol=1e-10, atol=1e-10)
        if km.n_iter_ < T:   # scikit-learn stopped on stable labels
            r0 = oracle.lloyd(X, C0, T, tol=0.0, lib=lib)
            assert r0["iters"] == km.n_iter_, (r0["iters"], km.n_iter_)


# ------------------------------------------------------------------ brute force
def _objective(X, C, L):
    return float(((X.astype(np.float64) - C[L]) ** 2).sum())


def pin_assign_bruteforce(lib):
    """For fixed centroids the labels minimise sum_i d(x_i, c_L(i)) over all
    k^n labelings."""
    for seed in range(4):
        X, C = _rand_case(10 + seed, 6, 2, 3)
        lab, dmin, d2, J = oracle.assign(X, C, lib=lib)
        best, bestL = None, None
        for L in itertools.product(range(3), repeat=6):
            v = _objective(X, C, np.array(L))
            if best is None or v < best:
                best, bestL = v, L
        assert tuple(lab.tolist()) == bestL
        np.testing.assert_allclose(J, best, rtol=1e-12)


def pin_lloyd_bruteforce(lib):
    """Over all labelings with non-empty clusters: the global optimum is a
    Lloyd fixed point, and Lloyd from any start ends at J >= the optimum."""
    for seed in range(3):
        n, k = 8, 3
        rng = np.random.default_rng(20 + seed)
        X = rng.normal(0, 2, (n, 2)).astype(np.float32)
        Xd = X.astype(np.float64)
        best, bestL = None, None
        for L in itertools.product(range(k), repeat=n):
            L = np.array(L)
            if len(set(L.tolist())) < k:
                continue
            C = np.stack([Xd[L == j].mean(0) for j in range(k)])
            v = _objective(X, C, L)
            if best is None or v < best - 1e-12:
                best, bestL = v, L
        Copt = np.stack([Xd[bestL == j].mean(0) for j in range(k)])
        lab, _, _, J = oracle.assign(X, Copt, lib=lib)
        assert np.array_equal(lab, bestL)
        np.testing.assert_allclose(J, best, rtol=1e-12)
        r = oracle.lloyd(X, Copt, 2, lib=lib)
        np.testing.assert_allclose(r["C"], Copt, rtol=1e-12, atol=1e-12)
        for s in range(5):
            C0 = Xd[np.random.default_rng(s).choice(n, k, replace=False)]
            r = oracle.lloyd(X, C0, 30, tol=0.0, lib=lib)
            assert r["J"][-1] >= best - 1e-9


# ---------------------------------------------------------------- closed forms
def pin_k1_closed_form(lib):
    """k = 1: the centroid is the global mean and J_1 = n * sum_f var_f."""
    X, _ = _rand_case(5, 1000, 6, 1)
    Xd = X.astype(np.float64)
    r = oracle.lloyd(X, np.zeros((1, 6)), 2, lib=lib)
    np.testing.assert_allclose(r["C"][0], Xd.mean(0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["J"][1], len(X) * Xd.var(0).sum(), rtol=1e-12)
    np.testing.assert_allclose(r["J"][0], (Xd ** 2).sum(), rtol=1e-12)
    assert r["counts"].tolist() == [1000]


def pin_k_equals_n(lib):
    """k = n distinct samples initialised at the samples: identity labels, J = 0."""
    X, _ = _rand_case(6, 50, 3, 1)
    r = oracle.lloyd(X, X.astype(np.float64), 3, lib=lib)
    assert r["labels"].tolist() == list(range(50))
    assert np.all(r["J"] == 0.0)
    assert np.array_equal(r["C"], X.astype(np.float64))


def pin_blobs_recovered(lib):
    """Well-separated blobs, one initial centroid per blob: labels recover the
    generating blob of every sample."""
    rng = np.random.default_rng(7)
    k, d, n = 5, 3, 600
    centers = np.arange(k)[:, None] * 100.0 + np.zeros((k, d))
    ids = rng.integers(0, k, n)
    X = (centers[ids] + rng.normal(0, 1, (n, d))).astype(np.float32)
    C0 = np.stack([X[np.flatnonzero(ids == j)[0]] for j in range(k)]).astype(np.float64)
    r = oracle.lloyd(X, C0, 5, lib=lib)
    assert np.array_equal(r["labels"], ids)


# ------------------------------------------------------------------ invariants
def pin_scale_invariance(lib):
    """Scaling samples and centroids by 2^m is exact in floating point: labels
    unchanged, J scaled by 4^m, centroids by 2^m, all bit for bit."""
    X, C = _rand_case(8, 500, 5, 7)
    r = oracle.lloyd(X, C, 6, lib=lib)
    for m in (-3, 5):
        s = 2.0 ** m
        r2 = oracle.lloyd((X * np.float32(s)).astype(np.float32), C * s, 6, lib=lib)
        assert np.array_equal(r2["labels"], r["labels"])
        assert np.array_equal(r2["J"], r["J"] * s * s)
        assert np.array_equal(r2["C"], r["C"] * s)


def pin_permutation(lib):
    """Permuting the samples permutes the labels; centroids agree up to the
    order of the FP64 sums."""
    X, C = _rand_case(9, 700, 4, 6)
    perm = np.random.default_rng(1).permutation(len(X))
    r = oracle.lloyd(X, C, 5, lib=lib)
    r2 = oracle.lloyd(X[perm], C, 5, lib=lib)
    assert np.array_equal(r2["labels"], r["labels"][perm])
    np.testing.assert_allclose(r2["C"], r["C"], rtol=1e-12, atol=1e-12)
    assert np.array_equal(r2["counts"], r["counts"])


def pin_lloyd_invariants(lib):
    """J non-increasing; centroid = mean of its members; counts sum to n and
    equal the label histogram; labels are the nearest centroid of C_{T-1}."""
    X, C = _rand_case(11, 3000, 8, 12, spread=5.0)
    r = oracle.lloyd(X, C, 15, lib=lib)
    J = r["J"]
    assert np.all(np.diff(J) <= 1e-9 * J[:-1]), J
    L = r["labels"]
    assert r["counts"].sum() == len(X)
    assert np.array_equal(r["counts"], np.bincount(L, minlength=12))
    Xd = X.astype(np.float64)
    for j in range(12):
        if r["counts"][j]:
            np.testing.assert_allclose(r["C"][j], Xd[L == j].mean(0), rtol=1e-12, atol=1e-12)


ALL_PINS = [
    pin_golden_assign, pin_golden_lloyd, pin_golden_tolerance, pin_near_tie_margin, pin_golden_empty, pin_assign_vs_scipy,
    pin_lloyd_vs_sklearn, pin_assign_bruteforce, pin_lloyd_bruteforce,
    pin_k1_closed_form, pin_k_equals_n, pin_blobs_recovered, pin_scale_invariance,
    pin_permutation, pin_lloyd_invariants,
]


def pin_tie_duplicates(lib):
    """Duplicate centroid rows tie exactly for every sample: the lowest index
    must win, so the later copies stay empty."""
    X, C = _rand_case(12, 200, 3, 4)
    C2 = np.concatenate([C, C[::-1]], 0)         # rows 4..7 duplicate rows 3..0
    lab, _, _, _ = oracle.assign(X, C2, lib=lib)
    lab1, _, _, _ = oracle.assign(X, C, lib=lib)
    assert np.array_equal(lab, lab1)


ALL_PINS.append(pin_tie_duplicates)


def pin_objective(lib):
    """J of given labels: the hand-worked value for the nearest labels, and
    scipy's distances summed over arbitrary labels."""
    from scipy.spatial.distance import cdist
    g = _golden("assign_pythagorean.json")
    X = np.array(g["X"], np.float32)
    C = np.array(g["C"], np.float64)
    assert oracle.objective(X, C, g["labels"], lib=lib) == g["J"]
    assert oracle.objective(X, C, [1, 1, 0, 1], lib=lib) == 100 + 25 + 100 + 225
    X, C = _rand_case(21, 400, 6, 9)
    L = np.random.default_rng(22).integers(0, 9, 400)
    D = cdist(X.astype(np.float64), C, "sqeuclidean")
    np.testing.assert_allclose(oracle.objective(X, C, L, lib=lib), D[np.arange(400), L].sum(), rtol=1e-13)


ALL_PINS.append(pin_objective)
