"""Pins of the application oracles (``oracle/ml_oracle.c``) against facts
fixed outside them.

Each ``pin_*`` function raises AssertionError when the oracle at ``lib``
disagrees with:
  - hand-worked values (``tests/golden/spade_1d.json``, ``nb_gda.json``);
  - independent library routines: scipy's pairwise L1 / squared Euclidean
    distances, scikit-learn's MultinomialNB (alpha = 1) and
    LinearDiscriminantAnalysis (its pooled covariance), numpy's biased
    covariance;
  - a second, set-based statement of the SPADE result (visited rows form
    the greedy in-order cover of the approximation-width graph; each
    density is the count of the earliest visited row that covers the
    sample) evaluated from scipy distances;
  - special cases and invariants (approximation width 0: every row visited
    and every density is its kernel count; identical samples; probabilities
    summing to one; translation of the samples).

``test_ml_oracle_mutants.py`` runs them against broken copies of the oracle.
"""
from __future__ import annotations

import json
import os

import numpy as np
from scipy.spatial.distance import cdist

from oracle import ml

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _cloud(seed, n, d, scale=1.0, grid=None):
    """Small samples; with ``grid`` the coordinates are multiples of 1/grid,
    so distances between samples are exact in FP64 and ties with the widths
    can be placed on purpose."""
    rng = np.random.default_rng(seed)
    if grid:
        return (rng.integers(0, 4 * grid, (n, d)) / grid).astype(np.float32)
    return (rng.normal(0.0, scale, (n, d))).astype(np.float32)


# ------------------------------------------------------------------ SPADE
def pin_spade_golden(lib):
    g = _golden("spade_1d.json")
    X = np.array(g["X"], np.float32)
    dens, proc = ml.spade_densities(X, g["apprx_width"], g["kernel_width"], lib=lib)
    assert dens.tolist() == g["densities"], dens
    assert proc.tolist() == g["processed"], proc
    X2 = np.array(g["X2"], np.float32)
    dens, proc = ml.spade_densities(X2, g["apprx_width2"], g["kernel_width2"], "l1", lib=lib)
    assert dens.tolist() == g["densities2_l1"] and proc.tolist() == g["processed2_l1"], (dens, proc)
    dens, proc = ml.spade_densities(X2, g["apprx_width2"] ** 2, g["kernel_width2"] ** 2, "sqeuclidean", lib=lib)
    assert dens.tolist() == g["densities2_sq"] and proc.tolist() == g["processed2_sq"], (dens, proc)


def _spade_setwise(X, a, w, metric):
    """The same result stated over sets, from scipy's distances: row i is
    visited iff no earlier visited row lies within a of it; its count is
    |{j : D_ij < a or D_ij < w}|; every sample's density is the count of the
    earliest visited row within a of it (itself when it is visited)."""
    D = cdist(X.astype(np.float64), X.astype(np.float64), "cityblock" if metric == "l1" else "sqeuclidean")
    n = X.shape[0]
    counts = ((D < a) | (D < w)).sum(axis=1)
    visited = np.zeros(n, bool)
    for i in range(n):
        visited[i] = not np.any(visited[:i] & (D[:i, i] < a))
    dens = np.empty(n, np.int64)
    for j in range(n):
        if visited[j]:
            dens[j] = counts[j]
        else:
            p = np.flatnonzero(visited[:j] & (D[:j, j] < a))[0]
            dens[j] = counts[p]
    return dens, visited


def pin_spade_setwise(lib):
    for seed, n, d, metric, grid in [(1, 300, 3, "l1", 4), (2, 250, 5, "l1", None), (3, 200, 2, "sqeuclidean", 8),
                                     (4, 220, 4, "sqeuclidean", None)]:
        X = _cloud(seed, n, d, grid=grid)
        D = cdist(X.astype(np.float64), X.astype(np.float64), "cityblock" if metric == "l1" else "sqeuclidean")
        nn = np.sort(D, axis=1)[:, 1]
        a = float(np.median(nn)) * 1.5
        w = float(np.median(nn)) * 5.0
        if grid:                       # widths on the grid: some distances equal them exactly
            q = grid if metric == "l1" else grid * grid
            a = max(1.0, np.round(a * q)) / q
            w = max(2.0, np.round(w * q)) / q
            assert np.any(D == a) or np.any(D == w)
        ref_d, ref_v = _spade_setwise(X, a, w, metric)
        dens, proc = ml.spade_densities(X, a, w, metric, lib=lib)
        assert np.array_equal(proc, ref_v), (seed, np.flatnonzero(proc != ref_v)[:5])
        assert np.array_equal(dens, ref_d), (seed, np.flatnonzero(dens != ref_d)[:5])
        assert 0 < proc.sum() < n


def pin_spade_special_cases(lib):
    X = _cloud(5, 150, 3)
    D = cdist(X.astype(np.float64), X.astype(np.float64), "cityblock")
    # no approximation: every row is visited and its density is its kernel count
    for w in (0.5, 2.0):
        dens, proc = ml.spade_densities(X, 0.0, w, lib=lib)
        assert proc.all()
        assert np.array_equal(dens, (D < w).sum(axis=1))
    # an approximation width above every distance: row 0 covers everything
    dens, proc = ml.spade_densities(X, float(D.max()) + 1.0, 1.0, lib=lib)
    assert proc.tolist() == [True] + [False] * (len(X) - 1)
    assert (dens == len(X)).all()
    # identical samples: one visited row, density n
    Z = np.ones((40, 6), np.float32)
    dens, proc = ml.spade_densities(Z, 0.1, 0.2, lib=lib)
    assert proc.sum() == 1 and (dens == 40).all()
    # a single sample
    dens, proc = ml.spade_densities(np.zeros((1, 3), np.float32), 1.0, 2.0, lib=lib)
    assert dens.tolist() == [1] and proc.tolist() == [True]


# ------------------------------------------------------------- L1 assign
def pin_assign_metric_golden(lib):
    g = _golden("nb_gda.json")["assign_l1"]
    X = np.array(g["X"], np.float32)
    C = np.array(g["C"], np.float64)
    lab, d1, d2 = ml.assign_metric(X, C, "l1", lib=lib)
    assert lab.tolist() == g["labels_l1"] and d1.tolist() == g["dmin_l1"] and d2.tolist() == g["d2nd_l1"]
    lab, _, _ = ml.assign_metric(X, C, "sqeuclidean", lib=lib)
    assert lab.tolist() == g["labels_sq"], lab


def pin_assign_metric_scipy(lib):
    for metric, sp in (("l1", "cityblock"), ("sqeuclidean", "sqeuclidean")):
        X = _cloud(7, 500, 9)
        C = _cloud(8, 13, 9).astype(np.float64)
        C[5] = C[2]                                    # duplicate centroid: lowest index wins
        D = cdist(X.astype(np.float64), C, sp)
        lab, d1, d2 = ml.assign_metric(X, C, metric, lib=lib)
        assert np.array_equal(lab, np.argmin(D, axis=1))
        np.testing.assert_allclose(d1, D.min(axis=1), rtol=1e-13, atol=0)
        Ds = np.sort(D, axis=1)
        np.testing.assert_allclose(d2, Ds[:, 1], rtol=1e-13, atol=0)
        assert not np.any(lab == 5)


# -------------------------------------------------------------- class sums, NB
def pin_nb_golden(lib):
    g = _golden("nb_gda.json")["nb"]
    X = np.array(g["X"], np.float32)
    prior, phi = ml.nb_train(X, g["y"], g["C"], lib=lib)
    assert prior.tolist() == g["prior"], prior
    want = np.array(g["phi_num"], np.float64) / np.array(g["phi_den"], np.float64)[:, None]
    assert np.array_equal(phi, want), phi
    S, cnt = ml.class_sums(X, g["y"], g["C"], lib=lib)
    assert cnt.tolist() == [2, 2, 0] and S.tolist() == [[3, 1, 1], [0, 3, 1], [0, 0, 0]]


def pin_nb_sklearn(lib):
    from sklearn.naive_bayes import MultinomialNB
    rng = np.random.default_rng(11)
    n, d, C = 600, 40, 4
    X = rng.poisson(rng.uniform(0.1, 3.0, d), (n, d)).astype(np.float32)
    y = rng.integers(0, C, n).astype(np.int32)
    prior, phi = ml.nb_train(X, y, C, lib=lib)
    m = MultinomialNB(alpha=1.0).fit(X.astype(np.float64), y)
    np.testing.assert_allclose(np.log(phi), m.feature_log_prob_, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(np.log(prior), m.class_log_prior_, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(phi.sum(axis=1), 1.0, rtol=1e-12)
    # the per-class reduce: sums against a masked numpy sum (exact: integer counts)
    S, cnt = ml.class_sums(X, y, C, lib=lib)
    for c in range(C):
        assert np.array_equal(S[c], X[y == c].astype(np.float64).sum(axis=0))
        assert cnt[c] == (y == c).sum()


# ----------------------------------------------------------------- GDA
def pin_gda_golden(lib):
    g = _golden("nb_gda.json")["gda"]
    X = np.array(g["X"], np.float32)
    prior, mu, sigma = ml.gda_train(X, g["y"], g["C"], lib=lib)
    assert prior.tolist() == g["prior"] and mu.tolist() == g["mu"] and sigma.tolist() == g["sigma"], (prior, mu, sigma)


def pin_gda_sklearn(lib):
    from sklearn.discriminant_analysis import LinearDiscriminantAnalysis
    rng = np.random.default_rng(12)
    n, d, C = 800, 7, 3
    y = rng.integers(0, C, n).astype(np.int32)
    centers = rng.uniform(-5, 5, (C, d))
    A = rng.normal(0, 1, (d, d))
    X = (centers[y] + rng.normal(0, 1, (n, d)) @ A).astype(np.float32)
    prior, mu, sigma = ml.gda_train(X, y, C, lib=lib)
    lda = LinearDiscriminantAnalysis(solver="lsqr", store_covariance=True).fit(X.astype(np.float64), y)
    np.testing.assert_allclose(mu, lda.means_, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(prior, lda.priors_, rtol=1e-12)
    np.testing.assert_allclose(sigma, lda.covariance_, rtol=1e-10, atol=1e-12)
    assert np.array_equal(sigma, sigma.T)
    assert np.linalg.eigvalsh(sigma).min() > 0


def pin_gda_special_cases(lib):
    rng = np.random.default_rng(13)
    X = (np.round(rng.normal(3.0, 2.0, (300, 5)) * 256) / 256).astype(np.float32)   # + 64 stays exact
    # one class: the biased sample covariance
    prior, mu, sigma = ml.gda_train(X, np.zeros(300, np.int32), 1, lib=lib)
    np.testing.assert_allclose(sigma, np.cov(X.astype(np.float64).T, bias=True), rtol=1e-11, atol=1e-12)
    assert prior.tolist() == [1.0]
    # a translation moves the means and leaves the covariance (power-of-two shift: exact in FP32)
    y = rng.integers(0, 2, 300).astype(np.int32)
    _, mu0, s0 = ml.gda_train(X, y, 2, lib=lib)
    _, mu1, s1 = ml.gda_train((X + np.float32(64.0)).astype(np.float32), y, 2, lib=lib)
    np.testing.assert_allclose(mu1, mu0 + 64.0, rtol=1e-13)
    np.testing.assert_allclose(s1, s0, rtol=1e-9, atol=1e-10)
    # an empty class: prior 0, mean 0, covariance of the others unchanged
    p3, mu3, s3 = ml.gda_train(X, y, 3, lib=lib)
    assert p3[2] == 0.0 and (mu3[2] == 0).all() and np.array_equal(s3, s0)


ALL_ML_PINS = [pin_spade_golden, pin_spade_setwise, pin_spade_special_cases, pin_assign_metric_golden,
               pin_assign_metric_scipy, pin_nb_golden, pin_nb_sklearn, pin_gda_golden, pin_gda_sklearn,
               pin_gda_special_cases]
