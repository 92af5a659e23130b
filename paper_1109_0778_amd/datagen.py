"""Seeded synthetic Gaussian-blob inputs for k-means.

This module only draws random numbers; it holds none of the clustering
arithmetic.  Both the CPU oracle (through the tests) and the GPU path consume
its output, so the two sides always see bit-identical FP32 inputs.

Recipe (one generator per instance, numpy PCG64 ``default_rng(seed)``), in
draw order:

1. ``centers = uniform(-10, 10, (B, d))``
2. anisotropic case only: ``sig = uniform(0.5, 3.0, (B, d))`` (per blob, per
   feature); otherwise every blob has the scalar ``sigma``.
3. ``blob = integers(0, B, n)`` (equal weights, i.i.d.)
4. ``X = centers[blob] + sig[blob] * standard_normal((n, d))``, drawn in
   fixed chunks of 2**20 rows (the chunked draw equals the one-shot draw), and
   rounded once from FP64 to FP32.
5. initial centroids: the first ``k`` points (``init="first"``) or ``k``
   distinct points drawn with ``choice(n, k, replace=False)``
   (``init="sample"``).

The named workloads follow the shapes of the k-means configurations the
library is measured on (Lloyd 1982 applied to Gaussian-blob data; the paper's
own applications use dense row-major sample matrices, section 4.1).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

CHUNK_ROWS = 1 << 20


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    k: int
    blobs: int
    sigma: float
    seed: int
    iters: int
    init: str = "sample"         # "first" or "sample"
    aniso: bool = False          # per-blob, per-feature sigma ~ U(0.5, 3)
    precision: str = "fp32"      # distance arithmetic the workload names


# The five workloads, by size.  ``precision`` is the arithmetic the workload
# asks the distance step to use.
WORKLOADS = {
    "small": Workload("small", 4096, 8, 8, 8, 1.0, 0, 10, init="first"),
    "plain": Workload("plain", 1 << 20, 64, 64, 64, 1.0, 1, 20),
    "bf16": Workload("bf16", 1 << 22, 128, 1024, 1024, 2.0, 2, 20, precision="bf16"),
    "fp8": Workload("fp8", 1 << 24, 32, 256, 256, 1.0, 3, 15, aniso=True, precision="fp8"),
}

BATCH_COUNT = 512
BATCH_ITERS = 25


def blobs(n: int, d: int, k: int, n_blobs: int, sigma: float, seed: int,
          init: str = "sample", aniso: bool = False, chunk_rows: int = CHUNK_ROWS,
          return_ids: bool = False):
    """Draw ``X`` (n x d FP32, C-contiguous) and initial centroids ``C0`` (k x d FP32)."""
    return _blobs(np.random.default_rng(seed), n, d, k, n_blobs, sigma, init,
                  aniso, chunk_rows, return_ids)


def _blobs(rng, n, d, k, n_blobs, sigma, init="sample", aniso=False,
           chunk_rows=CHUNK_ROWS, return_ids=False):
    if not (1 <= k <= n):
        raise ValueError("need 1 <= k <= n")
    centers = rng.uniform(-10.0, 10.0, (n_blobs, d))
    if aniso:
        sig = rng.uniform(0.5, 3.0, (n_blobs, d))
    else:
        sig = np.full((n_blobs, d), float(sigma))
    blob = rng.integers(0, n_blobs, n)
    X = np.empty((n, d), dtype=np.float32)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        b = blob[r0:r1]
        z = rng.standard_normal((r1 - r0, d))
        X[r0:r1] = (centers[b] + sig[b] * z).astype(np.float32)
    if init == "first":
        C0 = X[:k].copy()
    elif init == "sample":
        idx = rng.choice(n, k, replace=False)
        C0 = X[idx].copy()
    else:
        raise ValueError(f"unknown init {init!r}")
    if return_ids:
        return X, C0, blob.astype(np.int32)
    return X, C0


def workload(name: str, n: int | None = None):
    """Inputs of a named workload; ``n`` optionally truncates to the first rows
    drawn with the same recipe (a different, smaller draw, same distribution)."""
    w = WORKLOADS[name]
    nn = w.n if n is None else n
    return blobs(nn, w.d, w.k, w.blobs, w.sigma, w.seed, init=w.init, aniso=w.aniso)


@dataclass(frozen=True)
class Instance:
    seed: int
    n: int
    d: int
    k: int


def _instance_shape(rng, seed: int) -> Instance:
    n = int(round(float(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))))
    d = int(rng.choice(np.array([16, 32, 64])))
    k = int(rng.integers(4, 129))
    return Instance(seed, n, d, k)


def batch_instance_shape(seed: int) -> Instance:
    """Shape of batched instance ``seed``: n log-uniform in [1e3, 2e5], d in
    {16, 32, 64}, k uniform in [4, 128] (the first three draws of its stream)."""
    return _instance_shape(np.random.default_rng(seed), seed)


def batch_instance(seed: int):
    """Inputs of batched instance ``seed``: after its shape, the same stream
    draws its own blobs (B = k, sigma 1) and sampled initial centroids."""
    rng = np.random.default_rng(seed)
    s = _instance_shape(rng, seed)
    X, C0 = _blobs(rng, s.n, s.d, s.k, s.k, 1.0, init="sample")
    return s, X, C0


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# --------------------------------------------------------------- cytometry
# Synthetic stand-in for the flow-cytometry matrices of the section 4.1
# downsampling step (the datasets are not available): P cell populations with
# Dirichlet(0.7) weights, per-population per-marker means U(0, 5) and standard
# deviations U(0.09, 0.37) (arcsinh-like marker scale), samples drawn i.i.d.
# from the mixture and rounded once to FP32.  With n = 235,000 rows (the
# section's row length) and d = 32 markers the median nearest-neighbour L1
# distance is about 4.4, so the two widths of the section's generated code
# (6.689027961000001 and 22.296759870000002, 1.5 and 5 times a median
# nearest-neighbour distance of 4.459) sit where they sat on its data.
SPADE_APPRX_WIDTH = 6.689027961000001
SPADE_KERNEL_WIDTH = 22.296759870000002
SPADE_N, SPADE_D, SPADE_POPS, SPADE_SEED = 235_000, 32, 24, 7


def cytometry(n: int = SPADE_N, d: int = SPADE_D, pops: int = SPADE_POPS, seed: int = SPADE_SEED,
              sd_lo: float = 0.09, sd_hi: float = 0.37):
    """``X`` (n x d FP32) and the population of every row."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.full(pops, 0.7))
    mu = rng.uniform(0.0, 5.0, (pops, d))
    sd = rng.uniform(sd_lo, sd_hi, (pops, d))
    pop = rng.choice(pops, n, p=w)
    X = mu[pop] + sd[pop] * rng.standard_normal((n, d))
    return np.ascontiguousarray(X, dtype=np.float32), pop


# ----------------------------------------------------- classification data
# Labelled samples for the section 4.2 training applications (their datasets
# are not available).  Labels are i.i.d. uniform over k classes.
def nb_counts(n: int, d: int, k: int, seed: int, rate_hi: float = 5.0):
    """Naive Bayes input: per-sample feature counts, ``X[i, f] ~
    Poisson(rate[y_i, f])`` with ``rate ~ U(0, rate_hi)`` per class and
    feature, as FP32 (exact integers); returns ``(X, y)``."""
    rng = np.random.default_rng(seed)
    rate = rng.uniform(0.0, rate_hi, (k, d))
    y = rng.integers(0, k, n).astype(np.int32)
    X = rng.poisson(rate[y]).astype(np.float32)
    return np.ascontiguousarray(X), y


def gda_classes(n: int, d: int, k: int, seed: int):
    """GDA input: class means ``U(-5, 5)^d``, one shared covariance
    ``A A^T`` with ``A`` having i.i.d. ``N(0, 1/d)`` entries plus the
    identity; ``X = mu[y] + eps A^T`` with ``eps ~ N(0, I)``, rounded once
    to FP32; returns ``(X, y)``."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-5.0, 5.0, (k, d))
    A = np.eye(d) + rng.standard_normal((d, d)) / np.sqrt(d)
    y = rng.integers(0, k, n).astype(np.int32)
    X = mu[y] + rng.standard_normal((n, d)) @ A.T
    return np.ascontiguousarray(X, dtype=np.float32), y
