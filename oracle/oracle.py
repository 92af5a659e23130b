"""ctypes front end of the C oracle (``kmeans_oracle.c``) -- test infrastructure.

Every function takes FP32 samples (widened exactly to FP64 inside) and FP64
or FP32 centroids, and returns FP64 results.  See ``kmeans_oracle.c`` for the
definition each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(_HERE, "kmeans_oracle.c")
LIB_PATH = os.path.join(_HERE, "libkmeans_oracle.so")

# Plain FP64: no contraction into FMA, no reassociation.
CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-shared", "-fPIC"]


def build(src: str = SRC_PATH, out: str = LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *extra, src, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


_LIB = {}


def _lib(path: str = LIB_PATH):
    if path not in _LIB:
        if path == LIB_PATH and (not os.path.exists(path)
                                 or os.path.getmtime(path) < os.path.getmtime(SRC_PATH)):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.orc_assign.restype = ctypes.c_double
        lib.orc_assign.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P]
        lib.orc_update.restype = ctypes.c_int
        lib.orc_update.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_lloyd.restype = ctypes.c_int
        lib.orc_lloyd.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, P, P, P, P, P]
        lib.orc_objective.restype = ctypes.c_double
        lib.orc_objective.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        lib.orc_num_threads.restype = ctypes.c_int
        _LIB[path] = lib
    return _LIB[path]


def _f32(a):
    a = np.ascontiguousarray(a)
    if a.dtype != np.float32:
        raise TypeError("samples must be FP32")
    return a


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def assign(X, C, lib: str = LIB_PATH):
    """Labels, nearest distance, second-nearest distance (all FP64) and J."""
    X = _f32(X)
    C = _f64(C)
    n, d = X.shape
    k = C.shape[0]
    labels = np.empty(n, np.int32)
    dmin = np.empty(n, np.float64)
    d2 = np.empty(n, np.float64)
    J = _lib(lib).orc_assign(_p(X), _p(C), n, d, k, _p(labels), _p(dmin), _p(d2))
    return labels, dmin, d2, J


def update(X, labels, C_old, lib: str = LIB_PATH):
    """New centroids (FP64) and counts (int64) from given labels."""
    X = _f32(X)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    C_old = _f64(C_old)
    n, d = X.shape
    k = C_old.shape[0]
    C_new = np.empty((k, d), np.float64)
    counts = np.empty(k, np.int64)
    rc = _lib(lib).orc_update(_p(X), _p(labels), _p(C_old), n, d, k, _p(C_new), _p(counts))
    if rc != 0:
        raise ValueError(f"orc_update failed ({rc}): label out of range")
    return C_new, counts


def lloyd(X, C0, max_iter: int, tol: float = -1.0, lib: str = LIB_PATH):
    """Lloyd iterations.  Returns dict with C (C_T), labels (L_{T-1}), counts,
    J (J_0..J_{T-1}), changed and iters."""
    X = _f32(X)
    C0 = _f64(C0)
    n, d = X.shape
    k = C0.shape[0]
    C = np.empty((k, d), np.float64)
    labels = np.empty(n, np.int32)
    counts = np.empty(k, np.int64)
    J = np.zeros(max(max_iter, 1), np.float64)
    ch = np.zeros(max(max_iter, 1), np.int64)
    it = _lib(lib).orc_lloyd(_p(X), _p(C0), n, d, k, max_iter, tol, _p(C), _p(labels),
                             _p(counts), _p(J), _p(ch))
    if it < 0:
        raise MemoryError("orc_lloyd failed")
    return {"C": C, "labels": labels, "counts": counts, "J": J[:it].copy(),
            "changed": ch[:it].copy(), "iters": it}


def objective(X, C, labels, lib: str = LIB_PATH) -> float:
    """J of given labels against C (FP64)."""
    X = _f32(X)
    C = _f64(C)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n, d = X.shape
    J = _lib(lib).orc_objective(_p(X), _p(C), _p(labels), n, d, C.shape[0])
    if J < 0:
        raise ValueError("label out of range")
    return float(J)


def near_tie_margin(dmin, d2nd):
    """Relative top-2 margin (d2 - d1) / (d1 + d2); 0 for exact ties at a
    shared zero distance, +inf when there is no second centroid."""
    dmin = np.asarray(dmin, np.float64)
    d2nd = np.asarray(d2nd, np.float64)
    den = dmin + d2nd
    with np.errstate(invalid="ignore", divide="ignore"):
        m = (d2nd - dmin) / den
    m = np.where(den == 0.0, 0.0, m)
    m = np.where(np.isinf(d2nd), np.inf, m)
    return m


def num_threads(lib: str = LIB_PATH) -> int:
    return int(_lib(lib).orc_num_threads())
