"""ctypes front end of ``ml_oracle.c`` -- test infrastructure.

FP64 oracles of the applications that reuse the k-means building blocks:
SPADE's density step (paper section 4.1), nearest centroid under L1 or
squared Euclidean distance, per-class sums, multinomial naive Bayes and
Gaussian discriminant analysis training (the section 4.2 applications).
Every function takes FP32 samples (widened exactly inside) and returns FP64
results; see ``ml_oracle.c`` for the definition each follows.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .oracle import build as _build_c

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(_HERE, "ml_oracle.c")
LIB_PATH = os.path.join(_HERE, "libml_oracle.so")

METRICS = {"l1": 0, "sqeuclidean": 1}


def build(src: str = SRC_PATH, out: str = LIB_PATH) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    return _build_c(src, out)


_LIB = {}


def _lib(path: str = LIB_PATH):
    if path not in _LIB:
        if path == LIB_PATH and (not os.path.exists(path)
                                 or os.path.getmtime(path) < os.path.getmtime(SRC_PATH)):
            build()
        lib = ctypes.CDLL(path)
        P, I64, I32, F64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.orc_spade_densities.restype = I64
        lib.orc_spade_densities.argtypes = [P, I64, I32, F64, F64, I32, P, P]
        lib.orc_assign_metric.restype = None
        lib.orc_assign_metric.argtypes = [P, P, I64, I32, I32, I32, P, P, P]
        lib.orc_class_sums.restype = I32
        lib.orc_class_sums.argtypes = [P, P, I64, I32, I32, P, P]
        lib.orc_nb_train.restype = I32
        lib.orc_nb_train.argtypes = [P, P, I64, I32, I32, P, P]
        lib.orc_gda_train.restype = I32
        lib.orc_gda_train.argtypes = [P, P, I64, I32, I32, P, P, P]
        _LIB[path] = lib
    return _LIB[path]


def _f32(a):
    a = np.ascontiguousarray(a)
    if a.dtype != np.float32 or a.ndim != 2:
        raise TypeError("samples must be a 2-D FP32 array")
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def spade_densities(X, apprx_width: float, kernel_width: float, metric: str = "l1", lib: str = LIB_PATH):
    """SPADE densities (int32) and the processed-row mask (bool)."""
    X = _f32(X)
    n, d = X.shape
    dens = np.empty(n, np.int32)
    proc = np.empty(n, np.int8)
    r = _lib(lib).orc_spade_densities(_p(X), n, d, float(apprx_width), float(kernel_width),
                                      METRICS[metric], _p(dens), _p(proc))
    if r < 0:
        raise MemoryError("orc_spade_densities failed")
    return dens, proc.astype(bool)


def assign_metric(X, C, metric: str = "l1", lib: str = LIB_PATH):
    """Labels, nearest and second-nearest distances (FP64) under ``metric``."""
    X = _f32(X)
    C = np.ascontiguousarray(C, dtype=np.float64)
    n, d = X.shape
    k = C.shape[0]
    lab = np.empty(n, np.int32)
    d1 = np.empty(n, np.float64)
    d2 = np.empty(n, np.float64)
    _lib(lib).orc_assign_metric(_p(X), _p(C), n, d, k, METRICS[metric], _p(lab), _p(d1), _p(d2))
    return lab, d1, d2


def class_sums(X, y, C: int, lib: str = LIB_PATH):
    X = _f32(X)
    y = _i32(y)
    n, d = X.shape
    S = np.empty((C, d), np.float64)
    cnt = np.empty(C, np.int64)
    if _lib(lib).orc_class_sums(_p(X), _p(y), n, d, C, _p(S), _p(cnt)) != 0:
        raise ValueError("label outside [0, C)")
    return S, cnt


def nb_train(X, y, C: int, lib: str = LIB_PATH):
    """Multinomial naive Bayes: (prior[C], phi[C, d]) in FP64."""
    X = _f32(X)
    y = _i32(y)
    n, d = X.shape
    prior = np.empty(C, np.float64)
    phi = np.empty((C, d), np.float64)
    if _lib(lib).orc_nb_train(_p(X), _p(y), n, d, C, _p(prior), _p(phi)) != 0:
        raise ValueError("label outside [0, C)")
    return prior, phi


def gda_train(X, y, C: int, lib: str = LIB_PATH):
    """GDA: (prior[C], mu[C, d], sigma[d, d]) in FP64."""
    X = _f32(X)
    y = _i32(y)
    n, d = X.shape
    prior = np.empty(C, np.float64)
    mu = np.empty((C, d), np.float64)
    sigma = np.empty((d, d), np.float64)
    if _lib(lib).orc_gda_train(_p(X), _p(y), n, d, C, _p(prior), _p(mu), _p(sigma)) != 0:
        raise ValueError("label outside [0, C)")
    return prior, mu, sigma
