"""Thin ctypes binding of ``libkmeans_mi355x.so`` (argument marshalling only).

Every function mirrors the C entry point of the same name in
``include/kmeans_mi355x.h``: tensors are passed as device pointers, the stream
is torch's current HIP stream unless one is given, and a non-OK status raises
``KMeansError`` carrying ``km_last_error()``.  PyTorch provides device memory
(tensors, the plan workspace) and streams; all arithmetic runs in the
library's kernels.  There is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmeans_mi355x.so")

KM_OK, KM_EINVAL, KM_ENOTSUP, KM_EHIP, KM_EWORKSPACE = 0, -1, -2, -3, -4
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2}

# Entry points the header declares (checked by the ABI tests).
EXPORTS = ["km_plan_create", "km_plan_workspace_bytes", "km_plan_set_workspace",
           "km_plan_destroy", "km_last_error", "kmeans_assign", "kmeans_update",
           "kmeans_lloyd", "kmeans_lloyd_static", "km_plan_enable_timing", "km_plan_kernel_times", "km_plan_recheck_count",
           "km_plan_use_graphs", "km_plan_set_validate", "km_batch_create", "km_batch_workspace_bytes", "km_batch_set_workspace",
           "km_batch_set_schedule", "km_batch_use_graphs", "km_batch_destroy", "kmeans_lloyd_batched",
           "spade_workspace_bytes", "spade_densities", "spade_stats", "km_class_sums", "nb_train",
           "gda_workspace_bytes", "gda_train", "kmeans_assign_metric", "km_batch_num_classes",
           "km_batch_class_info", "km_batch_set_class_schedule", "km_batch_use_persistent",
           "km_batch_persistent_status"]
LAYOUTS = {"row": 0, "feature": 1}
METRICS = {"l1": 0, "sqeuclidean": 1}


class KmInstance(ctypes.Structure):
    """km_instance of the C header."""
    _fields_ = [("X", ctypes.c_void_p), ("C", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("obj_hist", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("d", ctypes.c_int32), ("k", ctypes.c_int32)]


class KMeansError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1109_0778_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, F64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.km_plan_create.restype = I32
        L.km_plan_create.argtypes = [I64, I32, I32, I32, ctypes.POINTER(P)]
        L.km_plan_workspace_bytes.restype = ctypes.c_size_t
        L.km_plan_workspace_bytes.argtypes = [P]
        L.km_plan_set_workspace.restype = I32
        L.km_plan_set_workspace.argtypes = [P, P, ctypes.c_size_t]
        L.km_plan_destroy.restype = None
        L.km_plan_destroy.argtypes = [P]
        L.km_last_error.restype = ctypes.c_char_p
        L.km_last_error.argtypes = []
        L.kmeans_assign.restype = I32
        L.kmeans_assign.argtypes = [P, P, P, P, P, P, P]
        L.kmeans_update.restype = I32
        L.kmeans_update.argtypes = [P, P, P, P, P, P, P]
        L.kmeans_lloyd.restype = I32
        L.kmeans_lloyd.argtypes = [P, P, P, P, P, P, I32, F64, ctypes.POINTER(I32), P]
        L.kmeans_lloyd_static.restype = I32
        L.kmeans_lloyd_static.argtypes = [P, P, P, P, P, P, I32, F64, ctypes.POINTER(I32), P]
        L.km_plan_enable_timing.restype = I32
        L.km_plan_enable_timing.argtypes = [P, I32]
        L.km_plan_kernel_times.restype = I32
        L.km_plan_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_float), I32, ctypes.POINTER(I32)]
        L.km_batch_create.restype = I32
        L.km_batch_create.argtypes = [ctypes.POINTER(KmInstance), I32, I32, ctypes.POINTER(P)]
        L.km_batch_workspace_bytes.restype = ctypes.c_size_t
        L.km_batch_workspace_bytes.argtypes = [P]
        L.km_batch_set_workspace.restype = I32
        L.km_batch_set_workspace.argtypes = [P, P, ctypes.c_size_t]
        L.km_batch_set_schedule.restype = I32
        L.km_batch_set_schedule.argtypes = [P, I32, I32]
        L.km_batch_use_graphs.restype = I32
        L.km_batch_use_graphs.argtypes = [P, I32]
        L.km_batch_destroy.restype = None
        L.km_batch_destroy.argtypes = [P]
        L.kmeans_lloyd_batched.restype = I32
        L.kmeans_lloyd_batched.argtypes = [P, I32, P]
        L.km_plan_use_graphs.restype = I32
        L.km_plan_use_graphs.argtypes = [P, I32]
        L.km_plan_set_validate.restype = I32
        L.km_plan_set_validate.argtypes = [P, I32]
        L.km_plan_recheck_count.restype = I32
        L.km_plan_recheck_count.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), P]
        L.spade_workspace_bytes.restype = ctypes.c_size_t
        L.spade_workspace_bytes.argtypes = [I64, I32]
        L.spade_densities.restype = I32
        L.spade_densities.argtypes = [P, I64, I32, F64, F64, I32, P, P, ctypes.POINTER(I64), P, ctypes.c_size_t, P]
        L.spade_stats.restype = I32
        L.spade_stats.argtypes = [P, I64, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), P]
        L.km_class_sums.restype = I32
        L.km_class_sums.argtypes = [P, P, P, P, P, P]
        L.nb_train.restype = I32
        L.nb_train.argtypes = [P, P, P, P, P, P]
        L.gda_workspace_bytes.restype = ctypes.c_size_t
        L.gda_workspace_bytes.argtypes = [P]
        L.gda_train.restype = I32
        L.gda_train.argtypes = [P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.km_batch_num_classes.restype = I32
        L.km_batch_num_classes.argtypes = [P]
        L.km_batch_class_info.restype = I32
        L.km_batch_class_info.argtypes = [P, I32] + [ctypes.POINTER(I32)] * 4
        L.km_batch_set_class_schedule.restype = I32
        L.km_batch_set_class_schedule.argtypes = [P, I32, I32]
        L.km_batch_use_persistent.restype = I32
        L.km_batch_use_persistent.argtypes = [P, I32]
        L.km_batch_persistent_status.restype = I32
        L.km_batch_persistent_status.argtypes = [P, ctypes.POINTER(I32)]
        L.kmeans_assign_metric.restype = I32
        L.kmeans_assign_metric.argtypes = [P, P, I32, I32, P, P, P, P, P]
        _lib = L
    return _lib


def _check(status: int):
    if status != KM_OK:
        raise KMeansError(status, lib().km_last_error().decode())


def _ptr(t, dtype, what, numel=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


class Plan:
    """km_plan plus a workspace tensor it owns (allocated by torch)."""

    def __init__(self, n: int, d: int, k: int, precision: str = "fp32", device=None,
                 bind_workspace: bool = True):
        import torch
        self.n, self.d, self.k, self.precision = int(n), int(d), int(k), precision
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        with torch.cuda.device(dev):
            h = ctypes.c_void_p()
            _check(lib().km_plan_create(self.n, self.d, self.k, PRECISIONS[precision], ctypes.byref(h)))
            self._h = h
            self.workspace = None
            if not bind_workspace:
                return
            nbytes = int(lib().km_plan_workspace_bytes(h))
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            off = (-raw.data_ptr()) % 256
            self.workspace = raw[off:off + nbytes]
            _check(lib().km_plan_set_workspace(h, self.workspace.data_ptr(), nbytes))

    @property
    def handle(self):
        return self._h

    @property
    def workspace_bytes(self) -> int:
        return int(lib().km_plan_workspace_bytes(self._h))

    def use_graphs(self, enable: bool = True):
        """km_plan_use_graphs: capture kmeans_lloyd calls into HIP graphs."""
        _check(lib().km_plan_use_graphs(self._h, int(bool(enable))))

    def set_validate(self, enable: bool = True):
        """km_plan_set_validate: kmeans_update rejects labels outside [0, k)."""
        _check(lib().km_plan_set_validate(self._h, int(bool(enable))))

    def rebind_workspace(self):
        """Allocate a fresh workspace tensor and bind it (km_plan_set_workspace)."""
        import torch
        nbytes = self.workspace_bytes
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes]
        _check(lib().km_plan_set_workspace(self._h, self.workspace.data_ptr(), nbytes))

    def enable_timing(self, cap: int):
        """km_plan_enable_timing: time up to ``cap`` launches of the per-sample pass."""
        _check(lib().km_plan_enable_timing(self._h, int(cap)))

    def kernel_times(self, cap: int = 4096):
        """km_plan_kernel_times: per-launch durations (ms) recorded so far."""
        buf = (ctypes.c_float * cap)()
        cnt = ctypes.c_int32(0)
        _check(lib().km_plan_kernel_times(self._h, buf, cap, ctypes.byref(cnt)))
        return [float(buf[i]) for i in range(min(cap, cnt.value))]

    def recheck_count(self, stream=None):
        """km_plan_recheck_count: (samples the last mixed-precision assign queued for the
        exact recheck, how many of them were full scans)."""
        v = ctypes.c_int64(0)
        f = ctypes.c_int64(0)
        _check(lib().km_plan_recheck_count(self._h, ctypes.byref(v), ctypes.byref(f), _stream(stream)))
        return int(v.value), int(f.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().km_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kmeans_assign(plan: Plan, X, C, labels, mindist=None, objective=None, stream=None):
    import torch
    n, d, k = plan.n, plan.d, plan.k
    _check(lib().kmeans_assign(
        plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(C, torch.float32, "C", k * d),
        _ptr(labels, torch.int32, "labels", n), _ptr(mindist, torch.float32, "mindist", n),
        _ptr(objective, torch.float64, "objective", 1), _stream(stream)))


def kmeans_update(plan: Plan, X, labels, C_old, C_new, counts=None, stream=None):
    import torch
    n, d, k = plan.n, plan.d, plan.k
    _check(lib().kmeans_update(
        plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(labels, torch.int32, "labels", n),
        _ptr(C_old, torch.float32, "C_old", k * d), _ptr(C_new, torch.float32, "C_new", k * d),
        _ptr(counts, torch.int64, "counts", k), _stream(stream)))


def kmeans_lloyd(plan: Plan, X, C, labels, counts=None, obj_hist=None, max_iter: int = 1,
                 tol: float = -1.0, stream=None) -> int:
    """Runs Lloyd iterations in place on C; returns iters_done."""
    import torch
    n, d, k = plan.n, plan.d, plan.k
    if obj_hist is not None and obj_hist.numel() < max_iter:
        raise ValueError("obj_hist needs max_iter entries")
    it = ctypes.c_int32(0)
    _check(lib().kmeans_lloyd(
        plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(C, torch.float32, "C", k * d),
        _ptr(labels, torch.int32, "labels", n), _ptr(counts, torch.int64, "counts", k),
        _ptr(obj_hist, torch.float64, "obj_hist"), int(max_iter), float(tol), ctypes.byref(it),
        _stream(stream)))
    return int(it.value)


def kmeans_lloyd_static(plan: Plan, X, C, labels, counts=None, obj_hist=None, max_iter: int = 1,
                        tol: float = -1.0, stream=None) -> int:
    """kmeans_lloyd on the library's static scratch (no workspace); returns iters_done."""
    import torch
    n, d, k = plan.n, plan.d, plan.k
    if obj_hist is not None and obj_hist.numel() < max_iter:
        raise ValueError("obj_hist needs max_iter entries")
    it = ctypes.c_int32(0)
    _check(lib().kmeans_lloyd_static(
        plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(C, torch.float32, "C", k * d),
        _ptr(labels, torch.int32, "labels", n), _ptr(counts, torch.int64, "counts", k),
        _ptr(obj_hist, torch.float64, "obj_hist"), int(max_iter), float(tol), ctypes.byref(it),
        _stream(stream)))
    return int(it.value)


STATIC_SCRATCH_BYTES = 64 << 20   # KM_STATIC_SCRATCH_BYTES


class Batch:
    """km_batch over a list of instances, each a dict of tensors X (n x d,
    FP32), C (k x d, FP32, updated in place), labels (n, int32) and optional
    counts (k, int64) and obj_hist (>= iterations, FP64); plus a workspace
    tensor the batch owns."""

    def __init__(self, instances, precision: str = "fp32", device=None):
        import torch
        self.instances = instances
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        arr = (KmInstance * len(instances))()
        for i, t in enumerate(instances):
            X, C = t["X"], t["C"]
            n, d = X.shape
            k = C.shape[0]
            arr[i] = KmInstance(_ptr(X, torch.float32, "X"), _ptr(C, torch.float32, "C", k * d),
                                _ptr(t["labels"], torch.int32, "labels", n),
                                _ptr(t.get("counts"), torch.int64, "counts", k),
                                _ptr(t.get("obj_hist"), torch.float64, "obj_hist"), n, d, k)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().km_batch_create(arr, len(instances), PRECISIONS[precision], ctypes.byref(h)))
        self._h = h
        self._bind()

    def _bind(self):
        import torch
        nbytes = int(lib().km_batch_workspace_bytes(self._h))
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes]
        _check(lib().km_batch_set_workspace(self._h, self.workspace.data_ptr(), nbytes))

    @property
    def handle(self):
        return self._h

    def set_schedule(self, tiles_per_block: int, order: int):
        """km_batch_set_schedule, then a workspace of the new size is bound."""
        _check(lib().km_batch_set_schedule(self._h, int(tiles_per_block), int(order)))
        self._bind()

    def use_graphs(self, enable: bool = True):
        _check(lib().km_batch_use_graphs(self._h, int(bool(enable))))

    def use_persistent(self, enable: bool = True):
        """km_batch_use_persistent, then a workspace of the new size is bound."""
        _check(lib().km_batch_use_persistent(self._h, int(bool(enable))))
        self._bind()

    def persistent_aborted(self) -> bool:
        """km_batch_persistent_status (synchronous): whether a wait of the last
        persistent launch exceeded its bound."""
        v = ctypes.c_int32(0)
        _check(lib().km_batch_persistent_status(self._h, ctypes.byref(v)))
        return bool(v.value)

    def classes(self):
        """[(d8, lds_bytes, instances, tiles_per_block)] of the shape classes."""
        out = []
        for c in range(int(lib().km_batch_num_classes(self._h))):
            v = [ctypes.c_int32(0) for _ in range(4)]
            _check(lib().km_batch_class_info(self._h, c, *[ctypes.byref(x) for x in v]))
            out.append(tuple(int(x.value) for x in v))
        return out

    def set_class_schedule(self, cls: int, tiles_per_block: int):
        """km_batch_set_class_schedule, then a workspace of the new size is bound."""
        _check(lib().km_batch_set_class_schedule(self._h, int(cls), int(tiles_per_block)))
        self._bind()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().km_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kmeans_lloyd_batched(batch: Batch, iterations: int, stream=None):
    for t in batch.instances:
        h = t.get("obj_hist")
        if h is not None and h.numel() < iterations:
            raise ValueError("obj_hist needs one entry per iteration")
    _check(lib().kmeans_lloyd_batched(batch.handle, int(iterations), _stream(stream)))


def _workspace(nbytes, device):
    import torch
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


def spade_densities(X, apprx_width: float, kernel_width: float, metric: str = "l1", densities=None,
                    visited=None, workspace=None, stream=None):
    """spade_densities: returns (densities, visited_count, workspace); the
    workspace is allocated here when not given."""
    import torch
    n, d = X.shape
    if densities is None:
        densities = torch.empty(n, dtype=torch.int32, device=X.device)
    nbytes = int(lib().spade_workspace_bytes(n, d))
    if nbytes == 0:
        raise KMeansError(KM_EINVAL, f"bad shape n={n}, d={d}")
    if workspace is None:
        workspace = _workspace(nbytes, X.device)
    cnt = ctypes.c_int64(0)
    _check(lib().spade_densities(_ptr(X, torch.float32, "X", n * d), n, d, float(apprx_width),
                                 float(kernel_width), METRICS[metric], _ptr(densities, torch.int32, "densities", n),
                                 _ptr(visited, torch.int8, "visited", n), ctypes.byref(cnt),
                                 workspace.data_ptr(), workspace.numel(), _stream(stream)))
    return densities, int(cnt.value), workspace


def spade_stats(workspace, n: int, d: int, stream=None):
    """spade_stats: (batches, candidate rows formed) of the last call on ``workspace``."""
    b = ctypes.c_int64(0)
    c = ctypes.c_int64(0)
    _check(lib().spade_stats(workspace.data_ptr(), n, d, ctypes.byref(b), ctypes.byref(c), _stream(stream)))
    return int(b.value), int(c.value)


def km_class_sums(plan: Plan, X, labels, S, counts=None, stream=None):
    import torch
    n, d, k = plan.n, plan.d, plan.k
    _check(lib().km_class_sums(plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(labels, torch.int32, "labels", n),
                               _ptr(S, torch.float64, "S", k * d), _ptr(counts, torch.int64, "counts", k),
                               _stream(stream)))


def nb_train(plan: Plan, X, labels, prior, phi, stream=None):
    import torch
    n, d, k = plan.n, plan.d, plan.k
    _check(lib().nb_train(plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(labels, torch.int32, "labels", n),
                          _ptr(prior, torch.float64, "prior", k), _ptr(phi, torch.float64, "phi", k * d),
                          _stream(stream)))


def gda_train(plan: Plan, X, labels, prior, mu, sigma, workspace=None, stream=None):
    """gda_train; returns the GDA workspace (allocated here when not given)."""
    import torch
    n, d, k = plan.n, plan.d, plan.k
    nbytes = int(lib().gda_workspace_bytes(plan.handle))
    if workspace is None:
        workspace = _workspace(nbytes, X.device)
    _check(lib().gda_train(plan.handle, _ptr(X, torch.float32, "X", n * d), _ptr(labels, torch.int32, "labels", n),
                           _ptr(prior, torch.float64, "prior", k), _ptr(mu, torch.float64, "mu", k * d),
                           _ptr(sigma, torch.float64, "sigma", d * d), workspace.data_ptr(), workspace.numel(),
                           _stream(stream)))
    return workspace


def kmeans_assign_metric(plan: Plan, X, C, labels, metric: str = "l1", layout: str = "row", mindist=None,
                         objective=None, stream=None):
    """kmeans_assign_metric; X is n x d (layout "row") or d x n ("feature")."""
    import torch
    n, d, k = plan.n, plan.d, plan.k
    _check(lib().kmeans_assign_metric(
        plan.handle, _ptr(X, torch.float32, "X", n * d), LAYOUTS[layout], METRICS[metric],
        _ptr(C, torch.float32, "C", k * d), _ptr(labels, torch.int32, "labels", n),
        _ptr(mindist, torch.float32, "mindist", n), _ptr(objective, torch.float64, "objective", 1),
        _stream(stream)))
