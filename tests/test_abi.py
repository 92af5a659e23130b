"""The C-ABI library: it loads, exports every entry point the header declares,
and rejects bad arguments on the host before touching a device (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1109_0778_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(",
                             src, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def L():
    return binding.lib()


def test_header_declares_the_binding_exports():
    assert _declared() == set(binding.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = _declared() - exported
    assert not missing, missing
    for name in _declared():
        assert hasattr(L, name)


def test_header_is_valid_c():
    for h in HEADERS:
        subprocess.run(["gcc", "-fsyntax-only", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-x", "c", h], check=True)


def _create(L, n, d, k, prec=0):
    h = ctypes.c_void_p()
    st = L.km_plan_create(n, d, k, prec, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("n,d,k", [(0, 4, 1), (-5, 4, 1), (1 << 31, 4, 2), (100, 0, 2), (100, 1025, 2),
                                   (100, 4, 0), (100, 4, 101), (100, 4, -1)])
def test_plan_create_rejects_bad_shapes(L, n, d, k):
    st, h = _create(L, n, d, k)
    assert st == binding.KM_EINVAL
    assert not h.value
    assert L.km_last_error().decode()


def test_plan_create_rejects_unknown_precision(L):
    st, h = _create(L, 100, 4, 3, 7)
    assert st == binding.KM_EINVAL and not h.value


@pytest.mark.parametrize("n,d,k,prec", [(20000, 4, 16385, 1), (20000, 4, 16385, 2),
                                        (1 << 30, 128, 786433, 0)])   # more label chunks than the partition holds
def test_plan_create_reports_unsupported(L, n, d, k, prec):
    st, h = _create(L, n, d, k, prec)
    assert st == binding.KM_ENOTSUP and not h.value
    assert L.km_last_error().decode()


def test_null_handles(L):
    assert L.km_plan_workspace_bytes(None) == 0
    L.km_plan_destroy(None)
    assert L.km_plan_set_workspace(None, None, 0) == binding.KM_EINVAL
    assert L.kmeans_assign(None, None, None, None, None, None, None) == binding.KM_EINVAL
    assert L.kmeans_update(None, None, None, None, None, None, None) == binding.KM_EINVAL
    it = ctypes.c_int32(-7)
    assert L.kmeans_lloyd(None, None, None, None, None, None, 3, -1.0, ctypes.byref(it), None) == binding.KM_EINVAL
    assert it.value == -7  # outputs untouched on error
    assert L.km_plan_create(10, 2, 2, 0, None) == binding.KM_EINVAL


def test_valid_shape_without_device_fails_cleanly(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(L, 1000, 8, 4)
    assert st == binding.KM_EHIP and not h.value
    assert "hip" in L.km_last_error().decode().lower()
