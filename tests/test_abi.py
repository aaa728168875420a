"""CPU-side checks of the C ABI: the library loads, exports every function
include/kk.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1309_4349_amd import kk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:kk_status|void|const char \*)\s*\*?\s*(kk_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("kk_create", "kk_sweep", "kk_energy", "kk_cluster_hist"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = kk.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) <= set(kk.EXPORTS) | {n for n in _declared() if n.startswith("kk_batch") or n.startswith("kk_serve")}


@pytest.mark.parametrize("L,x,w,layout", [
    (0, 0.5, 0.5, 0), (6, 0.5, 0.5, 0), (3, 0.5, 0.5, 0), (64, -0.1, 0.5, 0), (64, 1.5, 0.5, 0),
    (64, 0.5, float("nan"), 0), (64, 0.5, float("inf"), 0), (100, 0.5, 0.5, 2), (64, 0.5, 0.5, 7),
    (65540, 0.5, 0.5, 0), (32772, 0.5, 0.5, 0),
])
def test_create_rejects_invalid_arguments(L, x, w, layout):
    lib = kk.load()
    h = ctypes.c_void_p(1)
    st = lib.kk_create_ex(ctypes.byref(h), L, x, w, 1, layout, None)
    assert st == kk.KK_EINVAL
    assert h.value is None
    assert lib.kk_last_error()


def test_null_handle_calls_are_rejected():
    lib = kk.load()
    assert lib.kk_sweep(None, 1) == kk.KK_EINVAL
    assert lib.kk_energy(None, None, None) == kk.KK_EINVAL
    n = ctypes.c_size_t()
    assert lib.kk_cluster_hist(None, 1, None, 0, ctypes.byref(n)) == kk.KK_EINVAL
    lib.kk_destroy(None)
