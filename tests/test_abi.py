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
    assert set(_declared()) == set(kk.EXPORTS)


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


def test_null_handles_of_the_batch_server_and_tuner_calls_are_rejected():
    lib = kk.load()
    w, r, u = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    d = ctypes.c_double()
    n = ctypes.c_size_t()
    assert lib.kk_autotune(None, 5, ctypes.byref(w), ctypes.byref(r), ctypes.byref(u), ctypes.byref(d)) == kk.KK_EINVAL
    assert lib.kk_batch_create(None, None, 0, None) == kk.KK_EINVAL
    h = ctypes.c_void_p(1)
    assert lib.kk_batch_create(ctypes.byref(h), None, 0, None) == kk.KK_EINVAL and h.value is None
    assert lib.kk_batch_run(None) == kk.KK_EINVAL
    assert lib.kk_batch_autotune(None, 5, None, None, None) == kk.KK_EINVAL
    assert lib.kk_batch_sim(None, 0, ctypes.byref(h)) == kk.KK_EINVAL
    assert lib.kk_batch_info(None, None, None, None) == kk.KK_EINVAL
    lib.kk_batch_destroy(None)
    assert lib.kk_server_create(None, None) == kk.KK_EINVAL
    assert lib.kk_server_now(None, ctypes.byref(d)) == kk.KK_EINVAL
    rep = kk.Replica(64, 1, 0.5, 0.5, 1, 10)
    jid = ctypes.c_uint64()
    assert lib.kk_server_submit(None, ctypes.byref(rep), -1.0, ctypes.byref(jid)) == kk.KK_EINVAL
    assert lib.kk_server_step(None, ctypes.byref(n), ctypes.byref(n)) == kk.KK_EINVAL
    assert lib.kk_server_poll(None, None, 0, ctypes.byref(n)) == kk.KK_EINVAL
    assert lib.kk_server_job_hist(None, 1, None, 0, ctypes.byref(n)) == kk.KK_EINVAL
    assert lib.kk_server_job_lattice(None, 1, None, 0) == kk.KK_EINVAL
    assert lib.kk_server_release(None, 1) == kk.KK_EINVAL
    st = kk.ServerStats()
    assert lib.kk_server_get_stats(None, ctypes.byref(st)) == kk.KK_EINVAL
    lib.kk_server_destroy(None)
    assert lib.kk_last_error()


@pytest.mark.parametrize("L,H,scheme,x,w", [
    (8, 8, 0, 0.5, 0.5), (12, 6, 0, 0.5, 0.5), (0, 12, 0, 0.5, 0.5), (12, 0, 0, 0.5, 0.5),
    (11, 7, 1, 0.5, 0.5), (10, 8, 1, 0.5, 0.5), (14, 14, 1, 0.5, 0.5), (10, 7, 2, 0.5, 0.5),
    (12, 12, 0, -0.5, 0.5), (10, 7, 1, 0.5, float("nan")), (65540, 4, 0, 0.5, 0.5), (65532, 65532, 0, 0.5, 0.5),
])
def test_triangular_create_rejects_invalid_arguments(L, H, scheme, x, w):
    # shapes outside the 16-class schedule (L % 8 == 4, H % 4 == 0) or the 7-site cover
    # (L % 7 in {3, 5}, H % 7 == 0), unknown schemes, bad compositions, omegas and sizes
    lib = kk.load()
    h = ctypes.c_void_p(1)
    st = lib.kk_create_triangular_ex(ctypes.byref(h), L, H, scheme, x, w, 1, None)
    assert st == kk.KK_EINVAL
    assert h.value is None
    assert lib.kk_last_error()
    if H == L and scheme == 0:
        assert lib.kk_create_triangular(ctypes.byref(h), L, x, w, 1, None) == kk.KK_EINVAL


def test_null_handles_of_the_geometry_calls_are_rejected():
    lib = kk.load()
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    T = (ctypes.c_uint64 * 11)()
    assert lib.kk_shape(None, ctypes.byref(a), ctypes.byref(b)) == kk.KK_EINVAL
    assert lib.kk_geometry(None, ctypes.byref(a)) == kk.KK_EINVAL
    assert lib.kk_tri_thresholds(None, T) == kk.KK_EINVAL
    assert lib.kk_tri_set_tile(None, 64, 64) == kk.KK_EINVAL
    assert lib.kk_tri_get_tile(None, ctypes.byref(a), ctypes.byref(b)) == kk.KK_EINVAL
    assert lib.kk_restart(None, 0) == kk.KK_EINVAL
    assert lib.kk_create_triangular_ex(None, 12, 12, 0, 0.5, 0.5, 1, None) == kk.KK_EINVAL


def test_borrowed_batch_handles_describe_a_square_lattice():
    b = kk._Borrowed(None, 64, 0.5, 1)
    assert (b.L, b.H, b.geometry) == (64, 64, "square")


def test_header_compiles_as_c99(tmp_path):
    # the boundary is a C ABI: the header must stand alone in a C translation unit
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_kk.c"
    src.write_text('#include "kk.h"\n'
                   "int use(kk_sim *h, kk_tri_batch *b) {\n"
                   "    kk_observables o; kk_tri_replica r; kk_replica q; (void)r; (void)q;\n"
                   "    if (kk_tri_batch_run(b) != KK_OK) return 1;\n"
                   "    return kk_observe(h, 1, &o) == KK_OK ? (int)KK_TRI_MPKK : (int)KK_START_SEGREGATED;\n"
                   "}\n")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"), "-c",
                    str(src), "-o", str(tmp_path / "use_kk.o")], check=True)


def _job_bytes(L, layout, keep):
    lib = kk.load()
    r = kk.Replica(L, layout, 0.5, 0.5, 1, 10, 0)
    out = ctypes.c_uint64()
    st = lib.kk_server_job_bytes(ctypes.byref(r), keep, ctypes.byref(out))
    assert st == kk.KK_OK, lib.kk_last_error()
    return out.value


@pytest.mark.parametrize("L", [128, 256, 1024, 2048, 32768])
def test_server_job_charge_bounds_every_phase(L):
    # The server admits a job by its charge, so the charge must cover the most
    # a job's handle holds at once: its two lattice buffers plus either the
    # placement keys (8 B per site) or, while it retires, the labelling arrays
    # (8 B per site) and, when a bit-packed lattice is copied out, the
    # one-byte-per-site unpack buffer beside them.
    N = L * L
    bits = _job_bytes(L, kk.LAYOUT_BITPACKED, 0)
    bits_keep = _job_bytes(L, kk.LAYOUT_BITPACKED, 1)
    assert bits >= 2 * (N // 8) + 8 * N
    assert bits_keep >= 2 * (N // 8) + 8 * N + N
    assert 0 < bits_keep - bits <= N
    i8 = _job_bytes(L, kk.LAYOUT_INT8, 0)
    assert i8 == _job_bytes(L, kk.LAYOUT_INT8, 1) >= 2 * N + 8 * N
    assert _job_bytes(L, kk.LAYOUT_AUTO, 1) == bits_keep   # L % 32 == 0: auto is bit-packed
    # small tables only on top
    assert bits_keep < 2 * (N // 8) + 9 * N + 4 * (N // 4096 + 1) + (1 << 20)


def test_server_job_charge_rejects_invalid_jobs():
    lib = kk.load()
    out = ctypes.c_uint64()
    for L, layout in ((0, 0), (6, 1), (100, 2), (64, 5), (32772, 1)):
        r = kk.Replica(L, layout, 0.5, 0.5, 1, 10, 0)
        assert lib.kk_server_job_bytes(ctypes.byref(r), 0, ctypes.byref(out)) == kk.KK_EINVAL
    assert lib.kk_server_job_bytes(None, 0, ctypes.byref(out)) == kk.KK_EINVAL
