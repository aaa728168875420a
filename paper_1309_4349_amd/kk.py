"""Thin ctypes binding of libkk (include/kk.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libkk.so.  Loading fails loudly when the library has not been
built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkk.so")

KK_OK, KK_EINVAL, KK_ENOMEM, KK_EDEVICE, KK_ESTATE, KK_ETRUNC = range(6)
LAYOUT_AUTO, LAYOUT_INT8, LAYOUT_BITPACKED = 0, 1, 2
_LAYOUTS = {"auto": LAYOUT_AUTO, "int8": LAYOUT_INT8, "bitpacked": LAYOUT_BITPACKED}
START_RANDOM, START_SEGREGATED = 0, 1
TRI_CLASSES, TRI_MPKK = 0, 1
_SCHEMES = {"classes": TRI_CLASSES, "mpkk": TRI_MPKK}
_STARTS = {"random": START_RANDOM, "segregated": START_SEGREGATED}

EXPORTS = [
    "kk_create", "kk_create_ex", "kk_create_triangular", "kk_create_triangular_ex", "kk_shape", "kk_tri_thresholds",
    "kk_tri_set_tile", "kk_tri_get_tile", "kk_tri_autotune",
    "kk_geometry", "kk_restart", "kk_sweep", "kk_sweep_async", "kk_sync", "kk_energy", "kk_cluster_hist",
    "kk_get_lattice", "kk_set_lattice", "kk_observe", "kk_sweep_series", "kk_stats", "kk_thresholds", "kk_info",
    "kk_set_tile", "kk_get_tile", "kk_autotune",
    "kk_stream", "kk_sweep_timed", "kk_destroy", "kk_last_error",
    "kk_batch_create", "kk_batch_run", "kk_batch_sim", "kk_batch_info", "kk_batch_autotune", "kk_batch_destroy",
    "kk_batch_cluster_hists", "kk_batch_set_tile",
    "kk_tri_batch_create", "kk_tri_batch_run", "kk_tri_batch_sim", "kk_tri_batch_info", "kk_tri_batch_destroy",
    "kk_server_create", "kk_server_now", "kk_server_submit", "kk_server_step", "kk_server_poll",
    "kk_server_job_hist", "kk_server_job_lattice", "kk_server_release", "kk_server_get_stats",
    "kk_server_destroy", "kk_server_job_bytes", "kk_sweep_noalloc", "kk_valu_issue_cycles",
]


class KKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libkk status {status}: {msg}")
        self.status = status


class HistEntry(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint64), ("count", ctypes.c_uint64)]


class Observables(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_uint64), ("n_unlike", ctypes.c_uint64), ("energy_kT", ctypes.c_double),
                ("similar_exact", ctypes.c_double), ("similar_sampled", ctypes.c_double),
                ("n_clusters", ctypes.c_uint64), ("size_number_avg", ctypes.c_double),
                ("size_weight_avg", ctypes.c_double), ("size_max", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Replica(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("layout", ctypes.c_uint32), ("composition", ctypes.c_double),
                ("omega_kT", ctypes.c_double), ("seed", ctypes.c_uint64), ("sweeps", ctypes.c_uint64),
                ("start", ctypes.c_uint32)]


class TriReplica(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("H", ctypes.c_uint32), ("scheme", ctypes.c_uint32),
                ("start", ctypes.c_uint32), ("composition", ctypes.c_double), ("omega_kT", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("sweeps", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("keep_lattice", ctypes.c_uint32), ("chunk_sweeps", ctypes.c_uint64),
                ("hip_stream", ctypes.c_void_p)]


class JobResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("L", ctypes.c_uint32),
                ("sweeps", ctypes.c_uint64), ("attempts", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("n_unlike", ctypes.c_uint64), ("energy_kT", ctypes.c_double),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("hist_entries", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "steps", "queued", "active",
                                               "bytes_in_use", "peak_bytes", "budget", "attempts")] + \
               [("gpu_busy_s", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libkk.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with __graft_entry__.build() "
                                "or python paper_1309_4349_amd/build.py")
    lib = ctypes.CDLL(path)
    P, U32, U64, D, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    szp = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "kk_create": [PP, U32, D, D, U64],
        "kk_create_ex": [PP, U32, D, D, U64, U32, P],
        "kk_create_triangular": [PP, U32, D, D, U64, P],
        "kk_create_triangular_ex": [PP, U32, U32, U32, D, D, U64, P],
        "kk_shape": [P, u32p, u32p],
        "kk_tri_set_tile": [P, U32, U32],
        "kk_tri_get_tile": [P, u32p, u32p],
        "kk_tri_autotune": [P, U32, u32p, u32p, dp],
        "kk_tri_thresholds": [P, u64p],
        "kk_geometry": [P, u32p],
        "kk_restart": [P, U32],
        "kk_sweep": [P, U64],
        "kk_sweep_async": [P, U64],
        "kk_sync": [P],
        "kk_energy": [P, u64p, dp],
        "kk_cluster_hist": [P, I, ctypes.POINTER(HistEntry), ctypes.c_size_t, szp],
        "kk_get_lattice": [P, P, ctypes.c_size_t],
        "kk_observe": [P, I, ctypes.POINTER(Observables)],
        "kk_sweep_series": [P, U64, U64, I, ctypes.POINTER(Observables)],
        "kk_set_lattice": [P, P, ctypes.c_size_t, U64],
        "kk_stats": [P, u64p, u64p, u64p],
        "kk_thresholds": [P, u64p],
        "kk_info": [P, u32p, u32p],
        "kk_set_tile": [P, U32, U32, U32],
        "kk_get_tile": [P, u32p, u32p, u32p],
        "kk_autotune": [P, U32, u32p, u32p, u32p, dp],
        "kk_stream": [P, PP],
        "kk_sweep_timed": [P, U64, dp, u64p],
        "kk_batch_create": [PP, ctypes.POINTER(Replica), ctypes.c_size_t, P],
        "kk_batch_run": [P],
        "kk_batch_sim": [P, ctypes.c_size_t, PP],
        "kk_batch_cluster_hists": [P, ctypes.c_int],
        "kk_batch_set_tile": [P, U32, U32, U32],
        "kk_batch_info": [P, szp, szp, szp],
        "kk_batch_autotune": [P, U32, u32p, u32p, dp],
        "kk_tri_batch_create": [PP, ctypes.POINTER(TriReplica), ctypes.c_size_t, P],
        "kk_tri_batch_run": [P],
        "kk_tri_batch_sim": [P, ctypes.c_size_t, PP],
        "kk_tri_batch_info": [P, szp, szp, szp, szp],
        "kk_server_create": [PP, ctypes.POINTER(ServerConfig)],
        "kk_server_now": [P, dp],
        "kk_server_submit": [P, ctypes.POINTER(Replica), D, u64p],
        "kk_server_step": [P, szp, szp],
        "kk_server_poll": [P, ctypes.POINTER(JobResult), ctypes.c_size_t, szp],
        "kk_server_job_hist": [P, U64, ctypes.POINTER(HistEntry), ctypes.c_size_t, szp],
        "kk_server_job_lattice": [P, U64, P, ctypes.c_size_t],
        "kk_server_release": [P, U64],
        "kk_server_get_stats": [P, ctypes.POINTER(ServerStats)],
        "kk_sweep_noalloc": [P, U32, U32, D, U64, U64, U64, P, P],
        "kk_server_job_bytes": [ctypes.POINTER(Replica), U32, u64p],
        "kk_valu_issue_cycles": [dp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.kk_destroy.argtypes = [P]
    lib.kk_destroy.restype = None
    lib.kk_batch_destroy.argtypes = [P]
    lib.kk_batch_destroy.restype = None
    lib.kk_tri_batch_destroy.argtypes = [P]
    lib.kk_tri_batch_destroy.restype = None
    lib.kk_server_destroy.argtypes = [P]
    lib.kk_server_destroy.restype = None
    lib.kk_last_error.argtypes = []
    lib.kk_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int):
    if st != KK_OK:
        raise KKError(st, load().kk_last_error().decode(errors="replace"))


def sweep_noalloc(lattice_ptr: int, L: int, layout: str, omega: float, seed: int, t0: int, n: int,
                  accepted_ptr: int = 0, stream: int = 0):
    """kk_sweep_noalloc: n sweeps of a caller-held device lattice (device pointers as ints),
    enqueued on `stream` without waiting; adds the accepted count into *accepted_ptr."""
    _check(load().kk_sweep_noalloc(ctypes.c_void_p(lattice_ptr), L, _LAYOUTS[layout], float(omega),
                                   seed & (2**64 - 1), t0, n, ctypes.c_void_p(accepted_ptr or None),
                                   ctypes.c_void_p(stream or None)))


class Sim:
    """One lattice simulation owned by libkk (device memory and stream).

    geometry "square": the L x L torus (L % 4 == 0); "triangular": the paper's
    six-neighbour lattice with helical boundaries, `rows` rows of L sites
    (default L), int8, swept by scheme "classes" (the conflict-free 16-class
    schedule: L % 8 == 4, rows % 4 == 0) or "mpkk" (the paper's literal
    7-domain MPKK, a comparison variant: L % 7 in {3, 5}, rows % 7 == 0)."""

    def __init__(self, L: int, composition: float, omega: float, seed: int, layout: str = "auto",
                 stream: Optional[int] = None, geometry: str = "square", rows: Optional[int] = None,
                 scheme: str = "classes"):
        lib = load()
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream else None
        if geometry == "square":
            _check(lib.kk_create_ex(ctypes.byref(h), L, float(composition), float(omega), seed & (2**64 - 1),
                                    _LAYOUTS[layout], st))
        elif geometry == "triangular":
            if layout not in ("auto", "int8"):
                raise ValueError("the triangular lattice is stored one byte per site")
            _check(lib.kk_create_triangular_ex(ctypes.byref(h), L, rows or L, _SCHEMES[scheme], float(composition),
                                               float(omega), seed & (2**64 - 1), st))
        else:
            raise ValueError(f"unknown geometry {geometry!r}")
        self.geometry = geometry
        self._h = h
        self.H = (rows or L) if geometry == "triangular" else L
        self.L = L
        self.omega = float(omega)
        self.seed = seed

    def close(self):
        if getattr(self, "_h", None):
            load().kk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tri_set_tile(self, cols: int, rows: int = 0):
        """Whole-sweep tile of the triangular class schedule (cols = 0: one launch per class)."""
        _check(load().kk_tri_set_tile(self._h, cols, rows or cols))

    def tri_get_tile(self) -> Tuple[int, int]:
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().kk_tri_get_tile(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def tri_autotune(self, trial_sweeps: int = 20) -> Tuple[int, int, float]:
        """Time the triangular tiles and keep the fastest; returns (cols, rows, us_per_sweep)."""
        a, b, us = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_double()
        _check(load().kk_tri_autotune(self._h, trial_sweeps, ctypes.byref(a), ctypes.byref(b), ctypes.byref(us)))
        return a.value, b.value, us.value

    def restart(self, start: str = "random"):
        """Back to a starting lattice ("random" or "segregated"), t = 0."""
        _check(load().kk_restart(self._h, _STARTS[start]))

    # -- the path -------------------------------------------------------------
    def sweep(self, n: int):
        _check(load().kk_sweep(self._h, n))

    def sweep_async(self, n: int):
        _check(load().kk_sweep_async(self._h, n))

    def sync(self):
        _check(load().kk_sync(self._h))

    def sweep_timed(self, n: int) -> Tuple[float, int]:
        ms = ctypes.c_double()
        nl = ctypes.c_uint64()
        _check(load().kk_sweep_timed(self._h, n, ctypes.byref(ms), ctypes.byref(nl)))
        return ms.value, nl.value

    def energy(self) -> Tuple[int, float]:
        n = ctypes.c_uint64()
        e = ctypes.c_double()
        _check(load().kk_energy(self._h, ctypes.byref(n), ctypes.byref(e)))
        return n.value, e.value

    def cluster_hist(self, species: int = 1) -> List[Tuple[int, int]]:
        lib = load()
        need = ctypes.c_size_t()
        st = lib.kk_cluster_hist(self._h, species, None, 0, ctypes.byref(need))
        if st not in (KK_OK, KK_ETRUNC):
            _check(st)
        buf = (HistEntry * max(1, need.value))()
        _check(lib.kk_cluster_hist(self._h, species, buf, need.value, ctypes.byref(need)))
        return [(int(buf[i].size), int(buf[i].count)) for i in range(need.value)]

    def observe(self, species: int = 1) -> dict:
        o = Observables()
        _check(load().kk_observe(self._h, species, ctypes.byref(o)))
        return o.as_dict()

    def series(self, every: int, count: int, species: int = 1) -> List[dict]:
        buf = (Observables * max(1, count))()
        _check(load().kk_sweep_series(self._h, every, count, species, buf))
        return [buf[i].as_dict() for i in range(count)]

    def get_lattice(self) -> np.ndarray:
        out = np.empty((self.H, self.L), dtype=np.uint8)
        _check(load().kk_get_lattice(self._h, out.ctypes.data, out.size))
        return out

    def set_lattice(self, s: np.ndarray, sweep_t: int = 0):
        s = np.ascontiguousarray(s, dtype=np.uint8)
        if s.shape != (self.H, self.L):
            raise ValueError(f"lattice must be {self.H} rows of {self.L}")
        _check(load().kk_set_lattice(self._h, s.ctypes.data, s.size, sweep_t))

    def stats(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().kk_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def thresholds(self) -> np.ndarray:
        """7 entries (square) or 11 (triangular)."""
        tri = self.geometry == "triangular"
        out = np.zeros(11 if tri else 7, dtype=np.uint64)
        fn = load().kk_tri_thresholds if tri else load().kk_thresholds
        _check(fn(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out

    def info(self) -> Tuple[int, str]:
        L, lay = ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().kk_info(self._h, ctypes.byref(L), ctypes.byref(lay)))
        return L.value, {LAYOUT_INT8: "int8", LAYOUT_BITPACKED: "bitpacked"}[lay.value]

    def set_tile(self, words: int, rows: int, units_per_thread: int = 2):
        _check(load().kk_set_tile(self._h, words, rows, units_per_thread))

    def get_tile(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().kk_get_tile(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, trial_sweeps: int = 20) -> Tuple[int, int, int, float]:
        """Time the candidate tiles, keep the fastest; returns (words, rows, units_per_thread, us_per_sweep)."""
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        us = ctypes.c_double()
        _check(load().kk_autotune(self._h, trial_sweeps, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                  ctypes.byref(us)))
        return a.value, b.value, c.value, us.value

    def stream(self) -> int:
        p = ctypes.c_void_p()
        _check(load().kk_stream(self._h, ctypes.byref(p)))
        return p.value or 0


class _Borrowed(Sim):
    """A replica handle owned by a Batch or TriBatch (never destroyed from Python)."""

    def __init__(self, handle, L, omega, seed, H=None, geometry="square"):
        self._h = handle
        self.L = L
        self.H = H or L
        self.geometry = geometry
        self.omega = omega
        self.seed = seed

    def close(self):
        self._h = None


class Batch:
    """Many replicas advanced together (kk_batch_*).  `jobs` are objects with
    L, composition, omega, seed, sweeps and layout attributes, and optionally
    start ("random" or "segregated")."""

    def __init__(self, jobs, stream: Optional[int] = None):
        lib = load()
        arr = (Replica * len(jobs))()
        for i, j in enumerate(jobs):
            arr[i] = _replica(j)
        h = ctypes.c_void_p()
        _check(lib.kk_batch_create(ctypes.byref(h), arr, len(jobs), ctypes.c_void_p(stream) if stream else None))
        self._h = h
        self.jobs = list(jobs)

    def run(self):
        _check(load().kk_batch_run(self._h))

    def sim(self, i: int) -> Sim:
        h = ctypes.c_void_p()
        _check(load().kk_batch_sim(self._h, i, ctypes.byref(h)))
        j = self.jobs[i]
        return _Borrowed(h, j.L, float(j.omega), j.seed)

    def set_tile(self, words: int, rows: int, units_per_thread: int = 2) -> None:
        """Fix the tile caps of the tiled replicas (what autotune would choose) and re-plan."""
        _check(load().kk_batch_set_tile(self._h, words, rows, units_per_thread))

    def cluster_hists(self, species: int = 1) -> None:
        """Label every replica's clusters of `species` with one device wait; the
        histograms are then returned by sim(i).cluster_hist(species)."""
        _check(load().kk_batch_cluster_hists(self._h, species))

    def autotune(self, trial_sweeps: int = 10) -> Tuple[int, int, float]:
        """Pick the tile size of the tiled replicas by timing; returns (words, rows, ms_per_sweep)."""
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        ms = ctypes.c_double()
        _check(load().kk_batch_autotune(self._h, trial_sweeps, ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms)))
        return a.value, b.value, ms.value

    def info(self):
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().kk_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"resident": a.value, "tiled": b.value, "tile_jobs": c.value}

    def close(self):
        if getattr(self, "_h", None):
            load().kk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TriBatch:
    """Many triangular lattices advanced together (kk_tri_batch_*).  `jobs` are
    objects with L, composition, omega, seed and sweeps attributes, and
    optionally rows (default L), scheme ("classes" or "mpkk") and start."""

    def __init__(self, jobs, stream: Optional[int] = None):
        lib = load()
        arr = (TriReplica * len(jobs))()
        for i, j in enumerate(jobs):
            arr[i] = TriReplica(j.L, getattr(j, "rows", 0) or j.L, _SCHEMES[getattr(j, "scheme", "classes")],
                                _STARTS[getattr(j, "start", "random")], float(j.composition), float(j.omega),
                                j.seed & (2**64 - 1), int(j.sweeps))
        h = ctypes.c_void_p()
        _check(lib.kk_tri_batch_create(ctypes.byref(h), arr, len(jobs), ctypes.c_void_p(stream) if stream else None))
        self._h = h
        self.jobs = list(jobs)

    def run(self):
        _check(load().kk_tri_batch_run(self._h))

    def sim(self, i: int) -> Sim:
        h = ctypes.c_void_p()
        _check(load().kk_tri_batch_sim(self._h, i, ctypes.byref(h)))
        j = self.jobs[i]
        return _Borrowed(h, j.L, float(j.omega), j.seed, H=getattr(j, "rows", 0) or j.L, geometry="triangular")

    def info(self):
        r, a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().kk_tri_batch_info(self._h, ctypes.byref(r), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"resident": r.value, "batched": a.value, "plain": b.value, "tile_jobs": c.value}

    def close(self):
        if getattr(self, "_h", None):
            load().kk_tri_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _replica(j) -> Replica:
    return Replica(j.L, _LAYOUTS[getattr(j, "layout", "auto")], float(j.composition), float(j.omega),
                   j.seed & (2**64 - 1), int(j.sweeps), _STARTS[getattr(j, "start", "random")])


VALU_PROBES = ("xor", "bitop3", "alignbit", "add", "mad_u64_u32", "mul_lo", "fma_f32", "lshl", "bcnt")


def valu_issue_cycles() -> dict:
    """kk_valu_issue_cycles: SIMD cycles per wave64 instruction of each probed kind."""
    out = (ctypes.c_double * len(VALU_PROBES))()
    _check(load().kk_valu_issue_cycles(out))
    return {k: out[i] for i, k in enumerate(VALU_PROBES)}


def server_job_bytes(job, keep_lattice: bool = False) -> int:
    """kk_server_job_bytes: the device bytes the job server charges a job at admission."""
    out = ctypes.c_uint64()
    r = _replica(job)
    _check(load().kk_server_job_bytes(ctypes.byref(r), 1 if keep_lattice else 0, ctypes.byref(out)))
    return out.value


class Server:
    """Job server (kk_server_*): FIFO admission under an HBM budget and
    continuous batching in chunks of sweeps."""

    def __init__(self, hbm_budget_bytes: int = 0, max_active: int = 0, chunk_sweeps: int = 0,
                 keep_lattice: bool = False, stream: Optional[int] = None):
        lib = load()
        cfg = ServerConfig(hbm_budget_bytes, max_active, 1 if keep_lattice else 0, chunk_sweeps,
                           ctypes.c_void_p(stream) if stream else None)
        h = ctypes.c_void_p()
        _check(lib.kk_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h
        self.keep_lattice = keep_lattice
        self.L = {}

    def now(self) -> float:
        t = ctypes.c_double()
        _check(load().kk_server_now(self._h, ctypes.byref(t)))
        return t.value

    def submit(self, job, arrival: float = -1.0) -> int:
        r = _replica(job)
        jid = ctypes.c_uint64()
        _check(load().kk_server_submit(self._h, ctypes.byref(r), float(arrival), ctypes.byref(jid)))
        self.L[jid.value] = job.L
        return jid.value

    def step(self) -> Tuple[int, int]:
        a, q = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().kk_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, cap: int = 256) -> List[dict]:
        buf = (JobResult * cap)()
        n = ctypes.c_size_t()
        _check(load().kk_server_poll(self._h, buf, cap, ctypes.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def job_hist(self, job_id: int) -> List[Tuple[int, int]]:
        lib = load()
        need = ctypes.c_size_t()
        st = lib.kk_server_job_hist(self._h, job_id, None, 0, ctypes.byref(need))
        if st not in (KK_OK, KK_ETRUNC):
            _check(st)
        buf = (HistEntry * max(1, need.value))()
        _check(lib.kk_server_job_hist(self._h, job_id, buf, need.value, ctypes.byref(need)))
        return [(int(buf[i].size), int(buf[i].count)) for i in range(need.value)]

    def job_lattice(self, job_id: int) -> np.ndarray:
        L = self.L[job_id]
        out = np.empty((L, L), dtype=np.uint8)
        _check(load().kk_server_job_lattice(self._h, job_id, out.ctypes.data, out.size))
        return out

    def release(self, job_id: int):
        _check(load().kk_server_release(self._h, job_id))
        self.L.pop(job_id, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().kk_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().kk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
