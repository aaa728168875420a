"""CPU oracle for the Kawasaki lattice sweeps -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product.  The arithmetic lives in
``kk_oracle.c`` (plain C, built with gcc by :func:`build`); this module only
marshals numpy arrays into it.  ``enumerate4x4`` is the one pure-Python
helper: it lists all states of a small lattice for exact Boltzmann sums.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from itertools import combinations

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kk_oracle.c")
_LIB = os.path.join(_HERE, "libkkoracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``kk_oracle.c`` into ``libkkoracle.so`` with gcc (OpenMP on)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u16p = ctypes.POINTER(ctypes.c_uint16)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    c_int_p = ctypes.POINTER(ctypes.c_int)
    U32, U64, D = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "ko_philox4x32_10": (None, [u32p, u32p, u32p]),
        "ko_thresholds": (None, [D, u64p]),
        "ko_sweep_randoms": (None, [U32, U64, U64, u16p]),
        "ko_ext_word": (U32, [U64, U64, U32, U32]),
        "ko_phase_order": (None, [U64, U64, c_int_p]),
        "ko_site_class": (ctypes.c_int, [U32, U32]),
        "ko_local_dnab": (ctypes.c_int, [u8p, U32, U32, U32, U32]),
        "ko_lattice_hash": (U64, [u8p, U32]),
        "ko_sweeps": (U64, [u8p, U32, D, U64, U64, U64, u64p]),
        "ko_energy": (U64, [u8p, U32]),
        "ko_n_ones": (U64, [U32, D]),
        "ko_init_key": (U64, [U64, U32, U32]),
        "ko_init": (ctypes.c_int, [u8p, U32, D, U64]),
        "ko_init_rect": (ctypes.c_int, [u8p, U32, U32, D, U64]),
        "ko_n_ones_rect": (U64, [U32, U32, D]),
        "ko_cluster_counts": (U64, [u8p, U32, ctypes.c_int, u64p]),
        "ko_seq_kawasaki": (U64, [u8p, U32, D, U64, U64]),
        "ko_tri_seq_kawasaki": (U64, [u8p, U32, U32, D, U64, U64]),
        "ko_set_threads": (ctypes.c_int, [ctypes.c_int]),
        "ko_mpkk_k": (ctypes.c_int, [U64, U64, ctypes.c_int]),
        "ko_mpkk_domain_randoms": (None, [U64, U64, ctypes.c_int, U64, u32p, u32p]),
        "ko_mpkk_iteration": (ctypes.c_int64, [u8p, U32, U32, ctypes.c_int, u32p, u32p, u64p]),
        "ko_mpkk_steps": (U64, [u8p, U32, U32, D, U64, U64, U64]),
        "ko_similar_sampled": (U64, [u8p, U32, U64, U64]),
        "ko_tri_thresholds": (None, [D, u64p]),
        "ko_tri_phase_order": (None, [U64, U64, c_int_p]),
        "ko_tri_site_randoms": (None, [U64, U64, U64, u32p, u32p]),
        "ko_tri_local_dnab": (ctypes.c_int, [u8p, U32, U32, U64, U32]),
        "ko_tri_sweeps": (U64, [u8p, U32, U32, D, U64, U64, U64]),
        "ko_tri_energy": (U64, [u8p, U32, U32]),
        "ko_tri_cluster_counts": (U64, [u8p, U32, U32, ctypes.c_int, u64p]),
        "ko_tri_similar_sampled": (U64, [u8p, U32, U32, U64, U64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _ring(s: np.ndarray) -> np.ndarray:
    """A triangular helical lattice: H rows of L sites, shape (H, L)."""
    if s.dtype != np.uint8 or s.ndim != 2 or not s.flags.c_contiguous:
        raise ValueError("lattice must be a C-contiguous 2-D uint8 array")
    return s


def _lattice(s: np.ndarray) -> np.ndarray:
    if s.dtype != np.uint8 or s.ndim != 2 or s.shape[0] != s.shape[1] or not s.flags.c_contiguous:
        raise ValueError("lattice must be a C-contiguous square uint8 array")
    return s


# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().ko_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def thresholds(omega: float) -> np.ndarray:
    T = np.zeros(7, dtype=np.uint64)
    _load().ko_thresholds(float(omega), _ptr(T, ctypes.c_uint64))
    return T


def sweep_randoms(L: int, seed: int, t: int) -> np.ndarray:
    """(L, L) uint16 array, per site (direction << 10) | u10 for sweep t."""
    r = np.zeros((L, L), dtype=np.uint16)
    _load().ko_sweep_randoms(L, seed, t, _ptr(r, ctypes.c_uint16))
    return r


def ext_word(seed: int, t: int, x: int, y: int) -> int:
    return int(_load().ko_ext_word(seed, t, x, y))


def phase_order(seed: int, t: int) -> list:
    p = (ctypes.c_int * 8)()
    _load().ko_phase_order(seed, t, p)
    return list(p)


def site_class(x: int, y: int) -> int:
    return int(_load().ko_site_class(x, y))


def local_dnab(s: np.ndarray, x: int, y: int, direction: int) -> int:
    s = _lattice(s)
    return int(_load().ko_local_dnab(_ptr(s, ctypes.c_uint8), s.shape[0], x, y, direction))


def lattice_hash(s: np.ndarray) -> int:
    s = _lattice(s)
    return int(_load().ko_lattice_hash(_ptr(s, ctypes.c_uint8), s.shape[0]))


def sweeps(s: np.ndarray, omega: float, seed: int, t0: int, n: int, trace: bool = False):
    """Run n sweeps in place from sweep counter t0.

    Returns the accepted-exchange count, or (count, per-sweep hashes)."""
    s = _lattice(s)
    L = s.shape[0]
    tr = np.zeros(max(n, 1), dtype=np.uint64) if trace else None
    acc = _load().ko_sweeps(_ptr(s, ctypes.c_uint8), L, float(omega), seed, t0, n,
                            _ptr(tr, ctypes.c_uint64) if trace else None)
    if acc == 2**64 - 1:
        raise MemoryError("oracle sweep allocation failed")
    return (int(acc), tr[:n]) if trace else int(acc)


def energy(s: np.ndarray) -> int:
    s = _lattice(s)
    return int(_load().ko_energy(_ptr(s, ctypes.c_uint8), s.shape[0]))


def n_ones(L: int, composition: float) -> int:
    return int(_load().ko_n_ones(L, float(composition)))


def init_key(seed: int, x: int, y: int) -> int:
    return int(_load().ko_init_key(seed, x, y))


def init(L: int, composition: float, seed: int) -> np.ndarray:
    s = np.zeros((L, L), dtype=np.uint8)
    if _load().ko_init(_ptr(s, ctypes.c_uint8), L, float(composition), seed) != 0:
        raise MemoryError("oracle init allocation failed")
    return s


def n_ones_rect(L: int, H: int, composition: float) -> int:
    return int(_load().ko_n_ones_rect(L, H, float(composition)))


def init_rect(L: int, H: int, composition: float, seed: int) -> np.ndarray:
    """The random start on H rows of L sites (shape (H, L))."""
    s = np.zeros((H, L), dtype=np.uint8)
    if _load().ko_init_rect(_ptr(s, ctypes.c_uint8), L, H, float(composition), seed) != 0:
        raise MemoryError("oracle init allocation failed")
    return s


def cluster_counts(s: np.ndarray, species: int = 1) -> np.ndarray:
    """Dense counts: out[k] = number of clusters of exactly k sites."""
    s = _lattice(s)
    L = s.shape[0]
    counts = np.zeros(L * L + 1, dtype=np.uint64)
    r = _load().ko_cluster_counts(_ptr(s, ctypes.c_uint8), L, int(species), _ptr(counts, ctypes.c_uint64))
    if r == 2**64 - 1:
        raise MemoryError("oracle cluster allocation failed")
    return counts


def cluster_hist(s: np.ndarray, species: int = 1):
    """Sparse histogram: list of (size, count) pairs, ascending by size."""
    c = cluster_counts(s, species)
    nz = np.nonzero(c)[0]
    return [(int(k), int(c[k])) for k in nz]


def similar_sampled(s: np.ndarray, seed: int, t: int) -> int:
    """Count of sites whose randomly drawn neighbour is of the same type
    (the random-neighbour estimate of the similar first-neighbour fraction is
    this count over the number of sites)."""
    s = _lattice(s)
    return int(_load().ko_similar_sampled(_ptr(s, ctypes.c_uint8), s.shape[0], seed, t))


def observables(s: np.ndarray, omega: float, species: int, seed: int, t: int) -> dict:
    """The observables of one lattice state, from their definitions:
    N_AB and E/kT = omega * N_AB; the exact similar first-neighbour fraction
    1 - N_AB / (2N) (each of the 2N bonds joins like or unlike sites) and its
    random-neighbour estimate; the number of clusters of `species`, the
    number-average size sum s h(s) / sum h(s), the weight-average size
    sum s^2 h(s) / sum s h(s) and the largest size.  Sums are exact integers;
    each ratio is one correctly rounded division."""
    s = _lattice(s)
    N = s.shape[0] * s.shape[0]
    return _observables_of(energy(s), 2 * N, cluster_counts(s, species), similar_sampled(s, seed, t), N, omega)


def _observables_of(nab: int, bonds: int, c: np.ndarray, same: int, N: int, omega: float) -> dict:
    sizes = np.nonzero(c)[0]
    n_cl = int(sum(int(c[k]) for k in sizes))
    s1 = int(sum(int(k) * int(c[k]) for k in sizes))
    s2 = int(sum(int(k) * int(k) * int(c[k]) for k in sizes))
    return {
        "n_unlike": nab, "energy_kT": omega * nab,
        "similar_exact": 1.0 - nab / bonds,
        "similar_sampled": same / N,
        "n_clusters": n_cl,
        "size_number_avg": s1 / n_cl if n_cl else 0.0,
        "size_weight_avg": s2 / s1 if s1 else 0.0,
        "size_max": int(sizes.max()) if len(sizes) else 0,
    }


# --------------------------------------------------------------------------
# Triangular lattice, helical boundaries (sites i = y*L + x on one ring,
# neighbours i +- 1, i +- L, i +- (L - 1) mod N); L % 8 == 4.
# --------------------------------------------------------------------------
def tri_thresholds(omega: float) -> np.ndarray:
    T = np.zeros(11, dtype=np.uint64)
    _load().ko_tri_thresholds(float(omega), _ptr(T, ctypes.c_uint64))
    return T


def tri_phase_order(seed: int, t: int) -> list:
    p = (ctypes.c_int * 16)()
    _load().ko_tri_phase_order(seed, t, p)
    return list(p)


def tri_site_randoms(seed: int, t: int, i: int):
    d, u = ctypes.c_uint32(), ctypes.c_uint32()
    _load().ko_tri_site_randoms(seed, t, i, ctypes.byref(d), ctypes.byref(u))
    return d.value, u.value


def tri_local_dnab(s: np.ndarray, i: int, direction: int) -> int:
    s = _ring(s)
    return int(_load().ko_tri_local_dnab(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], i, direction))


def tri_sweeps(s: np.ndarray, omega: float, seed: int, t0: int, n: int) -> int:
    s = _ring(s)
    return int(_load().ko_tri_sweeps(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], float(omega), seed, t0, n))


def tri_energy(s: np.ndarray) -> int:
    s = _ring(s)
    return int(_load().ko_tri_energy(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0]))


def tri_cluster_counts(s: np.ndarray, species: int = 1) -> np.ndarray:
    s = _ring(s)
    H, L = s.shape
    counts = np.zeros(L * H + 1, dtype=np.uint64)
    r = _load().ko_tri_cluster_counts(_ptr(s, ctypes.c_uint8), L, H, int(species), _ptr(counts, ctypes.c_uint64))
    if r == 2**64 - 1:
        raise MemoryError("oracle cluster allocation failed")
    return counts


def tri_cluster_hist(s: np.ndarray, species: int = 1):
    c = tri_cluster_counts(s, species)
    nz = np.nonzero(c)[0]
    return [(int(k), int(c[k])) for k in nz]


def tri_similar_sampled(s: np.ndarray, seed: int, t: int) -> int:
    s = _ring(s)
    return int(_load().ko_tri_similar_sampled(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], seed, t))


def tri_observables(s: np.ndarray, omega: float, species: int, seed: int, t: int) -> dict:
    """observables() on the triangular lattice: 3N bonds, six-connected
    clusters, the six-neighbour random draw."""
    s = _ring(s)
    N = s.shape[0] * s.shape[1]
    return _observables_of(tri_energy(s), 3 * N, tri_cluster_counts(s, species), tri_similar_sampled(s, seed, t),
                           N, omega)


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's per-class loops (n <= 0: unchanged); returns the count in force."""
    return int(_load().ko_set_threads(int(n)))


def init_segregated(L: int, composition: float, H: int = 0) -> np.ndarray:
    """The non-random start (Results, Figs. 10-11), read as full segregation:
    the first n1 sites in index order y*L + x hold type 1 (H rows; 0 = L)."""
    H = H or L
    s = np.zeros(L * H, dtype=np.uint8)
    s[: n_ones_rect(L, H, composition)] = 1
    return s.reshape(H, L)


def tri_seq_kawasaki(s: np.ndarray, omega: float, rng_seed: int, n_steps: int) -> int:
    """Sequential random-site Kawasaki on the triangular helical lattice."""
    s = _ring(s)
    return int(_load().ko_tri_seq_kawasaki(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], float(omega), rng_seed,
                                            n_steps))


# --------------------------------------------------------------------------
# The paper's literal MPKK: 7-site domains covering H rows of L sites
# (L = 3 or 5 mod 7, H = 0 mod 7), 7 iterations per step with k drawn with
# replacement, every domain of an iteration deciding from the state at its
# start.
# --------------------------------------------------------------------------
def mpkk_k(seed: int, t: int, j: int) -> int:
    return int(_load().ko_mpkk_k(seed, t, j))


def mpkk_domain_randoms(seed: int, t: int, j: int, m: int):
    d, u = ctypes.c_uint32(), ctypes.c_uint32()
    _load().ko_mpkk_domain_randoms(seed, t, j, m, ctypes.byref(d), ctypes.byref(u))
    return d.value, u.value


def mpkk_iteration(s: np.ndarray, k: int, dirs, us, T) -> int:
    """One synchronous iteration with explicit directions and uniforms (one per domain)."""
    s = _ring(s)
    M = s.size // 7
    d = np.ascontiguousarray(dirs, dtype=np.uint32)
    u = np.ascontiguousarray(us, dtype=np.uint32)
    T = np.ascontiguousarray(T, dtype=np.uint64)
    if d.shape != (M,) or u.shape != (M,) or T.shape != (11,):
        raise ValueError("need one direction and one uniform per domain and 11 thresholds")
    r = _load().ko_mpkk_iteration(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], int(k), _ptr(d, ctypes.c_uint32),
                                  _ptr(u, ctypes.c_uint32), _ptr(T, ctypes.c_uint64))
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return int(r)


def mpkk_steps(s: np.ndarray, omega: float, seed: int, t0: int, n: int) -> int:
    s = _ring(s)
    r = _load().ko_mpkk_steps(_ptr(s, ctypes.c_uint8), s.shape[1], s.shape[0], float(omega), seed, t0, n)
    if r == 2**64 - 1:
        raise MemoryError("oracle allocation failed")
    return int(r)


def seq_kawasaki(s: np.ndarray, omega: float, rng_seed: int, n_steps: int) -> int:
    s = _lattice(s)
    return int(_load().ko_seq_kawasaki(_ptr(s, ctypes.c_uint8), s.shape[0], float(omega), rng_seed, n_steps))


def enumerate_states(L: int, n1: int):
    """All (L, L) 0/1 lattices with exactly n1 ones, as an (M, L*L) uint8 array."""
    N = L * L
    combos = list(combinations(range(N), n1))
    out = np.zeros((len(combos), N), dtype=np.uint8)
    for i, c in enumerate(combos):
        out[i, list(c)] = 1
    return out
