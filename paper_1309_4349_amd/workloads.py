"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds parameters and seeded draws only: lattice side, composition,
interaction omega (in kT), seeds, sweep counts, replica tables and job
arrival traces.  None of the simulation's arithmetic lives here; both the
HIP library and the CPU oracle receive what it produces as plain inputs.

The paper's own runs use no public dataset: lattices start random or
segregated, 400x400 is its headline size and it compares runs of 1e4 and 1e7
steps on lattices up to 100x100 (Introduction; Results, "MPKK vs. Kawasaki
method").  The workloads below are the standing synthetic stand-ins.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MASTER_SEED = 0x13094349
U64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One splitmix64 output for state x (Steele, Lea, Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & U64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & U64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & U64
    return z ^ (z >> 31)


def job_seed(config: int, index: int) -> int:
    """Per-job Philox seed: splitmix64(master ^ (config << 32 | index))."""
    return splitmix64(MASTER_SEED ^ (((config & 0xFFFFFFFF) << 32) | (index & 0xFFFFFFFF)))


@dataclass
class Job:
    L: int
    composition: float
    omega: float
    seed: int
    sweeps: int
    layout: str = "int8"          # "int8" or "bitpacked"
    hist_every: int = 0           # take a cluster histogram every k sweeps (0: only at the end)
    arrival: float = 0.0          # serving: arrival time in seconds from trace start
    tag: str = ""
    start: str = "random"         # "random" or "segregated"

    @property
    def sites(self) -> int:
        return self.L * self.L

    @property
    def attempts(self) -> int:
        return self.sites * self.sweeps


# --------------------------------------------------------------------------
# The five standing workloads.
# --------------------------------------------------------------------------
def small_64() -> Job:
    """64x64, 50:50, omega 0.5 kT, 1000 sweeps, int8."""
    return Job(L=64, composition=0.5, omega=0.5, seed=job_seed(0, 0), sweeps=1000, layout="int8",
               tag="64x64 int8 x=0.5 omega=0.5 1000 sweeps")


def grid_400(sweeps: int = 100_000) -> List[Job]:
    """400x400 int8, compositions {0.3,0.5,0.7} x omega {0.3,0.6,0.9,1.2}, histogram every 1000."""
    jobs = []
    idx = 0
    for x in (0.3, 0.5, 0.7):
        for w in (0.3, 0.6, 0.9, 1.2):
            jobs.append(Job(L=400, composition=x, omega=w, seed=job_seed(1, idx), sweeps=sweeps,
                            layout="int8", hist_every=1000, tag=f"400x400 int8 x={x} omega={w}"))
            idx += 1
    return jobs


def big_4096(sweeps: int = 10_000) -> Job:
    """4096x4096 bit-packed, 50:50, omega 0.88 kT (just below demixing), 1e4 sweeps."""
    return Job(L=4096, composition=0.5, omega=0.88, seed=job_seed(2, 0), sweeps=sweeps,
               layout="bitpacked", tag="4096x4096 bitpacked x=0.5 omega=0.88")


def batch_replicas(n: int = 256, sweeps: int = 10_000, seed: int = MASTER_SEED ^ 3,
                   offgrid: bool = False) -> List[Job]:
    """Replica table: L = 64 * 16**U (log-uniform 64..1024), x ~ U[0.2,0.8], omega ~ U[0.2,1.4].

    Replicas with L_raw >= 256 are bit-packed with L rounded to a multiple of
    32; the rest are stored as int8, with L rounded to a multiple of 32 as
    well (whole 32-site words per row) or, with `offgrid`, to a multiple of 4
    (the same draws, so the same replicas up to the rounding of the small ones)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        raw = 64.0 * 16.0 ** rng.random()
        layout = "bitpacked" if raw >= 256.0 else "int8"
        step = 4 if (offgrid and layout == "int8") else 32
        L = int(round(raw / step)) * step
        L = max(64, min(1024, L))
        x = float(rng.uniform(0.2, 0.8))
        w = float(rng.uniform(0.2, 1.4))
        jobs.append(Job(L=L, composition=x, omega=w, seed=job_seed(3, i), sweeps=sweeps, layout=layout,
                        tag=f"replica {i}"))
    return jobs


def serving_trace(n_jobs: int = 1000, rate: float = 200.0, sweeps_lo: float = 1e3, sweeps_hi: float = 1e5,
                  sides=(128, 256, 512, 1024, 2048), seed: int = MASTER_SEED ^ 4,
                  sweep_scale: float = 1.0) -> List[Job]:
    """Poisson arrivals (mean `rate` jobs/s); L uniform over `sides`; sweeps log-uniform.

    `sweep_scale` shrinks every job's sweep count by the same factor (for
    short rehearsals); the arrival process is unchanged."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for i in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        L = int(rng.choice(np.asarray(sides)))
        sw = math.exp(rng.uniform(math.log(sweeps_lo), math.log(sweeps_hi)))
        sw = max(1, int(round(sw * sweep_scale)))
        x = float(rng.uniform(0.2, 0.8))
        w = float(rng.uniform(0.2, 1.4))
        layout = "bitpacked" if L >= 256 else "int8"
        jobs.append(Job(L=L, composition=x, omega=w, seed=job_seed(4, i), sweeps=sw, layout=layout,
                        arrival=t, tag=f"job {i}"))
    return jobs


# --------------------------------------------------------------------------
# Seeded lattices for tests that start from a given state.
# --------------------------------------------------------------------------
def random_lattice(L: int, composition: float, seed: int) -> np.ndarray:
    """A uniformly random (L, L) uint8 0/1 lattice with round(c*L*L) ones (numpy generator)."""
    rng = np.random.default_rng(seed)
    N = L * L
    n1 = int(math.floor(composition * N + 0.5))
    flat = np.zeros(N, dtype=np.uint8)
    flat[rng.permutation(N)[:n1]] = 1
    return flat.reshape(L, L)


def segregated_lattice(L: int, composition: float) -> np.ndarray:
    """Non-random start: the first round(c*N) sites in row-major order are type 1 (a slab)."""
    N = L * L
    n1 = int(math.floor(composition * N + 0.5))
    flat = np.zeros(N, dtype=np.uint8)
    flat[:n1] = 1
    return flat.reshape(L, L)
