"""GPU: batches of triangular lattices -- every replica, batched (one launch
per sweep over the tiles of all replicas) or run on its own (literal MPKK,
lattices too small for a tile), equals the same replica alone and the oracle,
over two runs in a row."""
from dataclasses import dataclass

import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk

pytestmark = pytest.mark.gpu


@dataclass
class TJ:
    L: int
    rows: int
    scheme: str
    start: str
    composition: float
    omega: float
    seed: int
    sweeps: int


JOBS = [TJ(100, 100, "classes", "random", 0.5, 0.9, 11, 10), TJ(204, 204, "classes", "segregated", 0.35, 0.6, 12, 7),
        TJ(404, 412, "classes", "random", 0.5, -0.4, 13, 12), TJ(76, 76, "classes", "random", 0.4, 1.1, 14, 5),
        TJ(101, 84, "mpkk", "random", 0.5, 0.5, 15, 4), TJ(124, 84, "classes", "random", 0.5, 0.7, 16, 0),
        TJ(132, 200, "classes", "segregated", 0.6, 0.0, 17, 9)]


def test_tri_batch_equals_alone_and_oracle():
    print(f"case tri batch of {len(JOBS)}", flush=True)
    b = kk.TriBatch(JOBS)
    info = b.info()
    # fewer than 64 small rings: those whose default is the whole ring (100^2, 76^2, 124 x 84) and the
    # MPKK replica run on their own; 204^2, 404 x 412 and 132 x 200 share the tile launches
    assert (info["resident"], info["batched"], info["plain"]) == (0, 3, 4) and info["tile_jobs"] > 50
    b.run()
    b.run()   # the second run continues from the first
    for i, j in enumerate(JOBS):
        print(f"  replica {i}: {j}", flush=True)
        alone = kk.Sim(j.L, j.composition, j.omega, j.seed, geometry="triangular", rows=j.rows, scheme=j.scheme)
        alone.restart(j.start)
        alone.sweep(2 * j.sweeps)
        s = b.sim(i)
        assert np.array_equal(s.get_lattice(), alone.get_lattice())
        assert s.stats() == alone.stats()
        assert s.energy() == alone.energy()
        alone.close()
        if j.L * j.rows <= 50000:
            ref = oracle.init_segregated(j.L, j.composition, j.rows) if j.start == "segregated" else \
                oracle.init_rect(j.L, j.rows, j.composition, j.seed)
            run = oracle.tri_sweeps if j.scheme == "classes" else oracle.mpkk_steps
            acc = run(ref, j.omega, j.seed, 0, 2 * j.sweeps)
            assert np.array_equal(s.get_lattice(), ref)
            assert s.stats()[2] == acc
    b.close()


def test_tri_batch_rejects_bad_replicas():
    for bad in (TJ(8, 8, "classes", "random", 0.5, 1.0, 1, 3), TJ(10, 8, "mpkk", "random", 0.5, 1.0, 1, 3),
                TJ(100, 100, "classes", "sideways", 0.5, 1.0, 1, 3)):
        with pytest.raises((kk.KKError, KeyError)):
            kk.TriBatch([bad])


def test_tri_batch_resident_replicas():
    # 72 small rings (whole ring in one workgroup each), uneven sizes, sweeps and starts, plus two tiled ones
    jobs = [TJ(12 + 8 * (i % 12), 12 + 8 * ((5 * i) % 12), "classes", "segregated" if i % 3 == 0 else "random",
               0.2 + 0.6 * ((7 * i) % 10) / 10, -0.5 + 1.7 * (i % 9) / 8, 100 + i, (3 * i) % 11) for i in range(72)]
    jobs += [TJ(404, 404, "classes", "random", 0.5, 0.8, 999, 6), TJ(10, 14, "mpkk", "random", 0.5, 0.6, 998, 5)]
    print(f"case tri batch resident, {len(jobs)} replicas", flush=True)
    b = kk.TriBatch(jobs)
    info = b.info()
    # the 404^2 ring (163,216 B) does not fit one workgroup: it is tiled; MPKK runs on its own
    assert (info["resident"], info["batched"], info["plain"]) == (72, 1, 1)
    b.run()
    b.run()
    for i, j in enumerate(jobs):
        alone = kk.Sim(j.L, j.composition, j.omega, j.seed, geometry="triangular", rows=j.rows, scheme=j.scheme)
        alone.restart(j.start)
        alone.sweep(2 * j.sweeps)
        s = b.sim(i)
        assert np.array_equal(s.get_lattice(), alone.get_lattice()), i
        assert s.stats() == alone.stats(), i
        alone.close()
        if i % 10 == 0:
            ref = oracle.init_segregated(j.L, j.composition, j.rows) if j.start == "segregated" else \
                oracle.init_rect(j.L, j.rows, j.composition, j.seed)
            oracle.tri_sweeps(ref, j.omega, j.seed, 0, 2 * j.sweeps)
            assert np.array_equal(s.get_lattice(), ref), i
    b.close()


def test_tri_batch_keeps_its_tiles_when_a_replica_changes_its_own():
    # the batch's job table was built for each replica's tile at creation; a
    # replica whose handle is re-tiled between runs still runs on that table
    jobs = [TJ(404, 412, "classes", "random", 0.5, 0.7, 21, 4), TJ(204, 204, "classes", "random", 0.4, 0.9, 22, 3)]
    b = kk.TriBatch(jobs)
    b.run()
    b.sim(0).tri_set_tile(96, 160)
    b.sim(1).tri_set_tile(0)
    b.run()
    for i, j in enumerate(jobs):
        ref = oracle.init_rect(j.L, j.rows, j.composition, j.seed)
        acc = oracle.tri_sweeps(ref, j.omega, j.seed, 0, 2 * j.sweeps)
        s = b.sim(i)
        assert np.array_equal(s.get_lattice(), ref)
        assert s.stats() == (2 * j.sweeps, 2 * j.sweeps * j.L * j.rows, acc)
    b.close()
