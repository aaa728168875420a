"""GPU parity over the full sweep counts of the standing square-torus workloads.

The expected values in tests/golden/fullsize_*.json were written by
tests/golden/make_fullsize.py, which runs only the CPU oracle: for each of the
twelve 400 x 400 runs (10^5 sweeps) N_AB and a digest of the species-1
cluster-size histogram after every 1000 sweeps, and for the 4096 x 4096 run
(10^4 sweeps) N_AB and the lattice hash after every 1000 sweeps; each run ends
with its lattice hash, N_AB, accepted count and both species' histograms.
The paper takes its cluster statistics regularly during a run (Materials and
Methods, "Cluster Analysis methods"; Results, "Cluster Analysis").  Here the
plain single-lattice path and the batch engine run the same workloads in the
launch configuration the benchmark uses (default tiles) and must reproduce
every recorded value exactly."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
from make_fullsize import OUT_400, OUT_4096, hist_digest  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load(path):
    with open(path) as f:
        return json.load(f)


def _pairs(h):
    return [tuple(int(v) for v in p) for p in h]


def _check_cadence(rec, got_nab, got_hist, k):
    want = rec["cadence"][k]
    assert got_nab == want["n_unlike"], (rec["tag"], want["t"], got_nab, want["n_unlike"])
    assert hist_digest(got_hist) == want["hist1"], (rec["tag"], want["t"])
    assert sum(c for _, c in got_hist) == want["n_clusters1"]


def _check_final(rec, sim, accepted):
    s = sim.get_lattice()
    assert oracle.lattice_hash(s) == rec["lattice_hash"], rec["tag"]
    assert sim.energy()[0] == rec["n_unlike"]
    assert accepted == rec["accepted"]
    assert sim.cluster_hist(1) == _pairs(rec["hist1"])
    assert sim.cluster_hist(0) == _pairs(rec["hist0"])


@pytest.mark.parametrize("idx", range(12))
def test_400_full_run_matches_oracle_goldens(idx):
    rec = _load(OUT_400)["runs"][idx]
    job = wl.grid_400()[idx]
    assert (rec["L"], rec["composition"], rec["omega"], rec["seed"], rec["sweeps"]) == \
        (job.L, job.composition, job.omega, job.seed, job.sweeps)
    say(f"case {job.tag}: {job.sweeps} sweeps, histogram every {job.hist_every}, plain path")
    sim = kk.Sim(job.L, job.composition, job.omega, job.seed, layout="int8")
    for k in range(job.sweeps // job.hist_every):
        sim.sweep(job.hist_every)
        _check_cadence(rec, sim.energy()[0], sim.cluster_hist(1), k)
    assert sim.stats()[0] == job.sweeps
    _check_final(rec, sim, sim.stats()[2])
    sim.close()


def test_400_grid_batched_matches_oracle_goldens():
    recs = _load(OUT_400)["runs"]
    jobs = wl.grid_400(sweeps=1000)
    say(f"case 400^2 grid: {len(jobs)} runs batched, 100 rounds of 1000 sweeps")
    b = kk.Batch(jobs)
    b.autotune(5)
    for k in range(100):
        b.run()
        for i, rec in enumerate(recs):
            s = b.sim(i)
            _check_cadence(rec, s.energy()[0], s.cluster_hist(1), k)
    for i, rec in enumerate(recs):
        s = b.sim(i)
        assert s.stats()[0] == 100_000
        _check_final(rec, s, s.stats()[2])
    b.close()


def test_4096_full_run_matches_oracle_goldens():
    rec = _load(OUT_4096)
    job = wl.big_4096()
    assert (rec["L"], rec["composition"], rec["omega"], rec["seed"], rec["sweeps"]) == \
        (job.L, job.composition, job.omega, job.seed, job.sweeps)
    say(f"case {job.tag}: {job.sweeps} sweeps, lattice hash every 1000")
    sim = kk.Sim(job.L, job.composition, job.omega, job.seed, layout="bitpacked")
    for k, want in enumerate(rec["cadence"]):
        sim.sweep(1000)
        assert sim.stats()[0] == want["t"]
        assert sim.energy()[0] == want["n_unlike"], (want["t"],)
        assert oracle.lattice_hash(sim.get_lattice()) == want["lattice_hash"], (want["t"],)
    _check_final(rec, sim, sim.stats()[2])
    sim.close()
