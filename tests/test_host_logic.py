"""CPU checks of the host-side logic: seeded workload generators and the
serving summary (no GPU, no oracle)."""
import math

import numpy as np
import pytest

from paper_1309_4349_amd import workloads as wl


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0 (Steele, Lea, Flood 2014): first output
    assert wl.splitmix64(0) == 0xE220A8397B1DCDAF


def test_job_seeds_are_distinct_and_deterministic():
    seeds = {wl.job_seed(c, i) for c in range(5) for i in range(300)}
    assert len(seeds) == 5 * 300
    assert wl.job_seed(3, 7) == wl.job_seed(3, 7)


def test_batch_replica_table():
    jobs = wl.batch_replicas()
    assert len(jobs) == 256 and jobs == wl.batch_replicas()
    for j in jobs:
        assert j.L % 32 == 0 and 64 <= j.L <= 1024
        assert 0.2 <= j.composition <= 0.8 and 0.2 <= j.omega <= 1.4
        assert j.layout in ("int8", "bitpacked") and j.sweeps == 10_000
    # log-uniform side: about a quarter of the replicas fall in each factor-of-2 band
    bands = np.histogram([math.log2(j.L / 64) for j in jobs], bins=[0, 1, 2, 3, 4.01])[0]
    assert all(40 <= b <= 90 for b in bands), bands


def test_serving_trace_is_poisson_with_the_stated_mix():
    jobs = wl.serving_trace(n_jobs=2000, rate=200.0)
    t = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    # exponential gaps: mean 1/rate, coefficient of variation 1
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.08
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1
    assert {j.L for j in jobs} == {128, 256, 512, 1024, 2048}
    sw = np.log([j.sweeps for j in jobs])
    assert sw.min() >= math.log(1e3) - 1e-9 and sw.max() <= math.log(1e5) + 1e-9
    assert abs(sw.mean() - 0.5 * (math.log(1e3) + math.log(1e5))) < 0.15
    for j in jobs:
        assert j.layout == ("bitpacked" if j.L >= 256 else "int8")


def test_grid_and_standing_workloads():
    g = wl.grid_400()
    assert len(g) == 12 and {(j.composition, j.omega) for j in g} == {
        (x, w) for x in (0.3, 0.5, 0.7) for w in (0.3, 0.6, 0.9, 1.2)}
    assert all(j.L == 400 and j.layout == "int8" and j.hist_every == 1000 for j in g)
    b = wl.big_4096()
    assert (b.L, b.layout, b.composition, b.omega, b.sweeps) == (4096, "bitpacked", 0.5, 0.88, 10_000)


def test_serving_summary_percentiles():
    from paper_1309_4349_amd import serve

    jobs = [wl.Job(L=64, composition=0.5, omega=1.0, seed=i, sweeps=10, arrival=0.1 * i) for i in range(100)]
    res = [{"id": i + 1, "status": 0, "t_arrival": 10.0 + 0.1 * i, "t_admit": 10.0 + 0.1 * i,
            "t_done": 10.0 + 0.1 * i + (i + 1) * 0.01, "attempts": 64 * 64 * 10} for i in range(100)]
    out = serve.summarize(jobs, res, t0=10.0, stats={"steps": 5, "peak_bytes": 1, "budget": 2, "gpu_busy_s": 1.0})
    assert out["jobs"] == 100 and out["failed"] == 0
    assert out["latency_p50_s"] == pytest.approx(np.percentile([(i + 1) * 0.01 for i in range(100)], 50))
    assert out["latency_p99_s"] == pytest.approx(np.percentile([(i + 1) * 0.01 for i in range(100)], 99))
    assert out["attempts"] == 100 * 64 * 64 * 10


def test_runner_arguments():
    from paper_1309_4349_amd import run
    a = run.parse(["--geometry", "square", "--L", "64", "--sweeps", "10", "--every", "5", "--start", "segregated"])
    assert (a.geometry, a.L, a.sweeps, a.every, a.start, a.scheme) == ("square", 64, 10, 5, "segregated", "classes")
    with pytest.raises(SystemExit):
        run.parse(["--every", "0"])
