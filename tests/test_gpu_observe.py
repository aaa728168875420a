"""GPU: the observables (N_AB, exact and random-neighbour similar-neighbour
fractions, cluster-size averages) equal the oracle's, bit for bit, and a
time series equals sweeping and observing step by step."""
import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,layout,x,w,n", [
    (64, "bitpacked", 0.5, 0.9, 30), (100, "int8", 0.3, 1.2, 17), (36, "int8", 0.0, 0.5, 3),
    (128, "int8", 1.0, 0.5, 2), (256, "bitpacked", 0.7, 0.6, 11), (4, "int8", 0.5, 0.4, 5),
])
def test_observe_matches_oracle(L, layout, x, w, n):
    print(f"case observe L={L} {layout} x={x}", flush=True)
    seed = wl.job_seed(21, L)
    s = kk.Sim(L, x, w, seed, layout=layout)
    s.sweep(n)
    ref = oracle.init(L, x, seed)
    oracle.sweeps(ref, w, seed, 0, n)
    for species in (0, 1):
        got = s.observe(species)
        want = oracle.observables(ref, w, species, seed, n)
        assert got["sweep"] == n
        for k, v in want.items():
            assert got[k] == v, (species, k, got[k], v)
    s.close()


def test_series_equals_step_by_step():
    L, x, w, seed = 96, 0.4, 0.8, 77
    a = kk.Sim(L, x, w, seed, layout="bitpacked")
    ser = a.series(every=7, count=5, species=1)
    b = kk.Sim(L, x, w, seed, layout="bitpacked")
    for i in range(5):
        b.sweep(7)
        assert ser[i] == b.observe(1), i
    assert [r["sweep"] for r in ser] == [7, 14, 21, 28, 35]
    a.close()
    b.close()


def test_observe_4096_properties():
    # full size: the sampled fraction scatters around the exact one by O(1/L)
    job = wl.big_4096(20)
    s = kk.Sim(job.L, job.composition, job.omega, job.seed, layout="bitpacked")
    s.sweep(job.sweeps)
    o = s.observe(1)
    N = job.L * job.L
    assert o["similar_exact"] == 1.0 - o["n_unlike"] / (2 * N)
    assert abs(o["similar_sampled"] - o["similar_exact"]) < 5 * 0.5 / job.L
    assert o["size_number_avg"] * o["n_clusters"] == pytest.approx(oracle.n_ones(job.L, job.composition))
    assert o["size_max"] <= N and o["size_weight_avg"] >= o["size_number_avg"]
    s.close()
