"""GPU: cluster-size histograms through the one-wait paths.

A batch labels every replica with one device wait (kk_batch_cluster_hists);
each replica's histogram must equal the oracle's labelling of its lattice, for
both species, and a later kk_cluster_hist on the replica must return it without
relabelling.  A single handle's histogram copies the small sizes, the count of
large clusters and the first large sizes back in one go; a lattice with more
large clusters than that first copy holds takes the second copy, checked here
against the closed form of a striped lattice, on a single handle and as one
replica of a batch."""
import sys

import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def jobs():
    specs = [(64, "int8", 0.5, 0.5, 30), (96, "bitpacked", 0.3, 1.2, 17), (128, "int8", 0.7, -0.4, 25),
             (160, "bitpacked", 0.45, 0.0, 9), (100, "int8", 0.6, 0.9, 14), (320, "int8", 0.35, 1.1, 8),
             (512, "bitpacked", 0.5, 0.88, 6), (68, "int8", 0.4, 0.3, 19)]
    return [wl.Job(L=L, composition=x, omega=w, seed=wl.job_seed(91, i), sweeps=n, layout=lay)
            for i, (L, lay, x, w, n) in enumerate(specs)]


@pytest.mark.parametrize("species", [1, 0])
def test_batch_cluster_hists_match_the_oracle(species):
    js = jobs()
    say(f"case batch histograms of {len(js)} replicas, species {species}")
    b = kk.Batch(js)
    for rnd in range(2):
        b.run()
        b.cluster_hists(species)
        for i, j in enumerate(js):
            s = b.sim(i)
            got = s.cluster_hist(species)
            assert got == oracle.cluster_hist(s.get_lattice(), species), (rnd, i, j.L)
    b.close()


def test_batch_cluster_hists_follow_the_lattice():
    js = jobs()[:3]
    b = kk.Batch(js)
    b.run()
    b.cluster_hists(1)
    before = [b.sim(i).cluster_hist(1) for i in range(len(js))]
    b.run()  # the lattices change: the held histograms must not be returned
    after = [b.sim(i).cluster_hist(1) for i in range(len(js))]
    for i in range(len(js)):
        assert after[i] == oracle.cluster_hist(b.sim(i).get_lattice(), 1)
    assert after != before
    with pytest.raises(kk.KKError) as e:
        b.cluster_hists(2)
    assert e.value.status == kk.KK_EINVAL
    b.close()


def test_more_large_clusters_than_the_first_copy():
    # columns of species 1 one site wide, separated by columns of species 0:
    # L / 2 clusters of L sites each, more than the 1024 large sizes copied
    # back with the histogram
    L = 4160
    say(f"case striped {L}^2 lattice")
    s = kk.Sim(L, 0.5, 0.5, 1, layout="int8")
    lat = np.zeros((L, L), dtype=np.uint8)
    lat[:, 0::2] = 1
    s.set_lattice(lat, 0)
    assert s.cluster_hist(1) == [(L, L // 2)]
    assert s.cluster_hist(0) == [(L, L // 2)]
    s.close()


def test_batch_cluster_hists_with_some_replicas_held():
    # replicas whose histogram is already held are left out of the labelling
    # launches; the others' result rows must still land on their own handles
    js = jobs()
    say(f"case batch histograms, {len(js)} replicas, two held beforehand")
    b = kk.Batch(js)
    b.run()
    held = {1: b.sim(1).cluster_hist(1), 5: b.sim(5).cluster_hist(1)}
    b.cluster_hists(1)
    for i in range(len(js)):
        s = b.sim(i)
        want = oracle.cluster_hist(s.get_lattice(), 1)
        assert s.cluster_hist(1) == want, i
        if i in held:
            assert held[i] == want, i
    b.close()


def test_batch_replica_with_more_large_clusters_than_the_first_copy():
    # the striped lattice of the single-handle case, as one replica of a batch
    # beside an ordinary one: its histogram takes the second copy
    L = 4160
    js = [wl.Job(L=L, composition=0.5, omega=0.5, seed=wl.job_seed(92, 0), sweeps=1, layout="int8"),
          wl.Job(L=96, composition=0.4, omega=0.7, seed=wl.job_seed(92, 1), sweeps=3, layout="int8")]
    say(f"case batch with a striped {L}^2 replica")
    b = kk.Batch(js)
    b.run()
    lat = np.zeros((L, L), dtype=np.uint8)
    lat[:, 0::2] = 1
    b.sim(0).set_lattice(lat, 1)
    for species in (1, 0):
        b.cluster_hists(species)
        assert b.sim(0).cluster_hist(species) == [(L, L // 2)]
        s = b.sim(1)
        assert s.cluster_hist(species) == oracle.cluster_hist(s.get_lattice(), species)
    b.close()
