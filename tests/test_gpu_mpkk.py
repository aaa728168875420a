"""GPU: the paper's literal MPKK (7-site domain cover, synchronous
iterations) and the conflict-free schedule on rectangular helical rings equal
the oracle bit for bit -- lattice, accepted exchanges, N_AB, cluster
histograms and observables -- including the smallest covers (3 x 7, 5 x 7),
ragged grids and a segregated restart."""
import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _check(s, ref, w, seed, n, sweeps_fn):
    acc = sweeps_fn(ref, w, seed, 0, n)
    s.sweep(n)
    H, L = ref.shape
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (n, n * L * H, acc)
    assert s.energy()[0] == oracle.tri_energy(ref)
    for species in (0, 1):
        assert s.cluster_hist(species) == oracle.tri_cluster_hist(ref, species)
        got = s.observe(species)
        for k, v in oracle.tri_observables(ref, w, species, seed, n).items():
            assert got[k] == v, (species, k, got[k], v)


@pytest.mark.parametrize("L,H,x,w,n", [
    (10, 7, 0.5, 1.0, 12), (3, 7, 0.4, 0.5, 9), (5, 7, 0.6, 0.8, 10), (12, 14, 0.3, 0.6, 20),
    (52, 56, 0.5, 0.5, 15), (404, 420, 0.5, 0.55, 5), (17, 63, 0.2, -0.4, 7), (24, 35, 0.5, 0.0, 6),
])
def test_mpkk_matches_oracle(L, H, x, w, n):
    print(f"case mpkk {L}x{H} x={x} w={w} n={n}", flush=True)
    seed = wl.job_seed(61, L * 1000 + H)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    ref = oracle.init_rect(L, H, x, seed)
    assert np.array_equal(s.get_lattice(), ref)
    assert np.array_equal(s.thresholds(), oracle.tri_thresholds(w))
    _check(s, ref, w, seed, n, oracle.mpkk_steps)
    s.close()


@pytest.mark.parametrize("L,H,x,w,n", [
    (12, 8, 0.5, 0.9, 10), (20, 28, 0.4, 0.6, 8), (44, 100, 0.5, 1.1, 6), (4, 12, 0.5, 0.3, 9),
])
def test_rectangular_classes_match_oracle(L, H, x, w, n):
    print(f"case classes {L}x{H} x={x}", flush=True)
    seed = wl.job_seed(62, L * 1000 + H)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H)
    ref = oracle.init_rect(L, H, x, seed)
    assert np.array_equal(s.get_lattice(), ref)
    _check(s, ref, w, seed, n, oracle.tri_sweeps)
    s.close()


def test_mpkk_segregated_restart_and_resume():
    L, H, x, w, seed = 52, 56, 0.45, 0.7, 31
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    s.sweep(3)
    s.restart("segregated")
    ref = oracle.init_segregated(L, x, H)
    assert np.array_equal(s.get_lattice(), ref)
    oracle.mpkk_steps(ref, w, seed, 0, 9)
    s.sweep(4)
    snap = s.get_lattice()
    s.sweep(5)
    assert np.array_equal(s.get_lattice(), ref)
    b = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    b.set_lattice(snap, 4)
    b.sweep(5)
    assert np.array_equal(b.get_lattice(), ref)
    s.close()
    b.close()


def test_invalid_shapes_are_rejected():
    for L, H, scheme in ((11, 7, "mpkk"), (10, 8, "mpkk"), (12, 6, "classes"), (8, 8, "classes"), (10, 0, "mpkk")):
        with pytest.raises(kk.KKError):
            kk.Sim(L, 0.5, 1.0, 1, geometry="triangular", rows=H, scheme=scheme)


def test_mpkk_full_size_4098x4095():
    # the benchmarked configuration: 4098 x 4095 ring, x = 0.5, omega = 0.88
    L, H, x, w, seed = 4098, 4095, 0.5, 0.88, 0x13094349
    print("case mpkk full size 4098x4095", flush=True)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    ref = oracle.init_rect(L, H, x, seed)
    assert np.array_equal(s.get_lattice(), ref)
    acc = oracle.mpkk_steps(ref, w, seed, 0, 2)
    s.sweep(2)
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (2, 2 * L * H, acc)
    s.sweep(48)
    got = s.get_lattice()
    assert int(got.sum()) == oracle.n_ones_rect(L, H, x)
    assert s.energy()[0] == oracle.tri_energy(got)
    s.close()


@pytest.mark.parametrize("L,H,tile,x,w,n", [
    (66, 70, (16, 16), 0.5, 0.8, 4), (80, 63, (30, 17), 0.45, 1.2, 5), (101, 84, (40, 20), 0.5, 0.5, 3),
    (404, 420, (128, 96), 0.3, -0.6, 3), (234, 238, (192, 192), 0.5, 0.0, 2),
    # N/7 odd: the ring end breaks the pairing of consecutive domains in one window row
    (59, 63, (17, 21), 0.5, 0.9, 4), (73, 77, (31, 35), 0.4, 1.0, 3), (409, 413, (96, 96), 0.5, 0.7, 3),
])
def test_mpkk_whole_step_tiles_match_oracle(L, H, tile, x, w, n):
    # one launch per step on LDS windows (flip marks keep each iteration synchronous)
    print(f"case mpkk tiles {L}x{H} tile={tile}", flush=True)
    seed = wl.job_seed(63, L * 1000 + H)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H, scheme="mpkk")
    s.tri_set_tile(*tile)
    assert s.tri_get_tile() == tile
    ref = oracle.init_rect(L, H, x, seed)
    acc = oracle.mpkk_steps(ref, w, seed, 0, n)
    ms, launches = s.sweep_timed(n)
    assert launches == n
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (n, n * L * H, acc)
    assert s.cluster_hist(0) == oracle.tri_cluster_hist(ref, 0)
    s.tri_set_tile(0)       # back to one launch per iteration mid-run
    s.sweep(2)
    oracle.mpkk_steps(ref, w, seed, n, 2)
    assert np.array_equal(s.get_lattice(), ref)
    s.close()
