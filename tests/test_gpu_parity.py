"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is bit-exact: lattice, accepted-move count, N_AB and the
cluster histogram.  The decomposition is conflict-free, so the result does
not depend on tiling, and the counter-based random numbers make a run
independent of how its sweeps are split across calls."""
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


def run_pair(L, x, w, seed, nsweeps, layout="auto", tile=None):
    say(f"case L={L} x={x} omega={w} seed={seed:#x} sweeps={nsweeps} layout={layout} tile={tile}")
    sim = kk.Sim(L, x, w, seed, layout=layout)
    if tile is not None:
        sim.set_tile(*tile)
    ref = oracle.init(L, x, seed)
    assert np.array_equal(sim.get_lattice(), ref), "initial placement differs"
    acc_ref = oracle.sweeps(ref, w, seed, 0, nsweeps) if nsweeps else 0
    if nsweeps:
        sim.sweep(nsweeps)
    got = sim.get_lattice()
    return sim, got, ref, acc_ref


def check_all(sim, got, ref, acc_ref, nsweeps):
    L = ref.shape[0]
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError(f"lattice differs at {len(bad)} sites, first {bad[:5].tolist()}")
    sweeps, attempts, accepted = sim.stats()
    assert sweeps == nsweeps and attempts == nsweeps * L * L
    assert accepted == acc_ref
    nab, e = sim.energy()
    assert nab == oracle.energy(ref)
    assert e == pytest.approx(sim.omega * nab)
    for sp in (0, 1):
        assert sim.cluster_hist(sp) == oracle.cluster_hist(ref, sp)


def test_small_64_config_bitexact():
    job = wl.small_64()
    for layout in ("int8", "bitpacked"):
        sim, got, ref, acc = run_pair(job.L, job.composition, job.omega, job.seed, job.sweeps, layout)
        check_all(sim, got, ref, acc, job.sweeps)
        assert sim.info() == (64, layout)
        sim.close()


@pytest.mark.parametrize("L", [4, 8, 12, 20, 28, 32, 36, 60, 64, 68, 96, 100, 132, 160, 260])
def test_sizes_and_wraps(L):
    sim, got, ref, acc = run_pair(L, 0.4, 0.7, 0xC0FFEE + L, 12, "int8")
    check_all(sim, got, ref, acc, 12)


@pytest.mark.parametrize("omega", [0.0, 0.3, 0.88, 1.2, 3.0, -0.7, -2.0, 1e-13, 40.0])
def test_omegas(omega):
    for layout in ("int8", "bitpacked"):
        sim, got, ref, acc = run_pair(96, 0.55, omega, 0xBEEF, 15, layout)
        check_all(sim, got, ref, acc, 15)


@pytest.mark.parametrize("x", [0.0, 0.03, 0.3, 0.5, 0.7, 0.97, 1.0])
def test_compositions(x):
    sim, got, ref, acc = run_pair(64, x, 0.9, 0x5A5A, 10, "bitpacked")
    check_all(sim, got, ref, acc, 10)
    assert int(got.sum()) == oracle.n_ones(64, x)


@pytest.mark.parametrize("tile", [(0, 0, 1), (1, 16, 1), (2, 32, 2), (2, 64, 1), (4, 64, 2), (1, 2, 1),
                                  (8, 256, 2), (3, 40, 2)])
def test_tile_shapes_give_identical_results(tile):
    L = 128
    sim, got, ref, acc = run_pair(L, 0.5, 0.88, 0x7777, 9, "bitpacked", tile=tile)
    check_all(sim, got, ref, acc, 9)


def test_int8_and_bitpacked_agree():
    a = kk.Sim(224, 0.35, 1.1, 42, layout="int8")
    b = kk.Sim(224, 0.35, 1.1, 42, layout="bitpacked")
    a.sweep(40)
    b.sweep(40)
    assert np.array_equal(a.get_lattice(), b.get_lattice())
    assert a.stats() == b.stats()


def test_split_sweeps_and_resume_are_exact():
    L, seed = 160, 99
    a = kk.Sim(L, 0.5, 0.6, seed, layout="bitpacked")
    a.sweep(30)
    b = kk.Sim(L, 0.5, 0.6, seed, layout="bitpacked")
    b.sweep(7)
    b.sweep(23)
    assert np.array_equal(a.get_lattice(), b.get_lattice())
    # checkpoint after 30, resume in a fresh handle, continue to 50
    snap = a.get_lattice()
    a.sweep(20)
    c = kk.Sim(L, 0.1, 0.6, seed, layout="int8")   # composition is overwritten by the checkpoint
    c.set_lattice(snap, 30)
    c.sweep(20)
    assert np.array_equal(a.get_lattice(), c.get_lattice())
    assert c.stats()[0] == 50


def test_set_lattice_roundtrip_and_validation():
    s = wl.random_lattice(64, 0.3, 5)
    sim = kk.Sim(64, 0.5, 0.5, 1, layout="bitpacked")
    sim.set_lattice(s, 123)
    assert np.array_equal(sim.get_lattice(), s)
    assert sim.stats()[0] == 123
    ref = s.copy()
    acc = oracle.sweeps(ref, 0.5, 1, 123, 5)
    sim.sweep(5)
    assert np.array_equal(sim.get_lattice(), ref)
    bad = s.copy()
    bad[0, 0] = 2
    with pytest.raises(kk.KKError):
        sim.set_lattice(bad)


def test_thresholds_match_oracle():
    for w in (0.0, 0.2, 0.5, 0.88, 1.4, -0.3, 1e-13):
        sim = kk.Sim(32, 0.5, w, 3)
        assert list(sim.thresholds()) == list(oracle.thresholds(w))
        sim.close()


def test_segregated_start_relaxes_identically():
    L = 128
    s = wl.segregated_lattice(L, 0.5)
    sim = kk.Sim(L, 0.5, 0.9, 11, layout="bitpacked")
    sim.set_lattice(s, 0)
    ref = s.copy()
    for chunk in (1, 2, 5, 10, 20):
        acc_ref = oracle.sweeps(ref, 0.9, 11, sim.stats()[0], chunk)
        sim.sweep(chunk)
        assert np.array_equal(sim.get_lattice(), ref)
