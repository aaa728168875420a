"""GPU parity across the 32-bit boundary of the sweep counter.

Every Philox counter carries the sweep's low 32 bits in one word and its next
28 bits in the fourth word beside the stream tag, so sweeps at t >= 2^32 are
the first to put a non-zero high part there.  Each case resumes at
t = 2^32 - 3 and runs 6 sweeps (or MPKK steps) across the boundary, on every
kernel family, against the oracle bit for bit.  The last case checks that the
library refuses a run that would carry the counter to 2^60."""
import sys

import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu

T0 = (1 << 32) - 3
N = 6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _square(L, x, w, seed, layout, tile=None):
    say(f"case square L={L} layout={layout} tile={tile} t0=2^32-3")
    s0 = wl.random_lattice(L, x, seed)
    sim = kk.Sim(L, 0.5, w, seed, layout=layout)
    if tile is not None:
        sim.set_tile(*tile)
    sim.set_lattice(s0, T0)
    ref = s0.copy()
    acc = oracle.sweeps(ref, w, seed, T0, N)
    # split across the boundary so that one call ends just before it
    sim.sweep(2)
    sim.sweep(N - 2)
    assert np.array_equal(sim.get_lattice(), ref)
    assert sim.stats()[0] == T0 + N
    assert sim.stats()[2] == acc
    assert sim.energy()[0] == oracle.energy(ref)
    assert sim.cluster_hist(1) == oracle.cluster_hist(ref, 1)
    got = sim.observe(1)
    for k, v in oracle.observables(ref, w, 1, seed, T0 + N).items():
        assert got[k] == v, (k, got[k], v)
    sim.close()


@pytest.mark.parametrize("layout", ["int8", "bitpacked"])
def test_square_resident_across_2_32(layout):
    _square(64, 0.5, 0.7, 0xB0DA + 1, layout)


@pytest.mark.parametrize("layout,tile", [("int8", (2, 16, 2)), ("bitpacked", (2, 32, 2)),
                                         ("bitpacked", (1, 16, 1))])
def test_square_tiles_across_2_32(layout, tile):
    _square(128, 0.45, 0.9, 0xB0DA + 2, layout, tile)


def test_square_default_tile_large_across_2_32():
    _square(1024, 0.5, 0.88, 0xB0DA + 3, "bitpacked")


def _ring(L, H, scheme, tile, w, seed):
    say(f"case {scheme} {L}x{H} tile={tile} t0=2^32-3")
    s0 = oracle.init_rect(L, H, 0.5, seed)
    sim = kk.Sim(L, 0.5, w, seed, geometry="triangular", rows=H, scheme=scheme)
    if tile is not None:
        sim.tri_set_tile(*tile)
    sim.set_lattice(s0, T0)
    ref = s0.copy()
    fn = oracle.mpkk_steps if scheme == "mpkk" else oracle.tri_sweeps
    acc = fn(ref, w, seed, T0, N)
    sim.sweep(3)
    sim.sweep(N - 3)
    assert np.array_equal(sim.get_lattice(), ref)
    assert sim.stats()[0] == T0 + N
    assert sim.stats()[2] == acc
    assert sim.energy()[0] == oracle.tri_energy(ref)
    assert sim.cluster_hist(1) == oracle.tri_cluster_hist(ref, 1)
    got = sim.observe(1)
    for k, v in oracle.tri_observables(ref, w, 1, seed, T0 + N).items():
        assert got[k] == v, (k, got[k], v)
    sim.close()


@pytest.mark.parametrize("L,H,tile", [(100, 100, None), (100, 100, (0, 0)), (204, 204, (64, 64))])
def test_triangular_across_2_32(L, H, tile):
    _ring(L, H, "classes", tile, 0.6, 0xB0DA + 4)


@pytest.mark.parametrize("tile", [None, (0, 0), (48, 40)])
def test_mpkk_across_2_32(tile):
    _ring(122, 126, "mpkk", tile, 0.5, 0xB0DA + 5)


def test_counter_limit_refused():
    say("case counter limit 2^60")
    lim = 1 << 60
    for geometry in ("square", "triangular"):
        L = 64 if geometry == "square" else 68
        s0 = wl.random_lattice(L, 0.5, 3)
        sim = kk.Sim(L, 0.5, 0.5, 3, geometry=geometry)
        with pytest.raises(kk.KKError):
            sim.set_lattice(s0, lim)
        sim.set_lattice(s0, lim - 3)
        ref = s0.copy()
        sim.sweep(2)                        # t: 2^60 - 3 -> 2^60 - 1, still a valid resume point
        with pytest.raises(kk.KKError):
            sim.sweep(1)                    # would leave the counter at 2^60
        with pytest.raises(kk.KKError):
            sim.sweep_async(5)
        with pytest.raises(kk.KKError):
            sim.series(1, 1)
        assert sim.stats()[0] == lim - 1    # the refused calls ran nothing
        if geometry == "square":
            oracle.sweeps(ref, 0.5, 3, lim - 3, 2)
        else:
            oracle.tri_sweeps(ref, 0.5, 3, lim - 3, 2)
        assert np.array_equal(sim.get_lattice(), ref)
        sim.sweep(0)
        sim.close()
