"""GPU: the triangular lattice with helical boundaries (the paper's model)
equals the oracle bit for bit -- lattice, accepted exchanges, N_AB, cluster
histograms of both species and the observables -- over sizes from one site
per class (L = 4) to many blocks with a ragged last one; runs resume exactly."""
import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,x,w,n", [
    (4, 0.5, 0.4, 9), (12, 0.3, 1.1, 20), (20, 0.5, 0.8, 15), (100, 0.4, 1.0, 12),
    (204, 0.5, 0.6, 6), (36, 0.0, 1.0, 3), (28, 1.0, 1.0, 3), (60, 0.5, -0.7, 8), (44, 0.5, 0.0, 5),
])
def test_tri_sweeps_match_oracle(L, x, w, n):
    print(f"case tri L={L} x={x} w={w} n={n}", flush=True)
    seed = wl.job_seed(41, L)
    s = kk.Sim(L, x, w, seed, geometry="triangular")
    ref = oracle.init(L, x, seed)
    assert np.array_equal(s.get_lattice(), ref)
    acc = oracle.tri_sweeps(ref, w, seed, 0, n)
    s.sweep(n)
    assert np.array_equal(s.get_lattice(), ref)
    sw, att, got_acc = s.stats()
    assert (sw, att, got_acc) == (n, n * L * L, acc)
    assert s.energy()[0] == oracle.tri_energy(ref)
    for species in (0, 1):
        assert s.cluster_hist(species) == oracle.tri_cluster_hist(ref, species)
        got = s.observe(species)
        want = oracle.tri_observables(ref, w, species, seed, n)
        for k, v in want.items():
            assert got[k] == v, (species, k, got[k], v)
    assert np.array_equal(s.thresholds(), oracle.tri_thresholds(w))
    s.close()


def test_tri_resume_and_series():
    L, x, w, seed = 52, 0.45, 0.9, 123
    a = kk.Sim(L, x, w, seed, geometry="triangular")
    a.sweep(7)
    snap = a.get_lattice()
    a.sweep(11)
    b = kk.Sim(L, x, w, seed + 1, geometry="triangular")
    b.close()
    b = kk.Sim(L, x, w, seed, geometry="triangular")
    b.set_lattice(snap, 7)
    b.sweep(11)
    assert np.array_equal(a.get_lattice(), b.get_lattice())
    c = kk.Sim(L, x, w, seed, geometry="triangular")
    ser = c.series(every=6, count=3, species=1)
    d = kk.Sim(L, x, w, seed, geometry="triangular")
    for i in range(3):
        d.sweep(6)
        assert ser[i] == d.observe(1), i
    for h in (a, b, c, d):
        h.close()


def test_tri_large_sampled_sites():
    # a large ring: whole-lattice invariants plus a sampled recount of N_AB
    L, x, w, seed = 1028, 0.5, 1.0, 99
    s = kk.Sim(L, x, w, seed, geometry="triangular")
    ref = oracle.init(L, x, seed)
    oracle.tri_sweeps(ref, w, seed, 0, 4)
    s.sweep(4)
    got = s.get_lattice()
    assert np.array_equal(got, ref)
    assert int(got.sum()) == oracle.n_ones(L, x)
    assert s.energy()[0] == oracle.tri_energy(ref)
    s.close()


def test_tri_rejects_square_only_calls():
    s = kk.Sim(12, 0.5, 1.0, 1, geometry="triangular")
    for call in (lambda: s.get_tile(), lambda: s.set_tile(8, 64, 1), lambda: s.autotune(2)):
        with pytest.raises(kk.KKError):
            call()
    s.close()
    for L in (8, 16, 0, 6):
        with pytest.raises(kk.KKError):
            kk.Sim(L, 0.5, 1.0, 1, geometry="triangular")


@pytest.mark.parametrize("L,H,tile,x,w,n", [
    (100, 100, (16, 16), 0.5, 0.8, 7), (124, 84, (40, 18), 0.45, 1.2, 5), (204, 204, (128, 128), 0.5, 0.6, 6),
    (404, 412, (256, 256), 0.3, 0.9, 4), (404, 404, (96, 160), 0.5, -0.5, 5), (132, 200, (66, 134), 0.5, 0.0, 3),
])
def test_tri_whole_sweep_tiles_match_oracle(L, H, tile, x, w, n):
    # one launch per sweep on LDS windows: ragged tiles, rectangles, windows across row ends
    print(f"case tri tiles L={L} H={H} tile={tile}", flush=True)
    seed = wl.job_seed(43, L * 1000 + H)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H)
    s.tri_set_tile(*tile)
    assert s.tri_get_tile() == tile
    ref = oracle.init_rect(L, H, x, seed)
    acc = oracle.tri_sweeps(ref, w, seed, 0, n)
    ms, launches = s.sweep_timed(n)
    assert launches == n
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (n, n * L * H, acc)
    assert s.energy()[0] == oracle.tri_energy(ref)
    assert s.cluster_hist(1) == oracle.tri_cluster_hist(ref, 1)
    # switching to one launch per class mid-run continues the same chain
    s.tri_set_tile(0)
    s.sweep(2)
    oracle.tri_sweeps(ref, w, seed, n, 2)
    assert np.array_equal(s.get_lattice(), ref)
    s.close()


def test_tri_default_tiles_and_rejections():
    s = kk.Sim(4092, 0.5, 0.88, 5, geometry="triangular")
    assert s.tri_get_tile() == (256, 256)
    assert kk.Sim(1028, 0.5, 0.88, 5, geometry="triangular").tri_get_tile() == (61, 69)   # 17 x 15 tiles
    for bad in ((15, 64), (64, 15), (4092, 64), (400, 400)):
        with pytest.raises(kk.KKError):
            s.tri_set_tile(*bad)
    s.close()
    assert kk.Sim(100, 0.5, 1.0, 1, geometry="triangular").tri_get_tile() == (100, 100)   # the whole ring
    assert kk.Sim(148, 0.5, 1.0, 1, geometry="triangular").tri_get_tile() == (16, 16)
    assert kk.Sim(76, 0.5, 1.0, 1, geometry="triangular").tri_get_tile() == (76, 76)
    assert kk.Sim(76, 0.5, 1.0, 1, geometry="triangular", rows=2400).tri_get_tile() == (0, 0)   # no tile fits
    m = kk.Sim(10, 0.5, 1.0, 1, geometry="triangular", rows=7, scheme="mpkk")
    with pytest.raises(kk.KKError):
        m.tri_set_tile(16, 16)
    m.close()


def test_tri_full_size_4092():
    # the benchmarked configuration: 4092^2, x = 0.5, omega = 0.88, default 256 x 256 tiles
    L, x, w, seed = 4092, 0.5, 0.88, 0x13094349
    print("case tri full size 4092", flush=True)
    s = kk.Sim(L, x, w, seed, geometry="triangular")
    assert s.tri_get_tile() == (256, 256)
    ref = oracle.init(L, x, seed)
    assert np.array_equal(s.get_lattice(), ref)
    acc = oracle.tri_sweeps(ref, w, seed, 0, 3)
    s.sweep(3)
    got = s.get_lattice()
    assert np.array_equal(got, ref)
    assert s.stats() == (3, 3 * L * L, acc)
    # a longer run: composition, N_AB recount, histogram sum rule, resume
    s.sweep(197)
    got = s.get_lattice()
    assert int(got.sum()) == oracle.n_ones(L, x)
    assert s.energy()[0] == oracle.tri_energy(got)
    h = s.cluster_hist(1)
    assert sum(k * c for k, c in h) == oracle.n_ones(L, x)
    b = kk.Sim(L, x, w, seed, geometry="triangular")
    b.set_lattice(got, 200)
    s.sweep(5)
    b.sweep(5)
    assert np.array_equal(s.get_lattice(), b.get_lattice())
    s.close()
    b.close()


@pytest.mark.parametrize("L,H,scheme", [(404, 404, "classes"), (404, 420, "mpkk"), (76, 84, "classes")])
def test_tri_autotune_restores_state_and_keeps_results(L, H, scheme):
    seed = wl.job_seed(44, L * 1000 + H)
    s = kk.Sim(L, 0.5, 0.7, seed, geometry="triangular", rows=H, scheme=scheme)
    s.sweep(3)
    before = (s.get_lattice(), s.stats())
    cols, rows, us = s.tri_autotune(4)
    assert us > 0 and (cols, rows) == s.tri_get_tile()
    assert np.array_equal(s.get_lattice(), before[0]) and s.stats() == before[1]
    ref = oracle.init_rect(L, H, 0.5, seed)
    run = oracle.tri_sweeps if scheme == "classes" else oracle.mpkk_steps
    acc = run(ref, 0.7, seed, 0, 7)
    s.sweep(4)
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (7, 7 * L * H, acc)
    s.close()
    with pytest.raises(kk.KKError):
        kk.Sim(64, 0.5, 0.7, 1).tri_autotune(2)


@pytest.mark.parametrize("L,H,scheme", [(1028, 1028, "classes"), (1027, 1029, "mpkk")])
def test_tri_autotune_never_loses_to_the_default_tile(L, H, scheme):
    # the default tile (here a grid-cut rectangle) is one of the timed candidates,
    # so the tuned tile is never measurably slower than it
    print(f"case tri autotune vs default {L}x{H} {scheme}", flush=True)
    s = kk.Sim(L, 0.5, 0.88, 5, geometry="triangular", rows=H, scheme=scheme)
    default = s.tri_get_tile()
    assert default[0] != default[1] or default[0] not in (320, 256, 192, 160, 128, 96, 64, 48, 32, 16)
    s.sweep(5)
    ms_def, n_def = s.sweep_timed(60)
    cols, rows, us = s.tri_autotune(20)
    ms_tuned, n_tuned = s.sweep_timed(60)
    assert ms_tuned <= 1.25 * ms_def, ((cols, rows, ms_tuned), (default, ms_def))
    s.close()


def test_runner_series_and_resume(tmp_path):
    import io
    import json

    from paper_1309_4349_amd import run
    lat = tmp_path / "lat.npy"
    hist = tmp_path / "hist.json"
    buf = io.StringIO()
    args = run.parse(["--geometry", "triangular", "--L", "100", "--x", "0.4", "--omega", "0.9", "--seed", "17",
                      "--sweeps", "25", "--every", "10", "--start", "segregated", "--lattice-out", str(lat),
                      "--hist-out", str(hist)])
    recs = run.run(args, out=buf)
    assert [r["sweep"] for r in recs] == [10, 20, 25]
    assert [json.loads(x)["sweep"] for x in buf.getvalue().splitlines()] == [10, 20, 25]
    ref = oracle.init_segregated(100, 0.4)
    oracle.tri_sweeps(ref, 0.9, 17, 0, 25)
    assert np.array_equal(np.load(lat), ref)
    assert [tuple(e) for e in json.load(open(hist))] == oracle.tri_cluster_hist(ref, 1)
    for k, v in oracle.tri_observables(ref, 0.9, 1, 17, 25).items():
        assert recs[-1][k] == v
    # resume for 5 more sweeps
    recs2 = run.run(run.parse(["--geometry", "triangular", "--L", "100", "--x", "0.4", "--omega", "0.9", "--seed",
                               "17", "--sweeps", "5", "--every", "5", "--resume", str(lat), "--resume-sweep", "25"]),
                    out=io.StringIO())
    oracle.tri_sweeps(ref, 0.9, 17, 25, 5)
    assert recs2[-1]["sweep"] == 30 and recs2[-1]["n_unlike"] == oracle.tri_energy(ref)


@pytest.mark.parametrize("L,H,x,w,n", [(100, 100, 0.5, 0.9, 12), (204, 204, 0.4, 0.6, 5), (300, 124, 0.5, -0.3, 4),
                                       (28, 20, 0.5, 1.0, 1030), (12, 12, 0.5, 0.4, 3)])
def test_tri_whole_ring_matches_oracle(L, H, x, w, n):
    # the whole ring in one workgroup, up to 1024 sweeps per launch
    print(f"case tri whole ring {L}x{H} n={n}", flush=True)
    seed = wl.job_seed(45, L * 1000 + H)
    s = kk.Sim(L, x, w, seed, geometry="triangular", rows=H)
    s.tri_set_tile(L, H)
    assert s.tri_get_tile() == (L, H)
    ref = oracle.init_rect(L, H, x, seed)
    acc = oracle.tri_sweeps(ref, w, seed, 0, n)
    ms, launches = s.sweep_timed(n)
    assert launches == (n + 1023) // 1024
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (n, n * L * H, acc)
    s.tri_set_tile(0)
    s.sweep(2)
    oracle.tri_sweeps(ref, w, seed, n, 2)
    assert np.array_equal(s.get_lattice(), ref)
    s.close()
    with pytest.raises(kk.KKError):
        kk.Sim(404, 0.5, 0.5, 1, geometry="triangular").tri_set_tile(404, 404)   # 163,216 B: too large
