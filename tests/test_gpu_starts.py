"""GPU: the segregated (non-random) start equals the oracle's bit for bit on
both geometries and layouts, restarting reproduces a fresh handle, and the
average cluster size does not depend on the starting condition (Results,
"Cluster Analysis", Figs. 10-11)."""
import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("geometry,L,layout,x,w,n", [
    ("square", 64, "bitpacked", 0.5, 0.9, 12), ("square", 100, "int8", 0.3, 0.6, 9),
    ("square", 96, "bitpacked", 0.37, 1.1, 7), ("square", 36, "int8", 1.0, 0.5, 2),
    ("triangular", 20, "int8", 0.5, 0.8, 10), ("triangular", 100, "int8", 0.41, 0.4, 6),
])
def test_segregated_start_matches_oracle(geometry, L, layout, x, w, n):
    print(f"case segregated {geometry} L={L} {layout} x={x}", flush=True)
    seed = wl.job_seed(51, L)
    s = kk.Sim(L, x, w, seed, layout=layout, geometry=geometry)
    s.sweep(3)
    s.restart("segregated")
    ref = oracle.init_segregated(L, x)
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (0, 0, 0)
    acc = (oracle.sweeps if geometry == "square" else oracle.tri_sweeps)(ref, w, seed, 0, n)
    s.sweep(n)
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (n, n * L * L, acc)
    energy = oracle.energy if geometry == "square" else oracle.tri_energy
    assert s.energy()[0] == energy(ref)
    # back to the random start: the same as a fresh handle
    s.restart("random")
    f = kk.Sim(L, x, w, seed, layout=layout, geometry=geometry)
    assert np.array_equal(s.get_lattice(), f.get_lattice())
    s.sweep(4)
    f.sweep(4)
    assert np.array_equal(s.get_lattice(), f.get_lattice()) and s.stats() == f.stats()
    s.close()
    f.close()


def _batch_means(v, nb=10):
    b = np.asarray(v[: len(v) // nb * nb]).reshape(nb, -1).mean(1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nb)


@pytest.mark.parametrize("geometry,omega", [("square", 0.6), ("triangular", 0.4)])
def test_average_cluster_size_does_not_depend_on_start(geometry, omega):
    # 100 x 100, x = 0.5, below the demixing point of each lattice; after a
    # burn-in the weight- and number-average cluster sizes of runs from the two
    # starts agree within 5 combined batch-means standard errors
    L, x = 100, 0.5
    out = {}
    for start in ("random", "segregated"):
        s = kk.Sim(L, x, omega, 2024, layout="int8", geometry=geometry)
        s.restart(start)
        s.sweep(20000)
        ser = s.series(every=25, count=400, species=1)
        out[start] = ser
        s.close()
    for key in ("size_weight_avg", "size_number_avg", "similar_exact"):
        ma, sa = _batch_means([r[key] for r in out["random"]])
        mb, sb = _batch_means([r[key] for r in out["segregated"]])
        print(f"{geometry} {key}: random {ma:.4f} +- {sa:.4f}, segregated {mb:.4f} +- {sb:.4f}", flush=True)
        assert abs(ma - mb) < 5 * np.hypot(sa, sb) + 1e-12, (key, ma, sa, mb, sb)
