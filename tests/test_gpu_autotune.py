"""GPU: the tile autotuner leaves the simulation exactly where it was, keeps
the fastest tile on the handle and hands it to later handles of the same
shape; sweeps after tuning still match the oracle bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1309_4349_amd import kk

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,layout", [(132, "int8"), (256, "bitpacked"), (608, "bitpacked")])
def test_autotune_restores_state_and_caches(L, layout):
    print(f"case autotune L={L} {layout}", flush=True)
    x, w, seed = 0.4, 0.9, 4242 + L
    s = kk.Sim(L, x, w, seed, layout=layout)
    s.sweep(7)
    lat0, st0, e0 = s.get_lattice(), s.stats(), s.energy()
    words, rows, ku, us = s.autotune(4)
    assert us > 0
    assert np.array_equal(s.get_lattice(), lat0)
    assert s.stats() == st0 and s.energy() == e0
    assert s.get_tile() == (words, rows, ku)
    s.sweep(9)
    ref = oracle.init(L, x, seed)
    acc = oracle.sweeps(ref, w, seed, 0, 16)
    assert np.array_equal(s.get_lattice(), ref)
    assert s.stats() == (16, 16 * L * L, acc)
    s2 = kk.Sim(L, 0.5, 0.3, 1, layout=layout)
    assert s2.get_tile() == (words, rows, ku)
    s2.close()
    s.close()
