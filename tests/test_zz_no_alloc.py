"""GPU: kk_sweep_noalloc (sweeps of a caller-held device lattice, no
allocation) against kk_sweep on a handle holding the same lattice at the same
sweep counter: lattice and accepted count bit for bit, over several calls in a
row with successively smaller inputs (each call reuses the scratch array the
previous one left behind), on both layouts, the tiled and the resident
kernels and both parities of the launch count."""
import sys

import numpy as np
import pytest
import torch

from paper_1309_4349_amd import kk
from paper_1309_4349_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _to_device(s, layout):
    if layout == "int8":
        return torch.from_numpy(np.ascontiguousarray(s, dtype=np.uint8)).cuda()
    # bit b of word g of a row holds site 32 g + b
    words = np.packbits(s, axis=1, bitorder="little").view("<u4")
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int32)).cuda()


def _from_device(buf, L, layout):
    a = buf.cpu().numpy()
    if layout == "int8":
        return a.reshape(L, L).astype(np.uint8)
    return np.unpackbits(np.ascontiguousarray(a).view(np.uint8).reshape(L, L // 8), axis=1,
                         bitorder="little").astype(np.uint8)


# successively smaller lattices: tiled halo kernel (odd and even launch
# counts), then the whole-lattice resident kernel (one launch, then two)
CASES = [(1024, "bitpacked", 0.88, 0xA11, 9), (400, "int8", 0.6, 0xA12, 6), (128, "bitpacked", 1.2, 0xA13, 3),
         (64, "int8", 0.5, 0xA14, 300)]


def _reference(L, layout, w, seed, s0, t0, n):
    ref = kk.Sim(L, 0.5, w, seed, layout=layout)
    ref.set_lattice(s0, t0)
    a0 = ref.stats()[2]
    ref.sweep(n)
    out = ref.get_lattice(), ref.stats()[2] - a0
    ref.close()
    return out


def test_noalloc_matches_kk_sweep_on_calls_in_a_row():
    torch.cuda.set_device(0)
    side = torch.cuda.Stream()
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    for i, (L, layout, w, seed, n) in enumerate(CASES):
        t0 = 17 + i
        say(f"case noalloc L={L} layout={layout} omega={w} sweeps={n} t0={t0}")
        s0 = wl.random_lattice(L, 0.45, seed)
        want, want_acc = _reference(L, layout, w, seed, s0, t0, n)
        buf = _to_device(s0, layout)
        acc.zero_()
        torch.cuda.synchronize()
        stream = side if i % 2 else torch.cuda.current_stream()
        kk.sweep_noalloc(buf.data_ptr(), L, layout, w, seed, t0, n, acc.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        got = _from_device(buf, L, layout)
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            raise AssertionError(f"L={L}: lattice differs at {len(bad)} sites, first {bad[:5].tolist()}")
        assert int(acc.item()) == want_acc
        assert int(got.sum()) == int(s0.sum())


def test_noalloc_repeat_accumulates_and_splits_exactly():
    # two calls that split a run equal one call; the count accumulates
    torch.cuda.set_device(0)
    L, layout, w, seed = 256, "bitpacked", 0.7, 0xA15
    say(f"case noalloc split L={L}")
    s0 = wl.random_lattice(L, 0.5, seed)
    want, want_acc = _reference(L, layout, w, seed, s0, 5, 7)
    buf = _to_device(s0, layout)
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    kk.sweep_noalloc(buf.data_ptr(), L, layout, w, seed, 5, 4, acc.data_ptr())
    kk.sweep_noalloc(buf.data_ptr(), L, layout, w, seed, 9, 3, acc.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(_from_device(buf, L, layout), want)
    assert int(acc.item()) == want_acc


def test_noalloc_refuses_what_does_not_fit():
    torch.cuda.set_device(0)
    say("case noalloc limits")
    big = torch.zeros(4096 * 4096, dtype=torch.uint8, device="cuda")   # 16 MiB int8: beyond the scratch
    with pytest.raises(kk.KKError):
        kk.sweep_noalloc(big.data_ptr(), 4096, "int8", 0.5, 1, 0, 1)
    with pytest.raises(kk.KKError):
        kk.sweep_noalloc(big.data_ptr(), 100, "bitpacked", 0.5, 1, 0, 1)   # bit-packed needs L % 32 == 0
    with pytest.raises(kk.KKError):
        kk.sweep_noalloc(0, 64, "int8", 0.5, 1, 0, 1)
    with pytest.raises(kk.KKError):
        kk.sweep_noalloc(big.data_ptr(), 64, "int8", 0.5, 1, (1 << 60) - 2, 2)
    torch.cuda.synchronize()
    assert int(big.sum().item()) == 0   # nothing ran
