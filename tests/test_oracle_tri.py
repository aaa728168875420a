"""Pins of the oracle's triangular lattice with helical boundaries (the
paper's own model): every check here is independent of the oracle's code --
numpy recounts over a rolled flat array, brute-force conflict checks, exact
Boltzmann sums by enumeration, closed forms, and a pure-Python BFS."""
import math
from itertools import combinations

import numpy as np
import pytest

OFFS = lambda L: (1, -1, L, -L, L - 1, -(L - 1))  # noqa: E731  (d = 0..5)


def nb(i, d, L, H=None):
    return (i + OFFS(L)[d]) % (L * (H or L))


def np_energy(s):
    L = s.shape[1]
    f = s.ravel()
    return int(sum(np.count_nonzero(f != np.roll(f, -k)) for k in (1, L, L - 1)))


def test_energy_matches_a_rolled_recount(orc):
    for L, x, seed in ((4, 0.5, 1), (12, 0.3, 2), (20, 0.5, 3), (28, 0.7, 4)):
        s = orc.init(L, x, seed)
        assert orc.tri_energy(s) == np_energy(s)
    for L, H in ((12, 8), (10, 7), (5, 14)):
        s = orc.init_rect(L, H, 0.4, L + H)
        assert s.shape == (H, L) and int(s.sum()) == orc.n_ones_rect(L, H, 0.4)
        assert orc.tri_energy(s) == np_energy(s)
    z = np.zeros((12, 12), np.uint8)
    assert orc.tri_energy(z) == 0
    z[5, 5] = 1                       # one isolated site: all 6 bonds unlike
    assert orc.tri_energy(z) == 6


def _conflicts(L, H=None):
    H = H or L
    N = L * H
    hits = 0
    for c in range(16):
        centres = list(range(c, N, 16))
        for i1, i2 in combinations(centres, 2):
            for d1 in range(6):
                w1 = {i1, nb(i1, d1, L, H)}
                for d2 in range(6):
                    b2 = nb(i2, d2, L, H)
                    r2 = {i2, b2} | {nb(i2, d, L, H) for d in range(6)} | {nb(b2, d, L, H) for d in range(6)}
                    w2 = {i2, b2}
                    b1 = nb(i1, d1, L, H)
                    r1 = w1 | {nb(i1, d, L, H) for d in range(6)} | {nb(b1, d, L, H) for d in range(6)}
                    hits += bool(w1 & r2) or bool(w2 & r1)
    return hits


@pytest.mark.parametrize("L,H", [(12, 12), (20, 20), (12, 8), (20, 4), (4, 12)])
def test_classes_are_conflict_free_for_L_4_mod_8(L, H):
    assert _conflicts(L, H) == 0


@pytest.mark.parametrize("L,H", [(8, 8), (12, 6)])
def test_classes_conflict_for_other_sizes(L, H):
    # the negative controls: the pin has teeth
    assert _conflicts(L, H) > 0


def test_local_dnab_matches_a_full_recount(orc):
    rng = np.random.default_rng(5)
    for L in (4, 12, 20):
        s = orc.init(L, 0.5, L)
        for _ in range(60):
            i = int(rng.integers(L * L))
            d = int(rng.integers(6))
            b = nb(i, d, L)
            t = s.copy().ravel()
            t[i], t[b] = t[b], t[i]
            want = np_energy(t.reshape(L, L)) - np_energy(s) if s.ravel()[i] != s.ravel()[b] else 0
            assert orc.tri_local_dnab(s, i, d) == want


def test_thresholds_closed_form(orc):
    T = orc.tri_thresholds(math.log(2) / 2)   # exp(-omega (10 - 2n)) = 2^(n - 5)
    for n in range(11):
        want = 2 ** 32 if n >= 5 else 2 ** (32 + n - 5)
        assert abs(int(T[n]) - want) <= 1, n
    assert np.all(orc.tri_thresholds(0.0) == 2 ** 32)
    w = 0.83
    assert np.array_equal(orc.tri_thresholds(w)[::-1], orc.tri_thresholds(-w))
    assert np.all(np.diff(orc.tri_thresholds(1.1).astype(np.float64)) >= 0)


def test_directions_are_uniform_and_phase_orders_are_permutations(orc):
    cnt = np.zeros(6)
    for i in range(6000):
        cnt[orc.tri_site_randoms(9, 3, i)[0]] += 1
    chi2 = ((cnt - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 25.0    # 5 degrees of freedom, p ~ 1e-4
    first = np.zeros(16)
    for t in range(1600):
        p = orc.tri_phase_order(4, t)
        assert sorted(p) == list(range(16))
        first[p[0]] += 1
    assert ((first - 100.0) ** 2 / 100.0).sum() < 50.0   # 15 dof


def _levels(L, n1, omega):
    st = np.zeros((math.comb(L * L, n1), L * L), np.uint8)
    for r, c in enumerate(combinations(range(L * L), n1)):
        st[r, list(c)] = 1
    nab = np.array([np_energy(x.reshape(L, L)) for x in st])
    lv, deg = np.unique(nab, return_counts=True)
    w = deg * np.exp(-omega * lv)
    return lv, w / w.sum()


def test_chain_samples_the_exact_boltzmann_law_4x4(orc):
    L, n1, omega = 4, 8, 0.5
    lv, p = _levels(L, n1, omega)
    s = orc.init(L, 0.5, 77)
    orc.tri_sweeps(s, omega, 11, 0, 200)
    M = 40000
    seen = np.zeros(len(lv))
    idx = {int(v): k for k, v in enumerate(lv)}
    for t in range(M):
        orc.tri_sweeps(s, omega, 11, 200 + t, 1)
        seen[idx[orc.tri_energy(s)]] += 1
    for k in range(len(lv)):
        mu = M * p[k]
        # generous bound for correlated samples: 6 standard deviations, or a Poisson band for rare levels
        tol = 6 * math.sqrt(mu * 4) if mu > 200 else 6 * math.sqrt(mu) + 10
        assert abs(seen[k] - mu) < tol, (lv[k], seen[k], mu)


def test_two_particles_on_12x12_bind_with_the_exact_weight(orc):
    # 2 sites of type 1 among 144: adjacent pairs (N_AB = 10) vs apart (12)
    L, omega = 12, 1.0
    N = L * L
    A = N * 6 // 2
    B = math.comb(N, 2) - A
    p_adj = A * math.exp(-10 * omega) / (A * math.exp(-10 * omega) + B * math.exp(-12 * omega))
    s = np.zeros((L, L), np.uint8)
    s[0, 0] = s[6, 6] = 1
    orc.tri_sweeps(s, omega, 3, 0, 100)
    M = 20000
    adj = 0
    for t in range(M):
        orc.tri_sweeps(s, omega, 3, 100 + t, 1)
        adj += orc.tri_energy(s) == 10
    # batch-means error bar
    assert abs(adj / M - p_adj) < 0.03, (adj / M, p_adj)


def test_zero_omega_mixes_to_the_random_subset_mean(orc):
    L = 12
    N = L * L
    s = np.zeros((L, L), np.uint8)
    s.ravel()[: N // 2] = 1          # segregated start
    n1 = N // 2
    orc.tri_sweeps(s, 0.0, 8, 0, 50)
    vals = []
    for t in range(2000):
        orc.tri_sweeps(s, 0.0, 8, 50 + t, 1)
        vals.append(orc.tri_energy(s))
    exact = 3 * N * 2 * n1 * (N - n1) / (N * (N - 1))
    assert abs(np.mean(vals) - exact) < 5 * np.std(vals) / math.sqrt(len(vals) / 10)


def _bfs_hist(s, species):
    H, L = s.shape
    N = L * H
    f = s.ravel()
    seen = np.zeros(N, bool)
    sizes = {}
    for i in range(N):
        if f[i] != species or seen[i]:
            continue
        seen[i] = True
        stack, n = [i], 0
        while stack:
            c = stack.pop()
            n += 1
            for d in range(6):
                j = nb(c, d, L, H)
                if f[j] == species and not seen[j]:
                    seen[j] = True
                    stack.append(j)
        sizes[n] = sizes.get(n, 0) + 1
    return sorted(sizes.items())


def test_clusters_match_a_python_bfs(orc):
    for L, x, seed in ((12, 0.4, 1), (20, 0.55, 2), (28, 0.3, 3)):
        s = orc.init(L, x, seed)
        orc.tri_sweeps(s, 1.0, seed, 0, 5)
        for sp in (0, 1):
            assert orc.tri_cluster_hist(s, sp) == _bfs_hist(s, sp)
    for L, H in ((12, 8), (10, 7)):
        s = orc.init_rect(L, H, 0.5, 9)
        for sp in (0, 1):
            assert orc.tri_cluster_hist(s, sp) == _bfs_hist(s, sp)


def test_similar_sampled_is_unbiased(orc):
    L = 28
    N = L * L
    assert orc.tri_similar_sampled(np.ones((L, L), np.uint8), 1, 0) == N
    s = orc.init(L, 0.5, 6)
    exact = 1.0 - orc.tri_energy(s) / (3 * N)
    fr = np.array([orc.tri_similar_sampled(s, 2, t) for t in range(300)]) / N
    assert abs(fr.mean() - exact) < 5 * fr.std(ddof=1) / math.sqrt(len(fr))


def test_sweeps_conserve_composition_and_are_deterministic(orc):
    a = orc.init(20, 0.35, 5)
    b = a.copy()
    n1 = int(a.sum())
    acc_a = orc.tri_sweeps(a, 0.7, 5, 0, 30)
    acc_b = orc.tri_sweeps(b, 0.7, 5, 0, 30)
    assert acc_a == acc_b and np.array_equal(a, b) and int(a.sum()) == n1
    c = orc.init(20, 0.35, 5)
    orc.tri_sweeps(c, 0.7, 5, 0, 12)
    orc.tri_sweeps(c, 0.7, 5, 12, 18)   # split runs resume exactly
    assert np.array_equal(a, c)


def test_observables_of_special_lattices(orc):
    L = 12
    N = L * L
    o = orc.tri_observables(np.ones((L, L), np.uint8), 0.5, 1, 3, 0)
    assert (o["n_unlike"], o["similar_exact"], o["similar_sampled"]) == (0, 1.0, 1.0)
    assert (o["n_clusters"], o["size_max"], o["size_number_avg"], o["size_weight_avg"]) == (1, N, N, N)
    # isolated type-1 sites: one schedule class (no two of its sites are neighbours)
    s = np.zeros(N, np.uint8)
    s[::16] = 1                        # a class: no two of its sites are neighbours
    o = orc.tri_observables(s.reshape(L, L), 1.0, 1, 3, 0)
    k = N // 16
    assert o["n_unlike"] == 6 * k and o["energy_kT"] == 6.0 * k
    assert o["similar_exact"] == 1.0 - 6 * k / (3 * N)
    assert (o["n_clusters"], o["size_max"], o["size_number_avg"], o["size_weight_avg"]) == (k, 1, 1.0, 1.0)
    o0 = orc.tri_observables(s.reshape(L, L), 1.0, 0, 3, 0)
    assert o0["n_clusters"] == 1 and o0["size_max"] == N - k
