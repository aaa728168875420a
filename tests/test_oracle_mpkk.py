"""Pins of the oracle's literal MPKK (the paper's 7-site domain cover with k
drawn with replacement, every domain of an iteration deciding from the
lattice as it stood when the iteration began): the cover is a partition for
the allowed sizes (with a negative control), a hand-worked iteration in which
two exchanges that are each neutral on the old state together break a bond,
accept-everything at U = 0, the lone-particle move rate, random mixing at
omega = 0, uniform k draws, and exact resume."""
import math

import numpy as np
import pytest


def offs(L):
    return (1, -1, L, -L, L - 1, -(L - 1))


def domains(L, H, k):
    N = L * H
    return [[c] + [(c + o) % N for o in offs(L)] for c in range(k, N, 7)]


@pytest.mark.parametrize("L,H", [(10, 7), (12, 14), (5, 7), (3, 7), (17, 21), (404, 420)])
def test_domains_partition_the_ring(L, H):
    N = L * H
    for k in range(7):
        sites = [q for d in domains(L, H, k) for q in d]
        assert sorted(sites) == list(range(N)), k


@pytest.mark.parametrize("L,H", [(11, 7), (10, 8), (14, 14)])
def test_domains_overlap_for_other_sizes(L, H):
    # negative control: L % 7 not in {3, 5}, or H % 7 != 0
    N = L * H
    sites = [q for d in domains(L, H, 0) for q in d]
    assert sorted(sites) != list(range(N))


def test_worked_conflict_example(orc):
    # 10 x 7 ring (N = 70, offsets +-1, +-10, +-9), k = 0: centres 0, 7, ..., 63.
    # Type 1 at 10, 21, 22.  Domain 3 (centre 21) proposes 21 <-> 20 (d = 1),
    # domain 0 (centre 0) proposes 0 <-> 10 (d = 2); the other domains pair
    # like sites.  With U = 2^32 - 1 only exchanges with dN_AB <= 0 pass.
    # On the old lattice: 21 -> 20 loses the bond to 22 but gains one to 10
    # (n = 4 + 1 = 5, dN_AB = 0); 10 -> 0 keeps the lone particle lone
    # (n = 0 + 5, dN_AB = 0).  Both pass, leaving type 1 at 0, 20, 22: three
    # lone particles, N_AB 16 -> 18.  In either sequential order the second
    # exchange would see the first and be refused (dN_AB = +2), N_AB staying 16.
    L, H = 10, 7
    s = np.zeros((H, L), np.uint8)
    s.ravel()[[10, 21, 22]] = 1
    assert orc.tri_energy(s) == 16
    dirs = np.zeros(10, np.uint32)
    dirs[0], dirs[3] = 2, 1
    us = np.full(10, 2**32 - 1, np.uint32)
    acc = orc.mpkk_iteration(s, 0, dirs, us, orc.tri_thresholds(1.0))
    assert acc == 2
    assert sorted(np.flatnonzero(s.ravel())) == [0, 20, 22]
    assert orc.tri_energy(s) == 18


def test_u_zero_accepts_every_unlike_proposal(orc):
    L, H = 12, 14
    N = L * H
    rng = np.random.default_rng(3)
    for k in range(7):
        s = orc.init_rect(L, H, 0.45, 11 + k)
        old = s.ravel().copy()
        dirs = rng.integers(0, 6, N // 7).astype(np.uint32)
        c = k + 7 * np.arange(N // 7)
        b = (c + np.array(offs(L))[dirs]) % N
        want = old.copy()
        want[c], want[b] = old[b], old[c]
        acc = orc.mpkk_iteration(s, k, dirs, np.zeros(N // 7, np.uint32), orc.tri_thresholds(0.7))
        assert np.array_equal(s.ravel(), want)
        assert acc == int(np.count_nonzero(old[c] != old[b]))


def test_lone_particle_moves_twice_per_step(orc):
    # a lone particle's exchanges never change N_AB, so every proposal moves
    # it: per iteration it is the centre (1/7) or its centre's chosen
    # neighbour (6/7 * 1/6) -> 2/7; 7 iterations -> 2 moves per step,
    # variance 7 * (2/7)(5/7) = 10/7 per step
    L, H = 12, 14
    s = np.zeros((H, L), np.uint8)
    s.ravel()[40] = 1
    S = 20000
    acc = orc.mpkk_steps(s, 1.3, 8, 0, S)
    assert abs(acc - 2 * S) < 5 * math.sqrt(10 * S / 7), acc
    assert int(s.sum()) == 1


def test_zero_omega_mixes_to_the_random_subset_mean(orc):
    # at omega = 0 every unlike proposal is taken: each iteration applies a set
    # of disjoint transpositions, a symmetric move, so the uniform law over
    # placements is stationary
    L, H = 10, 14
    N = L * H
    s = orc.init_segregated(L, 0.5, H)
    n1 = int(s.sum())
    orc.mpkk_steps(s, 0.0, 4, 0, 100)
    vals = []
    for t in range(3000):
        orc.mpkk_steps(s, 0.0, 4, 100 + t, 1)
        vals.append(orc.tri_energy(s))
    exact = 3 * N * 2 * n1 * (N - n1) / (N * (N - 1))
    assert abs(np.mean(vals) - exact) < 5 * np.std(vals) / math.sqrt(len(vals) / 10)


def test_k_draws_are_uniform_and_steps_resume(orc):
    cnt = np.zeros(7)
    for t in range(2000):
        for j in range(7):
            cnt[orc.mpkk_k(5, t, j)] += 1
    assert ((cnt - 2000.0) ** 2 / 2000.0).sum() < 30.0     # 6 dof
    dcnt = np.zeros(6)
    for m in range(6000):
        dcnt[orc.mpkk_domain_randoms(5, 3, 2, m)[0]] += 1
    assert ((dcnt - 1000.0) ** 2 / 1000.0).sum() < 25.0
    a = orc.init_rect(12, 14, 0.4, 2)
    b = a.copy()
    n1 = int(a.sum())
    acc = orc.mpkk_steps(a, 0.8, 2, 0, 40)
    acc2 = orc.mpkk_steps(b, 0.8, 2, 0, 15) + orc.mpkk_steps(b, 0.8, 2, 15, 25)
    assert np.array_equal(a, b) and acc == acc2 and int(a.sum()) == n1
