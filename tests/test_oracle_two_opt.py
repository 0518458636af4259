"""Pins of the oracle's 2-opt (Sec. 5.7: neighbour lists and don't-look bits,
after Bentley) and an end-to-end sanity bar for the whole method."""
import itertools

import numpy as np
import pytest

from paper_2003_11902_amd import instances as I


def improving_2opt_moves(d, tour):
    """All (i, j) whose 2-opt exchange shortens the tour (brute force)."""
    t = np.asarray(tour, dtype=np.int64)
    n = len(t)
    out = []
    for i in range(n):
        for j in range(i + 2, n):
            if i == 0 and j == n - 1:
                continue
            a, a1, c, c1 = t[i], t[i + 1], t[j], t[(j + 1) % n]
            if d[a, a1] + d[c, c1] - d[a, c] - d[a1, c1] > 0:
                out.append((i, j))
    return out


def test_uncrosses_a_square(orc):
    xy = np.array([[0, 0], [10, 0], [10, 10], [0, 10]], dtype=np.float64)
    d = I.distance_matrix(xy)
    nn = orc.nearest(d, 3)
    t, length = orc.two_opt_tour(d, nn, np.array([0, 2, 1, 3]))
    assert length == 40 and sorted(t.tolist()) == [0, 1, 2, 3]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_full_lists_reach_2opt_local_optimum(orc, seed):
    """With full neighbour lists, repeating the search until it makes no move
    leaves no improving 2-opt exchange; every pass keeps a permutation, reports
    its true length and never lengthens the tour."""
    n = 40
    _, d = I.make_instance("uniform", n, seed=seed)
    nn = orc.nearest(d, n - 1)
    tour = np.random.default_rng(seed).permutation(n).astype(np.uint16)
    prev = orc.tour_length(d, tour)
    for _ in range(50):
        new, length = orc.two_opt_tour(d, nn, tour)
        assert sorted(new.tolist()) == list(range(n))
        t = new.astype(np.int64)
        assert length == int(d[t, np.roll(t, -1)].sum())
        assert length <= prev
        if length == prev:
            break
        tour, prev = new, length
    assert improving_2opt_moves(d, tour) == []


def test_short_lists_improve_a_random_tour(orc):
    n = 300
    _, d = I.make_instance("uniform", n, seed=4)
    nn = orc.nearest(d, 8)
    tour = np.random.default_rng(0).permutation(n).astype(np.uint16)
    l0 = orc.tour_length(d, tour)
    t, length = orc.two_opt_tour(d, nn, tour)
    assert length < 0.5 * l0
    assert sorted(t.tolist()) == list(range(n))


def brute_force_optimum(d):
    n = d.shape[0]
    best = None
    for perm in itertools.permutations(range(1, n)):
        if perm[0] > perm[-1]:
            continue
        t = (0,) + perm
        length = sum(int(d[t[k], t[(k + 1) % n]]) for k in range(n))
        best = length if best is None else min(best, length)
    return best


@pytest.mark.parametrize("ls_nn", [0, 4])
def test_mmas_finds_optimum_of_tiny_instances(orc, ls_nn):
    """Sanity bar, not an exact pin: on 9-city instances MMAS (with or without
    2-opt) reaches the brute-force optimum within 60 iterations for at least
    19 of 20 seeds."""
    hits = 0
    for seed in range(20):
        _, d = I.make_instance("uniform", 9, seed=100 + seed, side=1000.0)
        opt = brute_force_optimum(d)
        col = orc.Colony(d, ants=9, cand_len=4, rho=0.1, seed=seed, ls_nn=ls_nn)
        for it in range(60):
            col.iterate(it)
            if col.best()[1] == opt:
                break
        assert col.best()[1] >= opt
        hits += col.best()[1] == opt
    assert hits >= 19
