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


def read_order_example():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "two_opt_order6.txt")
    rows, tour, expected, length = [], None, None, None
    for line in open(path):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "tour":
            tour = [int(x) for x in line[1:]]
        elif line[0] == "expected":
            expected = [int(x) for x in line[1:]]
        elif line[0] == "length":
            length = int(line[1])
        else:
            rows.append([int(x) for x in line])
    return np.array(rows, dtype=np.int32), tour, expected, length


def test_search_order_worked_example(orc):
    """Reading 19 of Sec. 5.7's search order, pinned by a hand-derived run.

    Neighbour lists by (d, index): 0: 1 4 2 3 5; 1: 0 2 4 3 5; 2: 1 0 4 3 5;
    3: 4 0 5 1 2; 4: 3 0 1 2 5; 5: 3 4 0 1 2. Start tour T0 = [5 1 2 4 3 0]
    (length 25+7+15+4+11+22 = 84).

    City 0, successor a' = 5, d(0,5) = 22:
      c = 1: g1 = 22-4 = 18, c' = succ(1) = 2, gain = 18 + d(1,2) - d(5,2)
             = 18+7-31 = -6;
      c = 4: g1 = 22-6 = 16, c' = succ(4) = 3, gain = 16+4-12 = 8 > 0: move.
      The paths a'..c (positions 0-3, 4 cities) and c'..a (positions 4-5,
      2 cities): the shorter one is reversed, T1 = [5 1 2 4 0 3] (76).
    City 0 again, a' = succ(0) = 3, d(0,3) = 11:
      c = 1: g1 = 7, c' = 2, gain = 7+7-19 = -5;
      c = 4: g1 = 5, c' = succ(4) = 0 = a: skipped;
      c = 2: g1 = 1, c' = succ(2) = 4, gain = 1+15-4 = 12 > 0: move.
      Paths a'..c (positions 5,0,1,2: 4 cities) and c'..a (positions 3-4):
      the latter is reversed, T2 = [5 1 2 0 4 3] (64).
    City 0 again: successor 4 (d 6): c = 1: g1 = 2, gain = 2+7-15 = -6;
      c = 4: g1 = 0, stop. Predecessor 2 (d 10): c = 1: g1 = 6, c' =
      pred(1) = 5, gain = 6+25-31 = 0 (not positive); c = 4: c' = pred(4) =
      0 = a, skipped; c = 2: g1 = 0, stop. Its bit is set.
    Cities 1-5 then find no improving move either: T2 is 2-optimal (checked
    below by brute force), so the search ends with T2.

    Each alternative reading ends elsewhere (as a tour, not only as an
    array): predecessor first moves at city 0 with c = 1 (g1 = 11-4 = 7,
    c' = pred(1) = 5, gain = 7+25-12 = 20) and ends at [0 1 2 4 3 5];
    leaving city 0 after its first move ends at [3 4 2 1 0 5]; reversing the
    longer path first gives [4 2 1 5 3 0] and ends at [1 0 4 5 3 2]. All
    three have a different edge set from T2."""
    d, tour, expected, length = read_order_example()
    nn = orc.nearest(d, 5)
    assert nn.tolist() == [[1, 4, 2, 3, 5], [0, 2, 4, 3, 5], [1, 0, 4, 3, 5], [4, 0, 5, 1, 2], [3, 0, 1, 2, 5],
                           [3, 4, 0, 1, 2]]
    assert orc.tour_length(d, np.array(tour)) == 84
    t, L = orc.two_opt_tour(d, nn, np.array(tour))
    assert t.tolist() == expected and L == length == orc.tour_length(d, np.array(expected))
    assert improving_2opt_moves(d, expected) == []

    def edges(x):
        return {frozenset((x[i], x[(i + 1) % len(x)])) for i in range(len(x))}
    for other in ([0, 1, 2, 4, 3, 5], [3, 4, 2, 1, 0, 5], [1, 0, 4, 5, 3, 2]):
        assert edges(other) != edges(expected)
