"""Pins of the oracle on the asymmetric TSP (Sec. 2.1: d_ij may differ from
d_ji, so an edge (i,j) is an arc from i to j). Construction reads row i of
d for the step out of i, a tour's length sums d along its direction, and the
iteration best deposits on its n arcs (i, succ(i)) only, never on the
reversed arcs."""
import itertools

import numpy as np
import pytest

from paper_2003_11902_amd import instances as I


@pytest.fixture(scope="module")
def a60():
    _, d = I.make_instance("uniform", 60, seed=12)
    return I.asymmetric(d, 0.5, seed=3)


def arcs(tour):
    t = np.asarray(tour, dtype=np.int64)
    return t, np.roll(t, -1)


def test_asymmetric_recipe(a60):
    _, d = I.make_instance("uniform", 60, seed=12)
    n = 60
    off = ~np.eye(n, dtype=bool)
    assert np.all(np.diag(a60) == 0) and np.all(a60[off] >= 1)
    assert np.all(a60[off] >= d[off]) and np.all(a60[off] <= d[off] + 0.5 * d[off])
    assert (a60 != a60.T)[off].mean() > 0.9


def test_lengths_follow_the_tour_direction(orc, a60):
    col = orc.Colony(a60, ants=30, cand_len=8, seed=3, problem="atsp")
    col.iterate(0, nthreads=4)
    tours = col.tours().astype(np.int64)
    assert np.all(np.sort(tours, axis=1) == np.arange(60))
    a, b = tours, np.roll(tours, -1, axis=1)
    fwd = a60[a, b].sum(axis=1)
    assert np.array_equal(col.lengths(), fwd)
    assert np.any(a60[b, a].sum(axis=1) != fwd)  # the reverse direction differs


@pytest.mark.parametrize("deposit", ["iteration", "global"])
def test_sum_rule_arcs_only(orc, a60, deposit):
    """Trails far from both limits: the n arcs (i, succ(i)) of the tour that
    deposits gain 1/C, every other entry (the reversed arcs included) is just
    fl((1-rho) tau), the total grows by n/C and the trails turn asymmetric."""
    n = 60
    col = orc.Colony(a60, ants=20, cand_len=8, rho=0.1, seed=4, problem="atsp", deposit=deposit)
    col.prepare_choice()
    col.construct(0)
    L = col.lengths()
    tmin, tmax = orc.limits(0.1, int(L.min()), n, col.pdec)
    rng = np.random.default_rng(1)
    tau = rng.uniform(0.3, 0.6, size=(n, n)).astype(np.float32) * tmax
    tau = np.minimum(tau, tau.T)
    col.set_pheromone(tau)
    col.update()
    ib, C = col.iteration_best()
    gbt, C_gb = col.best()
    assert C_gb == C  # the first update: the iteration best is the global best
    new = col.pheromone().astype(np.float64)
    evap = ((np.float32(1.0) - np.float32(0.1)) * tau).astype(np.float64)
    a, b = arcs(col.tours()[ib])
    dep = np.zeros((n, n), bool)
    dep[a, b] = True
    assert dep.sum() == n and not np.any(dep & dep.T)
    assert np.array_equal(new[~dep], evap[~dep])
    assert np.array_equal(new[b, a], evap[b, a])
    assert np.allclose(new[dep] - evap[dep], 1.0 / C, rtol=1e-5)
    assert abs((new.sum() - evap.sum()) - n / C) < 1e-5 * n / C
    assert not np.array_equal(new, new.T)
    assert np.all((new >= tmin) & (new <= tmax))


def test_candidate_trails_arcs_only(orc, a60):
    """Candidate-only trails: entry (i, r) gains 1/C exactly when cand[i][r] is
    succ(i) on the iteration best; pred(i) on the list gains nothing."""
    n, cl = 60, 8
    col = orc.Colony(a60, ants=20, cand_len=cl, rho=0.1, seed=6, problem="atsp",
                     pher_mode=orc.PHER_CANDIDATES)
    col.prepare_choice()
    col.construct(0)
    L = col.lengths()
    tmin, tmax = orc.limits(0.1, int(L.min()), n, col.pdec)
    tau = np.random.default_rng(2).uniform(0.3, 0.6, size=(n, cl)).astype(np.float32) * tmax
    col.set_pheromone(tau)
    col.update()
    ib, C = col.iteration_best()
    t = col.tours()[ib].astype(np.int64)
    succ = np.empty(n, np.int64)
    pred = np.empty(n, np.int64)
    succ[t] = np.roll(t, -1)
    pred[np.roll(t, -1)] = t
    cand = col.cand().astype(np.int64)
    dep = cand == succ[:, None]
    back = cand == pred[:, None]
    assert dep.any() and back.any()
    new = col.pheromone().astype(np.float64)
    evap = ((np.float32(1.0) - np.float32(0.1)) * tau).astype(np.float64)
    assert np.array_equal(new[~dep], evap[~dep])
    assert np.allclose(new[dep] - evap[dep], 1.0 / C, rtol=1e-5)


def test_brute_force_optimum(orc):
    """20 asymmetric 7-city instances, full candidate lists: in at least 19 the
    colony's global best is the directed optimum over all 6! tours from city
    0, and in every one its length is the sum of d along its own direction."""
    n, hits = 7, 0
    for seed in range(20):
        _, d = I.make_instance("uniform", n, seed=300 + seed, side=100.0)
        d = I.asymmetric(d, 1.0, seed=400 + seed)
        assert not np.array_equal(d, d.T)
        best = min(sum(int(d[p[k], p[(k + 1) % n]]) for k in range(n))
                   for p in ((0,) + q for q in itertools.permutations(range(1, n))))
        col = orc.Colony(d, ants=2 * n, cand_len=n - 1, rho=0.1, seed=2, problem="atsp")
        for it in range(100):
            col.iterate(it, nthreads=1)
        t, C = col.best()
        t = np.asarray(t, np.int64)
        assert sorted(t.tolist()) == list(range(n))
        assert C == int(d[t, np.roll(t, -1)].sum()) and C >= best
        hits += C == best
    assert hits >= 19, hits


def test_two_opt_and_bad_problem_rejected(orc, a60):
    with pytest.raises(ValueError):
        orc.Colony(a60, ants=4, cand_len=8, ls_nn=4, problem="atsp")
    with pytest.raises(ValueError):
        orc.Colony(a60, ants=4, cand_len=8, problem=2)
