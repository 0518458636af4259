"""Pins of the pheromone update of Alg. 1 (Sec. 2.1): evaporation
tau <- max((1 - rho) tau, tau_min), deposit of 1/C_ib on the iteration best's
edges (both directions of a symmetric instance), the tau_max clamp, and the
global-best / limits bookkeeping."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I


@pytest.fixture(scope="module")
def d60():
    return I.make_instance("uniform", 60, seed=12)[1]


def edges(tour):
    t = np.asarray(tour, dtype=np.int64)
    return t, np.roll(t, -1)


def test_tours_valid_and_lengths_exact(orc, d60):
    col = orc.Colony(d60, ants=30, cand_len=8, seed=3)
    for it in range(3):
        col.iterate(it, nthreads=4)
        tours = col.tours().astype(np.int64)
        assert np.all(np.sort(tours, axis=1) == np.arange(60))
        a, b = tours, np.roll(tours, -1, axis=1)
        assert np.array_equal(col.lengths(), d60[a, b].sum(axis=1))
        ib, lib_ = col.iteration_best()
        L = col.lengths()
        assert lib_ == L.min() and ib == int(np.flatnonzero(L == L.min())[0])


def test_sum_rule_no_clamp(orc, d60):
    """With every trail far from both limits, the update is exactly
    fl(fl((1-rho) tau) + delta) on the 2n directed edges of the iteration best
    and fl((1-rho) tau) elsewhere; the total grows by 2n/C_ib."""
    n = 60
    col = orc.Colony(d60, ants=20, cand_len=8, rho=0.1, seed=4)
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
    new = col.pheromone().astype(np.float64)
    keep = np.float32(1.0) - np.float32(0.1)
    evap = (keep * tau).astype(np.float64)
    a, b = edges(col.tours()[ib])
    dep = np.zeros((n, n), bool)
    dep[a, b] = True
    dep[b, a] = True
    assert dep.sum() == 2 * n
    assert np.array_equal(new[~dep], evap[~dep])
    assert np.allclose(new[dep] - evap[dep], 1.0 / C, rtol=1e-5)
    assert abs((new.sum() - evap.sum()) - 2 * n / C) < 1e-5 * 2 * n / C
    assert np.array_equal(new, new.T)
    assert np.all((new >= tmin) & (new <= tmax))


def test_fixed_points_and_time_to_tau_min(orc, d60):
    """Repeating the update on fixed tours: deposited edges climb to
    Delta/rho = tau_max; other edges decay geometrically and hit tau_min after
    ceil(ln(tau_min/tau_0)/ln(1-rho)) updates (+-1 for FP32 rounding)."""
    n, rho = 60, 0.05
    col = orc.Colony(d60, ants=10, cand_len=8, rho=rho, seed=5)
    col.prepare_choice()
    col.construct(0)
    tau0 = col.pheromone()[0, 0]
    col.update()
    ib, C = col.iteration_best()
    tmin, tmax = col.limits()
    a, b = edges(col.tours()[ib])
    dep = np.zeros((n, n), bool)
    dep[a, b] = dep[b, a] = True
    off = ~dep & ~np.eye(n, dtype=bool)
    i0, j0 = np.argwhere(off)[0]
    hit = None
    for t in range(2, 3000):
        col.update()
        if hit is None and col.pheromone()[i0, j0] == tmin:
            hit = t
    expect = np.log(float(tmin) / float(tau0)) / np.log(1 - rho)
    assert abs(hit - np.ceil(expect)) <= 1, (hit, expect)
    tau = col.pheromone()
    assert np.all(tau[off] == tmin)
    # each update rounds twice (at most one ulp in all); the error of the FP32
    # recursion then settles within ulp/rho of the real fixed point Delta/rho
    assert np.all(np.abs(tau[dep] - tmax) <= (1 / rho + 2) * np.spacing(tmax))
    assert np.all(tau[dep] <= tmax)
    assert abs(float(tmax) - (1.0 / C) / np.float32(rho)) < 1e-6 * float(tmax)


def test_global_best_and_limits_bookkeeping(orc, d60):
    col = orc.Colony(d60, ants=12, cand_len=6, rho=0.02, seed=6)
    best = None
    for it in range(12):
        col.iterate(it)
        _, C = col.iteration_best()
        gb_tour, gb = col.best()
        best = C if best is None else min(best, C)
        assert gb == best
        t = gb_tour.astype(np.int64)
        assert int(d60[t, np.roll(t, -1)].sum()) == gb
        assert tuple(col.limits()) == orc.limits(0.02, gb, 60, col.pdec)
        tau = col.pheromone()
        tmin, tmax = col.limits()
        assert tau.min() >= tmin and tau.max() <= tmax


def test_candidate_mode_update(orc, d60):
    """Candidate-only trails follow the same rule on the stored (i, cand[i][r])
    entries."""
    n, cl = 60, 6
    col = orc.Colony(d60, ants=10, cand_len=cl, rho=0.1, seed=7, pher_mode=orc.PHER_CANDIDATES)
    col.prepare_choice()
    col.construct(0)
    tau = col.pheromone().copy()
    col.update()
    ib, C = col.iteration_best()
    tmin, tmax = col.limits()
    cand = col.cand().astype(np.int64)
    a, b = edges(col.tours()[ib])
    succ = np.empty(n, np.int64)
    pred = np.empty(n, np.int64)
    succ[a] = b
    pred[b] = a
    keep = np.float32(1.0) - np.float32(0.1)
    new = col.pheromone()
    for i in range(n):
        for r in range(cl):
            v = max(np.float32(keep * tau[i, r]), tmin)
            if cand[i, r] in (succ[i], pred[i]):
                v = np.float32(v + np.float32(1.0 / C))
            assert new[i, r] == min(v, tmax)


def test_global_best_deposit(orc, d60):
    """Sec. 2.1 lets the global best deposit instead of the iteration best: in
    an iteration whose best is worse than the global best, exactly the global
    best's 2n directed edges gain 1/C_gb (trails far from both limits), and
    the global best itself is unchanged."""
    n = 60
    col = orc.Colony(d60, ants=6, cand_len=4, rho=0.1, seed=8, deposit="global")
    col.iterate(0, nthreads=2)
    gbt, C_gb = col.best()
    for it in range(1, 40):
        col.prepare_choice()
        col.construct(it)
        if col.lengths().min() > C_gb:
            break
        col.update()
        gbt, C_gb = col.best()
    else:
        pytest.fail("no iteration with a worse iteration best")
    tmin, tmax = orc.limits(0.1, int(C_gb), n, col.pdec)
    rng = np.random.default_rng(2)
    tau = rng.uniform(0.3, 0.6, size=(n, n)).astype(np.float32) * tmax
    tau = np.minimum(tau, tau.T)
    col.set_pheromone(tau)
    ib_tour = col.tours()[int(np.argmin(col.lengths()))].copy()
    col.update()
    t2, C2 = col.best()
    assert C2 == C_gb and np.array_equal(t2, gbt)
    new = col.pheromone().astype(np.float64)
    evap = ((np.float32(1.0) - np.float32(0.1)) * tau).astype(np.float64)
    a, b = edges(gbt)
    dep = np.zeros((n, n), bool)
    dep[a, b] = True
    dep[b, a] = True
    assert np.array_equal(new[~dep], evap[~dep])
    assert np.allclose(new[dep] - evap[dep], 1.0 / C_gb, rtol=1e-5)
    # an edge of the iteration best that the global best lacks gets nothing
    ia, ibb = edges(ib_tour)
    only_ib = ~dep[ia, ibb]
    assert only_ib.any()
    assert np.array_equal(new[ia[only_ib], ibb[only_ib]], evap[ia[only_ib], ibb[only_ib]])
