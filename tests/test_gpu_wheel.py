"""The GPU's parallel roulette wheel (Sec. 4.2.1) judged by what defines it:
its selection probabilities. Its chunk prefix sums come from a wave scan, an
FP32 summation order of its own, so its tours equal a sequential-sum wheel's
only where no target falls within rounding of a chunk boundary. The tests:

- chi-square of the GPU's selection frequencies against Eq. (1) at a fixed
  trail state: whole tours of tiny instances, and the first two steps of
  every ant (candidate phase with visited candidates masked, fallbacks of
  two stages over up to 149 cities, candidate-only trails);
- with small integer weights every partial sum is exact in any order, so
  the GPU must pick exactly what the textbook sequential wheel picks at
  every step (one, two and three stages);
- against the oracle's wheel on the same trails: almost every tour equal,
  every tour valid.
"""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import make_pair, say
from tests.stat_util import chi2_arrays, chi2_ok, exact_tour_probs, ref_candidates, sequential_wheel_tours

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401  (fails loudly if not built)
    return torch


def wheel_colony(d, ants, cl, tau, alpha=1, beta=2, pher="dense", seed=9):
    from paper_2003_11902_amd import mmas as M
    g = M.Colony(d, ants, cand_len=cl, alpha=alpha, beta=beta, rho=0.1, seed=seed, pher=pher)
    g.set_selection("prwm")
    if tau is not None:
        g.set_pheromone(tau)
    return g


def gather_tours(g, iterations):
    """Tours of `iterations` constructions at one trail state (no update)."""
    out = []
    for it in range(iterations):
        g.construct(it)
        out.append(g.tours().copy())
    return np.concatenate(out)


@pytest.mark.parametrize("n,cl", [(5, 2), (6, 3), (6, 0)])
def test_whole_tour_distribution(gpu, n, cl):
    """Every ordered tour of a tiny instance against its exact probability
    (1/n) x the product of Eq. (1) over its steps."""
    _, d = I.make_instance("uniform", n, seed=40 + n, side=100.0)
    rng = np.random.default_rng(n + cl)
    tau = rng.uniform(0.2, 1.0, size=(n, n)).astype(np.float32)
    say(f"wheel whole tours n={n} cl={cl}")
    g = wheel_colony(d, 8192, cl, tau)
    tours = gather_tours(g, 24)
    keys, cnt = np.unique(tours, axis=0, return_counts=True)
    counts = {tuple(int(x) for x in k): int(c) for k, c in zip(keys, cnt)}
    chi2_ok(counts, exact_tour_probs(d, tau, cl, 1, 2), tours.shape[0])


def first_steps_expected(tours, W, cand):
    """Observed and expected counts of (current city, next city) for the
    first and second step of every tour, given its start (and first step):
    p(v) = W[c, v] / sum of W[c, u] over the eligible u (the unvisited
    candidates of c, or every unvisited city when none is left)."""
    n = W.shape[0]
    obs1 = np.zeros((n, n))
    exp1 = np.zeros((n, n))
    obs2 = np.zeros((n, n))
    exp2 = np.zeros((n, n))
    s, v1, v2 = tours[:, 0], tours[:, 1], tours[:, 2]
    np.add.at(obs1, (s, v1), 1)
    np.add.at(obs2, (v1, v2), 1)
    elig = np.zeros((n, n), bool)
    if cand is not None:
        elig[np.repeat(np.arange(n), cand.shape[1]), cand.ravel()] = True
    else:
        elig[:] = True
        np.fill_diagonal(elig, False)
    # step 1: from s every candidate (or every other city) is unvisited
    starts = np.bincount(s, minlength=n).astype(np.float64)
    P1 = np.where(elig, W, 0.0)
    exp1 += starts[:, None] * P1 / P1.sum(axis=1, keepdims=True)
    # step 2: from v1 with {s, v1} visited
    for a in range(tours.shape[0]):
        c, vis = v1[a], s[a]
        row = np.where(elig[c], W[c], 0.0)
        row[vis] = 0.0
        row[c] = 0.0
        if row.sum() == 0.0:  # every candidate visited: all unvisited cities
            row = W[c].copy()
            row[vis] = 0.0
            row[c] = 0.0
        exp2[c] += row / row.sum()
    return (obs1, exp1), (obs2, exp2)


@pytest.mark.parametrize("name,n,cl,pher,alpha,beta", [
    ("candidates200", 200, 32, "dense", 1, 2),      # candidate phase, visited candidates masked
    ("nolist150", 150, 0, "dense", 1, 2),           # two-stage fallbacks over 149 and 148 cities
    ("cand_only150_cl1", 150, 1, "candidates", 2, 3),  # fallback weights tau_min^alpha eta^beta
], ids=lambda x: x if isinstance(x, str) else "")
def test_first_steps_frequencies(gpu, name, n, cl, pher, alpha, beta):
    _, d = I.make_instance("uniform", n, seed=70 + n, side=1e4)
    rng = np.random.default_rng(n)
    if pher == "dense":
        tau = (10.0 ** rng.uniform(-1.5, 0.5, size=(n, n))).astype(np.float32)
        W = tau.astype(np.float64) ** alpha * (1.0 / np.where(d > 0, d, 1)) ** beta
    else:
        tau = None
    say(f"wheel first steps {name}")
    g = wheel_colony(d, 8192, cl, tau, alpha=alpha, beta=beta, pher=pher)
    if pher != "dense":
        # every edge off the lists weighs tau_min^alpha eta^beta; on the lists
        # tau_max^alpha eta^beta (untouched trails)
        tmin, tmax = (float(x) for x in g.limits())
        eta_b = (1.0 / np.where(d > 0, d, 1)) ** beta
        W = np.full((n, n), tmin ** alpha) * eta_b
        cand_l = ref_candidates(d, cl)
        W[np.repeat(np.arange(n), cl), cand_l.ravel()] = (tmax ** alpha) * eta_b[np.repeat(np.arange(n), cl),
                                                                                  cand_l.ravel()]
    tours = gather_tours(g, 32)
    cand = ref_candidates(d, cl) if cl else None
    (o1, e1), (o2, e2) = first_steps_expected(tours, W, cand)
    chi2_arrays(o1, e1)
    chi2_arrays(o2, e2)


@pytest.mark.parametrize("n,cl,ants", [(300, 8, 64), (300, 0, 16), (4200, 0, 2), (198, 32, 198)])
def test_integer_weights_equal_the_sequential_wheel(gpu, n, cl, ants):
    """alpha 1, beta 0 and integer trails make every partial sum exact: each
    GPU step must be the first eligible entry whose running total exceeds
    u times the total (up to three stages at n = 4200 without a list)."""
    from oracle import oracle as O
    _, d = I.make_instance("uniform", n, seed=60 + cl, side=1e5)
    rng = np.random.default_rng(n + cl)
    tau = rng.integers(1, 9, size=(n, n)).astype(np.float32)
    say(f"wheel integer weights n={n} cl={cl}")
    g = wheel_colony(d, ants, cl, tau, alpha=1, beta=0, seed=17)
    g.construct(4)
    cand = ref_candidates(d, cl) if cl else None
    L = O.lib()
    bad = sequential_wheel_tours(g.tours(), tau, cand, lambda s, it, a, k: L.orc_draw_word(s, it, a, k, 0), 17, 4)
    assert bad is None, f"ant {bad[0]} differs at step {bad[1]}"
    lengths = g.lengths()
    t = g.tours().astype(np.int64)
    assert np.array_equal(lengths, d[t, np.roll(t, -1, axis=1)].sum(axis=1))


@pytest.mark.parametrize("name,kind,n,seed,kw", [
    ("prwm198", "uniform", 198, 1, dict(ants=198, cand_len=32, pher="dense")),
    ("prwm_cand300", "clustered", 300, 2, dict(ants=64, cand_len=10, pher="candidates")),
    ("prwm_nolist130", "uniform", 130, 3, dict(ants=40, cand_len=0, pher="dense")),
    ("prwm_cl1", "clustered", 150, 4, dict(ants=20, cand_len=1, pher="dense")),
    ("prwm_big_fallback", "uniform", 1500, 5, dict(ants=8, cand_len=2, pher="dense")),
    ("prwm_atsp198", "uniform", 198, 6, dict(ants=198, cand_len=32, pher="dense", problem="atsp")),
    ("prwm1002", "clustered", 1002, 2, dict(ants=1002, cand_len=32, pher="dense")),
], ids=lambda x: x if isinstance(x, str) else "")
def test_agrees_with_the_oracle_wheel(gpu, name, kind, n, seed, kw):
    """From the same trails, the GPU's tours equal those of the oracle's
    sequential-sum wheel except where a target lands within rounding of a
    chunk boundary (measured between the two summation orders: 1 tour in
    1002 at n = 1002, none in the smaller cases): at least 98 % equal, and
    the fallback counts of the equal ones too. Every GPU tour, in this and
    three more iterations, is a permutation whose stored length is its
    length."""
    _, d = I.make_instance(kind, n, seed=seed, **({} if kind == "uniform" else dict(clusters=5, sigma=400.0)))
    if kw.get("problem") == "atsp":
        d = I.asymmetric(d, 0.5, seed=seed + 100)
    say(f"wheel vs oracle {name}")
    g, o = make_pair(d, rho=0.1, seed=seed, select="prwm", **kw)
    g.iterate(0)
    o.iterate(0, 8)
    gt, ot = g.tours(), o.tours()
    same = (gt == ot).all(axis=1)
    assert same.mean() >= 0.98, f"{(~same).sum()} of {same.size} tours differ"
    assert np.array_equal(g.lengths()[same], o.lengths()[same])
    gs, gn = g.fallback()
    os_, on = o.fallback()
    assert np.array_equal(gs[same], os_[same]) and np.array_equal(gn[same], on[same])
    for it in range(1, 5):
        t = g.tours().astype(np.int64)
        assert (np.sort(t, axis=1) == np.arange(n)).all(), it
        assert np.array_equal(g.lengths(), d[t, np.roll(t, -1, axis=1)].sum(axis=1)), it
        g.iterate(it)
    assert g.state().flags == 0
