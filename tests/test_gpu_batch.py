"""Batched construction: every instance of a batch must get exactly the tours
and trails of a single context driven with the same parameters, whatever the
launch shape, eagerly or replayed from a captured graph."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401
    return torch


def small_batch(count=9, seed=300, lo=40, hi=400, tabu="bitmask"):
    from paper_2003_11902_amd import mmas as M
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=count)
    dists, params = [], []
    for k in range(count):
        kind = "uniform" if k % 2 == 0 else "clustered"
        extra = {} if kind == "uniform" else dict(clusters=4, sigma=400.0)
        _, d = I.make_instance(kind, int(sizes[k]), seed=seed + k, **extra)
        dists.append(d)
        params.append(M.make_params(int(sizes[k]), int(sizes[k]) if k % 3 else 17, cand_len=(32, 8, 20)[k % 3],
                                    rho=0.05, seed=1000 + k, tabu=tabu))
    return dists, params


def singles(dists, params, iterations):
    from paper_2003_11902_amd import mmas as M
    out = []
    for d, p in zip(dists, params):
        c = M.Colony(d, p.ants, cand_len=p.cand_len, alpha=p.alpha, beta=p.beta, rho=p.rho, seed=p.seed,
                     tabu={0: "bitmask", 1: "compact", 2: "list"}[p.tabu])
        hist = []
        for it in range(iterations):
            c.iterate(it)
            hist.append((c.tours().copy(), c.pheromone().copy(), c.lengths().copy()))
        out.append(hist)
    return out


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
def test_batch_equals_single_instances(gpu, tabu):
    from paper_2003_11902_amd import mmas as M
    dists, params = small_batch(tabu=tabu)
    say(f"batch vs single {tabu}")
    ref = singles(dists, params, 3)
    b = M.Batch(dists, params)
    for it in range(3):
        b.step()
        b.synchronize()
        for i in range(len(dists)):
            v = b.instance(i)
            assert np.array_equal(v.tours(), ref[i][it][0]), (it, i)
            assert np.array_equal(v.pheromone(), ref[i][it][1]), (it, i)
    assert b.iteration() == 3


def test_launch_shapes_and_tuner_do_not_change_results(gpu):
    from paper_2003_11902_amd import mmas as M
    dists, params = small_batch(count=6, seed=400)
    ref = singles(dists, params, 2)
    shapes = [(1, -1, 64), (2, 0, 64), (8, -1, 64), (16, 0, 64), (16, 4096, 64),
              (2, -1, 32), (4, 0, 32), (8, -1, 32), (16, 4096, 32)]
    for apb, tb, lanes in shapes:
        say(f"shape {apb} {tb} {lanes}")
        b = M.Batch(dists, params)
        b.set_launch(apb, tb, lanes)
        for it in range(2):
            b.step()
        b.synchronize()
        for i in range(len(dists)):
            assert np.array_equal(b.instance(i).tours(), ref[i][1][0]), (apb, tb, lanes, i)
            assert np.array_equal(b.instance(i).lengths(), ref[i][1][2]), (apb, tb, lanes, i)
    for tabu in ("compact", "list", "bitmask"):
        say(f"tabu {tabu}")
        b = M.Batch(dists, params)
        b.set_tabu(tabu)
        b.set_launch(8, -1, 32)
        b.step()
        b.step()
        b.synchronize()
        for i in range(len(dists)):
            assert np.array_equal(b.instance(i).tours(), ref[i][1][0]), (tabu, i)
    b = M.Batch(dists, params)
    apb, tb, lanes, tabu = b.tune()
    assert apb in (4, 8, 16) and lanes in (32, 64) and tabu in (0, 1, 2)
    b.step()
    b.step()
    b.synchronize()
    for i in range(len(dists)):
        assert np.array_equal(b.instance(i).tours(), ref[i][1][0])
        assert np.array_equal(b.instance(i).pheromone(), ref[i][1][1])


def test_graph_replays_match_eager(gpu):
    """A captured step replayed several times, with host reads and syncs in
    between, matches the eager run at every iteration."""
    from paper_2003_11902_amd import mmas as M
    dists, params = small_batch(count=5, seed=500)
    ref = singles(dists, params, 4)
    b = M.Batch(dists, params)
    b.capture()
    for it in range(4):
        b.step()
        b.synchronize()
        for i in range(len(dists)):
            v = b.instance(i)
            assert np.array_equal(v.tours(), ref[i][it][0]), (it, i)
            assert np.array_equal(v.pheromone(), ref[i][it][1]), (it, i)
        assert b.iteration() == it + 1


def test_fallback_list_in_passes(gpu):
    """The batched kernel lists a bitmask fallback's unvisited cities in passes
    of at most 512; with short candidate lists on instances of 600-1500 cities
    many fallbacks see more than 512 unvisited cities and take several passes.
    Tours and trails equal those of single contexts (one full list) and, for
    one instance, the oracle's."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    dists, params = [], []
    for k, n in enumerate((600, 1100, 1500)):
        _, d = I.make_instance("uniform" if k != 1 else "clustered", n, seed=500 + k,
                               **({} if k != 1 else dict(clusters=6, sigma=300.0)))
        dists.append(d)
        params.append(M.make_params(n, 24, cand_len=4, rho=0.05, seed=2000 + k))
    say("batch fallback passes: n 600/1100/1500, cl 4")
    ref = singles(dists, params, 2)
    b = M.Batch(dists, params)
    for it in range(2):
        b.step()
        b.synchronize()
        for i in range(len(dists)):
            v = b.instance(i)
            assert np.array_equal(v.tours(), ref[i][it][0]), (it, i)
            assert np.array_equal(v.pheromone(), ref[i][it][1]), (it, i)
    # some fallback saw more than 512 unvisited cities: the fallback steps of
    # an ant are distinct steps k, so if every one had n - k <= 512, their
    # unvisited counts would sum to at most 512 + 511 + ... (steps terms)
    steps, nodes = b.instance(2).fallback()
    assert (nodes > steps * 512 - steps * (steps - 1) // 2).any()
    o = O.Colony(dists[2], 24, cand_len=4, rho=0.05, seed=2002)
    for it in range(2):
        o.iterate(it, 8)
    assert np.array_equal(b.instance(2).tours(), o.tours())
