"""GPU parity of the 2-opt local search (Sec. 5.7) and of whole iterations
with it, against the oracle's sequential first-improvement 2-opt."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import make_pair, run_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401
    return torch


def two_opt_pair(d, k, seed, ants=32, waves=0, random_tours=False):
    """2-opt of the same tours on the GPU and with the oracle: constructed
    tours, or random permutations written over them (many more moves)."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    import torch
    n = d.shape[0]
    g = M.Colony(d, ants, cand_len=16, rho=0.1, seed=seed, pher="candidates", ls_nn=k)
    g.set_two_opt_launch(waves)
    g.prepare_choice_info()
    g.construct(0)
    if random_tours:
        rng = np.random.default_rng(seed)
        perm = np.stack([rng.permutation(n) for _ in range(ants)]).astype(np.uint16)
        g.tensor(M.MMAS_BUF_TOURS).copy_(torch.from_numpy(perm.view(np.int16).ravel()).cuda())
        g.synchronize()
    before = g.tours().copy()
    g.two_opt()
    after, lengths = g.tours(), g.lengths()
    assert (g.state().flags & 16) == 0
    nn = O.nearest(d, k)
    for a in range(before.shape[0]):
        t, L = O.two_opt_tour(d, nn, before[a])
        assert np.array_equal(after[a], t), f"ant {a}"
        assert lengths[a] == L


@pytest.mark.parametrize("n,k,seed,waves", [(200, 8, 1, 0), (200, 8, 1, 1), (33, 32, 2, 0), (33, 32, 2, 2),
                                             (777, 8, 3, 0), (777, 8, 3, 4), (1500, 16, 4, 0), (1500, 16, 4, 8)])
def test_two_opt_matches_oracle_on_gpu_tours(gpu, n, k, seed, waves):
    """Construct on the GPU, then 2-opt each tour on the GPU and with the
    oracle; the tours and lengths must be identical for every launch shape."""
    _, d = I.make_instance("uniform", n, seed=seed, side=1e6)
    say(f"2-opt n={n} k={k} waves={waves}")
    two_opt_pair(d, k, seed, waves=waves)


@pytest.mark.parametrize("n,k,waves", [(300, 8, 0), (300, 1, 16), (64, 3, 1), (1000, 5, 0)])
def test_two_opt_from_random_tours(gpu, n, k, waves):
    """Random permutations need many moves and long reversals."""
    _, d = I.make_instance("clustered", n, seed=n + k, clusters=6, sigma=800.0)
    say(f"2-opt from random tours n={n} k={k} waves={waves}")
    two_opt_pair(d, k, 11, ants=16, waves=waves, random_tours=True)


def test_two_opt_without_lds_edge_lengths(gpu):
    """n large enough that the edge lengths do not fit in LDS beside the tour:
    the kernel reads every distance from HBM; same result."""
    _, d = I.make_instance("uniform", 20500, seed=12, side=1e6)
    say("2-opt n=20500 (edge lengths in HBM)")
    two_opt_pair(d, 8, 5, ants=4)


@pytest.mark.parametrize("tabu", ["bitmask", "compact"])
def test_iterations_with_two_opt(gpu, tabu):
    _, d = I.make_instance("uniform", 600, seed=7, side=1e6)
    say(f"iterations with 2-opt {tabu}")
    run_parity(d, 3, ants=40, cand_len=16, rho=0.02, seed=3, tabu=tabu, pher="candidates", ls_nn=8)


def test_two_opt_dense_trails(gpu):
    _, d = I.make_instance("clustered", 300, seed=8, clusters=5, sigma=500.0)
    run_parity(d, 3, ants=30, cand_len=12, rho=0.1, seed=4, ls_nn=8)


def test_search_order_worked_example(gpu):
    """The hand-derived 6-city run of the search order (see
    tests/test_oracle_two_opt.py): every ant starts from the same tour and
    must end at the derived 2-optimal tour, in every launch shape."""
    from paper_2003_11902_amd import mmas as M
    from tests.test_oracle_two_opt import read_order_example
    import torch
    d, tour, expected, length = read_order_example()
    for waves in (1, 4, 16):
        say(f"2-opt worked example, waves {waves}")
        g = M.Colony(d, 5, cand_len=5, rho=0.1, seed=1, pher="candidates", ls_nn=5)
        g.set_two_opt_launch(waves)
        g.construct(0)
        t0 = np.tile(np.array(tour, dtype=np.uint16), (5, 1))
        g.tensor(M.MMAS_BUF_TOURS).copy_(torch.from_numpy(t0.view(np.int16).ravel()).cuda())
        g.synchronize()
        g.two_opt()
        assert (g.tours() == np.array(expected, dtype=np.uint16)).all()
        assert (g.lengths() == length).all()
        assert (g.state().flags & 16) == 0
