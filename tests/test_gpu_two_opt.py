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


@pytest.mark.parametrize("n,k,seed", [(200, 8, 1), (33, 32, 2), (777, 8, 3), (1500, 16, 4)])
def test_two_opt_matches_oracle_on_gpu_tours(gpu, n, k, seed):
    """Construct on the GPU, then 2-opt each tour on the GPU and with the
    oracle; the tours and lengths must be identical."""
    from oracle import oracle as O
    _, d = I.make_instance("uniform", n, seed=seed, side=1e6)
    from paper_2003_11902_amd import mmas as M
    say(f"2-opt n={n} k={k}")
    g = M.Colony(d, 32, cand_len=16, rho=0.1, seed=seed, pher="candidates", ls_nn=k)
    g.prepare_choice_info()
    g.construct(0)
    before = g.tours().copy()
    g.two_opt()
    after, lengths = g.tours(), g.lengths()
    nn = O.nearest(d, k)
    for a in range(before.shape[0]):
        t, L = O.two_opt_tour(d, nn, before[a])
        assert np.array_equal(after[a], t), f"ant {a}"
        assert lengths[a] == L


@pytest.mark.parametrize("tabu", ["bitmask", "compact"])
def test_iterations_with_two_opt(gpu, tabu):
    _, d = I.make_instance("uniform", 600, seed=7, side=1e6)
    say(f"iterations with 2-opt {tabu}")
    run_parity(d, 3, ants=40, cand_len=16, rho=0.02, seed=3, tabu=tabu, pher="candidates", ls_nn=8)


def test_two_opt_dense_trails(gpu):
    _, d = I.make_instance("clustered", 300, seed=8, clusters=5, sigma=500.0)
    run_parity(d, 3, ants=30, cand_len=12, rho=0.1, seed=4, ls_nn=8)
