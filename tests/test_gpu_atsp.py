"""GPU parity on the asymmetric TSP (Sec. 2.1): the HIP library against the
oracle on asymmetric instances. Construction reads row i of d for the step
out of i and the deposit reaches the arcs (i, succ(i)) alone; tours and
lengths must match bit for bit and trails within 1e-6 relative (expected
bit-identical) at every iteration."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import run_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401  (fails loudly if not built)
    return torch


def asym(kind, n, seed, frac=0.5):
    extra = {} if kind == "uniform" else dict(clusters=5, sigma=400.0)
    _, d = I.make_instance(kind, n, seed=seed, **extra)
    return I.asymmetric(d, frac, seed=seed + 100)


@pytest.mark.parametrize("name,kind,n,kw", [
    ("bitmask198", "uniform", 198, dict(ants=198, cand_len=32, tabu="bitmask")),
    ("compact198", "uniform", 198, dict(ants=198, cand_len=32, tabu="compact")),
    ("list198", "uniform", 198, dict(ants=198, cand_len=32, tabu="list")),
    ("cand300", "clustered", 300, dict(ants=64, cand_len=10, pher="candidates")),
    ("nolist130", "uniform", 130, dict(ants=40, cand_len=0)),
    ("global150", "clustered", 150, dict(ants=6, cand_len=10, deposit="global")),
    ("big_fallback1500", "uniform", 1500, dict(ants=8, cand_len=2)),
], ids=lambda x: x if isinstance(x, str) else "")
def test_atsp_matches_oracle(gpu, name, kind, n, kw):
    d = asym(kind, n, seed=n)
    say(f"atsp {name}")
    g, o, _ = run_parity(d, 8, rho=0.1, seed=5, problem="atsp", **kw)
    tau = g.pheromone()
    if kw.get("pher", "dense") == "dense":
        assert not np.array_equal(tau, tau.T)


def test_atsp_workload_first_iterations(gpu):
    """The 1002-city asymmetric workload at full size (1002 ants, cl 32)."""
    _, d, w = I.workload_instance("clustered1002_atsp")
    say("atsp clustered1002_atsp")
    run_parity(d, 3, ants=w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=1, problem="atsp")


def test_asymmetric_matrix_needs_atsp(gpu):
    from paper_2003_11902_amd import mmas as M
    d = asym("uniform", 60, seed=2)
    with pytest.raises(M.MmasError) as e:
        M.Colony(d, 10, cand_len=8)
    assert e.value.status == M.MMAS_EINVAL
    g = M.Colony(d, 10, cand_len=8, problem="atsp")
    assert g.state().flags == 0
    # diagonal and sign checks still apply
    bad = d.copy()
    bad[3, 7] = 0
    with pytest.raises(M.MmasError):
        M.Colony(bad, 10, cand_len=8, problem="atsp")


def test_learned_heuristic_refuses_atsp(gpu):
    from paper_2003_11902_amd import mmas as M
    d = asym("uniform", 60, seed=3)
    g = M.Colony(d, 10, cand_len=8, problem="atsp")
    knn = gpu.zeros(60 * 16, dtype=gpu.int16, device="cuda")
    scores = gpu.zeros(60 * 16, dtype=gpu.float32, device="cuda")
    with pytest.raises(M.MmasError) as e:
        g.set_learned_heuristic(knn, scores)
    assert e.value.status == M.MMAS_EUNSUPPORTED


def test_batch_mixes_tsp_and_atsp(gpu):
    """A batch whose odd instances are asymmetric: every instance equals the
    oracle run alone with its own parameters."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    rng = np.random.default_rng(77)
    sizes = rng.integers(40, 300, size=6)
    dists, params, orcs = [], [], []
    for k, n in enumerate(int(x) for x in sizes):
        prob = "atsp" if k % 2 else "tsp"
        _, d = I.make_instance("uniform", n, seed=500 + k)
        if prob == "atsp":
            d = I.asymmetric(d, 0.5, seed=600 + k)
        dists.append(d)
        params.append(M.make_params(n, n, cand_len=16, rho=0.05, seed=700 + k, problem=prob))
        orcs.append(O.Colony(d, n, cand_len=16, rho=0.05, seed=700 + k, problem=prob))
    say("atsp batch")
    b = M.Batch(dists, params)
    for it in range(3):
        b.step()
        b.synchronize()
        for k, o in enumerate(orcs):
            o.iterate(it, 8)
            v = b.instance(k)
            assert np.array_equal(v.tours(), o.tours()), (it, k)
            assert np.array_equal(v.lengths(), o.lengths()), (it, k)
            assert np.array_equal(v.pheromone().view(np.uint32), o.pheromone().view(np.uint32)), (it, k)
