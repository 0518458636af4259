"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (the library's defaults, and the batch autotuner plus graph capture):

- n = 18512 with 2-opt: one whole iteration (construction with several waves
  per ant, 2-opt, update) of all 64 ants against the oracle;
- the batch of 256 instances (n in [100, 2000], ants = n): one tuned,
  captured step; three sampled instances (the smallest, the largest and one
  in between) against an oracle colony each;
- n = 3795 with 3795 ants and a learned heuristic: features bit-exact, then
  two whole iterations with the heuristic installed from oracle scores.
"""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import compare_iteration, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401
    return torch


def test_uniform18512_2opt_first_iteration(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    xy, d, w = I.workload_instance("uniform18512_2opt")
    say("uniform18512_2opt: one iteration, 64 ants, construction + 2-opt + update")
    g = M.Colony(d, w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=1, pher=w["pher"], ls_nn=w["ls_nn"])
    o = O.Colony(d, w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=1, pher_mode=O.PHER_CANDIDATES,
                 ls_nn=w["ls_nn"])
    g.iterate(0)
    o.iterate(0, 16)
    compare_iteration(g, o, 0)
    assert g.state().flags == 0
    t = g.tours()
    assert all(np.array_equal(np.sort(t[a]), np.arange(d.shape[0])) for a in (0, 31, 63))


def test_batched256_sampled_instances(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    insts = I.batch_instances(256)
    dists = [dd for _, dd in insts]
    params = [M.make_params(dd.shape[0], dd.shape[0], cand_len=32, rho=0.02, seed=1 + k)
              for k, dd in enumerate(dists)]
    say("batched256: tune, capture, one step")
    b = M.Batch(dists, params)
    b.tune()
    b.capture()
    b.step()
    b.synchronize()
    sizes = np.array([dd.shape[0] for dd in dists])
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), 128]
    for k in picks:
        n = dists[k].shape[0]
        say(f"  instance {k}: n = {n}")
        o = O.Colony(dists[k], n, cand_len=32, rho=0.02, seed=1 + k)
        o.iterate(0, 16)
        compare_iteration(b.instance(k), o, 0)


def test_uniform3795_learned_full_iterations(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    xy, d, w = I.workload_instance("uniform3795")
    n = d.shape[0]
    xy32 = xy.astype(np.float32)
    say("uniform3795: features, learned heuristic, 2 iterations with 3795 ants")
    knn, feat = O.knn_features(d, xy32)
    gk, _, gf = M.mmas_mlp_features(gpu.from_numpy(d).cuda(), gpu.from_numpy(xy32).cuda(), with_features=True)
    assert np.array_equal(gk.cpu().numpy().view(np.uint16), knn)
    assert np.array_equal(gf.cpu().numpy().view(np.uint32), feat.view(np.uint32))
    rng = np.random.default_rng(11)
    P = O.MLPParams(rng.normal(0, 0.4, (16, 128)), rng.normal(0, 0.1, 128), rng.normal(0, 0.09, (128, 128)),
                    rng.normal(0, 0.1, 128), rng.normal(0, 0.2, 128), rng.normal(0, 0.1))
    s = O.mlp_forward(O.bf16(O.pad_inputs(feat)), P, quantize=True).reshape(n, 16)
    heur = O.install_eta(d, knn, s, w["beta"])
    g = M.Colony(d, w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=4)
    g.set_learned_heuristic(gpu.from_numpy(knn.view(np.int16)).cuda(), gpu.from_numpy(s).cuda())
    assert np.array_equal(g.read(M.MMAS_BUF_HEUR).reshape(n, n).view(np.uint32), heur.view(np.uint32))
    o = O.Colony(d, w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=4)
    o.set_heuristic(heur)
    for it in range(2):
        g.iterate(it)
        o.iterate(it, 16)
        compare_iteration(g, o, it)
    assert g.state().flags == 0


def test_large_n_first_iteration(gpu):
    """n = 40000 (ids close to the 16-bit limit, per-ant LDS of 86 KB with the
    bitmask tabu, helper waves on the all-city fallbacks): one iteration of
    two ants with candidate-only trails against the oracle."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 40000, seed=77, side=1e6)
    say("n = 40000: one iteration, 2 ants, cl 8")
    g = M.Colony(d, 2, cand_len=8, rho=0.05, seed=9, pher="candidates")
    o = O.Colony(d, 2, cand_len=8, rho=0.05, seed=9, pher_mode=O.PHER_CANDIDATES)
    g.iterate(0)
    o.iterate(0, 2)
    compare_iteration(g, o, 0)
    assert g.state().flags == 0
