"""Parity over whole runs at the workloads' full sizes, in the launch
configuration bench.py times:

- n = 1002 clustered, 1002 ants, cl 32: all 500 iterations of Alg. 1 with the
  bitmask and the compact tabu, every iteration compared with the oracle
  (tours, lengths, fallback counts, trails bit for bit, limits, global best),
  so the converged-trail regime of the late iterations is covered;
- the batch of 256 instances (n in [100, 2000], ants = n): two tuned,
  graph-captured steps, every instance against its own oracle colony;
- the learned network at the n = 3795 size: 60720 edge rows (the last
  64-edge tile holds 48), forward scores and gradients element by element.
"""
import hashlib
import os

import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import compare_iteration, make_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401  (fails loudly if not built)
    return torch


def host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


@pytest.mark.parametrize("tabu", ["bitmask", "compact"])
def test_clustered1002_all_iterations(gpu, tabu):
    xy, d, w = I.workload_instance("clustered1002")
    threads = host_threads()
    say(f"clustered1002 {tabu}: {w['iterations']} iterations against the oracle ({threads} threads)")
    g, o = make_pair(d, ants=w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=2, tabu=tabu)
    identical = True
    for it in range(w["iterations"]):
        g.iterate(it)
        o.iterate(it, threads)
        identical &= compare_iteration(g, o, it)
        if it % 50 == 49 or it == w["iterations"] - 1:
            # how far the colony has converged: the share of trails within 100
            # times tau_min, and the share of ants that repeat the global best
            tau = g.pheromone()
            tmin, _ = g.limits()
            low = float(np.mean(tau <= 100 * tmin))
            gb = g.best()[1]
            say(f"  iteration {it}: equal so far; global best {gb}; trails near tau_min {low:.3f}; "
                f"ants on the best length {float(np.mean(g.lengths() == gb)):.3f}")
    assert identical, "trails agree within 1e-6 but are not bit-identical"
    assert g.state().flags == 0


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_batched256_every_instance_two_steps(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    insts = I.batch_instances(256)
    dists = [dd for _, dd in insts]
    params = [M.make_params(dd.shape[0], dd.shape[0], cand_len=32, rho=0.02, seed=1 + k)
              for k, dd in enumerate(dists)]
    threads = host_threads()
    say("batched256: tune, capture, two steps; all 256 instances against the oracle")
    b = M.Batch(dists, params)
    b.tune()
    b.capture()
    b.step()
    b.synchronize()
    first = []
    for k in range(len(dists)):
        v = b.instance(k)
        first.append(digest(v.tours(), v.lengths(), *v.fallback()))
    b.step()
    b.synchronize()
    for k, dd in enumerate(dists):
        n = dd.shape[0]
        o = O.Colony(dd, n, cand_len=32, rho=0.02, seed=1 + k)
        o.iterate(0, threads)
        ostep, onode = o.fallback()
        assert digest(o.tours(), o.lengths(), ostep, onode) == first[k], f"instance {k} (n = {n}), step 1"
        o.iterate(1, threads)
        compare_iteration(b.instance(k), o, 1)
        if k % 32 == 31:
            say(f"  instances 0..{k} equal")


def test_mlp_at_full_instance_size(gpu):
    """Forward scores and the gradient of every parameter, element by element
    within 1e-2 of the tensor's largest reference magnitude (and the
    relative Frobenius error below 1e-2), on the 60720 edges of the
    3795-city instance: 948 whole 64-edge tiles and a last one of 48."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    xy, d, w = I.workload_instance("uniform3795")
    knn, feat = O.knn_features(d, xy.astype(np.float32))
    X = O.bf16(O.pad_inputs(feat))
    E = X.shape[0]
    assert E == 60720 and E % 64 == 48
    rng = np.random.default_rng(12)
    P = O.MLPParams(rng.normal(0, 0.4, (16, 128)), rng.normal(0, 0.1, 128), rng.normal(0, 0.09, (128, 128)),
                    rng.normal(0, 0.1, 128), rng.normal(0, 0.2, 128), rng.normal(0, 0.1))
    f = rng.uniform(0, 1, E).astype(np.float32)
    say(f"mlp forward/backward at E = {E}")
    gX = gpu.from_numpy((X.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()
    flat = np.concatenate([P.W1.ravel(), P.b1, P.W2.ravel(), P.b2, P.w3, [P.b3]]).astype(np.float32)
    params = gpu.from_numpy(flat).cuda()
    packed = M.mmas_mlp_pack(params)

    def close(a, b, name):
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        scale = float(np.max(np.abs(b)))
        worst = float(np.max(np.abs(a - b)))
        fro = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        say(f"  {name}: max |diff| {worst:.3e} (bound {1e-2 * scale:.3e}), rel Frobenius {fro:.2e}")
        assert worst <= 1e-2 * scale, (name, worst, scale)
        assert fro < 1e-2, (name, fro)

    s_gpu = M.mmas_mlp_forward(gX, params, packed).cpu().numpy()
    s_ref = O.mlp_forward(X, P, quantize=True)
    close(s_gpu, s_ref, "scores")
    close(s_gpu[-48:], s_ref[-48:], "scores of the last tile")
    for groups in (256, 37):
        grad = M.mmas_mlp_grad(gX, gpu.from_numpy(f).cuda(), params, packed, groups=groups).cpu().numpy()
        loss_ref, gref = O.mlp_backward(X, f, P, quantize=True)
        assert abs(grad[-1] / E - loss_ref) < 1e-3 * abs(loss_ref)
        refs = [gref.W1.ravel(), gref.b1, gref.W2.ravel(), gref.b2, gref.w3, np.array([gref.b3])]
        off = 0
        for name, ref in zip(["W1", "b1", "W2", "b2", "w3", "b3"], refs):
            close(grad[off:off + ref.size], ref, f"grad {name} ({groups} groups)")
            off += ref.size
    # the tail's edges matter: dropping the last tile changes the gradient
    grad_head = M.mmas_mlp_grad(gX[:E - 48].contiguous(), gpu.from_numpy(f[:E - 48]).cuda(), params, packed,
                                groups=37).cpu().numpy()
    assert not np.array_equal(grad_head[:-1], grad[:-1])
