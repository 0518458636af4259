"""GPU parity of the learned heuristic: features and the installation are
bit-exact against the oracle; the bfloat16 MFMA forward and backward agree
with the oracle's float64 network (same bfloat16 rounding points) within a
relative Frobenius error of 1e-2 per tensor; Adam is bit-exact; a network
whose last layer is zero reproduces the plain method's tours exactly."""
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


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def flat_params(P):
    return np.concatenate([P.W1.ravel(), P.b1, P.W2.ravel(), P.b2, P.w3, [P.b3]]).astype(np.float32)


def rand_params(orc, seed):
    rng = np.random.default_rng(seed)
    return orc.MLPParams(rng.normal(0, 0.4, (16, 128)), rng.normal(0, 0.1, 128), rng.normal(0, 0.09, (128, 128)),
                         rng.normal(0, 0.1, 128), rng.normal(0, 0.2, 128), rng.normal(0, 0.1))


def split(g):
    g = np.asarray(g)
    o = 0
    out = []
    for size in (16 * 128, 128, 128 * 128, 128, 128, 1):
        out.append(g[o:o + size])
        o += size
    return out


@pytest.fixture(scope="module")
def inst(gpu):
    from oracle import oracle as O
    xy, d = I.make_instance("clustered", 700, seed=31, clusters=8, sigma=400.0)
    xy32 = xy.astype(np.float32)
    knn, feat = O.knn_features(d, xy32)
    return d, xy32, knn, feat


def test_features_bit_exact(gpu, inst):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    d, xy32, knn, feat = inst
    say("features")
    gk, gX, gf = M.mmas_mlp_features(gpu.from_numpy(d).cuda(), gpu.from_numpy(xy32).cuda(), with_features=True)
    assert np.array_equal(gk.cpu().numpy().view(np.uint16), knn)
    assert np.array_equal(gf.cpu().numpy().view(np.uint32), feat.view(np.uint32))
    X = O.bf16(O.pad_inputs(feat))
    assert np.array_equal((gX.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32), X)


def test_forward_and_backward_match_oracle(gpu, inst):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    d, xy32, knn, feat = inst
    P = rand_params(O, 7)
    X = O.bf16(O.pad_inputs(feat))
    E = X.shape[0]
    f = np.random.default_rng(3).uniform(0, 1, E).astype(np.float32)
    say(f"mlp forward/backward E={E}")
    gX = gpu.from_numpy((X.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()
    params = gpu.from_numpy(flat_params(P)).cuda()
    packed = M.mmas_mlp_pack(params)
    s_gpu = M.mmas_mlp_forward(gX, params, packed).cpu().numpy()
    s_ref = O.mlp_forward(X, P, quantize=True)
    assert rel_fro(s_gpu, s_ref) < 1e-2, rel_fro(s_gpu, s_ref)
    grad = M.mmas_mlp_grad(gX, gpu.from_numpy(f).cuda(), params, packed, groups=37).cpu().numpy()
    loss_ref, gref = O.mlp_backward(X, f, P, quantize=True)
    assert abs(grad[-1] / E - loss_ref) < 1e-3 * abs(loss_ref)
    names = ["W1", "b1", "W2", "b2", "w3", "b3"]
    refs = [gref.W1.ravel(), gref.b1, gref.W2.ravel(), gref.b2, gref.w3, np.array([gref.b3])]
    for name, a, b in zip(names, split(grad[:-1]), refs):
        e = rel_fro(a, b)
        say(f"  grad {name}: rel err {e:.2e}")
        assert e < 1e-2, (name, e)
    # deterministic: another grouping gives the same sums up to FP32 rounding;
    # the same grouping gives identical bits
    g2 = M.mmas_mlp_grad(gX, gpu.from_numpy(f).cuda(), params, packed, groups=37).cpu().numpy()
    assert np.array_equal(grad.view(np.uint32), g2.view(np.uint32))


def test_adam_bit_exact(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    rng = np.random.default_rng(5)
    P = M.mlp_param_count()
    p = rng.normal(size=P).astype(np.float32)
    m = np.zeros(P, np.float32)
    v = np.zeros(P, np.float32)
    gp, gm, gv = (gpu.from_numpy(a.copy()).cuda() for a in (p, m, v))
    for t in range(1, 4):
        g = rng.normal(size=P).astype(np.float32)
        O.adam(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, t)
        M.mmas_mlp_adam(gp, gpu.from_numpy(g).cuda(), gm, gv, 1e-3, t)
    assert np.array_equal(gp.cpu().numpy().view(np.uint32), p.view(np.uint32))
    assert np.array_equal(gv.cpu().numpy().view(np.uint32), v.view(np.uint32))


def test_install_bit_exact_and_zero_score_identity(gpu, inst):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    d, xy32, knn, feat = inst
    n = d.shape[0]
    s = np.random.default_rng(8).normal(0, 2, (n, 16)).astype(np.float32)
    g = M.Colony(d, 64, cand_len=32, rho=0.02, seed=3)
    g.set_learned_heuristic(gpu.from_numpy(knn.view(np.int16)).cuda(), gpu.from_numpy(s).cuda())
    heur = g.read(M.MMAS_BUF_HEUR).reshape(n, n)
    ref = O.install_eta(d, knn, s, 2)
    assert np.array_equal(heur.view(np.uint32), ref.view(np.uint32))
    # s = 0: the plain heuristic, hence the plain tours
    plain = M.Colony(d, 64, cand_len=32, rho=0.02, seed=3)
    zero = M.Colony(d, 64, cand_len=32, rho=0.02, seed=3)
    zero.set_learned_heuristic(gpu.from_numpy(knn.view(np.int16)).cuda(),
                               gpu.zeros((n, 16), dtype=gpu.float32, device="cuda"))
    for it in range(3):
        plain.iterate(it)
        zero.iterate(it)
        assert np.array_equal(plain.tours(), zero.tours())
        assert np.array_equal(plain.pheromone(), zero.pheromone())


def test_labels(gpu, inst):
    from paper_2003_11902_amd import mmas as M
    d, xy32, knn, feat = inst
    n = d.shape[0]
    rng = np.random.default_rng(9)
    tours = np.stack([rng.permutation(n) for _ in range(5)]).astype(np.uint16)
    lab = M.mmas_mlp_labels(gpu.from_numpy(tours.view(np.int16)).cuda(),
                            gpu.from_numpy(knn.view(np.int16)).cuda()).cpu().numpy()
    edges = [set() for _ in range(5)]
    for t in range(5):
        for k in range(n):
            a, b = int(tours[t, k]), int(tours[t, (k + 1) % n])
            edges[t].add((min(a, b), max(a, b)))
    for i in range(0, n, 29):
        for r in range(16):
            j = int(knn[i, r])
            exp = sum((min(i, j), max(i, j)) in e for e in edges) / 5
            assert lab[i, r] == np.float32(exp)


def test_pipeline_small(gpu):
    """Training data from batched runs, a few Adam steps and the time-to-gap
    evaluation run end to end; labels are shares of R tours (multiples of
    1/R) and every kNN row of an instance carries its tour edges."""
    from paper_2003_11902_amd import learned as L
    R = 2
    say("learned pipeline: 6 instances n in [120, 260], R=2, 5 iterations")
    X, F = L.training_set(count=6, n_lo=120, n_hi=260, base_seed=777, R=R, iterations=5, ants=64, log=say)
    assert X.shape[1] == 16 and X.shape[0] == F.shape[0] and X.shape[0] % 16 == 0
    f = F.cpu().numpy()
    assert np.all((f >= 0) & (f <= 1))
    assert np.all(np.isin(f * R, np.arange(R + 1)))
    # each tour has n edges, each seen from both ends when in both kNN lists:
    # the label mass per instance is at least n (one end) per tour share
    assert f.sum() >= 6 * 120 * 0.5
    params, hist = L.train(X, F, epochs=2, batch=4096, log=say)
    assert all(np.isfinite(hist))
    xy, d = I.make_instance("uniform", 200, seed=3)
    recs = L.time_to_gap(params, d, xy, seeds=[1], budget=20, ants=64, log=say)
    assert len(recs) == 1 and recs[0]["plain_len"] > 0


def test_learned_heuristic_reaches_plain_quality_sooner(gpu):
    """The gain of the trained network: trained on small generated instances
    (n 200-400), installed on an unseen 800-city instance, MMAS with the
    learned eta reaches the tour length plain MMAS has after 150 iterations
    in fewer than half as many iterations (deterministic: seeded data,
    fixed-order reductions)."""
    from paper_2003_11902_amd import learned as L
    say("learned gain: 64 training instances, eval n=800, budget 150")
    X, F = L.training_set(count=64, n_lo=200, n_hi=400, base_seed=4242, R=2, iterations=40, ants=64, log=say)
    params, hist = L.train(X, F, epochs=6, batch=8192, log=say)
    assert hist[-1] < hist[0]
    xy, d = I.make_instance("uniform", 800, seed=99)
    recs = L.time_to_gap(params, d, xy, seeds=[1, 2], budget=150, ants=200, log=say)
    for r in recs:
        assert r["learned_iters"] is not None and r["learned_iters"] < 75, r
