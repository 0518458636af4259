"""Pins of the oracle for the learned heuristic: features, the MLP forward
and backward (finite differences in float64), Adam's first step, the FP32 exp
and the installation eta = (1/d) 2 sigmoid(s)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2003_11902_amd import instances as I


def rand_params(orc, rng, scale=0.3):
    return orc.MLPParams(rng.normal(0, scale, (16, 128)), rng.normal(0, 0.1, 128),
                         rng.normal(0, scale / 4, (128, 128)), rng.normal(0, 0.1, 128),
                         rng.normal(0, scale, 128), rng.normal(0, 0.1))


def test_expf_accuracy(orc):
    xs = np.concatenate([np.linspace(-87, 88, 20001), np.linspace(-1, 1, 2001)]).astype(np.float32)
    got = np.array([orc.expf(x) for x in xs], dtype=np.float64)
    ref = np.exp(xs.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) <= 2.0
    assert orc.expf(0.0) == 1.0 and orc.expf(-200.0) == 0.0 and np.isinf(orc.expf(200.0))


def test_gelu_against_normal_cdf(orc):
    """With W1 = 0 and a bias c, every hidden unit is GELU(c) = c Phi(c); with
    W2 = 0 and bias 0 the second layer is GELU(0) = 0... so s = b3; with
    w3 = e_0 and W2 = I it is GELU(GELU(c))."""
    rng = np.random.default_rng(0)
    X = rng.normal(size=(4, 16)).astype(np.float32)
    for c in (-2.0, -0.5, 0.0, 0.7, 1.96, 3.0):
        g1 = c * stats.norm.cdf(c)
        P = orc.MLPParams(np.zeros((16, 128)), np.full(128, c), np.eye(128), np.zeros(128),
                          np.eye(128)[0], 0.25)
        s = orc.mlp_forward(X, P, quantize=False)
        assert np.allclose(s, g1 * stats.norm.cdf(g1) + 0.25, rtol=1e-6, atol=1e-7)


def test_zero_last_layer_scores_zero(orc):
    rng = np.random.default_rng(1)
    P = rand_params(orc, rng)
    P.w3[:] = 0
    P.b3 = np.float32(0)
    X = rng.normal(size=(50, 16)).astype(np.float32)
    assert np.all(orc.mlp_forward(X, P) == 0)


def test_backward_matches_central_differences(orc):
    """float64 network, weights with short mantissas so p +- h is exact."""
    rng = np.random.default_rng(2)
    P = rand_params(orc, rng)
    for a in P.arrays():
        a[...] = orc.bf16(a)
    P.b3 = np.float32(orc.bf16(np.array([P.b3], np.float32))[0])
    X = orc.bf16(rng.normal(size=(3, 16)).astype(np.float32))
    f = rng.uniform(size=3).astype(np.float32)
    loss, g = orc.mlp_backward(X, f, P, quantize=False)
    h = 2.0 ** -12
    names = ["W1", "b1", "W2", "b2", "w3"]
    for name, garr in zip(names, g.arrays()):
        arr = getattr(P, name)
        for idx in rng.choice(arr.size, size=6, replace=False):
            old = arr.flat[idx]
            arr.flat[idx] = old + h
            lp, _ = orc.mlp_backward(X, f, P, quantize=False)
            arr.flat[idx] = old - h
            lm, _ = orc.mlp_backward(X, f, P, quantize=False)
            arr.flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = float(garr.flat[idx])
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (name, idx, fd, an)
    # the bias of the output
    old = P.b3
    P.b3 = np.float32(old + h)
    lp, _ = orc.mlp_backward(X, f, P, quantize=False)
    P.b3 = np.float32(old - h)
    lm, _ = orc.mlp_backward(X, f, P, quantize=False)
    P.b3 = old
    assert abs((lp - lm) / (2 * h) - float(g.b3)) < 1e-8


def test_loss_is_bce_with_logits(orc):
    rng = np.random.default_rng(3)
    P = rand_params(orc, rng)
    X = rng.normal(size=(20, 16)).astype(np.float32)
    f = rng.uniform(size=20).astype(np.float32)
    s = orc.mlp_forward(X, P, quantize=False).astype(np.float64)
    loss, _ = orc.mlp_backward(X, f, P, quantize=False)
    p = 1 / (1 + np.exp(-s))
    ref = np.mean(-(f * np.log(p) + (1 - f) * np.log(1 - p)))
    assert abs(loss - ref) < 1e-5 * ref


def test_adam_first_step_is_sign(orc):
    rng = np.random.default_rng(4)
    p = rng.normal(size=100).astype(np.float32)
    g = rng.normal(size=100).astype(np.float32)
    m = np.zeros(100, np.float32)
    v = np.zeros(100, np.float32)
    p0 = p.copy()
    orc.adam(p, g, m, v, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1)
    assert np.allclose(p0 - p, 1e-3 * np.sign(g), rtol=1e-4)


def test_features_properties(orc):
    xy, d = I.make_instance("clustered", 300, seed=9, clusters=5, sigma=400.0)
    knn, feat = orc.knn_features(d, xy.astype(np.float32))
    n = 300
    assert np.array_equal(knn.astype(np.int64), np.argsort(d + np.eye(n, dtype=np.int64) * 10 ** 9, axis=1,
                                                           kind="stable")[:, :16])
    F = feat.reshape(n, 16, 8)
    assert np.all(F[:, :, 1] == (np.arange(16, dtype=np.float32) / np.float32(15))[None, :])
    # distances relative to the mean: they average to 1 over a row
    assert np.allclose(F[:, :, 0].mean(axis=1), 1.0, rtol=1e-5)
    # reverse rank < 1 exactly when i is among the 16 nearest of j
    for i in range(0, n, 37):
        for r in range(16):
            j = knn[i, r]
            assert (F[i, r, 2] < 1) == (i in knn[j])
    indeg = np.bincount(knn.ravel(), minlength=n)
    assert np.allclose(F[:, 0, 6], indeg / 16.0)
    # relative coordinates: (dx, dy) * dbar has length d_ij (up to rounding)
    dbar = d[np.arange(n)[:, None], knn].mean(axis=1)
    lens = np.hypot(F[:, :, 3], F[:, :, 4]) * dbar[:, None]
    assert np.allclose(lens, d[np.arange(n)[:, None], knn], atol=0.51 + 1e-3 * lens)


def test_install_identity_and_scaling(orc):
    xy, d = I.make_instance("uniform", 120, seed=10)
    knn, _ = orc.knn_features(d, xy.astype(np.float32))
    zero = np.zeros((120, 16), np.float32)
    col = orc.Colony(d, ants=1, cand_len=8, beta=2)
    plain = col.heuristic()
    assert np.array_equal(orc.install_eta(d, knn, zero, 2).view(np.uint32), plain.view(np.uint32))
    s = np.random.default_rng(0).normal(size=(120, 16)).astype(np.float32)
    h = orc.install_eta(d, knn, s, 1)
    i, r = 5, 3
    j = knn[i, r]
    assert math.isclose(h[i, j], (1 / d[i, j]) * 2 / (1 + math.exp(-s[i, r])), rel_tol=3e-7)
    # an unscored edge takes the multiplier of its row's lowest score
    mask = np.ones((120, 120), bool)
    mask[np.arange(120)[:, None], knn] = False
    np.fill_diagonal(mask, False)
    smin = s.astype(np.float64).min(axis=1)
    dd = np.where(np.eye(120, dtype=bool), 1, d).astype(np.float64)  # the diagonal is excluded below
    want = (1.0 / dd) * (2.0 / (1.0 + np.exp(-smin)))[:, None]
    assert np.allclose(h[mask], want[mask], rtol=1e-6)
    # the unscored multiplier h*d of a row is the smallest scored one
    mult = h * dd
    rows = np.arange(120)
    scored_min = mult[rows[:, None], knn].min(axis=1)
    for i in (0, 17, 119):
        assert np.allclose(mult[i][mask[i]], scored_min[i], rtol=1e-6)
