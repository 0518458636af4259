"""Helpers shared by the distribution tests: a chi-square check of observed
selection counts against exact probabilities, candidate lists straight from
the distances, and the exact probability of every tour of a tiny instance
under Eq. (1) restricted to the candidate list (Sec. 4.3). None of this is
the oracle's or the library's code."""
import itertools

import numpy as np
from scipy import stats


def chi2_ok(counts: dict, probs: dict, draws: int, pmin=1e-3):
    keys = sorted(probs)
    obs = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    exp = np.array([probs[k] for k in keys]) * draws
    # never a node outside the support
    assert sum(counts.values()) == obs.sum() == draws, "selected a node with zero probability"
    chi2_arrays(obs, exp, pmin)


def chi2_arrays(obs, exp, pmin=1e-3):
    """Pearson's test of observed against expected counts (same total); bins
    with an expectation below 5 are pooled into one."""
    obs = np.asarray(obs, dtype=np.float64).ravel()
    exp = np.asarray(exp, dtype=np.float64).ravel()
    assert np.all(obs[exp == 0] == 0), "a count where the probability is zero"
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    small = exp < 5
    if small.any():
        obs = np.append(obs[~small], obs[small].sum())
        exp = np.append(exp[~small], exp[small].sum())
    exp = exp * (obs.sum() / exp.sum())  # guard against float drift in the total
    p = stats.chisquare(obs, exp).pvalue
    assert p > pmin, (p, obs.size)
    return p


def ref_candidates(dist, cl):
    n = dist.shape[0]
    out = np.zeros((n, cl), dtype=np.int64)
    for i in range(n):
        js = np.array([j for j in range(n) if j != i])
        order = np.lexsort((js, dist[i, js]))  # by distance, then index
        out[i] = js[order][:cl]
    return out


def exact_tour_probs(dist, tau, cl, alpha, beta):
    """P(tour) = (1/n) * prod over steps of Eq. (1) restricted as in Sec. 4.3."""
    n = dist.shape[0]
    cands = ref_candidates(dist, cl)
    w = tau.astype(np.float64) ** alpha * (1.0 / np.where(dist > 0, dist, 1)) ** beta
    probs = {}
    for perm in itertools.permutations(range(n)):
        p = 1.0 / n
        vis = {perm[0]}
        for k in range(1, n):
            c = perm[k - 1]
            S = [j for j in cands[c] if j not in vis]
            if not S:
                S = [j for j in range(n) if j not in vis]
            p *= (w[c, perm[k]] / sum(w[c, j] for j in S)) if perm[k] in S else 0.0
            vis.add(perm[k])
        if p > 0:
            probs[perm] = p
    assert abs(sum(probs.values()) - 1.0) < 1e-9
    return probs


def u01(x):
    """random(0,1) of a 32-bit draw: (2 floor(x / 2^9) + 1) 2^-24, exact in FP32."""
    x = np.asarray(x, dtype=np.uint64)
    return ((2 * (x >> np.uint64(9)) + 1).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def sequential_wheel_tours(tours, tau, cand, draw, seed, it):
    """Checks tours built by the roulette wheel with integer weights (beta = 0,
    alpha = 1, tau holding small integers, so every partial sum is exact in
    FP32 whatever the order): the textbook wheel picks, among the eligible
    entries in order (the unvisited candidates by rank, else every unvisited
    node by index), the first whose running total exceeds fl(u * total).
    `draw(seed, it, ant, step)` gives the step's 32-bit draw (slot 0).
    Returns the first (ant, step) that disagrees, or None."""
    ants, n = tours.shape
    cl = cand.shape[1] if cand is not None else 0
    for a in range(ants):
        t = tours[a]
        vis = np.zeros(n, bool)
        vis[t[0]] = True
        for k in range(1, n):
            c = int(t[k - 1])
            elig = None
            if cl:
                cs = cand[c]
                cs = cs[~vis[cs]]
                if cs.size:
                    elig = cs
            if elig is None:
                elig = np.flatnonzero(~vis)
            w = tau[c, elig].astype(np.float64)
            cum = np.cumsum(w)
            u = u01(draw(seed, it, a, k))
            target = np.float32(u) * np.float32(cum[-1])
            pick = int(elig[int(np.argmax(cum > np.float64(target)))]) if (cum > target).any() \
                else int(elig[np.flatnonzero(w > 0)[-1]])
            if pick != int(t[k]):
                return a, k
            vis[pick] = True
    return None
