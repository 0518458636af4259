"""Seeded synthetic TSP instances: the one module that both the oracle tests and
the HIP path draw their inputs from.

It holds no arithmetic of the method (no heuristic, no pheromone, no sampling):
only city coordinates and the integer distance matrix built from them.

The paper's experiments use TSPLIB instances (Sec. 5, Tables 3-6, 9). They are
not reproduced here; these generators stand in for them with the same sizes and
the two spatial structures that matter for candidate lists: cities spread
uniformly over a square, and cities gathered in Gaussian clusters.

The asymmetric instances (the ATSP of Sec. 2.1) start from such a matrix and
add to each ordered pair (i, j) its own surcharge, floor(f u_ij d_ij) with
u_ij uniform in [0, 1): a one-way detour, so d_ij and d_ji differ while staying
positive.

Distances follow the usual Euclidean convention for integer instances,
d = floor(sqrt(dx^2 + dy^2) + 0.5), computed in float64. The problem statement
(Sec. 2.1) requires positive distances between distinct cities, so any city whose
rounded distance to an earlier city is 0 is redrawn.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_coords",
    "clustered_coords",
    "distance_matrix",
    "make_instance",
    "asymmetric",
    "WORKLOADS",
]


def _redraw_coincident(xy: np.ndarray, draw_one, rng) -> np.ndarray:
    """Redraw cities until every pair of distinct cities is at rounded distance >= 1."""
    xy = xy.copy()
    n = xy.shape[0]
    while True:
        d = distance_matrix(xy)
        d[np.arange(n), np.arange(n)] = 1
        bad_i, bad_j = np.nonzero(d <= 0)
        if bad_i.size == 0:
            return xy
        # redraw the later city of each coincident pair
        for k in np.unique(np.maximum(bad_i, bad_j)):
            xy[k] = draw_one(rng)


def uniform_coords(n: int, side: float, seed: int) -> np.ndarray:
    """n cities uniform in [0, side]^2 (float64), numpy PCG64 stream `seed`."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0.0, side, size=(n, 2))
    return _redraw_coincident(xy, lambda r: r.uniform(0.0, side, size=2), rng)


def clustered_coords(n: int, side: float, clusters: int, sigma: float, seed: int) -> np.ndarray:
    """n cities in `clusters` Gaussian clusters (std `sigma`) whose centres are
    uniform in [0, side]^2; each city picks its cluster uniformly; no clipping."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, side, size=(clusters, 2))
    which = rng.integers(0, clusters, size=n)
    xy = centres[which] + rng.normal(0.0, sigma, size=(n, 2))

    def one(r):
        return centres[r.integers(0, clusters)] + r.normal(0.0, sigma, size=2)

    return _redraw_coincident(xy, one, rng)


def distance_matrix(xy: np.ndarray) -> np.ndarray:
    """Integer Euclidean distances, nint rounding, int32, row-major n x n.

    Built row block by row block so that n = 18512 (1.37 GB of int32) does not
    need a float64 n x n temporary."""
    xy = np.asarray(xy, dtype=np.float64)
    n = xy.shape[0]
    out = np.empty((n, n), dtype=np.int32)
    block = max(1, (1 << 24) // max(n, 1))
    for s in range(0, n, block):
        e = min(n, s + block)
        dx = xy[s:e, None, 0] - xy[None, :, 0]
        dy = xy[s:e, None, 1] - xy[None, :, 1]
        out[s:e] = np.floor(np.sqrt(dx * dx + dy * dy) + 0.5).astype(np.int32)
    return out


def make_instance(kind: str, n: int, seed: int, side: float = 10000.0,
                  clusters: int = 20, sigma: float = 300.0):
    """Return (xy float64 [n,2], dist int32 [n,n]) for kind 'uniform' or 'clustered'."""
    if kind == "uniform":
        xy = uniform_coords(n, side, seed)
    elif kind == "clustered":
        xy = clustered_coords(n, side, clusters, sigma, seed)
    else:
        raise ValueError(f"unknown instance kind {kind!r}")
    return xy, distance_matrix(xy)


def asymmetric(dist: np.ndarray, frac: float, seed: int) -> np.ndarray:
    """d_ij + floor(frac * u_ij * d_ij) for i != j, u_ij uniform in [0, 1) from
    numpy PCG64 stream `seed` drawn row by row; the diagonal stays 0."""
    d = np.asarray(dist, dtype=np.int32)
    n = d.shape[0]
    rng = np.random.default_rng(seed)
    out = np.empty_like(d)
    for i in range(n):
        u = rng.random(n)
        row = d[i].astype(np.int64)
        out[i] = (row + np.floor(frac * u * row)).astype(np.int32)
    out[np.arange(n), np.arange(n)] = 0
    return out


# The synthetic workloads, sized like the paper's instances (d198, pr1002,
# d18512 and fl3795 by size only). Each entry is the recipe; the run parameters
# (ants, candidate list, rho, iterations, tabu) travel with it.
WORKLOADS = {
    "uniform198": dict(kind="uniform", n=198, seed=1, side=1e4, ants=198, cand_len=32,
                       alpha=1, beta=2, rho=0.02, iterations=20, ls_nn=0, pher="dense"),
    "clustered1002": dict(kind="clustered", n=1002, seed=2, side=1e4, clusters=20, sigma=300.0,
                          ants=1002, cand_len=32, alpha=1, beta=2, rho=0.02, iterations=500,
                          ls_nn=0, pher="dense"),
    "uniform18512_2opt": dict(kind="uniform", n=18512, seed=3, side=1e6, ants=64, cand_len=16,
                              alpha=1, beta=2, rho=0.02, iterations=200, ls_nn=8,
                              pher="candidates"),
    "uniform3795": dict(kind="uniform", n=3795, seed=5, side=1e4, ants=3795, cand_len=32,
                        alpha=1, beta=2, rho=0.02, iterations=500, ls_nn=0, pher="dense"),
    # the clustered 1002-city instance with one-way surcharges up to 50 %
    "clustered1002_atsp": dict(kind="clustered", n=1002, seed=2, side=1e4, clusters=20, sigma=300.0,
                               asym=0.5, asym_seed=7, problem="atsp", ants=1002, cand_len=32,
                               alpha=1, beta=2, rho=0.02, iterations=500, ls_nn=0, pher="dense"),
}


def workload_instance(name: str):
    """(xy, dist, recipe) for a named workload."""
    w = dict(WORKLOADS[name])
    kw = dict(kind=w["kind"], n=w["n"], seed=w["seed"], side=w.get("side", 1e4))
    if w["kind"] == "clustered":
        kw.update(clusters=w["clusters"], sigma=w["sigma"])
    xy, dist = make_instance(**kw)
    if w.get("asym"):
        dist = asymmetric(dist, w["asym"], w["asym_seed"])
    w.setdefault("problem", "tsp")
    return xy, dist, w


def batch_instances(count: int = 256, base_seed: int = 10000, n_lo: int = 100, n_hi: int = 2000):
    """The batched workload: instance k has n ~ U{n_lo..n_hi} (drawn from stream
    base_seed), uses seed base_seed + k, and is uniform when k is even and
    clustered (20 clusters, sigma 300) when k is odd."""
    rng = np.random.default_rng(base_seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for k in range(count):
        kind = "uniform" if k % 2 == 0 else "clustered"
        out.append(make_instance(kind, int(sizes[k]), base_seed + k))
    return out
