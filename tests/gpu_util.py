"""Helpers for the GPU parity tests: run the HIP library and the oracle side
by side on the same seeded instance and compare."""
import sys

import numpy as np

from paper_2003_11902_amd import instances as I


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(dist, ants, cand_len=32, alpha=1, beta=2, rho=0.02, seed=1, tabu="bitmask",
              pher="dense", ls_nn=0, deposit="iteration", select="wrs", problem="tsp"):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M

    g = M.Colony(dist, ants, cand_len=cand_len, alpha=alpha, beta=beta, rho=rho, seed=seed,
                 tabu=tabu, pher=pher, ls_nn=ls_nn, deposit=deposit, problem=problem)
    if select != "wrs":
        g.set_selection(select)
    o = O.Colony(dist, ants, cand_len=cand_len, alpha=alpha, beta=beta, rho=rho, seed=seed,
                 pher_mode=O.PHER_DENSE if pher == "dense" else O.PHER_CANDIDATES, ls_nn=ls_nn,
                 deposit=deposit, select=select, problem=problem)
    return g, o


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.maximum(np.abs(b), 1e-300)
    return float(np.max(np.abs(a - b) / den)) if a.size else 0.0


def compare_iteration(g, o, it, check_tau=True):
    """Tours bit-exact, lengths exact, trails within 1e-6 relative (expected
    bit-identical), limits and global best equal."""
    gt, ot = g.tours(), o.tours()
    if not np.array_equal(gt, ot):
        bad = np.flatnonzero((gt != ot).any(axis=1))
        a = int(bad[0])
        k = int(np.flatnonzero(gt[a] != ot[a])[0])
        raise AssertionError(f"iteration {it}: {bad.size} tours differ; ant {a} first at step {k}: "
                             f"gpu {gt[a, max(0, k-2):k+3]} oracle {ot[a, max(0, k-2):k+3]}")
    assert np.array_equal(g.lengths(), o.lengths()), f"iteration {it}: lengths differ"
    gs, os_ = g.fallback()
    ostep, onode = o.fallback()
    assert np.array_equal(gs, ostep) and np.array_equal(os_, onode), f"iteration {it}: fallback counts differ"
    if check_tau:
        gtau, otau = g.pheromone(), o.pheromone()
        e = rel_err(gtau, otau)
        assert e <= 1e-6, f"iteration {it}: pheromone rel err {e}"
        assert tuple(g.limits()) == tuple(o.limits()), f"iteration {it}: limits differ"
        assert g.best()[1] == o.best()[1]
        return bool(np.array_equal(gtau.view(np.uint32), otau.view(np.uint32)))
    return True


def run_parity(dist, iterations, nthreads=8, launch=None, **kw):
    """`launch` = (ants_per_block, table_rows, lanes_per_ant) for the GPU side."""
    g, o = make_pair(dist, **kw)
    if launch is not None:
        g.set_launch(*launch)
    identical = True
    for it in range(iterations):
        g.iterate(it)
        o.iterate(it, nthreads)
        identical &= compare_iteration(g, o, it)
    assert g.state().flags == 0
    return g, o, identical
