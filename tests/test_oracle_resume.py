"""Checkpoint and resume of Alg. 1 on the oracle: the state carried from one
iteration to the next is the trails, the trail limits and the global best;
draws are keyed by the iteration number, so a fresh colony restored after
iteration t and run from t repeats the uninterrupted run exactly."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I


def run(col, its):
    out = []
    for it in its:
        col.iterate(it, nthreads=4)
        out.append((col.tours().copy(), col.lengths().copy(), col.pheromone().copy(), col.best()[1]))
    return out


@pytest.mark.parametrize("kw", [
    dict(),
    dict(pher_mode=1, deposit="global"),
    dict(problem="atsp"),
], ids=["dense", "candidates-global", "atsp"])
def test_resume_repeats_the_uninterrupted_run(orc, kw):
    _, d = I.make_instance("clustered", 120, seed=9, clusters=4, sigma=500.0)
    if kw.get("problem") == "atsp":
        d = I.asymmetric(d, 0.5, seed=10)
    args = dict(ants=30, cand_len=10, rho=0.1, seed=7, **kw)
    full = run(orc.Colony(d, **args), range(12))
    first = orc.Colony(d, **args)
    run(first, range(5))
    ck = first.checkpoint()
    resumed = orc.Colony(d, **args)
    resumed.restore(ck)
    rest = run(resumed, range(5, 12))
    for (t1, l1, p1, b1), (t2, l2, p2, b2) in zip(full[5:], rest):
        assert np.array_equal(t1, t2) and np.array_equal(l1, l2) and b1 == b2
        assert np.array_equal(p1.view(np.uint32), p2.view(np.uint32))
    # without the restore the same iterations differ
    cold = run(orc.Colony(d, **args), range(5, 12))
    assert any(not np.array_equal(a[0], b[0]) for a, b in zip(full[5:], cold))
