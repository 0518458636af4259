"""Runtime services on the GPU. Checkpoint and resume (mmas_restore): a context restored from
a run stopped after iteration t-1 and driven from iteration t repeats the
uninterrupted run bit for bit, and both equal the oracle."""
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
    from paper_2003_11902_amd import mmas  # noqa: F401  (fails loudly if not built)
    return torch


def steps(col, its, oracle=False):
    out = []
    for it in its:
        if oracle:
            col.iterate(it, 8)
        else:
            col.iterate(it)
        out.append((col.tours().copy(), col.lengths().copy(), col.pheromone().copy(), col.best()[1]))
    return out


@pytest.mark.parametrize("name,kw", [
    ("dense", dict(pher="dense")),
    ("candidates_global", dict(pher="candidates", deposit="global")),
    ("atsp_list", dict(pher="dense", problem="atsp", tabu="list")),
], ids=lambda x: x if isinstance(x, str) else "")
def test_resume_repeats_the_run(gpu, name, kw):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("clustered", 300, seed=19, clusters=5, sigma=400.0)
    if kw.get("problem") == "atsp":
        d = I.asymmetric(d, 0.5, seed=20)
    say(f"resume {name}")
    args = dict(cand_len=16, rho=0.05, seed=3, **kw)
    full = steps(M.Colony(d, 80, **args), range(10))
    first = M.Colony(d, 80, **args)
    steps(first, range(4))
    ck = first.checkpoint()
    resumed = M.Colony(d, 80, **args)
    resumed.restore(ck)
    rest = steps(resumed, range(4, 10))
    okw = dict(cand_len=16, rho=0.05, seed=3, deposit=kw.get("deposit", "iteration"),
               problem=kw.get("problem", "tsp"),
               pher_mode=O.PHER_DENSE if kw["pher"] == "dense" else O.PHER_CANDIDATES)
    ref = steps(O.Colony(d, 80, **okw), range(10), oracle=True)
    for k, ((t1, l1, p1, b1), (t2, l2, p2, b2)) in enumerate(zip(full[4:], rest)):
        it = 4 + k
        assert np.array_equal(t1, t2) and np.array_equal(l1, l2) and b1 == b2, it
        assert np.array_equal(p1.view(np.uint32), p2.view(np.uint32)), it
        assert np.array_equal(t2, ref[it][0]) and b2 == ref[it][3], it
        assert np.array_equal(p2.view(np.uint32), ref[it][2].view(np.uint32)), it


def test_restore_rejects_bad_checkpoints(gpu):
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 50, seed=4)
    g = M.Colony(d, 10, cand_len=8)
    g.iterate(0)
    ck = g.checkpoint()
    bad_tour = dict(ck, gb_tour=np.zeros(50, np.uint16))
    with pytest.raises(M.MmasError) as e:
        g.restore(bad_tour)
    assert e.value.status == M.MMAS_EINVAL
    st = M.mmas_device_state.from_buffer_copy(ck["state"])
    st.tau_min = 0.0
    with pytest.raises(M.MmasError) as e:
        g.restore(dict(ck, state=st))
    assert e.value.status == M.MMAS_EINVAL
    tau = ck["pheromone"].copy()
    tau.reshape(-1)[3] = np.nan
    with pytest.raises(M.MmasError) as e:
        g.restore(dict(ck, pheromone=tau))
    assert e.value.status == M.MMAS_EINVAL
    g.restore(ck)  # the good checkpoint still restores
    assert g.best()[1] == ck["state"].gb_len


def test_per_call_timing(gpu):
    """mmas_set_timing: launch counts per kind and GPU milliseconds that agree
    with HIP events taken around the same construction calls."""
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 400, seed=6)
    g = M.Colony(d, 400, cand_len=16, ls_nn=8)
    g.iterate(0)
    assert all(v == (0.0, 0) for v in g.read_timing().values())  # off by default
    g.set_timing(True)
    ev = []
    for it in range(1, 6):
        a, b = gpu.cuda.Event(enable_timing=True), gpu.cuda.Event(enable_timing=True)
        g.prepare_choice_info()
        a.record(g.stream)
        g.construct(it)
        b.record(g.stream)
        g.two_opt()
        g.update_pheromone()
        ev.append((a, b))
    gpu.cuda.synchronize()
    t = g.read_timing(reset=True)
    assert t["construct"][1] == 5 and t["two_opt"][1] == 5 and t["update"][1] == 5
    assert t["choice"][1] == 0  # the fused update keeps choice_info current
    ref = sum(a.elapsed_time(b) for a, b in ev)
    assert t["construct"][0] > 0 and abs(t["construct"][0] - ref) <= 0.2 * ref + 0.05
    assert g.read_timing()["construct"] == (0.0, 0)  # reset
    g.set_timing(False)
    g.iterate(6)
    assert g.read_timing()["construct"] == (0.0, 0)


def test_update_needs_new_tours(gpu):
    """Alg. 1 deposits each iteration's tours once: a second update without a
    construction in between is refused, and the trails stay as they were."""
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 60, seed=8)
    g = M.Colony(d, 12, cand_len=8)
    g.iterate(0)
    tau = g.pheromone().copy()
    with pytest.raises(M.MmasError) as e:
        g.update_pheromone()
    assert e.value.status == M.MMAS_ESTATE
    assert np.array_equal(g.pheromone().view(np.uint32), tau.view(np.uint32))
    g.iterate(1)  # a construction re-arms it


def test_close_waits_for_enqueued_work(gpu):
    """Destroying a batch or a context right after an unsynchronised step
    leaves no work running on the stream that uses the workspace, and the
    workspace block is not handed out again before that work is done."""
    from paper_2003_11902_amd import mmas as M
    dists, params = [], []
    for k in range(6):
        _, d = I.make_instance("uniform", 300 + 50 * k, seed=40 + k)
        dists.append(d)
        params.append(M.make_params(d.shape[0], d.shape[0], cand_len=16, rho=0.05, seed=1 + k))
    b = M.Batch(dists, params)
    b.capture()
    for _ in range(3):
        b.step()
    st = b.stream
    b.close()
    assert st.query(), "the batch stream still had work after mmas_batch_destroy"
    del b
    side = gpu.cuda.Stream()
    _, d = I.make_instance("clustered", 500, seed=9, clusters=4, sigma=300.0)
    g = M.Colony(d, 500, cand_len=32, stream=side)
    g.prepare_choice_info()
    g.construct(0)
    g.close()
    assert side.query(), "the context's stream still had work after mmas_destroy"
