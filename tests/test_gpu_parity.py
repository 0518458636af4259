"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs. Tours and lengths must match bit for bit at every iteration; trails
within 1e-6 relative in FP32 (they are expected to be bit-identical, since
both sides round the same FP32 operations in the same order)."""
import numpy as np
import pytest

from paper_2003_11902_amd import instances as I
from tests.gpu_util import compare_iteration, make_pair, run_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401  (fails loudly if not built)
    return torch


def test_device_log_exhaustive(gpu):
    """The device logarithm equals the oracle's on all 2^23 values of u."""
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    k = np.arange(1 << 23, dtype=np.uint64)
    u = ((2 * k + 1).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    ref = O.logf_n(u)
    out = M.mmas_eval_log(gpu.from_numpy(u).cuda()).cpu().numpy()
    gpu.cuda.synchronize()
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))


def test_device_draws_match_oracle(gpu):
    from oracle import oracle as O
    from paper_2003_11902_amd import mmas as M
    rng = np.random.default_rng(0)
    m = 1 << 20
    it = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    ant = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
    step = rng.integers(0, 1 << 16, m).astype(np.uint32)
    slot = rng.integers(0, 1 << 18, m).astype(np.uint32)
    seed = 0x123456789ABCDEF
    ref = O.draw_words(seed, it, ant, step, slot)
    t = [gpu.from_numpy(a.view(np.int32)).cuda() for a in (it, ant, step, slot)]
    out = M.mmas_eval_draws(seed, *t).cpu().numpy().view(np.uint32)
    assert np.array_equal(out, ref)


def test_oracle_philox_matches_rocrand(gpu):
    """Pins the oracle's Philox4x32-10 to an independent implementation:
    rocRAND's PHILOX4_32_10 stream for seed s is the blocks at counters
    (i, 0, 0, 0), i = 0, 1, ..., key (s low, s high), words in order."""
    import ctypes as C
    from oracle import oracle as O
    try:
        lib = C.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("rocRAND not available")
    gen = C.c_void_p()
    if lib.rocrand_create_generator_host_blocking(C.byref(gen), 404) != 0:
        pytest.skip("rocRAND host generator unavailable")
    try:
        for seed in (0, 1, 0xDEADBEEF12345678):
            assert lib.rocrand_set_seed(gen, C.c_ulonglong(seed)) == 0
            out = np.zeros(4096, dtype=np.uint32)
            st = lib.rocrand_generate(gen, out.ctypes.data_as(C.c_void_p), C.c_size_t(out.size))
            if st != 0:
                pytest.skip(f"rocrand_generate status {st}")
            key = [seed & 0xFFFFFFFF, seed >> 32]
            ref = np.concatenate([O.philox([i, 0, 0, 0], key) for i in range(1024)])
            assert np.array_equal(out, ref), seed
    finally:
        lib.rocrand_destroy_generator(gen)


@pytest.mark.parametrize("workload", ["uniform198", "clustered1002"])
def test_setup_parity(gpu, workload):
    xy, d, w = I.workload_instance(workload)
    say(f"setup parity {workload}")
    g, o = make_pair(d, ants=w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=11)
    g.prepare_choice_info()
    o.prepare_choice()
    assert np.array_equal(g.cand(), o.cand())
    heur = g.read(5).reshape(g.n, g.n)
    assert np.array_equal(heur.view(np.uint32), o.heuristic().view(np.uint32))
    assert np.array_equal(g.read(9), o.nn_tour()[0])
    assert g.state().nn_len == o.nn_tour()[1]
    assert tuple(g.limits()) == tuple(o.limits())
    assert np.array_equal(g.pheromone(), o.pheromone())
    assert np.array_equal(g.choice().view(np.uint32), o.choice().view(np.uint32))
    assert np.array_equal(g.chc().view(np.uint32), o.chc().view(np.uint32))


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
def test_uniform198_full_run(gpu, tabu):
    """The n = 198 workload: 198 ants, cl 32, 20 iterations, every iteration."""
    xy, d, w = I.workload_instance("uniform198")
    say(f"uniform198 {tabu}")
    g, o, same = run_parity(d, w["iterations"], ants=w["ants"], cand_len=w["cand_len"],
                            rho=w["rho"], seed=1, tabu=tabu)
    assert same, "trails agree within 1e-6 but are not bit-identical"


CASES = [
    # (name, kind, n, instance seed, params)
    ("n3", "uniform", 3, 1, dict(ants=5, cand_len=32)),
    ("n4_cl1", "uniform", 4, 2, dict(ants=9, cand_len=1)),
    ("ragged37_cl8", "clustered", 37, 3, dict(ants=50, cand_len=8)),
    ("no_list130", "uniform", 130, 4, dict(ants=64, cand_len=0)),
    ("cl64_257", "uniform", 257, 5, dict(ants=33, cand_len=64)),
    ("cl_odd_101", "clustered", 101, 6, dict(ants=70, cand_len=13)),
    ("alpha0_beta0", "uniform", 90, 7, dict(ants=40, cand_len=10, alpha=0, beta=0)),
    ("alpha2_beta3", "uniform", 90, 8, dict(ants=40, cand_len=10, alpha=2, beta=3, rho=0.3)),
    ("cand_mode300", "uniform", 300, 9, dict(ants=64, cand_len=10, pher="candidates")),
    ("cand_mode_cl1", "clustered", 150, 10, dict(ants=20, cand_len=1, pher="candidates", rho=0.5)),
    ("one_ant", "uniform", 500, 11, dict(ants=1, cand_len=16)),
    ("ants_not_mult4", "uniform", 199, 12, dict(ants=1003 % 64 + 3, cand_len=32)),
    # group boundaries of the draws computed one group ahead (8 steps a group
    # for 17 <= cl <= 32, 16 for 9 <= cl <= 16): a tour of exactly two groups,
    # one step more, a whole number of groups, and one step past a 64-step
    # chunk of the tour
    ("groups_n24_cl20", "uniform", 24, 13, dict(ants=24, cand_len=20)),
    ("groups_n25_cl20", "clustered", 25, 14, dict(ants=24, cand_len=20)),
    ("groups_n21_cl20", "uniform", 21, 19, dict(ants=24, cand_len=20)),
    ("groups_n32_cl12", "uniform", 32, 15, dict(ants=24, cand_len=12)),
    ("groups_n33_cl12", "clustered", 33, 16, dict(ants=24, cand_len=12)),
    ("groups_n65_cl24", "uniform", 65, 17, dict(ants=40, cand_len=24)),
    ("groups_n129_cl16", "clustered", 129, 18, dict(ants=40, cand_len=16)),
]


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_edge_cases(gpu, case, tabu):
    name, kind, n, seed, kw = case
    _, d = I.make_instance(kind, n, seed=seed, side=1e4 if kind == "uniform" else 1e4,
                           **({} if kind == "uniform" else dict(clusters=4, sigma=400.0)))
    say(f"edge case {name} {tabu}")
    kw = dict(kw)
    kw.setdefault("rho", 0.1)
    run_parity(d, 6, tabu=tabu, seed=seed, **kw)


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
def test_clustered1002_first_iterations(gpu, tabu):
    """The n = 1002 workload (1002 ants, cl 32), first 4 iterations."""
    xy, d, w = I.workload_instance("clustered1002")
    say(f"clustered1002 {tabu}")
    g, o, _ = run_parity(d, 4, ants=w["ants"], cand_len=w["cand_len"], rho=w["rho"], seed=2, tabu=tabu)
    s, _ = g.fallback()
    assert s.sum() > 0  # the fallback really ran


def test_bitmask_equals_compact_and_repeatable(gpu):
    _, d = I.make_instance("clustered", 400, seed=21, clusters=6, sigma=300.0)
    from paper_2003_11902_amd import mmas as M
    runs = []
    for tabu in ("bitmask", "compact", "list", "bitmask"):
        g = M.Colony(d, 200, cand_len=12, rho=0.05, seed=5, tabu=tabu)
        tours = []
        for it in range(5):
            g.iterate(it)
            tours.append(g.tours())
        runs.append((np.stack(tours), g.pheromone()))
    for r in runs[1:]:
        assert np.array_equal(r[0], runs[0][0])
        assert np.array_equal(r[1], runs[0][1])


def test_error_paths(gpu):
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 50, seed=3)
    bad = d.copy()
    bad[3, 7] += 1
    with pytest.raises(M.MmasError) as e:
        M.Colony(bad, 10, cand_len=8)
    assert e.value.status == M.MMAS_EINVAL
    bad = d.copy()
    bad[3, 7] = bad[7, 3] = 0
    with pytest.raises(M.MmasError) as e:
        M.Colony(bad, 10, cand_len=8)
    assert e.value.status == M.MMAS_EINVAL
    g = M.Colony(d, 10, cand_len=8)
    with pytest.raises(M.MmasError) as e:
        g.update_pheromone()
    assert e.value.status == M.MMAS_ESTATE
    with pytest.raises(M.MmasError) as e:
        g.two_opt()
    assert e.value.status == M.MMAS_EUNSUPPORTED
    import ctypes as C
    ctx = C.c_void_p()
    p = M.make_params(50, 10, 8)
    need = M.mmas_workspace_bytes(p)
    assert M.lib.mmas_create(d.ctypes.data_as(C.c_void_p), C.byref(p), C.c_void_p(g.ws.data_ptr()),
                             need - 256, None, C.byref(ctx)) == M.MMAS_ENOSPACE
    assert g.best() == (None, -1)
    g.iterate(0)
    t, length = g.best()
    assert length > 0 and sorted(t.tolist()) == list(range(50))


@pytest.mark.parametrize("launch,tabu,pher,cl,ants", [
    ((1, 0, 64, 1), "bitmask", "dense", 32, 101),
    ((8, -1, 64, 1), "compact", "dense", 32, 101),
    ((16, 50, 64, 1), "bitmask", "candidates", 20, 64),
    ((2, -1, 32, 0), "bitmask", "dense", 32, 101),
    ((4, 0, 32, 0), "compact", "dense", 32, 101),
    ((8, 60, 32, 0), "bitmask", "candidates", 16, 64),
    ((16, -1, 32, 0), "compact", "candidates", 7, 33),
    ((4, -1, 32, 1), "bitmask", "dense", 0, 20),  # no list: 32 lanes fall back to one ant per wave
    ((0, -1, 64, 2), "bitmask", "dense", 32, 101),
    ((0, 0, 64, 4), "compact", "dense", 32, 64),
    ((0, 40, 64, 8), "bitmask", "candidates", 16, 33),
    ((0, -1, 64, 16), "compact", "candidates", 5, 20),
    ((0, -1, 64, 16), "bitmask", "dense", 0, 20),  # every step is a fallback
    ((4, -1, 64, 1), "list", "dense", 32, 101),
    ((8, -1, 32, 0), "list", "candidates", 16, 64),
    ((0, -1, 64, 8), "list", "dense", 0, 20),
    ((0, 0, 64, 0), "bitmask", "dense", 32, 101),  # waves from the ant count
    ((2, -1, 64, 0), "list", "candidates", 12, 63),  # a draw helper wave per ant; the last workgroup has one ant
    ((8, 0, 64, 0), "compact", "dense", 20, 101),  # eight ants and eight helpers a workgroup
    ((16, -1, 64, 0), "bitmask", "dense", 32, 101),  # sixteen asked for: eight with helpers
    ((0, 0, 64, 4), "bitmask", "dense", 16, 101),  # cl 9..16, rows from global memory
    ((0, 100, 64, 2), "compact", "dense", 9, 33),
    ((0, 0, 64, 8), "list", "candidates", 12, 64),
])
def test_launch_shapes_match_oracle(gpu, launch, tabu, pher, cl, ants):
    """Ants per workgroup, LDS table rows, two ants per wave (32 lanes each)
    and several waves per ant never change tours, lengths, fallback counts or
    trails; odd ant counts leave the last wave with one ant."""
    _, d = I.make_instance("clustered", 230, seed=77, clusters=5, sigma=500.0)
    say(f"launch {launch} {tabu} {pher} cl={cl} ants={ants}")
    run_parity(d, 3, launch=launch, ants=ants, cand_len=cl, rho=0.05, seed=9, tabu=tabu, pher=pher)


@pytest.mark.parametrize("pher", ["dense", "candidates"])
def test_global_best_deposit(gpu, pher):
    """The global-best deposit (Sec. 2.1): 25 iterations on 150 cities with few
    ants, so that many iterations have an iteration best worse than the
    global best; tours, lengths and trails equal the oracle's every
    iteration."""
    _, d = I.make_instance("clustered", 150, seed=31, clusters=5, sigma=400.0)
    say(f"global-best deposit {pher}")
    run_parity(d, 25, ants=6, cand_len=10, rho=0.1, seed=3, pher=pher, deposit="global")


def test_roulette_wheel_needs_bitmask(gpu):
    from paper_2003_11902_amd import mmas as M
    _, d = I.make_instance("uniform", 50, seed=3)
    g = M.Colony(d, 10, cand_len=8, tabu="compact")
    with pytest.raises(M.MmasError) as e:
        g.set_selection("prwm")
    assert e.value.status == M.MMAS_EUNSUPPORTED


@pytest.mark.parametrize("tabu", ["list", "compact", "bitmask"])
@pytest.mark.parametrize("cl,waves,pher", [(0, 0, "dense"), (0, 16, "dense"), (1, 4, "dense"), (3, 2, "candidates"),
                                             (0, 1, "dense"), (2, 1, "candidates")])
def test_wide_fallback_by_draw_blocks(gpu, tabu, cl, waves, pher):
    """Fallbacks of one wave per ant (keyed by list entries) or of several
    waves sharing them (keyed by draw blocks while most cities are unvisited,
    by list entries later): tours and trails equal the oracle's (no list or
    short lists, so fallbacks start early)."""
    _, d = I.make_instance("clustered", 600, seed=41, clusters=5, sigma=400.0)
    say(f"wide fallback {tabu} cl {cl} waves {waves} {pher}")
    run_parity(d, 3, ants=40, cand_len=cl, rho=0.1, seed=2, tabu=tabu, pher=pher, launch=(0, -1, 64, waves))


@pytest.mark.parametrize("n,pher,ants,waves", [(257, "dense", 40, 0), (1021, "dense", 20, 4),
                                               (64, "dense", 300, 4), (5, "dense", 3, 0), (1024, "dense", 8, 0),
                                               (600, "dense", 300, 0)])
def test_team_without_list(gpu, n, pher, ants, waves):
    """No candidate list, bitmask tabu, n <= 1024: the team launch (four waves
    per ant, one word of every draw block each, visited bits in registers) is
    taken by default or with four waves asked for; tours, lengths, fallback
    counts and trails equal the oracle's. The sizes cover a partial last
    round of blocks (257), four rounds (1021, 1024), one partial round (64,
    5), and more ants than SIMDs hold four waves each (300 ants: 1200 waves,
    asked for and by default)."""
    _, d = I.make_instance("uniform", n, seed=n + 3, side=1e5)
    say(f"team no list n={n} {pher} ants={ants} waves={waves}")
    run_parity(d, 3, ants=ants, cand_len=0, rho=0.1, seed=4, tabu="bitmask", pher=pher, launch=(0, -1, 64, waves))
