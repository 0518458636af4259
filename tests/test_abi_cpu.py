"""The C ABI without a GPU: the library loads, exports every entry point that
include/mmas.h declares, sizes workspaces, and rejects bad arguments before
any HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    text = open(os.path.join(ROOT, "include", "mmas.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mmas_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def M():
    from paper_2003_11902_amd import mmas
    return mmas


def test_exports_every_declared_symbol(M):
    names = declared_entry_points()
    assert len(names) >= 15
    for name in names:
        assert hasattr(M.lib, name), name
    assert set(names) == set(M.EXPORTED)


def test_struct_layouts_match_header(M):
    assert C.sizeof(M.mmas_params) == 64
    assert M.mmas_params.problem.offset == 56
    assert C.sizeof(M.mmas_device_state) == 48
    assert M.mmas_device_state.gb_len.offset == 24


def test_workspace_bytes(M):
    p = M.make_params(1002, 1002, 32)
    b = M.mmas_workspace_bytes(p)
    n = 1002
    # dist, heur, tau, choice and its reciprocal: five n*n arrays dominate
    assert 22 * n * n < b < 22 * n * n + (1 << 20)  # + tours (2 n ants)
    assert M.mmas_workspace_bytes(M.make_params(1002, 1002, 32, problem="atsp")) == b
    pc = M.make_params(18512, 64, 16, pher="candidates", ls_nn=8)
    bc = M.mmas_workspace_bytes(pc)
    assert 4 * 18512 ** 2 < bc < 4 * 18512 ** 2 + (16 << 20)


@pytest.mark.parametrize("kw", [
    dict(n=2), dict(n=65536), dict(ants=0), dict(cand_len=65), dict(cand_len=-1),
    dict(alpha=9), dict(beta=-1), dict(rho=0.0), dict(rho=1.0), dict(rho=float("nan")),
    dict(p_best=0.0), dict(p_best=1.0), dict(tabu=7), dict(pher=3),
    dict(pher="candidates", cand_len=0), dict(ls_nn=33), dict(n=10, ls_nn=10), dict(deposit=2), dict(tabu=3),
    dict(problem=2), dict(problem=-1), dict(problem="atsp", ls_nn=8),
])
def test_invalid_params_give_zero_workspace(M, kw):
    args = dict(n=100, ants=10, cand_len=8)
    args.update(kw)
    p = M.make_params(**args)
    assert M.mmas_workspace_bytes(p) == 0


def test_create_rejects_before_touching_the_gpu(M):
    p = M.make_params(10, 4, 4)
    ctx = C.c_void_p()
    dist = (C.c_int32 * 100)()
    # no workspace pointer, no output pointer, bad parameters
    assert M.lib.mmas_create(dist, C.byref(p), None, 1 << 20, None, C.byref(ctx)) == M.MMAS_EINVAL
    assert M.lib.mmas_create(dist, C.byref(p), C.c_void_p(256), 1 << 20, None, None) == M.MMAS_EINVAL
    bad = M.make_params(2, 4, 4)
    assert M.lib.mmas_create(dist, C.byref(bad), C.c_void_p(256), 1 << 20, None, C.byref(ctx)) == M.MMAS_EINVAL
    # misaligned workspace
    assert M.lib.mmas_create(dist, C.byref(p), C.c_void_p(4), 1 << 20, None, C.byref(ctx)) == M.MMAS_EINVAL
    # null contexts
    for name in ("mmas_prepare_choice_info", "mmas_two_opt", "mmas_update_pheromone", "mmas_synchronize"):
        assert getattr(M.lib, name)(None) == M.MMAS_EINVAL
    assert M.lib.mmas_construct(None, 0) == M.MMAS_EINVAL
    assert M.lib.mmas_restore(None, None, None, None) == M.MMAS_EINVAL
    assert M.lib.mmas_set_timing(None, 1) == M.MMAS_EINVAL
    assert M.lib.mmas_read_timing(None, None, None, 0) == M.MMAS_EINVAL
    assert M.lib.mmas_eval_log(None, None, 5, None) == M.MMAS_EINVAL
    M.lib.mmas_destroy(None)


def test_status_strings(M):
    for s in (0, -1, -2, -3, -4, -5):
        assert M.status_str(s)
    assert M.status_str(-99) == "unknown status"


def test_missing_library_fails_loudly(tmp_path):
    """Without the HIP library the binding refuses to import: there is no CPU
    fallback behind it."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MMAS_LIBRARY=str(tmp_path / "absent" / "libmmas.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_2003_11902_amd.mmas"], cwd=root, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr
