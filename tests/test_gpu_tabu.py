"""The construction's three tabu structures (Sec. 4.1) on their own, through
mmas_eval_tabu: the worked examples of the list and compact tabus (readings
C-18 and C-19) and random marking sequences against a plain set."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_11902_amd import mmas  # noqa: F401
    return torch


def run(gpu, tabu, n, marks):
    from paper_2003_11902_amd import mmas as M
    t = gpu.tensor(np.asarray(marks, dtype=np.int32)).cuda()
    return M.mmas_eval_tabu(tabu, n, t)


def test_list_tabu_worked_example(gpu):
    """Sec. 4.1's example: removing 2, 5 and 7 from 0..7 leaves indices 7, 6, 5
    for them (n - 1 - index recovers the visit order 0, 1, 2) and the
    unvisited list [0, 1, 6, 3, 4]."""
    visited, cells, left = run(gpu, "list", 8, [2, 5, 7])
    unv, idx = cells[:8], cells[8:]
    assert left == 5
    assert [int(idx[v]) for v in (2, 5, 7)] == [7, 6, 5]
    assert [8 - 1 - int(idx[v]) for v in (2, 5, 7)] == [0, 1, 2]
    assert unv[:5].tolist() == [0, 1, 6, 3, 4]
    assert np.flatnonzero(visited).tolist() == [2, 5, 7]


def test_compact_tabu_worked_example(gpu):
    """Sec. 4.1's compact tabu after removing 2, 5 and 7 from 0..7, with the
    sentinel n written for a relocated city (reading C-19): entries
    [0, 1, 6, 3, 4, 6, 2, 8], five unvisited, visited iff entries[u] > u."""
    visited, cells, left = run(gpu, "compact", 8, [2, 5, 7])
    assert left == 5
    assert cells.tolist() == [0, 1, 6, 3, 4, 6, 2, 8]
    assert sorted(cells[:5].tolist()) == [0, 1, 3, 4, 6]
    assert np.flatnonzero(visited).tolist() == [2, 5, 7]


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
@pytest.mark.parametrize("n", [1, 7, 33, 1000, 8192])
def test_random_marks_against_a_set(gpu, tabu, n):
    rng = np.random.default_rng(n)
    order = rng.permutation(n)
    for count in sorted({0, 1, n // 3, n - 1, n} - {-1}):
        if count < 0:
            continue
        marks = order[:count]
        visited, cells, left = run(gpu, tabu, n, marks)
        want = np.zeros(n, np.uint8)
        want[marks] = 1
        assert np.array_equal(visited, want), (tabu, n, count)
        assert left == n - count
        unvisited = set(np.flatnonzero(want == 0).tolist())
        if tabu == "bitmask":
            words = cells.view(np.uint32)
            bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:n]
            assert np.array_equal(bits, want)
        elif tabu == "compact":
            assert set(cells[:left].tolist()) == unvisited
        else:
            unv, idx = cells[:n], cells[n:]
            assert set(unv[:left].tolist()) == unvisited
            assert np.array_equal(unv[idx], np.arange(n))  # idx is unv's inverse
            # the visited cities sit after the list, the latest first
            assert unv[left:].tolist() == marks[::-1].tolist()


@pytest.mark.parametrize("tabu", ["bitmask", "compact", "list"])
def test_bad_marks_are_reported(gpu, tabu):
    assert run(gpu, tabu, 10, [3, 3])[2] == -1
    assert run(gpu, tabu, 10, [4, 10])[2] == -1
    assert run(gpu, tabu, 10, [-1])[2] == -1
