"""Host-side checks of bench.py: the one-GPU contract, the algorithmic byte
count behind the roofline figure, and the traffic record's guard."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n,cl,per_tour", [
    (198, 32, 39_012),        # uniform198
    (1002, 32, 198_204),      # clustered1002
    (18512, 16, 1_888_128),   # uniform18512_2opt
    (3795, 32, 751_218),      # uniform3795
])
def test_bytes_per_tour(bench, n, cl, per_tour):
    """Per tour without fallbacks: (n - 1) cl (2 + 4) for the candidate ids and
    choice_info of each step, 2n for the tour and 4n for its edge lengths."""
    assert bench.algorithmic_bytes(n, cl, 1, 0.0) == per_tour
    assert bench.algorithmic_bytes(n, cl, 10, 0.0) == 10 * per_tour
    # 4 B of choice_info per city enumerated in a fallback
    assert bench.algorithmic_bytes(n, cl, 1, 100.0) == per_tour + 400


def test_traffic_record_guard(bench):
    assert bench.measured_traffic("uniform198") is None
    v = bench.measured_traffic("clustered1002")
    assert v is None or v > 0


def test_cpu_model_is_text(bench):
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_native_oracle_build_gives_the_same_results(tmp_path):
    """The CPU baseline times the oracle built with -march=native; with
    contraction off it must compute exactly what the portable build does."""
    from oracle import build as OB
    native = OB.build(native=True)
    prog = (
        "import sys, numpy as np\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle import oracle as O\n"
        "if sys.argv[1] != '-': O.use_library(sys.argv[1])\n"
        "from paper_2003_11902_amd import instances as I\n"
        "_, d = I.make_instance('clustered', 300, seed=5, clusters=6, sigma=400.0)\n"
        "o = O.Colony(d, 60, cand_len=16, rho=0.05, seed=3)\n"
        "for it in range(3): o.iterate(it, 2)\n"
        "np.save(sys.argv[2], np.concatenate([o.tours().ravel().astype(np.int64), o.lengths(),\n"
        "        o.pheromone().view(np.uint32).ravel().astype(np.int64)]))\n")
    outs = []
    for lib, name in ((native, "native.npy"), ("-", "portable.npy")):
        r = subprocess.run([sys.executable, "-c", prog, lib, str(tmp_path / name)], capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        import numpy as np
        outs.append(np.load(tmp_path / name))
    assert (outs[0] == outs[1]).all()
