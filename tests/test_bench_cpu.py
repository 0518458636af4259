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
