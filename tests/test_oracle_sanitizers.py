"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (oracle/exercise.c) calls every oracle entry point over its option
combinations (list lengths 0, 1, 8 and n - 1, both trail stores, both
selections, both deposits, symmetric and asymmetric instances, 2-opt,
checkpoint and restore, the learned-heuristic pieces). Host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


def test_oracle_is_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "exercise")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-D_GNU_SOURCE", "-I", ORC,
           os.path.join(ORC, "exercise.c"), os.path.join(ORC, "mmas_oracle.c"),
           os.path.join(ORC, "learned_oracle.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr
    assert "all runs completed" in run.stdout
