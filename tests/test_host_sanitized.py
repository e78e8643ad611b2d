"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle (oracle/oracle.c) and the library's host sources (runtime,
C ABI, sampler, server, planner, autotuner) are rebuilt with
-fsanitize=address,undefined and their host-only paths -- argument
validation of every entry point, the planner, the Gray tables, the lossy
matrix check, and the oracle's formulas, sampler and isometry -- run in a
subprocess with the sanitizer runtime preloaded.  Any report fails the test.
The kernels' own per-lane code runs sanitized in the CPU emulation
(tests/test_emu.py)."""
import os
import subprocess
import sys

import pytest

from tests.sanitize import build_sanitized as S

HERE = os.path.dirname(os.path.abspath(__file__))


def _run(what):
    env = dict(os.environ, LD_PRELOAD=S.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    p = subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "run_host_paths.py"), what],
                       capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    return p.stdout


def test_oracle_under_sanitizers():
    S.build_oracle()
    assert "oracle paths ok" in _run("oracle")


def test_library_host_code_under_sanitizers():
    if not list(S.KOBJ.glob("*_hip.o")):
        pytest.skip("kernel objects not built (python -m paper_2309_07027_amd.build)")
    S.build_library()
    assert "library host paths ok" in _run("library")
