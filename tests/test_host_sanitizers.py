"""The library's host code (argument validation, the launch planner, the
Sobol direction-number expansion, the workspace layout) under
AddressSanitizer and UndefinedBehaviorSanitizer: a build with the host side
instrumented (device code unchanged) runs a few thousand random problems and
parameters, mostly valid, through the calls that need no GPU.  Any report
aborts the child process.  (GPU code cannot run under a sanitizer here.)"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2504_02627_amd import build
    rt = build.sanitizer_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime")
    lib = build.build_sanitized(tmp_path / "libchees_smc_san.so")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "_host_fuzz.py"), lib, "3000"],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host fuzz: 3000 cases" in r.stdout
    accepted = int(r.stdout.split("cases, ")[1].split()[0])
    assert accepted > 500            # the planner ran on many shapes
