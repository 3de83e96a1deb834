"""CPU check of the serving scheduler under ThreadSanitizer.

The admission logic of the serving loop (paper_2608_06669_amd/csrc/
scheduler.hpp) has no HIP calls; tests/scheduler_check.cpp drives it from
several threads with fake solves. Built with g++ -fsanitize=thread on the
host (no GPU code is involved), it must finish with no data race reported
and every invariant it checks holding.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_under_thread_sanitizer(tmp_path):
    exe = tmp_path / "scheduler_check"
    build = subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
         "-I", os.path.join(ROOT, "paper_2608_06669_amd", "csrc"),
         os.path.join(ROOT, "tests", "scheduler_check.cpp"), "-o", str(exe)],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-4000:]
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "0 failures" in run.stdout
