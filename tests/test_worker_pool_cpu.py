"""The batch worker pool (persistent host threads, csrc/worker_pool.h) under
ThreadSanitizer: 400 calls of 1-8 workers over stub jobs, every job run
exactly once by one of the called workers, no data race reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_worker_pool_tsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "pool_check"
    src = os.path.join(ROOT, "tests", "worker_pool_check.cpp")
    inc = os.path.join(ROOT, "paper_1809_04352_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-I", inc, src,
                    "-o", str(exe), "-pthread"], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
