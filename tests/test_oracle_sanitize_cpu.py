"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, no OpenMP) and driven through every entry point on a small cluster: no
report, certified labels equal the plain ones where decided, every crossing
edge gets a record."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_check"
    srcs = [os.path.join(ROOT, "oracle", "eses_oracle.c"),
            os.path.join(ROOT, "tests", "oracle_sanitize_check.c")]
    subprocess.run([gcc, "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *srcs,
                    "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=66",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=67")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.startswith("OK"), r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
