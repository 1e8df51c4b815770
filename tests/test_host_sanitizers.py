"""Host sanitizers on the oracle (C): AddressSanitizer + UndefinedBehavior-
Sanitizer on a small run of every oracle entry point, and ThreadSanitizer on
the same run with a pool of 4 worker threads.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def _build_and_run(tmp_path, flags):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "san")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-fno-omit-frame-pointer", *flags, "-I", ORACLE,
           os.path.join(HERE, "sanitizer_driver.c"), os.path.join(ORACLE, "oracle.c"), "-o", exe, "-lm",
           "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "WARNING" not in r.stderr, r.stderr


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])


def test_oracle_thread_pool_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"])
