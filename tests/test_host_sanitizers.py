"""Host sanitizers.  The oracle (C): AddressSanitizer + UndefinedBehavior-
Sanitizer on a small run of every oracle entry point, and ThreadSanitizer on
the same run with a pool of 4 worker threads.  The library's C ABI: its
argument checking (the host code of capi.cpp and what it calls) built with
AddressSanitizer + UndefinedBehaviorSanitizer and driven through ctypes by
the invalid-argument cases of test_abi.py.  CPU only: no case reaches a GPU
call."""
import os
import shutil
import subprocess
import sys

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


def test_capi_argument_checks_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from paper_1705_03666_amd import build as B
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    lib = B.build_host_sanitized(str(tmp_path / "san"))
    env = dict(os.environ, PDD_LIBRARY=lib, LD_PRELOAD=B.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the sanitized build is the one loaded, with the sanitizer runtime active
    probe = ("import ctypes as C\n"
             "from paper_1705_03666_amd import _abi\n"
             "L = _abi.load()\n"
             "assert _abi.LIB_PATH.endswith('libpdd_san.so'), _abi.LIB_PATH\n"
             "assert 'libpdd_san.so' in open('/proc/self/maps').read()\n"
             "C.CDLL(None).__asan_init\n"
             "print('sanitized library loaded')\n")
    root = os.path.dirname(HERE)
    r = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, cwd=root, timeout=300)
    assert r.returncode == 0 and "sanitized library loaded" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(HERE, "test_abi.py")], capture_output=True, text=True, env=env, cwd=root,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
