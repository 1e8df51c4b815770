"""The problem-specialised kernels compile for gfx950 (CPU only).

The library writes the source of a walk or branching kernel with a problem's
factor structure at run time and compiles it with hiprtc; on a GPU the tests
in test_gpu_parity.py check that those kernels give the table-driven kernels'
results.  Here a small host program (rtc_compile_check.cpp) links the
library's own source generators and compilation step (specialize.cpp and the
embedded device headers) and compiles a set of structures for gfx950 without
loading them, so a header that the runtime compiler cannot build, or a
generator that writes invalid source, fails on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_specialised_kernels_compile_for_gfx950(tmp_path):
    from paper_1705_03666_amd import build as B
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    objs = [os.path.join(B.BUILD, "specialize.o"), os.path.join(B.BUILD, B.RTC_SOURCE.replace(".cpp", ".o"))]
    if not all(os.path.exists(o) for o in objs):
        B.build(verbose=False)
    obj = str(tmp_path / "rtc_compile_check.o")
    exe = str(tmp_path / "rtc_compile_check")
    flags = [f for f in B.FLAGS if not f.startswith("--offload-arch")]
    subprocess.check_call([B._hipcc()] + flags + ["-c", os.path.join(HERE, "rtc_compile_check.cpp"), "-o", obj])
    subprocess.check_call([B._hipcc(), obj] + objs + ["-lhiprtc", "-o", exe])
    r = subprocess.run([exe, "gfx950"], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("ok ")]
    assert len(lines) == 8, r.stdout
    assert "FAIL" not in r.stdout
