"""The on-disk cache of problem-specialised kernels: an entry written by one
process is reused by the next, and a damaged or foreign entry under the same
name (truncated, a byte of the code object changed in place, another key) is
recompiled and replaced, with bitwise the same results every time.
Each step runs in a child process (the in-process cache would otherwise
answer first)."""
import glob
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import paper_1705_03666_amd as pdd
from workloads import configs as CF
P = CF.c2_problem()
nodes = CF.c2_nodes()[::32]
paths = np.full(len(nodes), 2000, np.int64)
t0 = time.perf_counter()
r = pdd.mc_interface(P, nodes, paths, 1e-3, 11, precision="fp32", specialize="on", schedule="persistent")
import torch
torch.cuda.synchronize()
print(json.dumps({"mean": r["mean"].cpu().numpy().tolist(), "steps": r["steps"].cpu().numpy().tolist(),
                  "seconds": time.perf_counter() - t0}), flush=True)
"""


def _valid_entry(path):
    """The entry's layout and checksum, restated: magic, little-endian uint64
    lengths of key, symbol and code object, their 64-bit FNV-1a checksum."""
    import struct
    with open(path, "rb") as f:
        d = f.read()
    if d[:8] != b"PDDJIT3\n" or len(d) < 40:
        return False
    nk, ns, nc, cs = struct.unpack("<4Q", d[8:40])
    if 40 + nk + ns + nc != len(d):
        return False
    h = 1469598103934665603
    for b in d[40:]:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h == cs


def _run(cache_dir):
    env = dict(os.environ, PDD_JIT_CACHE=str(cache_dir))
    p = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    return json.loads(p.stdout.strip().splitlines()[-1])


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_disk_cache_reuse_and_repair(gpu, tmp_path):
    print("jit cache: first process compiles", flush=True)
    first = _run(tmp_path)
    entries = glob.glob(str(tmp_path / "*.pddjit"))
    assert len(entries) == 1
    entry = entries[0]
    size = os.path.getsize(entry)
    assert size > 1000
    assert _valid_entry(entry)

    print("jit cache: second process loads the entry", flush=True)
    second = _run(tmp_path)
    assert second["mean"] == first["mean"] and second["steps"] == first["steps"]
    assert os.path.getsize(entry) == size

    print("jit cache: truncated entry", flush=True)
    with open(entry, "r+b") as f:
        f.truncate(size // 2)
    third = _run(tmp_path)
    assert third["mean"] == first["mean"] and third["steps"] == first["steps"]
    assert os.path.getsize(entry) == size          # rewritten whole

    head = 8 + 32                                  # magic, three lengths and the checksum
    with open(entry, "rb") as f:
        good = f.read()

    print("jit cache: a byte of the code object changed in place", flush=True)
    data = bytearray(good)
    data[-100] ^= 0x40                             # inside the code object; sizes unchanged
    with open(entry, "wb") as f:
        f.write(bytes(data))
    fourth = _run(tmp_path)
    assert fourth["mean"] == first["mean"] and fourth["steps"] == first["steps"]
    with open(entry, "rb") as f:
        again = f.read()
    assert again != bytes(data) and len(again) == len(good) and _valid_entry(entry)   # refused, rebuilt

    print("jit cache: entry of another key under the same name", flush=True)
    data = bytearray(good)
    data[head + 5] ^= 0x01                         # one byte of the stored key
    with open(entry, "wb") as f:
        f.write(bytes(data))
    fifth = _run(tmp_path)
    assert fifth["mean"] == first["mean"] and fifth["steps"] == first["steps"]
    with open(entry, "rb") as f:
        assert f.read()[head + 5] == good[head + 5]   # the true key again
    assert _valid_entry(entry)
    assert not glob.glob(str(tmp_path / "*.tmp*"))
