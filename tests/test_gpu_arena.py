"""The per-stream call arenas: calls without a cached graph plan keep their
scratch in one buffer per (device, stream) that grows when a call needs more.
Calls of growing and shrinking size, interleaved on two streams, queued back
to back without host synchronisation, and calls after pdd_release_workspace
must give exactly the results of the same calls made one at a time."""
import sys

import numpy as np
import pytest

from workloads import configs as CF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pdd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03666_amd as P
    P.library()
    return P


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _walk(pdd, P, nodes, paths):
    r = pdd.mc_interface(P, nodes, paths, 1e-3, 3, precision="fp32", schedule="persistent")
    return {k: r[k].clone() for k in ("mean", "m2", "n", "steps")}


def _tree(pdd, w, pts, trees):
    r = pdd.branching_eval(w.problem, pts, trees, 5, precision="fp32", schedule="persistent")
    return {k: r[k].clone() for k in ("mean", "m2", "n", "steps")}


def _same(a, b, what):
    for k in a:
        assert torch.equal(a[k], b[k]), (what, k)


def test_call_arena_reuse_growth_streams_and_release(pdd):
    P = CF.c1().problem
    nodes_all = torch.tensor(CF.c1().nodes, device="cuda")
    w4 = CF.c4(scale=0.01, n_points=64)
    pts = torch.tensor(w4.points, device="cuda")
    sizes = [(4, 500), (16, 4000), (2, 100), (16, 20000), (8, 50)]   # grows, shrinks, grows again

    log("arena: reference results, one call at a time")
    ref = []
    for n, p in sizes:
        ref.append(_walk(pdd, P, nodes_all[:n], np.full(n, p, np.int64)))
        torch.cuda.synchronize()
    ref_tree = [_tree(pdd, w4, pts[:k], t) for k, t in ((8, 300), (64, 2000), (4, 100))]
    torch.cuda.synchronize()

    log("arena: the same calls queued back to back on the current stream")
    got = [_walk(pdd, P, nodes_all[:n], np.full(n, p, np.int64)) for n, p in sizes]
    got_tree = [_tree(pdd, w4, pts[:k], t) for k, t in ((8, 300), (64, 2000), (4, 100))]
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(ref, got)):
        _same(a, b, f"walk {i}")
    for i, (a, b) in enumerate(zip(ref_tree, got_tree)):
        _same(a, b, f"tree {i}")

    log("arena: interleaved on two streams")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out1, out2 = [], []
    for i, (n, p) in enumerate(sizes):
        with torch.cuda.stream(s1 if i % 2 == 0 else s2):
            (out1 if i % 2 == 0 else out2).append(_walk(pdd, P, nodes_all[:n], np.full(n, p, np.int64)))
    with torch.cuda.stream(s2):
        t2 = _tree(pdd, w4, pts[:64], 2000)
    torch.cuda.synchronize()
    for j, i in enumerate(range(0, len(sizes), 2)):
        _same(ref[i], out1[j], f"stream 1 walk {i}")
    for j, i in enumerate(range(1, len(sizes), 2)):
        _same(ref[i], out2[j], f"stream 2 walk {i}")
    _same(ref_tree[1], t2, "stream 2 tree")

    log("arena: after pdd_release_workspace")
    pdd.release_workspace()
    again = _walk(pdd, P, nodes_all[:16], np.full(16, 20000, np.int64))
    again_tree = _tree(pdd, w4, pts[:64], 2000)
    torch.cuda.synchronize()
    _same(ref[3], again, "walk after release")
    _same(ref_tree[1], again_tree, "tree after release")
