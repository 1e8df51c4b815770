"""pdd_mc_interface_noalloc through the C ABI: the same node statistics as
pdd_mc_interface (persistent schedule, table-driven kernel) on two calls in a
row, the second smaller than the first, in FP32 and FP64; an input too large
for the fixed scratch area is refused before anything is enqueued; and the
calls map no device memory."""
import ctypes as C

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


def _call(pdd, entry, P, nodes, paths, dt, seed, precision, out):
    """One call of `entry` (pdd_mc_interface or pdd_mc_interface_noalloc) with
    the caller's output buffer; returns the status."""
    keep = []
    p = pdd._linear(P, keep)
    o = pdd._options(precision, None, 0, "persistent", 0, 0, 0, specialize="off")
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64))
    fn = getattr(pdd.library(), entry)
    return fn(C.byref(p), nodes.data_ptr(), nodes.shape[0], ph.ctypes.data_as(C.POINTER(C.c_int64)), float(dt),
              int(seed), C.byref(o), out.data_ptr(), torch.cuda.current_stream().cuda_stream)


def _cases():
    w5 = CF.c5(n_nodes=512)
    rng = np.random.default_rng(3)
    c2 = CF.c2_problem()
    c2_nodes = CF.c2_nodes()
    return [
        # FP32, polynomial c and f (the C5 walk): 512 nodes x 20000, then 37 ragged nodes
        ("fp32", w5.problem_template, (w5.nodes, np.full(512, 20000)),
         (w5.nodes[100:137], rng.integers(1, 3001, size=37)), 2e-3),
        # FP64 with generic terms in b, c, f (C2): 16 nodes x 4000, then 3 nodes
        ("fp64", c2, (c2_nodes[::16], np.full(16, 4000)), (c2_nodes[5:8], np.array([777, 1, 300])), 2e-3),
    ]


@pytest.mark.parametrize("case", [0, 1])
def test_noalloc_matches_mc_interface_on_two_calls(pdd, case):
    precision, P, first, second, dt = _cases()[case]
    for k, (nodes, paths) in enumerate((first, second)):
        nd = torch.tensor(nodes, device="cuda")
        out_a = torch.full((len(paths), 5), float("nan"), dtype=torch.float64, device="cuda")
        out_b = torch.full((len(paths), 5), float("nan"), dtype=torch.float64, device="cuda")
        print(f"noalloc case {case} call {k + 1}: {precision}, {len(paths)} nodes, {int(np.sum(paths))} paths",
              flush=True)
        assert _call(pdd, "pdd_mc_interface_noalloc", P, nd, paths, dt, 9, precision, out_a) == 0, \
            pdd.library().pdd_last_error()
        assert _call(pdd, "pdd_mc_interface", P, nd, paths, dt, 9, precision, out_b) == 0
        torch.cuda.synchronize()
        a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), k
        assert np.all(a[:, 2:].view(np.int64)[:, 0] == np.asarray(paths))


def test_noalloc_refuses_too_large_a_call_and_maps_no_memory(pdd):
    w5 = CF.c5(n_nodes=1024)
    P = w5.problem_template
    ndb = torch.tensor(w5.nodes, device="cuda")
    # 1024 nodes x 5e6 paths: about 5.9e5 work items, 37 MB of queue and
    # partials, beyond the 16 MiB fixed area
    big = np.full(1024, 5_000_000, np.int64)
    out = torch.full((1024, 5), float("nan"), dtype=torch.float64, device="cuda")
    st = _call(pdd, "pdd_mc_interface_noalloc", P, ndb, big, 1e-3, 1, "fp32", out)
    assert st == -2
    msg = pdd.library().pdd_last_error().decode()
    assert "fixed scratch area" in msg, msg
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
    # after a first call (which loads the library's code object), two calls
    # with preallocated outputs change the device's free memory by nothing
    nd = ndb[:64].contiguous()
    small = np.full(64, 3000, np.int64)
    outs = [torch.empty((64, 5), dtype=torch.float64, device="cuda") for _ in range(2)]
    assert _call(pdd, "pdd_mc_interface_noalloc", P, nd, small, 2e-3, 1, "fp32", outs[0]) == 0
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for o in outs:
        assert _call(pdd, "pdd_mc_interface_noalloc", P, nd, small, 2e-3, 1, "fp32", o) == 0
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert torch.equal(outs[0], outs[1])
