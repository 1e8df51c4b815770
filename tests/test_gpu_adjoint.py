"""GPU parity of the FP32 value+Jacobian and adjoint kernels (the timed
headline path) against the FP64 oracle, the library-side reductions of the
gradient (J^T w, the misfit loss, node moments), and the graph-plan cache.

FP32 tolerances follow the rule for the fast mode: node values within
4 sqrt(SE_gpu^2 + SE_oracle^2) + 1e-5, and every Jacobian entry within
4 sqrt(2) times its standard error (from the spread of the per-path
derivatives, computed by the oracle) + 1e-5."""
import sys

import numpy as np
import pytest

from workloads import configs as CF
from workloads.problem import factor, make_fun

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


def _c5_small(seed=0, n_nodes=5, deg_terms=True):
    rng = np.random.default_rng(seed)
    sh = CF.real_solid_harmonics_poly(7)
    tg, tf, tc = rng.standard_normal(64), rng.standard_normal(16), 0.1 * rng.standard_normal(16)
    tc[0] += 1.0
    P = CF.c5_problem(tg, tf, tc, sh)
    if deg_terms:
        P.f = make_fun([(0.7, [factor("sin", 1, a=2.0)])], poly_degree=3, poly=P.f.poly)
        P.c = make_fun([(0.3, [factor("cos", 0)])], poly_degree=3, poly=P.c.poly)
        P.g = make_fun([(0.5, [factor("tanh", 0), factor("pow", 1, power=2)])], poly_degree=7, poly=P.g.poly)
    return P, CF.c5_nodes(n_nodes)


def _jac_close(gj, oj, ose, what):
    bound = 4.0 * np.sqrt(2.0) * ose + 1e-5
    bad = np.abs(gj - oj) > bound
    assert not bad.any(), (what, int(bad.sum()), float(np.max(np.abs(gj - oj) / np.maximum(ose, 1e-300))))


@pytest.mark.parametrize("deg_terms", [False, True])
def test_fp32_forward_and_adjoint_kernels_walk_the_same_paths(pdd, deg_terms):
    """The FP32 forward, adjoint and value+Jacobian kernels take the same exit
    step on every path and agree on every path value to FP32 rounding, so the
    recomputed gradient is the derivative of the estimator the forward
    returned."""
    P, nodes = _c5_small(7, 6, deg_terms)
    paths = np.array([700, 257, 1024, 64, 333, 900], np.int64)
    dt, seed = 2e-3, 11
    kw = dict(precision="fp32", schedule="persistent", chunk_paths=256)
    f = pdd.mc_interface(P, nodes, paths, dt, seed, dump=True, **kw)
    v = pdd.mc_value_jacobian(P, nodes, paths, dt, seed, dump=True, **kw)
    a = pdd.mc_adjoint(P, nodes, paths, dt, seed, np.ones(6), dump=True, **kw)
    torch.cuda.synchronize()
    sf = f["path_steps"].cpu().numpy()
    for r, name in ((v, "value+Jacobian"), (a, "adjoint")):
        assert np.array_equal(r["path_steps"].cpu().numpy(), sf), name
        d = np.abs(r["phi"].cpu().numpy() - f["phi"].cpu().numpy())
        assert np.all(d <= 2e-6 * np.maximum(1.0, np.abs(f["phi"].cpu().numpy()))), (name, float(d.max()))
    assert np.array_equal(v["steps"].cpu().numpy(), f["steps"].cpu().numpy())


@pytest.mark.parametrize("deg_terms", [False, True])
def test_fp32_value_jacobian_matches_oracle_jacobian(pdd, orc, deg_terms):
    """Small case (several items per node, ragged tails): FP32 node values and
    every Jacobian entry against the FP64 oracle on the same QUAD24 streams."""
    P, nodes = _c5_small(5, 5, deg_terms)
    paths = np.array([4000, 2500, 6001, 3000, 1200], np.int64)
    dt, seed = 2e-3, 19
    r = pdd.mc_value_jacobian(P, nodes, paths, dt, seed, precision="fp32", schedule="persistent", chunk_paths=1024)
    torch.cuda.synchronize()
    o = orc.walk_jacobian(P, nodes, paths, dt, seed, layout=orc.QUAD24)
    gm, gs = r["mean"].cpu().numpy(), r["se"].cpu().numpy()
    assert np.all(np.abs(gm - o["stats"]["mean"]) <= 4.0 * np.sqrt(gs ** 2 + o["stats"]["se"] ** 2) + 1e-5)
    gj = r["jac"].cpu().numpy()
    assert gj.shape == o["jac"].shape
    _jac_close(gj, o["jac"], o["jac_se"], "jacobian")
    # same streams: the FP32-vs-FP64 difference itself is far below one SE
    rel = np.abs(gj - o["jac"]) / np.maximum(o["jac_se"], 1e-12)
    log(f"fp32 jacobian vs oracle (terms={deg_terms}): max {rel.max():.3e} SE, rms {np.sqrt(np.mean(rel ** 2)):.3e} SE")


def test_fp32_adjoint_matches_oracle_adjoint(pdd, orc):
    """The path-recomputing FP32 adjoint (gradient of sum_i w_i u_i) against
    the oracle's FP64 adjoint, each entry within 4 sqrt(2) of the standard
    error sqrt(sum_i w_i^2 se_ik^2) of the weighted sum."""
    P, nodes = _c5_small(6, 4)
    paths = np.array([3000, 1500, 5000, 2200], np.int64)
    dt, seed = 2e-3, 23
    w = np.array([0.5, -1.0, 2.0, 0.25])
    g = pdd.mc_adjoint(P, nodes, paths, dt, seed, w, precision="fp32", schedule="persistent", chunk_paths=1024)
    torch.cuda.synchronize()
    o = orc.walk_jacobian(P, nodes, paths, dt, seed, layout=orc.QUAD24)
    want = w @ o["jac"]
    se = np.sqrt((w[:, None] ** 2 * o["jac_se"] ** 2).sum(axis=0))
    got = np.concatenate([g[k].cpu().numpy() for k in ("g_coef", "g_poly", "f_coef", "f_poly", "c_coef", "c_poly")])
    _jac_close(got, want, se, "adjoint")


def test_headline_launch_sampled_nodes_match_oracle(pdd, orc):
    """The benchmark's timed call exactly: pdd_mc_value_jacobian in FP32 over
    C5 (4096 nodes x 1e5 paths, dt 1e-3) with the graph schedule and the
    library's schedule table; 6 sampled nodes re-run whole by the oracle on
    the same streams (node ids of the full batch)."""
    w = CF.c5()
    log("headline value+Jacobian launch: C5 4096 x 1e5, FP32, graph")
    r = pdd.mc_value_jacobian(w.problem_template, w.nodes, w.paths, w.dt, w.seed, precision="fp32",
                              schedule="graph")
    torch.cuda.synchronize()
    idx = np.array([0, 777, 1500, 2600, 3333, 4095])
    log("oracle Jacobian of 6 sampled nodes x 1e5 paths")
    o = orc.walk_jacobian(w.problem_template, w.nodes[idx], w.paths[idx], w.dt, w.seed, layout=orc.QUAD24,
                          node_ids=idx)
    gm, gs = r["mean"].cpu().numpy()[idx], r["se"].cpu().numpy()[idx]
    assert np.all(r["n"].cpu().numpy() == 100000) and int(r["censored"].sum()) == 0
    assert np.all(np.abs(gm - o["stats"]["mean"]) <= 4.0 * np.sqrt(gs ** 2 + o["stats"]["se"] ** 2) + 1e-5)
    gj = r["jac"].cpu().numpy()[idx]
    _jac_close(gj, o["jac"], o["jac_se"], "headline jacobian")
    # the misfit gradient of the timed step, formed in the library, against
    # the same contraction in FP64 on the host
    d = torch.zeros(len(w.nodes), dtype=torch.float64, device="cuda")
    m = pdd.misfit_gradient(r, d)
    torch.cuda.synchronize()
    u = r["mean"].cpu().numpy()
    J = r["jac"].cpu().numpy()
    assert np.allclose(m["loss"].cpu().numpy()[0], np.sum(u ** 2), rtol=1e-12)
    want = (2.0 * u) @ J
    assert np.allclose(m["grad"].cpu().numpy(), want, rtol=1e-10, atol=1e-10 * np.abs(want).max())


def test_jacobian_apply_and_misfit_gradient(pdd):
    """J^T w and the misfit loss / gradient against host FP64 sums, on ragged
    shapes (rows not a multiple of 4, columns not a multiple of 64, jac_ld >
    n_params); J^T w equals the recomputing adjoint with the same schedule."""
    P, nodes = _c5_small(4, 5)
    paths = np.array([150, 64, 201, 90, 33], np.int64)
    dt, seed = 1e-2, 17
    r = pdd.mc_value_jacobian(P, nodes, paths, dt, seed, precision="fp64", schedule="persistent", chunk_paths=50)
    wv = np.array([0.5, -1.0, 2.0, 0.25, 1.5])
    g = pdd.jacobian_apply(r["jac"], wv)
    adj = pdd.mc_adjoint(P, nodes, paths, dt, seed, wv, precision="fp64", schedule="persistent", chunk_paths=50)
    torch.cuda.synchronize()
    J = r["jac"].cpu().numpy()
    assert np.allclose(g.cpu().numpy(), wv @ J, rtol=1e-13, atol=1e-13 * np.abs(wv @ J).max())
    blocks = pdd.jacobian_blocks(P, g)
    for k in ("g_coef", "g_poly", "f_coef", "f_poly", "c_coef", "c_poly"):
        a, b = blocks[k].cpu().numpy(), adj[k].cpu().numpy()
        assert np.allclose(a, b, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(b).max())), k
    data = np.array([0.1, -0.3, 0.7, 0.0, 2.0])
    m = pdd.misfit_gradient(r, data)
    torch.cuda.synchronize()
    u = r["mean"].cpu().numpy()
    assert m["loss"].cpu().numpy()[0] == pytest.approx(float(np.sum((u - data) ** 2)), rel=1e-13)
    want = (2.0 * (u - data)) @ J
    assert np.allclose(m["grad"].cpu().numpy(), want, rtol=1e-12, atol=1e-13 * np.abs(want).max())
    # a strided view (ld > n_params) and a single row
    big = torch.zeros((7, 200), dtype=torch.float64, device="cuda")
    big[:, :130] = torch.tensor(np.random.default_rng(0).standard_normal((7, 130)), device="cuda")
    wv7 = np.random.default_rng(1).standard_normal(7)
    g7 = pdd.jacobian_apply(big[:, :130], wv7)
    g1 = pdd.jacobian_apply(big[:1, :130], wv7[:1])
    torch.cuda.synchronize()
    B = big.cpu().numpy()[:, :130]
    assert np.allclose(g7.cpu().numpy(), wv7 @ B, rtol=1e-13, atol=1e-14)
    assert np.allclose(g1.cpu().numpy(), wv7[0] * B[0], rtol=1e-15, atol=0)


def test_node_moments_are_the_unbiased_variance_and_se(pdd):
    P, nodes = _c5_small(2, 4, deg_terms=False)
    paths = np.array([1, 2, 500, 0], np.int64)
    r = pdd.mc_interface(P, nodes, paths, 2e-3, 3, precision="fp64", schedule="persistent")
    torch.cuda.synchronize()
    n = r["n"].cpu().numpy().astype(float)
    m2 = r["m2"].cpu().numpy()
    var = np.where(n > 1, m2 / np.maximum(n - 1, 1), 0.0)
    se = np.where(n > 0, np.sqrt(var / np.maximum(n, 1)), 0.0)
    assert np.array_equal(r["var"].cpu().numpy(), var)
    assert np.allclose(r["se"].cpu().numpy(), se, rtol=1e-15, atol=0)


def test_graph_plans_do_not_depend_on_caller_buffers(pdd):
    """Calls that differ only in their buffers (fresh coefficient tensors with
    new values, fresh outputs, all kept alive) replay one cached plan, each
    reading its own coefficients and writing its own output; plans stay
    bounded when the shapes differ."""
    P, nodes = _c5_small(3, 4, deg_terms=False)
    paths = np.full(4, 600, np.int64)
    dt = 2e-3
    pdd.release_workspace()
    assert pdd.cached_plan_count() == 0
    held = []
    rng = np.random.default_rng(5)
    for k in range(12):
        gp = torch.tensor(P.g.poly * (1.0 + 0.1 * rng.standard_normal()), device="cuda", dtype=torch.float64)
        nd = torch.tensor(nodes, device="cuda")
        a = pdd.mc_interface(P, nd, paths, dt, 4, precision="fp32", schedule="graph", coefs={"g_poly": gp})
        b = pdd.mc_interface(P, nd, paths, dt, 4, precision="fp32", schedule="persistent", coefs={"g_poly": gp})
        held.append((gp, nd, a, b))
    torch.cuda.synchronize()
    assert pdd.cached_plan_count() == 1
    for gp, nd, a, b in held:
        assert torch.equal(a["mean"], b["mean"])
    assert not torch.equal(held[0][2]["mean"], held[1][2]["mean"])
    # value+Jacobian and adjoint plans with fresh outputs / weights each call
    for k in range(3):
        wv = torch.tensor(rng.standard_normal(4), device="cuda")
        r = pdd.mc_value_jacobian(P, nodes, paths, dt, 4, precision="fp32", schedule="graph")
        g = pdd.mc_adjoint(P, nodes, paths, dt, 4, wv, precision="fp32", schedule="graph")
        h = pdd.mc_adjoint(P, nodes, paths, dt, 4, wv, precision="fp32", schedule="persistent")
        torch.cuda.synchronize()
        for key in ("g_poly", "f_poly", "c_poly"):
            assert torch.allclose(g[key], h[key], rtol=1e-12, atol=1e-14), key
        assert r["jac"].abs().sum() > 0
    assert pdd.cached_plan_count() == 3
    for s in range(30):
        pdd.mc_interface(P, nodes, paths, dt, 100 + s, precision="fp32", schedule="graph")
    torch.cuda.synchronize()
    assert pdd.cached_plan_count() <= 16
    pdd.release_workspace()
    assert pdd.cached_plan_count() == 0


def test_merge_estimates_equals_the_pooled_sample(pdd):
    """A second sample (another seed) of some nodes merged into an estimate
    gives the statistics of the pooled per-path values (mean, sum of squared
    deviations, counts) and the path-count weighted Jacobian."""
    P, nodes = _c5_small(8, 6, deg_terms=False)
    pa = np.array([500, 80, 1000, 3, 256, 700], np.int64)
    dt = 2e-3
    kw = dict(precision="fp64", schedule="persistent", chunk_paths=256, dump=True)
    a = pdd.mc_value_jacobian(P, nodes, pa, dt, 1, **kw)
    sel = np.array([4, 0, 2])
    pb = np.array([300, 41, 999], np.int64)
    b = pdd.mc_value_jacobian(P, nodes[sel], pb, dt, 2, **kw)
    torch.cuda.synchronize()
    ja, jb = a["jac"].cpu().numpy().copy(), b["jac"].cpu().numpy().copy()
    offa = np.concatenate([[0], np.cumsum(pa)])
    offb = np.concatenate([[0], np.cumsum(pb)])
    phia, phib = a["phi"].cpu().numpy(), b["phi"].cpu().numpy()
    stepsa, stepsb = a["steps"].cpu().numpy().copy(), b["steps"].cpu().numpy().copy()
    m = pdd.merge_estimates(a, b, sel)
    torch.cuda.synchronize()
    mean, m2, n = m["mean"].cpu().numpy(), m["m2"].cpu().numpy(), m["n"].cpu().numpy()
    J = m["jac"].cpu().numpy()
    for i in range(6):
        vals = phia[offa[i]:offa[i + 1]]
        want_j = ja[i]
        if i in sel:
            k = int(np.nonzero(sel == i)[0][0])
            vals = np.concatenate([vals, phib[offb[k]:offb[k + 1]]])
            want_j = (pa[i] * ja[i] + pb[k] * jb[k]) / (pa[i] + pb[k])
            assert m["steps"].cpu().numpy()[i] == stepsa[i] + stepsb[k]
        assert n[i] == len(vals)
        assert mean[i] == pytest.approx(vals.mean(), rel=1e-12, abs=1e-14)
        assert m2[i] == pytest.approx(np.sum((vals - vals.mean()) ** 2), rel=1e-10, abs=1e-12)
        assert np.allclose(J[i], want_j, rtol=1e-13, atol=1e-15)
    var = np.where(n > 1, m2 / np.maximum(n - 1, 1), 0.0)
    assert np.allclose(m["se"].cpu().numpy(), np.sqrt(var / n), rtol=1e-15)
