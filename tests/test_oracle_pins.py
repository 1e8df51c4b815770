"""Pins for the FP64 oracle: each test checks it against something other than
itself (an independent library, a closed form, a brute-force computation, an
ODE/PDE solve), chosen so that a dropped term, a wrong sign or a swapped index
in the oracle fails at least one of them."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, special, stats

from workloads import configs as CF
from workloads.problem import (BranchingProblem, LinearProblem, ball, box, const_fun, factor,
                               make_fun, zero_fun)

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def z_ok(est, se, exact, extra=0.0, k=4.0):
    return np.all(np.abs(np.asarray(est) - exact) <= k * np.asarray(se) + extra)


# ----------------------------------------------------------------------------- RNG
@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available to build the rocRAND host pin")
    out = tmp_path_factory.mktemp("pin") / "philox_pin"
    subprocess.check_call(["hipcc", "-O1", os.path.join(HERE, "philox_pin_rocrand.cpp"), "-o", str(out)])
    return str(out)


def test_philox_matches_rocrand_host_engine(orc, rocrand_pin):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
             (0x243F6A88, 0x05A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0)]
    for _ in range(200):
        c = rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF
        cases.append(tuple(int(v) for v in c))
    text = "\n".join(" ".join(f"{v:x}" for v in cs) for cs in cases) + "\n"
    res = subprocess.run([rocrand_pin], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for cs, line in zip(cases, lines):
        want = [int(v, 16) for v in line.split()]
        assert orc.philox(cs[:4], cs[4:]) == want


def test_uniform_lattices_are_open_and_exact(orc):
    # QUAD24 extremes and spacing
    assert orc.u_quad24(0) == 2.0 ** -24
    assert orc.u_quad24(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.u_quad24(1 << 9) - orc.u_quad24(0) == 2.0 ** -23
    assert orc.u_quad24(511) == orc.u_quad24(0)          # low 9 bits are dropped
    # PAIR52 extremes
    assert orc.u_pair52(0, 0) == 2.0 ** -53
    assert orc.u_pair52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u_pair52(0, 1 << 12) - orc.u_pair52(0, 0) == 2.0 ** -52
    # every QUAD24 value is a float32 exactly
    rng = np.random.default_rng(0)
    for w in rng.integers(0, 2 ** 32, size=2000):
        u = orc.u_quad24(int(w))
        assert 0.0 < u < 1.0 and float(np.float32(u)) == u


def test_walk_normals_are_standard_gaussian(orc):
    for layout in (orc.PAIR52, orc.QUAD24):
        z = np.array([orc.walk_normal(11, layout, 3, p, j) for p in range(40) for j in range(500)])
        assert abs(z.mean()) < 4.0 / math.sqrt(len(z))
        assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / len(z))
        assert abs(stats.skew(z)) < 4.0 * math.sqrt(6.0 / len(z))
        assert abs(stats.kurtosis(z)) < 4.0 * math.sqrt(24.0 / len(z))
        assert stats.kstest(z, "norm").pvalue > 1e-4


def test_walk_normal_index_layout(orc):
    """Normal j comes from block j // per_block and slot j % per_block: the pair
    (z_{2m}, z_{2m+1}) shares the radius, so z0^2 + z1^2 = -2 ln u_a."""
    seed, node, path = 5, 2, 9
    w = orc.philox([0, 0, path, node], [seed, 0])
    z0, z1 = orc.walk_normal(seed, orc.PAIR52, node, path, 0), orc.walk_normal(seed, orc.PAIR52, node, path, 1)
    ua = orc.u_pair52(w[0], w[1])
    assert z0 * z0 + z1 * z1 == pytest.approx(-2.0 * math.log(ua), rel=1e-13)
    z2, z3 = orc.walk_normal(seed, orc.QUAD24, node, path, 2), orc.walk_normal(seed, orc.QUAD24, node, path, 3)
    assert z2 * z2 + z3 * z3 == pytest.approx(-2.0 * math.log(orc.u_quad24(w[2])), rel=1e-13)
    # block 1 of the PAIR52 stream is counter word0 = 1
    w1 = orc.philox([1, 0, path, node], [seed, 0])
    z2p = orc.walk_normal(seed, orc.PAIR52, node, path, 2)
    ub = orc.u_pair52(w1[2], w1[3])
    r = math.sqrt(-2.0 * math.log(orc.u_pair52(w1[0], w1[1])))
    assert z2p == pytest.approx(r * math.cos(2 * math.pi * ub), rel=1e-14)


# ----------------------------------------------------------------------------- functions / domain
def test_fun_eval_matches_numpy(orc):
    f = CF.c2_problem().f
    rng = np.random.default_rng(1)
    for x, y in rng.uniform(-1, 1, size=(20, 2)):
        want = math.exp(y) * ((1 + 0.5 * x * x) * math.cos(x) + math.sin(math.pi * y) * math.sin(x)
                              - math.cos(math.pi * x) * math.cos(x))
        assert orc.fun_eval(f, 2, [x, y]) == pytest.approx(want, rel=1e-13, abs=1e-14)
    psi = CF.kpp_travelling_wave_problem().psi
    for x in np.linspace(-5, 5, 11):
        want = 1.0 - (1.0 + math.exp(x / math.sqrt(6.0))) ** -2
        assert orc.fun_eval(psi, 1, [x]) == pytest.approx(want, rel=1e-13)
    sh = CF.real_solid_harmonics_poly(7)
    theta = rng.standard_normal(64)
    g = make_fun([], poly_degree=7, poly=sh @ theta)
    pts = rng.uniform(-0.6, 0.6, size=(5, 3))
    vals = CF.real_solid_harmonic_values(pts) @ theta
    for p, v in zip(pts, vals):
        assert orc.fun_eval(g, 3, p) == pytest.approx(v, rel=1e-10, abs=1e-12)


# ----------------------------------------------------------------------------- linear walk
def _nystrom_1d(dt, sigma, b, c, f, g0, g1, x0, n=240):
    """Brute force for the discrete Euler chain on (0,1): the value function
    V(x) = f(x) dt + e^{-c(x) dt} E[ V(y) 1{0<y<1} + g0 1{y<=0} + g1 1{y>=1} ],
    y ~ N(x + b(x) dt, sigma^2 dt), solved by Gauss-Legendre Nystrom."""
    t, wq = np.polynomial.legendre.leggauss(n)
    y = 0.5 * (t + 1.0)
    wq = 0.5 * wq
    s = sigma * math.sqrt(dt)

    def row(x):
        m = x + b(x) * dt
        k = wq * np.exp(-0.5 * ((y - m) / s) ** 2) / (s * math.sqrt(2 * math.pi))
        p0 = special.ndtr((0.0 - m) / s)
        p1 = 1.0 - special.ndtr((1.0 - m) / s)
        return k, p0, p1

    A = np.zeros((n, n))
    rhs = np.zeros(n)
    for i, xi in enumerate(y):
        k, p0, p1 = row(xi)
        e = math.exp(-c(xi) * dt)
        A[i] = e * k
        rhs[i] = f(xi) * dt + e * (g0 * p0 + g1 * p1)
    V = np.linalg.solve(np.eye(n) - A, rhs)
    k, p0, p1 = row(x0)
    e = math.exp(-c(x0) * dt)
    return f(x0) * dt + e * (k @ V + g0 * p0 + g1 * p1)


def test_walk_matches_brute_force_euler_chain_1d(orc):
    """Pins the whole discrete scheme (left-point Z, Y update, drift, exit test,
    projection) against an independent integral-equation solve, no bias allowance."""
    dt, sigma = 1e-2, 1.0
    prob = LinearProblem(box((0.0,), (1.0,)), sigma,
                         [make_fun([(0.3, [])])],
                         make_fun([(0.5, []), (1.0, [factor("pow", 0)])]),       # c = 0.5 + x
                         make_fun([(1.0, []), (1.0, [factor("pow", 0)])]),       # f = 1 + x
                         make_fun([(1.0, [factor("exp", 0)])]))                  # g = e^x
    nodes = np.array([[0.2], [0.5], [0.77]])
    paths = np.full(3, 40000, np.int64)
    r = orc.walk(prob, nodes, paths, dt, 1)
    for i, x0 in enumerate(nodes[:, 0]):
        want = _nystrom_1d(dt, sigma, lambda x: 0.3, lambda x: 0.5 + x, lambda x: 1.0 + x,
                           1.0, math.e, x0)
        assert abs(r["mean"][i] - want) <= 4.0 * r["se"][i], (i, r["mean"][i], want, r["se"][i])


def test_walk_harmonic_data_reproduced(orc):
    """Eq. 2.1: harmonic g gives u = g (C1 data), up to 4 SE plus the O(sqrt dt)
    boundary bias (bounded by 0.6 sqrt(dt) |grad g|)."""
    w = CF.c1(dt=1e-3, scale=0.5)
    r = orc.walk(w.problem, w.nodes, w.paths, w.dt, 2)
    grad = math.e * math.sqrt(2.0)
    assert z_ok(r["mean"], r["se"], CF.c1_exact(w.nodes), extra=0.6 * math.sqrt(w.dt) * grad)


def test_walk_exit_time_bias_is_order_sqrt_dt(orc):
    """Euler-Maruyama plus a boundary test has an O(sqrt dt) weak error (Sec. 2.1,
    ingredients of PDD).  For the exit time from the unit ball the first-order
    term is the boundary-overshoot constant 0.5826 sigma sqrt(dt) |du/dn| with
    u = (1 - |x|^2)/d, |du/dn| = 2/d."""
    for d in (2, 3):
        prob = LinearProblem(ball(d), 1.0, [zero_fun()] * d, zero_fun(), const_fun(1.0), zero_fun())
        bias = []
        for dt in (1e-2, 2.5e-3, 6.25e-4):
            r = orc.walk(prob, np.zeros((1, d)), np.array([40000]), dt, 3)
            bias.append((r["mean"][0] - 1.0 / d, r["se"][0], dt))
        for (b1, s1, _), (b2, s2, _) in zip(bias, bias[1:]):
            assert 0.3 < b2 / b1 < 0.7, bias
        b, se, dt = bias[-1]
        assert abs(b / math.sqrt(dt) - 0.5826 * 2.0 / d) < 0.15 + 4 * se / math.sqrt(dt), bias


def test_boundary_corrected_walk_removes_the_sqrt_dt_bias(orc):
    """Gobet-Menozzi boundary shift (the corrected stopped-Euler schemes that
    Sec. 2.1 points to): stopping once X leaves D shrunk by c0 sigma sqrt(dt),
    c0 = -zeta(1/2)/sqrt(2 pi), cancels the first-order overshoot term.  Exit
    time from the 3-D unit ball, u = (1 - |x|^2)/3, dt = 4e-3, where the plain
    test is biased by about 0.5826 sqrt(dt) 2/3 = 0.025: the corrected
    estimate must sit within 4 SE plus an O(dt) allowance of the closed form
    and remove most of the plain bias (an outward shift or a wrong constant
    fails both)."""
    assert orc.GOBET_MENOZZI_C0 == pytest.approx(-special.zeta(0.5) / math.sqrt(2 * math.pi), rel=1e-15)
    prob = LinearProblem(ball(3), 1.0, [zero_fun()] * 3, zero_fun(), const_fun(1.0), zero_fun())
    x = np.array([[0.3, 0.0, 0.0], [0.0, 0.6, 0.0]])
    exact = (1.0 - (x ** 2).sum(axis=1)) / 3.0
    dt = 4e-3
    n = np.array([200000, 200000])
    plain = orc.walk(prob, x, n, dt, 11)
    corr = orc.walk(prob, x, n, dt, 11, boundary_shift=orc.GOBET_MENOZZI_C0)
    b_plain = plain["mean"] - exact
    b_corr = corr["mean"] - exact
    assert np.all(b_plain > 10 * plain["se"]), b_plain
    assert np.all(np.abs(b_corr) < 4 * corr["se"] + 0.5 * dt), (b_corr, corr["se"])
    assert np.all(np.abs(b_corr) < 0.25 * b_plain), (b_corr, b_plain)


def test_boundary_corrected_walk_harmonic_data_in_the_square(orc):
    """The same correction in a box (every face moved inward): harmonic data
    g = e^x sin y on [0,1]^2 (u = g) at dt = 1e-2, where the plain test is off
    by tens of SE near the face y = 1."""
    w = CF.c1()
    nd = w.nodes[[2, 13]]
    exact = CF.c1_exact(nd)
    n = np.array([100000, 100000])
    plain = orc.walk(w.problem, nd, n, 1e-2, 3)
    corr = orc.walk(w.problem, nd, n, 1e-2, 3, boundary_shift=orc.GOBET_MENOZZI_C0)
    assert np.max(np.abs(plain["mean"] - exact) / plain["se"]) > 10
    assert np.all(np.abs(corr["mean"] - exact) < 4 * corr["se"] + 1e-2 * 0.5)


def test_walk_on_spheres_reproduces_harmonic_data_in_the_square(orc):
    """Walk on Spheres (recommended in Sec. 2.1 for Laplace with Dirichlet
    data): u = g = e^x sin y on [0,1]^2 within 4 SE plus the eps-shell bias
    (at most eps |grad g|); the jump count grows like log(1/eps)."""
    w = CF.c1()
    nd = w.nodes[[1, 7, 14]]
    exact = CF.c1_exact(nd)
    eps = 1e-4
    r = orc.wos(w.problem, nd, np.full(3, 100000), eps, 5)
    assert np.all(np.abs(r["mean"] - exact) < 4 * r["se"] + eps * math.e * math.sqrt(2.0))
    jumps = r["steps"] / r["n"]
    r2 = orc.wos(w.problem, nd, np.full(3, 20000), 1e-2, 5)
    more = jumps - r2["steps"] / r2["n"]
    # log(1e-2 / 1e-4) = 4.6: the extra jumps per path are of that order
    assert np.all((more > 2.0) & (more < 12.0)), (jumps, more)


def test_walk_on_spheres_exit_law_from_the_centre_is_uniform(orc):
    """From the centre of the unit ball the first jump lands on the sphere,
    uniformly: E[x^4] = 1/5 and E[x^2 y^2] = 1/15 on S^2 (moments of the
    uniform law), with exactly one jump per path."""
    prob = LinearProblem(ball(3), 1.0, [zero_fun()] * 3, zero_fun(), zero_fun(),
                         make_fun([(1.0, [factor("pow", 0, power=4)])]))
    r = orc.wos(prob, np.zeros((1, 3)), np.array([200000]), 1e-6, 9)
    assert r["steps"][0] == r["n"][0]
    assert abs(r["mean"][0] - 0.2) < 4 * r["se"][0]
    prob.g = make_fun([(1.0, [factor("pow", 0, power=2), factor("pow", 1, power=2)])])
    r = orc.wos(prob, np.zeros((1, 3)), np.array([200000]), 1e-6, 10)
    assert abs(r["mean"][0] - 1.0 / 15.0) < 4 * r["se"][0]


def test_walk_on_spheres_matches_the_poisson_kernel(orc):
    """Off-centre start in the unit ball: the exit law is the harmonic
    measure, so E[g(X_tau)] is the Poisson integral of g, here for the
    non-harmonic g = x^4 at x0 = (0.5, 0, 0), by 1-D quadrature."""
    a = 0.5
    kern = lambda t: (1 - a * a) / (4 * math.pi * (1 + a * a - 2 * a * math.cos(t)) ** 1.5)
    want = 2 * math.pi * integrate.quad(lambda t: kern(t) * math.cos(t) ** 4 * math.sin(t), 0, math.pi,
                                        epsabs=1e-13)[0]
    prob = LinearProblem(ball(3), 1.0, [zero_fun()] * 3, zero_fun(), zero_fun(),
                         make_fun([(1.0, [factor("pow", 0, power=4)])]))
    r = orc.wos(prob, np.array([[a, 0.0, 0.0]]), np.array([300000]), 1e-5, 13)
    assert abs(r["mean"][0] - want) < 4 * r["se"][0] + 4e-5, (r["mean"][0], want, r["se"][0])


def test_walk_exit_time_ball(orc):
    """f = 1, g = 0, c = 0: the estimator is E[n dt] -> (1 - |x|^2)/d."""
    for d, x0 in ((2, [0.0, 0.0]), (3, [0.3, 0.0, 0.0])):
        dt = 1e-3
        prob = LinearProblem(ball(d), 1.0, [zero_fun()] * d, zero_fun(), const_fun(1.0), zero_fun())
        r = orc.walk(prob, np.array([x0]), np.array([20000]), dt, 3)
        exact = (1.0 - sum(v * v for v in x0)) / d
        # overshoot bias of the discrete exit time is O(sqrt(dt))
        assert z_ok(r["mean"], r["se"], exact, extra=0.6 * math.sqrt(dt) * 1.0)
        assert r["mean"][0] == pytest.approx(r["steps"][0] / r["n"][0] * dt, rel=1e-12)


def test_walk_killing_closed_forms(orc):
    """g = 1, c constant: E[exp(-c tau)] = I0(k r)/I0(k) in 2-D, sinh(k r)/(r sinh k)
    in 3-D, k = sqrt(2c) (centre: 0.638536 and 0.730834 for c = 1)."""
    dt = 1e-3
    for d, exact in ((2, 1.0 / special.i0(math.sqrt(2.0))), (3, math.sqrt(2.0) / math.sinh(math.sqrt(2.0)))):
        prob = LinearProblem(ball(d), 1.0, [zero_fun()] * d, const_fun(1.0), zero_fun(), const_fun(1.0))
        r = orc.walk(prob, np.zeros((1, d)), np.array([20000]), dt, 4)
        assert z_ok(r["mean"], r["se"], exact, extra=0.02)
    assert 1.0 / special.i0(math.sqrt(2.0)) == pytest.approx(0.638536, abs=1e-6)


def test_walk_full_feynman_kac_with_drift(orc):
    """C2: manufactured u = cos(x) e^y with drift, killing and source."""
    w = CF.c2(dt=1e-3, n_nodes=4)
    r = orc.walk(w.problem, w.nodes, np.full(4, 4000), w.dt, 5)
    assert z_ok(r["mean"], r["se"], CF.c2_exact(w.nodes), extra=0.03)


def test_walk_degenerate_cases(orc):
    w = CF.c1()
    nodes = np.array([[1.2, 0.3], [0.0, 0.5], [0.5, 0.5]])
    r = orc.walk(w.problem, nodes, np.array([5, 5, 5]), 1e-3, 0, max_steps=3, dump=True)
    # outside and on the boundary: tau = 0, phi = g(P(x))
    assert np.allclose(r["phi"][:5], math.exp(1.0) * math.sin(0.3), rtol=1e-15)
    assert np.allclose(r["phi"][5:10], math.sin(0.5), rtol=1e-15)
    assert r["steps"][0] == 0 and r["steps"][1] == 0
    # centre with max_steps = 3: every path censored after 3 steps
    assert r["censored"][2] == 5 and r["steps"][2] == 15


def test_censored_path_value_at_the_nearest_boundary_point(orc):
    """A path still inside D when max_steps is reached (R12) takes
    phi = g(P X) Y + Z, P the nearest boundary point: for a box the nearest
    face (only that coordinate moves), for a ball the radial point.  With
    sigma = 1e-12 a path does not move measurably in 3 steps, so P X is the
    hand-computed point below, and with constant c, f the left-point sums are
    Y = exp(-3 c dt), Z = f dt (1 + exp(-c dt) + exp(-2 c dt)).  Leaving an
    interior point unprojected, picking the wrong face or scaling the wrong
    way misses by more than 1 in every case."""
    dt, c, f = 0.1, 0.5, 2.0
    Y = math.exp(-3 * c * dt)
    Z = f * dt * (1.0 + math.exp(-c * dt) + math.exp(-2 * c * dt))
    cases = [
        # (domain, g as a graded-lex linear polynomial, node, nearest boundary point)
        (box((0.0,), (1.0,)), [3.0, 7.0], (0.3,), (0.0,)),
        (box((0.0,), (1.0,)), [3.0, 7.0], (0.8,), (1.0,)),
        (box((0, 0), (1, 1)), [0.0, 10.0, 100.0], (0.2, 0.5), (0.0, 0.5)),
        (box((0, 0), (1, 1)), [0.0, 10.0, 100.0], (0.5, 0.9), (0.5, 1.0)),
        (box((0, 0), (1, 1)), [0.0, 10.0, 100.0], (0.93, 0.4), (1.0, 0.4)),
        (box((0, 0), (1, 1)), [0.0, 10.0, 100.0], (0.5, 0.03), (0.5, 0.0)),
        (box((-1, 0, 0), (2, 1, 3)), [0.0, 1.0, 10.0, 100.0], (0.5, 0.5, 0.1), (0.5, 0.5, 0.0)),
        (box((-1, 0, 0), (2, 1, 3)), [0.0, 1.0, 10.0, 100.0], (1.7, 0.5, 1.5), (2.0, 0.5, 1.5)),
        (ball(2, 2.0, (1.0, -1.0)), [0.0, 10.0, 100.0], (1.3, -0.6), (2.2, 0.6)),
        (ball(3), [0.0, 1.0, 10.0, 100.0], (0.1, 0.2, -0.2), (1 / 3, 2 / 3, -2 / 3)),
    ]
    for dom, gpoly, node, proj in cases:
        d = dom.ndim
        g = make_fun([], poly_degree=1, poly=gpoly)
        prob = LinearProblem(dom, 1e-12, [zero_fun()] * d, const_fun(c), const_fun(f), g)
        r = orc.walk(prob, np.array([node]), np.array([6]), dt, 2, max_steps=3, dump=True)
        g_at = gpoly[0] + sum(gpoly[1 + k] * proj[k] for k in range(d))
        want = g_at * Y + Z
        assert r["censored"][0] == 6 and r["steps"][0] == 18, (node, r["censored"], r["steps"])
        assert np.allclose(r["phi"], want, rtol=0, atol=1e-8), (node, r["phi"][0], want)


def test_welford_matches_two_pass(orc):
    w = CF.c1(scale=0.05)
    r = orc.walk(w.problem, w.nodes, w.paths, w.dt, 0, dump=True)
    off = np.concatenate([[0], np.cumsum(w.paths)])
    for i in range(len(w.paths)):
        x = r["phi"][off[i]:off[i + 1]]
        assert r["mean"][i] == pytest.approx(x.mean(), rel=1e-13)
        assert r["var"][i] == pytest.approx(x.var(ddof=1), rel=1e-12)


# ----------------------------------------------------------------------------- branching
def test_branching_constant_data_logistic(orc):
    """Eq. 3.1 with psi = a constant: u' = beta (u^2 - u), so
    u(T) = 1 / (1 + (1/a - 1) e^{beta T}) (= 0.13619047142218818 for a = 0.3)."""
    exact = 1.0 / (1.0 + (1.0 / 0.3 - 1.0) * math.e)
    assert exact == pytest.approx(0.13619047142218818, rel=1e-15)
    B = CF.c4_problem("0.3")
    for layout in (orc.PAIR52, orc.QUAD24):
        r = orc.branching(B, np.zeros((2, 3)), 40000, 1, layout=layout)
        assert z_ok(r["mean"], r["se"], exact)
        # E[segments] = 2 e^{beta T} - 1 for binary branching
        segs = r["steps"].sum() / r["n"].sum()
        assert segs == pytest.approx(2 * math.e - 1, rel=0.02)


def test_branching_die_or_split(orc):
    """Sec. 3.1 die-or-split example (alpha_0 = alpha_2 = 1/2): constant data a gives
    u(t) = 1 - (1 - a)/(1 + (1 - a) t / 2) (0.48148148... for a = 0.3, t = 1)."""
    B = BranchingProblem(1, 1.0, 1.0, 1.0, (0.5, 0, 0.5, 0, 0), (0.5, 0, 0.5, 0, 0), const_fun(0.3), 0.3)
    r = orc.branching(B, np.zeros((1, 1)), 60000, 2)
    exact = 1.0 - 0.7 / (1.0 + 0.7 * 0.5)
    assert exact == pytest.approx(0.48148148148148148, rel=1e-15)
    assert z_ok(r["mean"], r["se"], exact)


def test_branching_marked_signed_polynomial_ode(orc):
    """Marked branching (Sec. 3.2) with a signed nonlinearity (the CVA
    polynomial) and q != alpha: constant data reduces the PDE to the ODE
    u' = beta (sum_i alpha_i u^i - u), solved here by scipy."""
    alpha = (0.0586, 0.5, 0.8199, 0.0, -0.4095)
    q = (0.25, 0.25, 0.25, 0.0, 0.25)
    a, beta, T = 0.6, 1.0, 0.5
    B = BranchingProblem(1, 1.0, beta, T, alpha, q, const_fun(a), a)
    sol = integrate.solve_ivp(lambda t, u: beta * (sum(al * u ** i for i, al in enumerate(alpha)) - u),
                              (0, T), [a], rtol=1e-12, atol=1e-14)
    exact = sol.y[0, -1]
    r = orc.branching(B, np.zeros((1, 1)), 100000, 3)
    assert z_ok(r["mean"], r["se"], exact)


def test_branching_paper_kpp_travelling_wave(orc):
    """The paper's KPP example: u_t = u_xx + u^2 - u (sigma = sqrt 2) with
    psi = 1 - (1 + e^{x/sqrt6})^-2 has u(x,t) = 1 - (1 + e^{x/sqrt6 - 5t/6})^-2.
    With sigma = 1 the estimate is clearly off, which pins the factor 1/2 in the
    generator."""
    B = CF.kpp_travelling_wave_problem()
    xs = np.array([[-2.0], [-1.0], [0.0], [1.0], [2.0]])
    exact = 1.0 - (1.0 + np.exp(xs[:, 0] / math.sqrt(6.0) - 5.0 / 6.0)) ** -2
    assert np.allclose(exact, [0.296300, 0.398074, 0.514108, 0.634339, 0.745773], atol=1e-6)
    r = orc.branching(B, xs, 40000, 4)
    assert z_ok(r["mean"], r["se"], exact)
    B1 = BranchingProblem(1, 1.0, B.beta, B.T, B.alpha, B.q, B.psi, 1.0)
    r1 = orc.branching(B1, xs, 40000, 4)
    assert np.max(np.abs(r1["mean"] - exact) / r1["se"]) > 6.0


def test_branching_dfs_matches_algorithm_31(orc):
    """Per-particle clocks and the global Exp(beta N_p) clock of Algorithm 3.1
    are equal in law (memorylessness)."""
    B = CF.c4_problem("tanh")
    pts = np.array([[-1.0, 0.0, 0.0], [0.3, 1.0, -1.0], [1.5, 0.0, 0.0]])
    a = orc.branching(B, pts, 40000, 5)
    b = orc.branching_alg31(B, pts, 40000, 6, max_particles=64)
    assert np.all(np.abs(a["mean"] - b["mean"]) <= 4.0 * np.sqrt(a["se"] ** 2 + b["se"] ** 2))


def _kpp_1d_reference(xq, T=1.0, L=12.0, n=1201):
    """u_t = 0.5 u_xx + u^2 - u on [-L, L], psi = (1 + tanh x)/2, method of lines
    (second-order differences, stiff BDF), end values held at psi's limits."""
    x = np.linspace(-L, L, n)
    h = x[1] - x[0]
    u0 = 0.5 * (1.0 + np.tanh(x))

    def rhs(t, u):
        du = np.zeros_like(u)
        du[1:-1] = 0.5 * (u[2:] - 2 * u[1:-1] + u[:-2]) / h ** 2 + u[1:-1] ** 2 - u[1:-1]
        return du

    from scipy.sparse import diags
    jac_pat = diags([1, 1, 1], [-1, 0, 1], shape=(n, n))
    sol = integrate.solve_ivp(rhs, (0, T), u0, method="BDF", rtol=1e-10, atol=1e-12, jac_sparsity=jac_pat)
    return np.interp(xq, x, sol.y[:, -1])


def test_branching_c4_against_pde_solve(orc):
    """C4's data depends on x_1 only, so the 3-D solution is the 1-D solution of
    u_t = 0.5 u_xx + u^2 - u; compared with a method-of-lines solve."""
    B = CF.c4_problem("tanh")
    pts = np.array([[-1.5, 0.2, 0.1], [0.0, -1.0, 1.0], [0.7, 0.0, 0.0], [2.0, 1.0, 1.0]])
    ref = _kpp_1d_reference(pts[:, 0])
    ref2 = _kpp_1d_reference(pts[:, 0], n=2401)
    assert np.max(np.abs(ref - ref2)) < 2e-5
    r = orc.branching(B, pts, 40000, 7)
    assert z_ok(r["mean"], r["se"], ref2, extra=1e-5)


def test_branching_pruning_redraws(orc):
    """A tiny segment cap forces redraws; every tree still ends with a value."""
    B = BranchingProblem(1, 1.0, 1.0, 1.0, (0, 0, 1, 0, 0), (0, 0, 1, 0, 0), const_fun(0.3), 0.3, max_segments=3)
    r = orc.branching(B, np.zeros((1, 1)), 2000, 8, dump=True)
    assert r["redrawn"] > 0
    assert r["n"][0] == 2000
    assert np.all(r["segments"] <= 3)


# ----------------------------------------------------------------------------- branching with a boundary
def test_branching_bvp_logistic_boundary_data_is_exact_at_every_time(orc):
    """Eq. 3.2 with constant initial data c and boundary data equal to the
    logistic solution L(s) of u' = beta (u^2 - u): u(x, t) = L(t) everywhere,
    and since L is constant in space the estimator is unbiased for any dt
    (optional stopping).  Pins the time argument t_i - tau of g, the per-time
    products and marks, and the rule that a particle dying after a sub-step
    branches before any boundary test (testing first looks ahead to the death
    time and leaves an O(dt) bias, about 5e-3 at dt = 0.1)."""
    times = (0.0, 0.25, 0.5, 1.0)
    for dom, dt in ((box((-0.5,), (0.5,)), 0.1), (box((-0.5,), (0.5,)), 1e-2), (ball(2, 0.6), 0.05),
                    (box((-0.5, -0.4, -0.3), (0.5, 0.4, 0.3)), 0.05)):
        B, Bd = CF.kpp_bvp_logistic(dom, 0.3, 1.0, dt, times)
        d = dom.ndim
        pts = np.zeros((2, d))
        pts[1, 0] = 0.3 if d > 1 else 0.2
        r = orc.branching_bvp(B, Bd, pts, 30000, 7, layout=orc.PAIR52 if d != 2 else orc.QUAD24)
        exact = CF.logistic(0.3, 1.0, np.asarray(times))[:, None]
        assert np.all(r["mean"][0] == 0.3)
        assert z_ok(r["mean"][1:], r["se"][1:], exact[1:]), (d, dt, (r["mean"] - exact) / np.maximum(r["se"], 1e-300))
    # time-reversed boundary data L(-s) is far off: the test above can tell
    # a wrong time argument of g apart
    B, Bd = CF.kpp_bvp_logistic(box((-0.5,), (0.5,)), 0.3, 1.0, 1e-2, times)
    wrong = CF.kpp_bvp_logistic(box((-0.5,), (0.5,)), 0.3, -1.0, 1e-2, times)[1].g
    Bw = type(Bd)(Bd.domain, wrong, Bd.g_sup, Bd.dt, Bd.times)
    rw = orc.branching_bvp(B, Bw, np.zeros((1, 1)), 30000, 7)
    exact = CF.logistic(0.3, 1.0, np.asarray(times))
    assert np.max(np.abs(rw["mean"][1:, 0] - exact[1:]) / rw["se"][1:, 0]) > 10.0


def test_branching_bvp_paper_travelling_wave_with_boundary(orc):
    """The paper's KPP travelling wave (Sec. 3.1) on a bounded interval with
    the wave itself as Dirichlet data on both ends: the wave is the exact
    solution of the boundary-value problem.  The discrete boundary test leaves
    an O(sqrt dt) overshoot bias, bounded by 0.5826 sigma sqrt(dt) max|u_x|."""
    times = (0.25, 0.5, 1.0)
    B, Bd = CF.kpp_bvp_travelling_wave(-1.0, 1.5, 1e-3, times)
    pts = np.array([[-0.6], [0.0], [0.8], [1.3]])
    r = orc.branching_bvp(B, Bd, pts, 30000, 11)
    exact = np.array([CF.travelling_wave(pts[:, 0], t) for t in times])
    ux = 2.0 * (4.0 / 27.0) / math.sqrt(6.0)   # max |u_x| of the wave (at e^z = 1/2)
    bias = 0.5826 * B.sigma * math.sqrt(Bd.dt) * ux
    assert z_ok(r["mean"], r["se"], exact, extra=bias), (r["mean"] - exact) / r["se"]
    # a reflected wave on the boundary (data of x -> -x) is clearly off
    Bm, Bdm = CF.kpp_bvp_travelling_wave(-1.5, 1.0, 1e-3, times)
    Bdx = type(Bd)(Bd.domain, Bdm.g, Bd.g_sup, Bd.dt, Bd.times)
    rx = orc.branching_bvp(B, Bdx, pts, 30000, 11)
    assert np.max(np.abs(rx["mean"] - exact) - 4 * rx["se"] - bias) > 0.0


def test_branching_bvp_boundary_correction_cuts_the_overshoot_bias(orc):
    """The walk's boundary correction applied per sub-step (domain shrunk by
    c0 sigma sqrt(h) after a sub-step of length h): on the travelling-wave
    problem at dt = 1e-2 the largest error against the exact solution falls
    to under half of the plain test's (0.0087 -> 0.0026 at 1e5 trees); on
    spatially constant data (logistic) both stay exact."""
    times = (0.25, 0.5, 1.0)
    B, Bd = CF.kpp_bvp_travelling_wave(-1.0, 1.5, 1e-2, times)
    pts = np.array([[-0.9], [-0.6], [0.0], [0.8], [1.3], [1.45]])
    exact = np.array([CF.travelling_wave(pts[:, 0], t) for t in times])
    err = {}
    for name, sh in (("plain", 0.0), ("corrected", orc.GOBET_MENOZZI_C0)):
        r = orc.branching_bvp(B, Bd, pts, 60000, 11, boundary_shift=sh)
        err[name] = np.max(np.abs(r["mean"] - exact))
    assert err["corrected"] < 0.5 * err["plain"], err
    Bl, Bdl = CF.kpp_bvp_logistic(box((-0.5,), (0.5,)), 0.3, 1.0, 0.05, times)
    rl = orc.branching_bvp(Bl, Bdl, np.array([[0.0], [0.3]]), 30000, 5, boundary_shift=orc.GOBET_MENOZZI_C0)
    assert z_ok(rl["mean"], rl["se"], CF.logistic(0.3, 1.0, np.asarray(times))[:, None])


def test_branching_bvp_free_space_times_match_single_time_estimator(orc):
    """Without a boundary the multi-time estimator at each output time t_i has
    the law of the free-space estimator run to T = t_i (Algorithm 3.1 reads one
    tree at every T_i); sub-steps at the output times must not change it."""
    B4 = CF.c4_problem("tanh")
    pts = np.array([[-0.7, 0.1, 0.0], [0.4, -0.5, 0.2]])
    times = (0.3, 0.7, 1.0)
    from workloads.problem import BranchingBoundary, free
    Bd = BranchingBoundary(free(3), const_fun(0.0), 0.0, 0.05, times)
    r = orc.branching_bvp(B4, Bd, pts, 30000, 13, layout=orc.QUAD24)
    for k, t in enumerate(times):
        Bt = BranchingProblem(3, B4.sigma, B4.beta, t, B4.alpha, B4.q, B4.psi, B4.psi_sup, B4.max_segments)
        o = orc.branching(Bt, pts, 30000, 14)
        assert np.all(np.abs(r["mean"][k] - o["mean"]) <= 4.0 * np.sqrt(r["se"][k] ** 2 + o["se"] ** 2)), t


def test_branching_bvp_start_outside_and_pruning(orc):
    """A start point outside the domain is stopped at time 0 (value g(P x, t_i));
    a tiny segment cap redraws trees and never leaves a tree without values."""
    times = (0.0, 0.5)
    B, Bd = CF.kpp_bvp_logistic(box((-0.5,), (0.5,)), 0.3, 1.0, 0.05, times)
    r = orc.branching_bvp(B, Bd, np.array([[0.9], [-2.0]]), 50, 1, dump=True)
    assert np.allclose(r["value"][:, :, 0], 0.3, rtol=1e-14)
    assert np.allclose(r["value"][:, :, 1], CF.logistic(0.3, 1.0, 0.5), rtol=1e-13)
    Bp = BranchingProblem(1, 1.0, 2.0, 1.0, B.alpha, B.q, B.psi, B.psi_sup, max_segments=3)
    Bd2 = type(Bd)(Bd.domain, Bd.g, Bd.g_sup, Bd.dt, (1.0,))
    rp = orc.branching_bvp(Bp, Bd2, np.zeros((1, 1)), 500, 2, dump=True)
    assert rp["redrawn"] > 0 and rp["n"][0, 0] == 500 and np.all(rp["segments"] <= 3)


# ----------------------------------------------------------------------------- adjoint
def _small_adjoint_problem(seed=0):
    rng = np.random.default_rng(seed)
    sh = CF.real_solid_harmonics_poly(7)
    tg = rng.standard_normal(64)
    tf = rng.standard_normal(16)
    tc = 0.1 * rng.standard_normal(16)
    tc[0] += 1.0
    P = CF.c5_problem(tg, tf, tc, sh)
    # add generic product terms so both coefficient kinds are exercised
    P.f = make_fun([(0.7, [factor("sin", 1, a=2.0)]), (-0.4, [factor("exp", 2)])], poly_degree=3, poly=P.f.poly)
    P.c = make_fun([(0.3, [factor("cos", 0)])], poly_degree=3, poly=P.c.poly)
    P.g = make_fun([(0.5, [factor("tanh", 0), factor("pow", 1, power=2)])], poly_degree=7, poly=P.g.poly)
    return P


def test_adjoint_matches_central_fd_with_common_random_numbers(orc):
    P = _small_adjoint_problem()
    nodes = CF.c5_nodes(6)
    paths = np.full(6, 150, np.int64)
    dt, seed = 1e-2, 21
    w = np.random.default_rng(2).standard_normal(6)
    adj = orc.walk_adjoint(P, nodes, paths, dt, seed, w)

    def objective(P2):
        return float(w @ orc.walk(P2, nodes, paths, dt, seed)["mean"])

    rng = np.random.default_rng(3)
    for name in ("g", "f", "c"):
        F = getattr(P, name)
        for kind in ("coef", "poly"):
            arr = F.coef if kind == "coef" else F.poly
            idx = rng.choice(len(arr), size=min(3, len(arr)), replace=False)
            for j in idx:
                h = 1e-3 * max(1.0, abs(arr[j]))
                vals = []
                for s in (+1, -1):
                    a2 = arr.copy()
                    a2[j] += s * h
                    F2 = F.with_coef(coef=a2) if kind == "coef" else F.with_coef(poly=a2)
                    P2 = LinearProblem(P.domain, P.sigma, P.b, P.c, P.f, P.g)
                    setattr(P2, name, F2)
                    vals.append(objective(P2))
                fd = (vals[0] - vals[1]) / (2 * h)
                got = adj[f"{name}_{kind}"][j]
                tol = 1e-9 * max(1.0, abs(fd)) if name != "c" else 1e-5 * max(1.0, abs(fd))
                assert abs(got - fd) <= tol, (name, kind, j, got, fd)


def test_adjoint_dot_product_with_directional_fd(orc):
    P = _small_adjoint_problem(1)
    nodes = CF.c5_nodes(4)
    paths = np.full(4, 100, np.int64)
    dt, seed = 1e-2, 5
    w = np.ones(4)
    adj = orc.walk_adjoint(P, nodes, paths, dt, seed, w)
    rng = np.random.default_rng(9)
    dirs = {k: rng.standard_normal(len(v)) for k, v in adj.items() if k != "stats"}
    h = 1e-4

    def shifted(s):
        P2 = LinearProblem(P.domain, P.sigma, P.b, P.c, P.f, P.g)
        for name in ("g", "f", "c"):
            F = getattr(P, name)
            setattr(P2, name, F.with_coef(coef=F.coef + s * h * dirs[f"{name}_coef"],
                                          poly=F.poly + s * h * dirs[f"{name}_poly"]))
        return float(w @ orc.walk(P2, nodes, paths, dt, seed)["mean"])

    fd = (shifted(+1) - shifted(-1)) / (2 * h)
    dot = sum(float(adj[k] @ dirs[k]) for k in dirs)
    assert dot == pytest.approx(fd, rel=1e-6)


def test_adjoint_analytic_solid_harmonic_gradient(orc):
    """c = f = 0 and g = sum theta_k r^l Y_k: u is linear in theta with
    du/dtheta_k = r^l Y_k(x) at the node (harmonic data reproduces itself)."""
    sh = CF.real_solid_harmonics_poly(7)
    theta = np.random.default_rng(4).standard_normal(64)
    P = CF.c5_problem(theta, np.zeros(16), np.zeros(16), sh)
    P.c, P.f = zero_fun(), zero_fun()
    node = np.array([[0.2, -0.1, 0.3]])
    n = 20000
    adj = orc.walk_adjoint(P, node, np.array([n]), 2.5e-3, 8, np.ones(1))
    g_mono = adj["g_poly"]            # E[x^alpha(X_tau)] per monomial
    grad_theta = sh.T @ g_mono
    exact = CF.real_solid_harmonic_values(node)[0]
    # each component is a mean of G_k(X_tau) (|G_k| <= ~1.3 on the sphere):
    # allow 4 SE of a bounded variable plus the sqrt(dt) exit bias
    tol = 4.0 * 1.3 / math.sqrt(n) + 0.03
    assert np.max(np.abs(grad_theta - exact)) < tol


def test_walk_jacobian_columns_are_walks_of_the_basis_functions(orc):
    """With c = 0 the derivative of one path value with respect to a
    coefficient of g is that basis function at the exit point, and with
    respect to one of f the path's integral of that basis function: each
    Jacobian column is the plain walk of the problem whose g (or f) is that
    basis function alone.  Its mean and standard error must equal that walk's
    (whose Welford statistics are pinned to a two-pass computation)."""
    P = _small_adjoint_problem(2)
    P.c = zero_fun()
    P.g = make_fun([(0.8, [factor("sin", 2)])], poly_degree=2, poly=np.arange(10) * 0.1 - 0.3)
    P.f = make_fun([(0.5, [factor("cos", 1)])], poly_degree=1, poly=np.array([0.2, -0.1, 0.4, 0.3]))
    nodes = CF.c5_nodes(3)
    paths = np.array([300, 150, 211], np.int64)
    dt, seed = 1e-2, 13
    ids = np.array([7, 40, 2])
    J = orc.walk_jacobian(P, nodes, paths, dt, seed, node_ids=ids)
    one = lambda n, k: np.eye(n)[k]
    col = 0
    cases = []
    for k in range(P.g.n_terms):
        cases.append(("g", P.g.with_coef(coef=one(P.g.n_terms, k), poly=np.zeros(len(P.g.poly)))))
    for m in range(len(P.g.poly)):
        cases.append(("g", P.g.with_coef(coef=np.zeros(P.g.n_terms), poly=one(len(P.g.poly), m))))
    for k in range(P.f.n_terms):
        cases.append(("f", P.f.with_coef(coef=one(P.f.n_terms, k), poly=np.zeros(len(P.f.poly)))))
    for m in range(len(P.f.poly)):
        cases.append(("f", P.f.with_coef(coef=np.zeros(P.f.n_terms), poly=one(len(P.f.poly), m))))
    assert J["jac"].shape == (3, len(cases) + len(P.c.poly) + P.c.n_terms)
    for name, F in cases:
        Pk = LinearProblem(P.domain, P.sigma, P.b, zero_fun(), F if name == "f" else zero_fun(),
                           F if name == "g" else zero_fun())
        r = orc.walk(Pk, nodes, paths, dt, seed, node_ids=ids)
        assert np.allclose(J["jac"][:, col], r["mean"], rtol=1e-12, atol=1e-14), (name, col)
        assert np.allclose(J["jac_se"][:, col], r["se"], rtol=1e-9, atol=1e-14), (name, col)
        col += 1
    assert np.array_equal(J["stats"]["steps"], orc.walk(P, nodes, paths, dt, seed, node_ids=ids)["steps"])


def test_walk_jacobian_weighted_rows_equal_the_adjoint(orc):
    """sum_i w_i J[i] is the gradient of sum_i w_i u_i, which the adjoint
    computes (pinned above by finite differences with common random
    numbers); with terms and polynomials in g, f and c."""
    P = _small_adjoint_problem(3)
    nodes = CF.c5_nodes(4)
    paths = np.array([120, 90, 150, 60], np.int64)
    dt, seed = 1e-2, 4
    w = np.array([0.5, -1.5, 2.0, 0.7])
    J = orc.walk_jacobian(P, nodes, paths, dt, seed)
    adj = orc.walk_adjoint(P, nodes, paths, dt, seed, w)
    want = np.concatenate([adj[k] for k in ("g_coef", "g_poly", "f_coef", "f_poly", "c_coef", "c_poly")])
    got = w @ J["jac"]
    assert np.allclose(got, want, rtol=1e-11, atol=1e-13 * np.abs(want).max())
