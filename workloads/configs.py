"""Seeded synthetic workloads with the shapes of the five benchmark problems.

Every generator returns plain data (problem description, node coordinates,
per-node path budgets, time step, path seed).  `scale` shrinks path budgets
(and, where stated, node counts) for tests; scale=1 is the full size.

Workload construction uses numpy's PCG64 (`default_rng`); the paths
themselves always draw from the counter-based generator inside the solvers.

  C1  2-D Laplace on the unit square, harmonic data g = e^x sin y,
      16 nodes on x = 0.5, 1e4 paths/node, dt = 1e-3.
  C2  2-D elliptic on the unit disk, L = 1/2 Lap + b.grad - c with
      b = (sin(pi y), cos(pi x)), c = 1 + x^2/2, f manufactured from
      u = cos(x) e^y; 256 nodes on the four chords x, y = +-1/3,
      1e6 paths/node, dt = 1e-4.
  C3  4096 nodes drawn from 8 subdomain layouts (unit square, unit disk,
      unit ball), log-uniform budgets in [1e3, 1e5], L = 1/2 Lap,
      g = sum of 8 harmonic polynomials with N(0,1) weights, dt = 1e-3.
  C4  KPP u_t = 1/2 Lap u + (u^2 - u) in R^3, T = 1, binary branching,
      psi = (1 + tanh x_1)/2, 1024 points in [-2,2]^3, 1e5 trees each.
  C5  3-D unit ball, 1/2 Lap u - c u = -f, g = sum_{k<64} theta_k r^l Y_k
      (real solid harmonics, l <= 7), c, f = 16-monomial expansions,
      4096 nodes on the three discs x_k = 0, |x| < 0.95, 1e5 paths/node,
      dt = 1e-3, loss sum_i (u_i - d_i)^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np

from .problem import (BranchingBoundary, BranchingProblem, Domain, Fun, LinearProblem, ball, box, const_fun,
                      factor, make_fun, monomial_exponents, n_monomials, zero_fun)


@dataclass
class LinearWorkload:
    name: str
    problem: LinearProblem
    nodes: np.ndarray       # (n, ndim) float64
    paths: np.ndarray       # (n,) int64
    dt: float
    seed: int


@dataclass
class BranchingWorkload:
    name: str
    problem: BranchingProblem
    points: np.ndarray      # (n, ndim)
    trees: int
    seed: int


def _budget(n: int, scale: float, floor: int = 2) -> int:
    return max(floor, int(round(n * scale)))


# --------------------------------------------------------------------------- C1
def c1(scale: float = 1.0, dt: float = 1e-3, seed: int = 0) -> LinearWorkload:
    g = make_fun([(1.0, [factor("exp", 0), factor("sin", 1)])])
    prob = LinearProblem(box((0.0, 0.0), (1.0, 1.0)), 1.0,
                         [zero_fun(), zero_fun()], zero_fun(), zero_fun(), g)
    nodes = np.array([[0.5, (k + 1) / 17.0] for k in range(16)], np.float64)
    paths = np.full(16, _budget(10_000, scale), np.int64)
    return LinearWorkload("C1 laplace unit square", prob, nodes, paths, dt, seed)


def c1_exact(nodes: np.ndarray) -> np.ndarray:
    return np.exp(nodes[:, 0]) * np.sin(nodes[:, 1])


# --------------------------------------------------------------------------- C2
def c2_problem() -> LinearProblem:
    pi = math.pi
    b0 = make_fun([(1.0, [factor("sin", 1, a=pi)])])
    b1 = make_fun([(1.0, [factor("cos", 0, a=pi)])])
    c = make_fun([(1.0, []), (0.5, [factor("pow", 0, power=2)])])
    # f = e^y [ (1 + x^2/2) cos x + sin(pi y) sin x - cos(pi x) cos x ]
    f = make_fun([
        (1.0, [factor("exp", 1), factor("cos", 0)]),
        (0.5, [factor("pow", 0, power=2), factor("exp", 1), factor("cos", 0)]),
        (1.0, [factor("exp", 1), factor("sin", 1, a=pi), factor("sin", 0)]),
        (-1.0, [factor("exp", 1), factor("cos", 0, a=pi), factor("cos", 0)]),
    ])
    g = make_fun([(1.0, [factor("cos", 0), factor("exp", 1)])])
    return LinearProblem(ball(2, 1.0), 1.0, [b0, b1], c, f, g)


def c2_nodes() -> np.ndarray:
    pts = []
    for h in (-1.0 / 3.0, 1.0 / 3.0):
        half = math.sqrt(1.0 - h * h)
        for k in range(64):
            s = -half + (k + 1) * 2.0 * half / 65.0
            pts.append((h, s))
        for k in range(64):
            s = -half + (k + 1) * 2.0 * half / 65.0
            pts.append((s, h))
    return np.asarray(pts, np.float64)


def c2(scale: float = 1.0, dt: float = 1e-4, seed: int = 0, n_nodes: Optional[int] = None) -> LinearWorkload:
    nodes = c2_nodes()
    if n_nodes is not None:
        nodes = nodes[np.linspace(0, len(nodes) - 1, n_nodes).round().astype(int)]
    paths = np.full(len(nodes), _budget(1_000_000, scale), np.int64)
    return LinearWorkload("C2 elliptic unit disk", c2_problem(), nodes, paths, dt, seed)


def c2_exact(nodes: np.ndarray) -> np.ndarray:
    return np.cos(nodes[:, 0]) * np.exp(nodes[:, 1])


# --------------------------------------------------------------------------- C3
def harmonic_basis_2d() -> np.ndarray:
    """Coefficients (8, 15) of Re z^n, Im z^n (n=1..4) as dense degree-4
    polynomials in (x, y), graded-lex order."""
    ex = monomial_exponents(2, 4)
    index = {(int(a), int(b)): i for i, (a, b, _) in enumerate(ex)}
    out = np.zeros((8, len(ex)))
    for n in range(1, 5):
        for k in range(n + 1):
            # (x + i y)^n = sum_k C(n,k) x^(n-k) (i y)^k ; i^k cycles 1, i, -1, -i
            cplx = math.comb(n, k) * (1j ** k)
            out[2 * (n - 1), index[(n - k, k)]] += cplx.real
            out[2 * (n - 1) + 1, index[(n - k, k)]] += cplx.imag
    return out


def harmonic_basis_3d() -> np.ndarray:
    """Coefficients (8, 10) of x, y, z, xy, yz, xz, x^2-y^2, 2z^2-x^2-y^2 as dense
    degree-2 polynomials in (x, y, z), graded-lex order."""
    ex = monomial_exponents(3, 2)
    index = {tuple(int(v) for v in e): i for i, e in enumerate(ex)}
    rows = [
        {(1, 0, 0): 1.0}, {(0, 1, 0): 1.0}, {(0, 0, 1): 1.0},
        {(1, 1, 0): 1.0}, {(0, 1, 1): 1.0}, {(1, 0, 1): 1.0},
        {(2, 0, 0): 1.0, (0, 2, 0): -1.0},
        {(0, 0, 2): 2.0, (2, 0, 0): -1.0, (0, 2, 0): -1.0},
    ]
    out = np.zeros((8, len(ex)))
    for r, row in enumerate(rows):
        for e, v in row.items():
            out[r, index[e]] = v
    return out


C3_LAYOUTS = [
    ("box2", 2), ("box2", 3), ("box2", 4),
    ("disk", 2), ("disk", 3), ("disk", 4),
    ("ball3", 2), ("ball3", 3),
]


def _layout_domain(kind: str):
    if kind == "box2":
        return box((0.0, 0.0), (1.0, 1.0))
    if kind == "disk":
        return ball(2, 1.0)
    return ball(3, 1.0)


def _interface_points(kind: str, parts: int, n: int, rng: np.random.Generator, margin: float = 1e-3) -> np.ndarray:
    """n points uniform on the union of the interior interfaces of a parts^d grid partition."""
    if kind == "box2":
        cuts = [k / parts for k in range(1, parts)]
        pts = []
        while len(pts) < n:
            h = cuts[rng.integers(len(cuts))]
            s = rng.uniform(margin, 1.0 - margin)
            pts.append((h, s) if rng.integers(2) == 0 else (s, h))
        return np.asarray(pts)
    cuts = [-1.0 + 2.0 * k / parts for k in range(1, parts)]
    ndim = 2 if kind == "disk" else 3
    if ndim == 2:
        w = np.array([2.0 * math.sqrt(1 - h * h) for h in cuts])
    else:
        w = np.array([math.pi * (1 - h * h) for h in cuts])
    w = w / w.sum()
    pts = []
    while len(pts) < n:
        h = cuts[rng.choice(len(cuts), p=w)]
        axis = int(rng.integers(ndim))
        rad = math.sqrt(1.0 - h * h)
        if ndim == 2:
            s = rng.uniform(-rad, rad)
            p = [0.0, 0.0]
            p[axis] = h
            p[1 - axis] = s
        else:
            rr = rad * math.sqrt(rng.uniform())
            th = rng.uniform(0, 2 * math.pi)
            p = [0.0, 0.0, 0.0]
            others = [k for k in range(3) if k != axis]
            p[axis] = h
            p[others[0]] = rr * math.cos(th)
            p[others[1]] = rr * math.sin(th)
        if np.linalg.norm(p) < 1.0 - margin:
            pts.append(tuple(p))
    return np.asarray(pts)


def c3(scale: float = 1.0, dt: float = 1e-3, seed: int = 0, n_nodes: int = 4096,
       workload_seed: int = 3) -> List[LinearWorkload]:
    """One LinearWorkload per layout (the union is the 4096-node batch)."""
    rng = np.random.default_rng(workload_seed)
    layout_of = rng.integers(len(C3_LAYOUTS), size=n_nodes)
    budgets = np.exp(rng.uniform(math.log(1e3), math.log(1e5), size=n_nodes))
    weights = rng.standard_normal((len(C3_LAYOUTS), 8))
    out = []
    for li, (kind, parts) in enumerate(C3_LAYOUTS):
        sel = np.nonzero(layout_of == li)[0]
        dom = _layout_domain(kind)
        ndim = dom.ndim
        pts = _interface_points(kind, parts, len(sel), rng)
        basis = harmonic_basis_2d() if ndim == 2 else harmonic_basis_3d()
        deg = 4 if ndim == 2 else 2
        g = make_fun([], poly_degree=deg, poly=weights[li] @ basis)
        prob = LinearProblem(dom, 1.0, [zero_fun() for _ in range(ndim)], zero_fun(), zero_fun(), g)
        paths = np.maximum(2, np.round(budgets[sel] * scale)).astype(np.int64)
        out.append(LinearWorkload(f"C3 {kind} {parts}^{ndim}", prob, pts.astype(np.float64), paths, dt, seed))
    return out


@dataclass
class BatchWorkload:
    """A heterogeneous batch: node i belongs to problems[node_problem[i]] and
    sits at nodes[i, :ndim] (rows padded to three coordinates)."""
    name: str
    problems: List[LinearProblem]
    node_problem: np.ndarray   # (n,) int32
    nodes: np.ndarray          # (n, 3)
    paths: np.ndarray          # (n,) int64
    dt: float
    seed: int
    exact: np.ndarray          # (n,) exact solution (harmonic data)


def c3_batch(scale: float = 1.0, dt: float = 1e-3, seed: int = 0, n_nodes: int = 4096,
             workload_seed: int = 3) -> BatchWorkload:
    """C3 as one batch: the same 4096 nodes, budgets and layouts as c3(), in
    the order they were drawn (node i of the batch is the i-th draw), so the
    eight layouts interleave in one node list."""
    rng = np.random.default_rng(workload_seed)
    layout_of = rng.integers(len(C3_LAYOUTS), size=n_nodes)
    parts = c3(scale, dt, seed, n_nodes, workload_seed)
    nodes = np.zeros((n_nodes, 3))
    paths = np.zeros(n_nodes, np.int64)
    exact = np.zeros(n_nodes)
    for li, w in enumerate(parts):
        sel = np.nonzero(layout_of == li)[0]
        nodes[sel, :w.problem.ndim] = w.nodes
        paths[sel] = w.paths
        exact[sel] = c3_exact(w)
    return BatchWorkload("C3 batch, 8 layouts", [w.problem for w in parts], layout_of.astype(np.int32), nodes,
                         paths, dt, seed, exact)


def eval_dense_poly(ndim: int, degree: int, coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Reference evaluation of a dense graded-lex polynomial (workload checks only)."""
    ex = monomial_exponents(ndim, degree)
    x3 = np.zeros((x.shape[0], 3))
    x3[:, :ndim] = x
    vals = np.prod(x3[:, None, :] ** ex[None, :, :], axis=2)
    return vals @ coef


def c3_exact(w: LinearWorkload) -> np.ndarray:
    """Exact solution at the nodes of one C3 layout: u = g (harmonic data,
    b = c = f = 0), g being a dense polynomial with no terms."""
    g = w.problem.g
    assert g.n_terms == 0 and g.poly_degree >= 0
    return eval_dense_poly(w.problem.ndim, g.poly_degree, np.asarray(g.poly), w.nodes)


# --------------------------------------------------------------------------- C4
def c4_problem(psi: str = "tanh", sigma: float = 1.0) -> BranchingProblem:
    if psi == "tanh":
        fpsi = make_fun([(0.5, []), (0.5, [factor("tanh", 0)])])
        sup = 1.0
    else:
        fpsi = const_fun(float(psi))
        sup = abs(float(psi))
    return BranchingProblem(3, sigma, 1.0, 1.0, (0.0, 0.0, 1.0, 0.0, 0.0),
                            (0.0, 0.0, 1.0, 0.0, 0.0), fpsi, sup, 127)


def c4(scale: float = 1.0, seed: int = 0, psi: str = "tanh", n_points: int = 1024,
       workload_seed: int = 4) -> BranchingWorkload:
    rng = np.random.default_rng(workload_seed)
    pts = rng.uniform(-2.0, 2.0, size=(n_points, 3))
    return BranchingWorkload("C4 KPP branching R^3", c4_problem(psi), pts,
                             _budget(100_000, scale), seed)


def kpp_travelling_wave_problem() -> BranchingProblem:
    """The paper's KPP example u_t = u_xx + u^2 - u (D = r = 1), which is the
    branching PDE with generator u_xx, i.e. sigma = sqrt(2), beta = 1, alpha_2 = 1,
    and initial data psi = 1 - (1 + e^{x/sqrt6})^-2.  Since
    (1 + e^s)^-1 = (1 - tanh(s/2))/2, psi = 3/4 + tanh(s/2)/2 - tanh(s/2)^2/4."""
    k = 1.0 / (2.0 * math.sqrt(6.0))
    psi = make_fun([(0.75, []), (0.5, [factor("tanh", 0, a=k)]),
                    (-0.25, [factor("tanh", 0, a=k, power=2)])])
    return BranchingProblem(1, math.sqrt(2.0), 1.0, 1.0, (0.0, 0.0, 1.0, 0.0, 0.0),
                            (0.0, 0.0, 1.0, 0.0, 0.0), psi, 1.0, 127)


# --------------------------------------------------------------------------- branching with a boundary
def travelling_wave(x, t):
    """The paper's KPP travelling wave u(x, t) = 1 - (1 + e^{x/sqrt6 - 5t/6})^-2."""
    return 1.0 - (1.0 + np.exp(np.asarray(x) / math.sqrt(6.0) - 5.0 * np.asarray(t) / 6.0)) ** -2


def kpp_bvp_travelling_wave(x1: float, x2: float, dt: float, times, max_segments: int = 255):
    """The paper's KPP example on the interval (x1, x2) with Dirichlet data
    equal to the travelling wave on both ends (eq. 3.2), so the travelling
    wave is the exact solution.  With z = x/sqrt6 - 5s/6 the wave is
    3/4 + T/2 - T^2/4, T = tanh(z/2); at an end point x_b it is a function of
    the time argument s alone, and g interpolates the two ends linearly in x:
    g(x, s) = sum_b w_b(x) u(x_b, s), w_1 = (x2 - x)/(x2 - x1), w_2 = (x - x1)/(x2 - x1)
    (coordinate index 1 is s)."""
    B = kpp_travelling_wave_problem()
    B = BranchingProblem(B.ndim, B.sigma, B.beta, float(max(times)), B.alpha, B.q, B.psi, B.psi_sup, max_segments)
    L = x2 - x1
    terms = []
    for xb, (wa, wb) in ((x1, (-1.0 / L, x2 / L)), (x2, (1.0 / L, -x1 / L))):
        w = factor("pow", 0, a=wa, b=wb)
        th = lambda p, xb=xb: factor("tanh", 1, a=-5.0 / 12.0, b=xb / (2.0 * math.sqrt(6.0)), power=p)
        terms += [(0.75, [w, factor("pow", 0, power=0)]), (0.5, [w, th(1)]), (-0.25, [w, th(2)])]
    Bd = BranchingBoundary(box((x1,), (x2,)), make_fun(terms), 1.0, float(dt), tuple(float(t) for t in times))
    return B, Bd


def kpp_bvp_logistic(domain: Domain, c: float, beta: float, dt: float, times, max_segments: int = 255):
    """Binary branching (alpha_2 = 1) with constant initial data c and boundary
    data equal to the logistic solution L(s) = 1 / (1 + ((1 - c)/c) e^{beta s})
    of u' = beta (u^2 - u): the solution is L(t) at every point, and the
    estimator is unbiased for any dt (the solution is constant in space).
    L(s) = 1/2 - tanh(beta s / 2 + ln((1 - c)/c) / 2) / 2."""
    d = domain.ndim
    B = BranchingProblem(d, 1.0, beta, float(max(times)), (0.0, 0.0, 1.0, 0.0, 0.0), (0.0, 0.0, 1.0, 0.0, 0.0),
                         const_fun(c), abs(c), max_segments)
    g = make_fun([(0.5, []), (-0.5, [factor("tanh", d, a=beta / 2.0, b=0.5 * math.log((1.0 - c) / c))])])
    return B, BranchingBoundary(domain, g, 1.0, float(dt), tuple(float(t) for t in times))


def logistic(c: float, beta: float, t):
    return 1.0 / (1.0 + (1.0 - c) / c * np.exp(beta * np.asarray(t)))


@dataclass
class BranchingBvpWorkload:
    name: str
    problem: BranchingProblem
    boundary: BranchingBoundary
    points: np.ndarray
    trees: int
    seed: int


def c6(scale: float = 1.0, seed: int = 0, n_points: int = 1024, dt: float = 1e-3) -> BranchingBvpWorkload:
    """The paper's KPP PDD setting (Sec. 3.1, Algorithm 3.1) on a bounded
    interval: u_t = u_xx + u^2 - u on (-5, 5) (the interval of the paper's
    error comparison) with travelling-wave initial and boundary data, 11
    output times 0, 0.1, .., 1 (the paper's Theta), n_points interior points
    evenly spaced (the interface nodes of a fine partition), 1e5 trees per
    point (the paper's N), boundary test every dt."""
    B, Bd = kpp_bvp_travelling_wave(-5.0, 5.0, dt, tuple(0.1 * k for k in range(11)))
    pts = (-5.0 + 10.0 * (np.arange(n_points) + 0.5) / n_points).reshape(-1, 1)
    return BranchingBvpWorkload("C6 KPP with boundary, 11 times", B, Bd, pts, _budget(100_000, scale), seed)


# --------------------------------------------------------------------------- C7
@dataclass
class CvaWorkload:
    """Inputs of the CVA construction of Sec. 3.3: u_t = 0.5 sigma^2 u_xx + f(u),
    u(., 0) = psi with |psi| <= psi_sup, at horizon T, branching rate beta.
    The branching problem itself (rescaling by psi_sup, polynomial fit of the
    rescaled nonlinearity, marks) is built by the library's host-side driver;
    this record holds only what goes into it."""
    name: str
    sigma: float
    nonlinearity: Callable[[np.ndarray], np.ndarray]
    psi: Fun
    psi_sup: float
    T: float
    beta: float
    points: np.ndarray
    trees: int
    seed: int


def c7_nonlinearity(u):
    """The CVA-type nonlinearity of Sec. 3.3 with r_0 = -1, r_1 = 1:
    f(u) = max(u, 0) - u (so the branching rate is 1)."""
    return np.maximum(u, 0.0) - u


def c7(scale: float = 1.0, seed: int = 0, n_points: int = 1024) -> CvaWorkload:
    """The CVA construction of Sec. 3.3 in one dimension (the paper leaves the
    operator, payoff and horizon open; chosen here): u_t = 0.5 u_xx + f(u),
    f = max(u, 0) - u, payoff psi = 2 tanh(x) (bounded, signed, psi_sup = 2),
    T = 0.5, beta = 1; 1024 points evenly spaced in [-3, 3], 1e5 trees each."""
    psi = make_fun([(2.0, [factor("tanh", 0)])])
    pts = np.linspace(-3.0, 3.0, n_points).reshape(-1, 1)
    return CvaWorkload("C7 CVA marked branching", 1.0, c7_nonlinearity, psi, 2.0, 0.5, 1.0, pts,
                       _budget(100_000, scale), seed)


def cva_reference_quartic(f: Callable[[np.ndarray], np.ndarray], psi_sup: float, n: int = 2001) -> np.ndarray:
    """Coefficients (increasing powers) of the quartic that Sec. 3.3's
    approximation step assigns to the rescaled nonlinearity
    v -> f(psi_sup v) / psi_sup on [-1, 1]: discrete least squares on n equally
    spaced points (the reading that reproduces every digit the paper prints for
    max(v, 0)), computed with numpy's own polynomial fit.  Used only to build
    reference solutions and expected values, independently of the library's
    driver."""
    from numpy.polynomial import polynomial as NP
    v = np.linspace(-1.0, 1.0, n)
    return NP.polyfit(v, np.asarray(f(psi_sup * v), dtype=np.float64) / psi_sup, 4)


def c7_reference(xq, L: float = 12.0, n: int = 2401) -> np.ndarray:
    """Method-of-lines solution (second-order differences, stiff BDF) at T of
    the PDE the C7 estimator represents: u_t = 0.5 u_xx + s P(u / s), P the
    quartic of `cva_reference_quartic`, s = psi_sup = 2, u(., 0) = 2 tanh x."""
    from scipy import integrate
    from scipy.sparse import diags
    w = c7(scale=1e-5, n_points=1)
    s, T = w.psi_sup, w.T
    a = cva_reference_quartic(w.nonlinearity, s)
    x = np.linspace(-L, L, n)
    h = x[1] - x[0]

    def rhs(t, u):
        du = np.zeros_like(u)
        v = u[1:-1] / s
        du[1:-1] = 0.5 * w.sigma ** 2 * (u[2:] - 2 * u[1:-1] + u[:-2]) / h ** 2 + s * sum(
            a[i] * v ** i for i in range(len(a)))
        return du

    sol = integrate.solve_ivp(rhs, (0, T), 2.0 * np.tanh(x), method="BDF", rtol=1e-10, atol=1e-12,
                              jac_sparsity=diags([1, 1, 1], [-1, 0, 1], shape=(n, n)))
    return np.interp(np.asarray(xq), x, sol.y[:, -1])


# --------------------------------------------------------------------------- C5
def real_solid_harmonics_poly(lmax: int = 7) -> np.ndarray:
    """Matrix (n_mono(3, lmax), (lmax+1)^2) whose column k holds the dense
    graded-lex coefficients of r^l Y_k(x/r), Y_k the real orthonormal
    spherical harmonics without the Condon-Shortley phase, ordered by
    l = 0..lmax, m = -l..l.  Obtained by an exact least-squares fit of each
    degree-l homogeneous polynomial against scipy's spherical harmonics."""
    from scipy.special import sph_harm_y
    ex = monomial_exponents(3, lmax)
    deg = ex.sum(axis=1)
    rng = np.random.default_rng(12345)
    pts = rng.standard_normal((400, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    pts *= rng.uniform(0.3, 1.0, size=(400, 1))
    r = np.linalg.norm(pts, axis=1)
    theta = np.arccos(np.clip(pts[:, 2] / r, -1, 1))
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    cols = []
    for l in range(lmax + 1):
        idx = np.nonzero(deg == l)[0]
        A = np.prod(pts[:, None, :] ** ex[None, idx, :], axis=2)
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            cs = (-1.0) ** abs(m)
            if m > 0:
                y = math.sqrt(2.0) * cs * Y.real
            elif m < 0:
                y = math.sqrt(2.0) * cs * Y.imag
            else:
                y = Y.real
            target = (r ** l) * y
            sol, *_ = np.linalg.lstsq(A, target, rcond=None)
            resid = np.max(np.abs(A @ sol - target))
            if resid > 1e-10:
                raise RuntimeError(f"solid harmonic fit failed l={l} m={m} resid={resid}")
            col = np.zeros(len(ex))
            col[idx] = sol
            cols.append(col)
    return np.stack(cols, axis=1)


def real_solid_harmonic_values(x: np.ndarray, lmax: int = 7) -> np.ndarray:
    """r^l Y_k(x/r) for all k (scipy evaluation), shape (n, (lmax+1)^2)."""
    from scipy.special import sph_harm_y
    r = np.linalg.norm(x, axis=1)
    theta = np.arccos(np.clip(x[:, 2] / np.where(r > 0, r, 1.0), -1, 1))
    phi = np.arctan2(x[:, 1], x[:, 0])
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            cs = (-1.0) ** abs(m)
            if m > 0:
                y = math.sqrt(2.0) * cs * Y.real
            elif m < 0:
                y = math.sqrt(2.0) * cs * Y.imag
            else:
                y = Y.real
            out.append((r ** l) * y)
    return np.stack(out, axis=1)


def c5_fc_selection() -> np.ndarray:
    """(20, 16) 0/1 matrix mapping the 16 expansion weights of c and f (the first
    16 graded-lex monomials) onto a dense cubic polynomial in 3 variables."""
    S = np.zeros((20, 16))
    S[np.arange(16), np.arange(16)] = 1.0
    return S


@dataclass
class AdjointWorkload:
    name: str
    problem_template: LinearProblem   # poly coefficient arrays filled from theta
    nodes: np.ndarray
    paths: np.ndarray
    dt: float
    seed: int
    theta_g: np.ndarray   # (64,)
    theta_f: np.ndarray   # (16,)
    theta_c: np.ndarray   # (16,)
    theta_star: Dict[str, np.ndarray]
    sh_matrix: np.ndarray  # (120, 64)
    fc_matrix: np.ndarray  # (20, 16)
    data_seed: int = 1000


def c5_theta(seed: int):
    rng = np.random.default_rng(seed)
    tg = rng.standard_normal(64)
    tf = rng.standard_normal(16)
    tc = 0.1 * rng.standard_normal(16)
    tc[0] += 1.0
    return tg, tf, tc


def c5_problem(theta_g, theta_f, theta_c, sh=None, sel=None) -> LinearProblem:
    sh = real_solid_harmonics_poly(7) if sh is None else sh
    sel = c5_fc_selection() if sel is None else sel
    g = make_fun([], poly_degree=7, poly=sh @ np.asarray(theta_g))
    f = make_fun([], poly_degree=3, poly=sel @ np.asarray(theta_f))
    c = make_fun([], poly_degree=3, poly=sel @ np.asarray(theta_c))
    return LinearProblem(ball(3, 1.0), 1.0, [zero_fun(), zero_fun(), zero_fun()], c, f, g)


def c5_nodes(n: int = 4096, workload_seed: int = 53, radius: float = 0.95) -> np.ndarray:
    rng = np.random.default_rng(workload_seed)
    axis = rng.integers(3, size=n)
    rr = radius * np.sqrt(rng.uniform(size=n))
    th = rng.uniform(0, 2 * math.pi, size=n)
    pts = np.zeros((n, 3))
    for i in range(n):
        others = [k for k in range(3) if k != axis[i]]
        pts[i, others[0]] = rr[i] * math.cos(th[i])
        pts[i, others[1]] = rr[i] * math.sin(th[i])
    return pts


def c5(scale: float = 1.0, dt: float = 1e-3, seed: int = 0, n_nodes: int = 4096) -> AdjointWorkload:
    sh = real_solid_harmonics_poly(7)
    sel = c5_fc_selection()
    tg, tf, tc = c5_theta(52)
    sg, sf, sc = c5_theta(51)
    nodes = c5_nodes(4096)[:n_nodes]
    paths = np.full(len(nodes), _budget(100_000, scale), np.int64)
    prob = c5_problem(tg, tf, tc, sh, sel)
    return AdjointWorkload("C5 adjoint unit ball", prob, nodes, paths, dt, seed, tg, tf, tc,
                           {"g": sg, "f": sf, "c": sc}, sh, sel)
