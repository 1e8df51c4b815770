"""Plain-data description of the problems the path solves.

This module only *describes* inputs: domains, coefficient functions as term
tables, interface nodes and path budgets.  It evaluates nothing of the method
(no walk, no estimator, no random numbers for paths); both the oracle and the
HIP library read these arrays and evaluate them with their own code.

Function encoding (shared input format, one per coefficient b_k, c, f, g, psi):

    F(x) = sum_t coef[t] * prod_j  fn[t,j]( a[t,j] * x[dim[t,j]] + b[t,j] ) ** power[t,j]
         + sum_m poly[m] * x^alpha_m

`fn` is one of POW (the identity, so the factor is (a*x+b)**power), EXP, SIN,
COS, TANH.  A factor with fn=POW and power=0 is the constant 1 (padding).
The polynomial part is dense in graded-lexicographic monomial order of total
degree <= poly_degree in `ndim` variables: degree 0 first, then within one
degree the exponent tuples in descending lexicographic order
(for 3 variables: 1; x, y, z; x^2, xy, xz, y^2, yz, z^2; x^3, ...).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

FN_POW, FN_EXP, FN_SIN, FN_COS, FN_TANH = 0, 1, 2, 3, 4
FN_NAMES = {"pow": FN_POW, "exp": FN_EXP, "sin": FN_SIN, "cos": FN_COS, "tanh": FN_TANH}

DOM_BOX, DOM_BALL, DOM_FREE = 0, 1, 2

MAX_FACTORS = 4


def monomial_exponents(ndim: int, degree: int) -> np.ndarray:
    """Exponent tuples of all monomials of total degree <= `degree` in
    graded-lexicographic order (see module docstring).  Shape (M, 3), unused
    dimensions get exponent 0."""
    out: List[Tuple[int, int, int]] = []
    for k in range(degree + 1):
        tuples = []
        if ndim == 1:
            tuples = [(k,)]
        elif ndim == 2:
            tuples = [(a, k - a) for a in range(k, -1, -1)]
        else:
            for a in range(k, -1, -1):
                for b in range(k - a, -1, -1):
                    tuples.append((a, b, k - a - b))
        for t in tuples:
            out.append(tuple(list(t) + [0] * (3 - ndim)))
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def n_monomials(ndim: int, degree: int) -> int:
    if degree < 0:
        return 0
    return len(monomial_exponents(ndim, degree))


@dataclass
class Fun:
    """One coefficient function in the term-table + dense-polynomial form."""
    fn: np.ndarray          # (T, F) int32
    dim: np.ndarray         # (T, F) int32
    power: np.ndarray       # (T, F) int32
    a: np.ndarray           # (T, F) float64
    b: np.ndarray           # (T, F) float64
    coef: np.ndarray        # (T,)   float64
    poly_degree: int = -1
    poly: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n_terms(self) -> int:
        return int(self.coef.shape[0])

    @property
    def n_factors(self) -> int:
        return int(self.fn.shape[1]) if self.fn.ndim == 2 else 0

    def n_mono(self, ndim: int) -> int:
        return n_monomials(ndim, self.poly_degree)

    def with_coef(self, coef=None, poly=None) -> "Fun":
        return Fun(self.fn, self.dim, self.power, self.a, self.b,
                   np.asarray(self.coef if coef is None else coef, dtype=np.float64),
                   self.poly_degree,
                   np.asarray(self.poly if poly is None else poly, dtype=np.float64))


def factor(fn: str, dim: int, a: float = 1.0, b: float = 0.0, power: int = 1):
    return (FN_NAMES[fn], int(dim), int(power), float(a), float(b))


def make_fun(terms: Sequence[Tuple[float, Sequence[tuple]]] = (),
             poly_degree: int = -1, poly: Optional[Sequence[float]] = None,
             n_factors: Optional[int] = None) -> Fun:
    """terms: list of (coef, [factor(...), ...]).  Empty factor list = constant."""
    nf = n_factors if n_factors is not None else max([1] + [len(fs) for _, fs in terms])
    if nf > MAX_FACTORS:
        raise ValueError("too many factors per term")
    T = len(terms)
    fnv = np.zeros((T, nf), np.int32)
    dimv = np.zeros((T, nf), np.int32)
    powv = np.zeros((T, nf), np.int32)
    av = np.ones((T, nf), np.float64)
    bv = np.zeros((T, nf), np.float64)
    coef = np.zeros(T, np.float64)
    for t, (c, fs) in enumerate(terms):
        coef[t] = c
        for j, (fn, d, p, a, b) in enumerate(fs):
            fnv[t, j], dimv[t, j], powv[t, j], av[t, j], bv[t, j] = fn, d, p, a, b
    pv = np.zeros(0) if poly is None else np.asarray(poly, np.float64)
    return Fun(fnv, dimv, powv, av, bv, coef, int(poly_degree), pv)


def zero_fun() -> Fun:
    return make_fun([])


def const_fun(v: float) -> Fun:
    return make_fun([(v, [])])


@dataclass
class Domain:
    kind: int               # DOM_BOX / DOM_BALL / DOM_FREE
    ndim: int
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    radius: float = 1.0


def box(lo, hi) -> Domain:
    d = len(lo)
    pad = lambda v: tuple(list(map(float, v)) + [0.0] * (3 - d))
    return Domain(DOM_BOX, d, lo=pad(lo), hi=pad(hi))


def ball(ndim: int, radius: float = 1.0, center=None) -> Domain:
    c = (0.0, 0.0, 0.0) if center is None else tuple(list(map(float, center)) + [0.0] * (3 - ndim))
    return Domain(DOM_BALL, ndim, center=c, radius=float(radius))


def free(ndim: int) -> Domain:
    return Domain(DOM_FREE, ndim)


@dataclass
class LinearProblem:
    """0.5*sigma^2*Lap(u) + b.grad(u) - c*u = -f in D,  u = g on the boundary."""
    domain: Domain
    sigma: float
    b: List[Fun]            # ndim entries
    c: Fun
    f: Fun
    g: Fun

    @property
    def ndim(self) -> int:
        return self.domain.ndim


@dataclass
class BranchingProblem:
    """u_t = 0.5*sigma^2*Lap(u) + beta*(sum_i alpha_i u^i - u),  u(x,0) = psi(x),
    evaluated at horizon T.  q is the offspring law used for sampling."""
    ndim: int
    sigma: float
    beta: float
    T: float
    alpha: Tuple[float, ...]     # length 5 (i = 0..4)
    q: Tuple[float, ...]         # length 5
    psi: Fun
    psi_sup: float
    max_segments: int = 127


@dataclass
class BranchingBoundary:
    """Dirichlet boundary and output times for the branching estimator
    (eq. 3.2, Algorithm 3.1): particles stop on the boundary of `domain`
    (BOX or BALL; FREE means no boundary) and contribute g(X_tau, t - tau) to
    every output time t >= tau.  `g` is evaluated at (x_0, .., x_{ndim-1}, s):
    a factor with coordinate index ndim reads the time argument s (the
    polynomial part is in x only).  `g_sup` bounds |g| (admissibility), `dt`
    is the step of the boundary test and `times` are the output times
    (increasing; the last one is the horizon)."""
    domain: Domain
    g: Fun
    g_sup: float
    dt: float
    times: Tuple[float, ...]
