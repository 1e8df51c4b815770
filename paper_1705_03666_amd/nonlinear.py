"""Polynomial-approximation driver for the marked branching estimator.

The branching representation covers semilinear PDEs whose nonlinearity is a
polynomial in u (eq. 3.1 and its marked form, Sec. 3.2).  Sec. 3.3 widens
that class by approximation: a nonlinearity such as v -> max(v, 0) is
replaced by a polynomial fitted on [-1, 1], after dividing u by ||psi||_inf
so that the solution stays in that interval (the CVA example, where a
degree-4 fit of max(v, 0) gives 0.0586 + 0.5 v + 0.8199 v^2 - 0.4095 v^4).
The signed coefficients need marks: offspring counts are drawn from a law q
and every branching multiplies the weight by alpha_I / q_I; the paper notes
that q does not change the expectation but does change the variance.

This module builds those inputs on the host (it runs no part of the Monte
Carlo path):

* `fit_polynomial` - least-squares polynomial on a uniform grid;
* `branching_form` - the coefficients alpha of beta (sum_i alpha_i u^i - u)
  for a polynomial nonlinearity and a branching rate beta;
* `variance_marks` - q_i proportional to |alpha_i|, which makes every mark
  +-sum|alpha| (no weight larger than needed), and `second_moment` to
  compare choices of q on constant data;
* `rescaled_problem` - the whole construction for
  u_t = 0.5 sigma^2 Lap u + f(u), u(., 0) = psi, |psi| <= psi_sup.
"""
from __future__ import annotations

from typing import Callable, Optional, Sequence

import numpy as np

from workloads.problem import BranchingProblem, Fun

MAX_DEGREE = 4          # offspring counts 0..4 (the library's alpha / q have five entries)


def fit_polynomial(f: Callable[[np.ndarray], np.ndarray], degree: int = 4, interval=(-1.0, 1.0),
                   n: int = 2001) -> np.ndarray:
    """Coefficients c_0..c_degree (increasing powers) of the least-squares
    polynomial through f at n equally spaced points of `interval`.  With the
    defaults and f = max(v, 0) this reproduces the coefficients printed in
    Sec. 3.3 to their four digits."""
    if not 0 <= degree <= MAX_DEGREE:
        raise ValueError(f"degree must be 0..{MAX_DEGREE}")
    x = np.linspace(float(interval[0]), float(interval[1]), int(n))
    V = np.vander(x, degree + 1, increasing=True)
    c, *_ = np.linalg.lstsq(V, np.asarray(f(x), dtype=np.float64), rcond=None)
    # coefficients at round-off level (a symmetry of f) are zero: a zero alpha
    # needs no offspring class
    c[np.abs(c) <= 1e-12 * max(1.0, float(np.abs(c).max()))] = 0.0
    return c


def branching_form(a: Sequence[float], beta: float) -> np.ndarray:
    """alpha (length 5) with sum_i a_i u^i = beta (sum_i alpha_i u^i - u):
    alpha_i = a_i / beta, plus 1 for i = 1."""
    a = np.asarray(a, dtype=np.float64)
    if a.shape[0] > MAX_DEGREE + 1:
        raise ValueError("nonlinearity of degree above 4")
    if not beta > 0.0:
        raise ValueError("beta must be positive")
    alpha = np.zeros(MAX_DEGREE + 1)
    alpha[:a.shape[0]] = a / beta
    alpha[1] += 1.0
    return alpha


def variance_marks(alpha: Sequence[float]) -> np.ndarray:
    """q_i = |alpha_i| / sum_j |alpha_j|: every mark alpha_I / q_I is then
    +-sum_j |alpha_j|, the smallest bound on |mark| any q can give."""
    a = np.abs(np.asarray(alpha, dtype=np.float64))
    s = a.sum()
    if not s > 0.0:
        raise ValueError("alpha is zero")
    return a / s


def second_moment(alpha: Sequence[float], q: Sequence[float], beta: float, T: float, psi0: float,
                  steps: int = 20000) -> float:
    """E[xi^2] of the marked estimator for constant initial data psi0 at time T:
    w' = beta (sum_i alpha_i^2 / q_i w^i - w), w(0) = psi0^2 (the square of the
    product over particles is again a product, with marks alpha_I^2 / q_I^2
    drawn with probability q_I).  Classical RK4; inf if it blows up."""
    al = np.asarray(alpha, dtype=np.float64)
    qq = np.asarray(q, dtype=np.float64)
    k2 = np.where(qq > 0, al ** 2 / np.where(qq > 0, qq, 1.0), 0.0)

    def rhs(w):
        return beta * (sum(k2[i] * w ** i for i in range(k2.shape[0])) - w)

    w = psi0 * psi0
    h = T / steps
    with np.errstate(over="ignore", invalid="ignore"):
        for _ in range(steps):
            k1 = rhs(w)
            k2_ = rhs(w + 0.5 * h * k1)
            k3 = rhs(w + 0.5 * h * k2_)
            k4 = rhs(w + h * k3)
            w = w + h / 6.0 * (k1 + 2 * k2_ + 2 * k3 + k4)
            if not np.isfinite(w) or w > 1e300:
                return float("inf")
    return float(w)


def rescaled_problem(ndim: int, sigma: float, f: Callable[[np.ndarray], np.ndarray], psi: Fun, psi_sup: float,
                     T: float, beta: float, degree: int = 4, q: Optional[Sequence[float]] = None,
                     max_segments: int = 127):
    """Marked branching problem for u_t = 0.5 sigma^2 Lap u + f(u) with
    u(., 0) = psi, |psi| <= psi_sup, through the rescaling of Sec. 3.3:
    v = u / psi_sup solves v_t = 0.5 sigma^2 Lap v + f(psi_sup v) / psi_sup
    with |v(., 0)| <= 1, and that nonlinearity is fitted on [-1, 1] by a
    polynomial of the given degree.  Returns (problem, scale): the estimate of
    u is scale times the estimate of the returned problem.  q defaults to
    variance_marks(alpha)."""
    s = float(psi_sup)
    if not s > 0.0:
        raise ValueError("psi_sup must be positive")
    a = fit_polynomial(lambda v: np.asarray(f(s * v)) / s, degree)
    alpha = branching_form(a, beta)
    qq = variance_marks(alpha) if q is None else np.asarray(q, dtype=np.float64)
    psi_v = psi.with_coef(coef=np.asarray(psi.coef) / s, poly=np.asarray(psi.poly) / s)
    prob = BranchingProblem(ndim, float(sigma), float(beta), float(T), tuple(float(v) for v in alpha),
                            tuple(float(v) for v in qq), psi_v, 1.0, max_segments)
    return prob, s
