"""Python front of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the library itself.  It shares
no code with the HIP path; the only common import is the `workloads` package
of plain input data.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

from workloads.problem import (BranchingBoundary, BranchingProblem, DOM_FREE, Fun, LinearProblem,
                               monomial_exponents)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
PAIR52, QUAD24 = 0, 1


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE",
               "-Wall", "-Wextra", src, "-o", LIB_PATH + ".tmp", "-lm", "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Factor(C.Structure):
    _fields_ = [("fn", C.c_int32), ("dim", C.c_int32), ("power", C.c_int32), ("pad", C.c_int32),
                ("a", C.c_double), ("b", C.c_double)]


class OFun(C.Structure):
    _fields_ = [("n_terms", C.c_int32), ("n_factors", C.c_int32), ("factors", C.POINTER(Factor)),
                ("coef", C.POINTER(C.c_double)), ("n_mono", C.c_int32), ("pad", C.c_int32),
                ("mono_exp", C.POINTER(C.c_int32)), ("mono_coef", C.POINTER(C.c_double))]


class ODomain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("center", C.c_double * 3), ("radius", C.c_double)]


class OLinear(C.Structure):
    _fields_ = [("dom", ODomain), ("sigma", C.c_double), ("b", OFun * 3), ("c", OFun), ("f", OFun),
                ("g", OFun), ("boundary_shift", C.c_double)]


# Gobet-Menozzi boundary-shift constant c0 = -zeta(1/2) / sqrt(2 pi) (the
# mean overshoot of a Gaussian random walk over a level, in units of its
# step standard deviation); zeta(1/2) = -1.4603545088095868...
GOBET_MENOZZI_C0 = 1.4603545088095868 / math.sqrt(2.0 * math.pi)


class OBranching(C.Structure):
    _fields_ = [("dim", C.c_int32), ("max_segments", C.c_int32), ("sigma", C.c_double),
                ("beta", C.c_double), ("T", C.c_double), ("alpha", C.c_double * 5),
                ("q", C.c_double * 5), ("psi", OFun)]


class OBranchBoundary(C.Structure):
    _fields_ = [("dom", ODomain), ("g", OFun), ("dt", C.c_double), ("n_times", C.c_int32), ("pad", C.c_int32),
                ("times", C.POINTER(C.c_double)), ("boundary_shift", C.c_double)]


class OStat(C.Structure):
    _fields_ = [("mean", C.c_double), ("m2", C.c_double), ("n", C.c_int64), ("steps", C.c_int64),
                ("censored", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_walk_normal.argtypes = [C.c_uint64, C.c_int, C.c_uint32, C.c_uint32, C.c_uint64]
        L.orc_walk_normal.restype = C.c_double
        L.orc_u_quad24.argtypes = [C.c_uint32]
        L.orc_u_quad24.restype = C.c_double
        L.orc_u_pair52.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u_pair52.restype = C.c_double
        L.orc_fun_eval.argtypes = [C.POINTER(OFun), dp]
        L.orc_fun_eval.restype = C.c_double
        L.orc_inside.argtypes = [C.POINTER(ODomain), dp]
        L.orc_project.argtypes = [C.POINTER(ODomain), dp, dp]
        L.orc_walk.argtypes = [C.POINTER(OLinear), dp, C.c_int64, ip, C.c_double, C.c_uint64, C.c_int,
                               C.c_int64, C.c_int, C.POINTER(OStat), dp, ip, ip]
        L.orc_wos.argtypes = [C.POINTER(OLinear), dp, C.c_int64, ip, C.c_double, C.c_uint64, C.c_int,
                              C.c_int64, C.c_int, C.POINTER(OStat), dp, ip, ip]
        L.orc_walk_adjoint.argtypes = [C.POINTER(OLinear), dp, C.c_int64, ip, C.c_double, C.c_uint64, C.c_int,
                                       C.c_int64, C.c_int, dp, dp, dp, dp, dp, dp, dp, C.POINTER(OStat)]
        L.orc_walk_jacobian.argtypes = [C.POINTER(OLinear), dp, C.c_int64, ip, C.c_double, C.c_uint64, C.c_int,
                                        C.c_int64, C.c_int, dp, dp, C.POINTER(OStat), ip]
        L.orc_branching_dfs.argtypes = [C.POINTER(OBranching), dp, C.c_int64, C.c_int64, C.c_uint64, C.c_int,
                                        C.c_int, C.POINTER(OStat), dp, ip, ip]
        L.orc_branching_alg31.argtypes = [C.POINTER(OBranching), dp, C.c_int64, C.c_int64, C.c_uint64, C.c_int,
                                          C.c_int, C.POINTER(OStat), ip]
        L.orc_branching_bvp.argtypes = [C.POINTER(OBranching), C.POINTER(OBranchBoundary), dp, C.c_int64, C.c_int64,
                                        C.c_uint64, C.c_int, C.c_int, C.POINTER(OStat), dp, ip, ip]
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def default_max_steps(dt: float) -> int:
    return int(np.ceil(100.0 / dt))


# --------------------------------------------------------------------------- marshalling
class _Keep:
    """Keeps numpy buffers alive while C structs point into them."""

    def __init__(self):
        self.refs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.refs.append(a)
        return a


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _ofun(F: Fun, ndim: int, keep: _Keep) -> OFun:
    o = OFun()
    T, nf = F.n_terms, max(1, F.n_factors)
    facs = (Factor * max(1, T * nf))()
    for t in range(T):
        for j in range(F.n_factors):
            k = t * nf + j
            facs[k].fn = int(F.fn[t, j]); facs[k].dim = int(F.dim[t, j]); facs[k].power = int(F.power[t, j])
            facs[k].a = float(F.a[t, j]); facs[k].b = float(F.b[t, j])
        for j in range(F.n_factors, nf):
            k = t * nf + j
            facs[k].fn = 0; facs[k].power = 0; facs[k].a = 1.0
    keep.refs.append(facs)
    o.n_terms = T
    o.n_factors = nf
    o.factors = C.cast(facs, C.POINTER(Factor))
    coef = keep.arr(F.coef if T else np.zeros(1), np.float64)
    o.coef = _ptr(coef, C.c_double)
    if F.poly_degree >= 0:
        ex = keep.arr(monomial_exponents(ndim, F.poly_degree), np.int32)
        pc = keep.arr(F.poly, np.float64)
        if len(pc) != len(ex):
            raise ValueError("polynomial coefficient count does not match its degree")
        o.n_mono = len(ex)
        o.mono_exp = _ptr(ex, C.c_int32)
        o.mono_coef = _ptr(pc, C.c_double)
    else:
        o.n_mono = 0
        ex = keep.arr(np.zeros(3), np.int32)
        pc = keep.arr(np.zeros(1), np.float64)
        o.mono_exp = _ptr(ex, C.c_int32)
        o.mono_coef = _ptr(pc, C.c_double)
    return o


def _odomain(D) -> ODomain:
    o = ODomain()
    o.kind, o.dim = int(D.kind), int(D.ndim)
    for k in range(3):
        o.lo[k], o.hi[k], o.center[k] = float(D.lo[k]), float(D.hi[k]), float(D.center[k])
    o.radius = float(D.radius)
    return o


def _olinear(P: LinearProblem, keep: _Keep, boundary_shift: float = 0.0) -> OLinear:
    o = OLinear()
    o.dom = _odomain(P.domain)
    o.sigma = float(P.sigma)
    o.boundary_shift = float(boundary_shift)
    from workloads.problem import zero_fun
    for k in range(3):
        o.b[k] = _ofun(P.b[k] if k < len(P.b) else zero_fun(), P.ndim, keep)
    o.c = _ofun(P.c, P.ndim, keep)
    o.f = _ofun(P.f, P.ndim, keep)
    o.g = _ofun(P.g, P.ndim, keep)
    return o


def _stats(arr) -> dict:
    n = np.array([s.n for s in arr], np.int64)
    mean = np.array([s.mean for s in arr])
    m2 = np.array([s.m2 for s in arr])
    var = np.where(n > 1, m2 / np.maximum(n - 1, 1), 0.0)
    return {"mean": mean, "m2": m2, "n": n, "var": var, "se": np.sqrt(var / np.maximum(n, 1)),
            "steps": np.array([s.steps for s in arr], np.int64),
            "censored": np.array([s.censored for s in arr], np.int64)}


# --------------------------------------------------------------------------- public API
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u_quad24(w: int) -> float:
    return float(lib().orc_u_quad24(w))


def u_pair52(whi: int, wlo: int) -> float:
    return float(lib().orc_u_pair52(whi, wlo))


def walk_normal(seed: int, layout: int, node: int, path: int, j: int) -> float:
    return float(lib().orc_walk_normal(seed, layout, node, path, j))


def fun_eval(F: Fun, ndim: int, x) -> float:
    keep = _Keep()
    o = _ofun(F, ndim, keep)
    xx = keep.arr(list(x) + [0.0] * (3 - len(x)), np.float64)
    return float(lib().orc_fun_eval(C.byref(o), _ptr(xx, C.c_double)))


def walk(P: LinearProblem, nodes, paths, dt: float, seed: int, layout: int = PAIR52,
         max_steps: Optional[int] = None, n_threads: Optional[int] = None, dump: bool = False,
         node_ids=None, boundary_shift: float = 0.0) -> dict:
    """Per-node sample mean / variance of the Feynman-Kac walk (optionally the
    per-path values and step counts, concatenated node after node).  node_ids
    gives the node index used in the random-number counters (default: the
    node's position), so a sample of a larger node set reproduces its paths.
    boundary_shift = GOBET_MENOZZI_C0 selects the boundary-corrected exit test."""
    keep = _Keep()
    o = _olinear(P, keep, boundary_shift)
    nodes = keep.arr(nodes, np.float64)
    paths = keep.arr(paths, np.int64)
    n = len(paths)
    out = (OStat * max(1, n))()
    total = int(paths.sum())
    phi = np.zeros(total if dump else 1)
    st = np.zeros(total if dump else 1, np.int64)
    rc = lib().orc_walk(C.byref(o), _ptr(nodes, C.c_double), n, _ptr(paths, C.c_int64), dt, seed, layout,
                        default_max_steps(dt) if max_steps is None else max_steps,
                        default_threads() if n_threads is None else n_threads, out,
                        _ptr(phi, C.c_double) if dump else None, _ptr(st, C.c_int64) if dump else None,
                        _ptr(keep.arr(node_ids, np.int64), C.c_int64) if node_ids is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the walk arguments")
    res = _stats(out[:n])
    if dump:
        res["phi"], res["path_steps"] = phi, st
    return res


def wos(P: LinearProblem, nodes, paths, eps: float, seed: int, layout: int = PAIR52,
        max_steps: int = 100000, n_threads: Optional[int] = None, dump: bool = False, node_ids=None) -> dict:
    """Walk on Spheres for Laplace's equation (b = c = f = 0): per-node mean /
    variance of g at the projected eps-shell exit point; steps = jumps.
    node_ids as in walk()."""
    keep = _Keep()
    o = _olinear(P, keep)
    nodes = keep.arr(nodes, np.float64)
    paths = keep.arr(paths, np.int64)
    n = len(paths)
    out = (OStat * max(1, n))()
    total = int(paths.sum())
    phi = np.zeros(total if dump else 1)
    st = np.zeros(total if dump else 1, np.int64)
    rc = lib().orc_wos(C.byref(o), _ptr(nodes, C.c_double), n, _ptr(paths, C.c_int64), eps, seed, layout,
                       max_steps, default_threads() if n_threads is None else n_threads, out,
                       _ptr(phi, C.c_double) if dump else None, _ptr(st, C.c_int64) if dump else None,
                       _ptr(keep.arr(node_ids, np.int64), C.c_int64) if node_ids is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the walk-on-spheres arguments")
    res = _stats(out[:n])
    if dump:
        res["phi"], res["path_steps"] = phi, st
    return res


def walk_adjoint(P: LinearProblem, nodes, paths, dt: float, seed: int, w, layout: int = PAIR52,
                 max_steps: Optional[int] = None, n_threads: Optional[int] = None,
                 boundary_shift: float = 0.0) -> dict:
    """Gradient of sum_i w_i * mean_i with respect to the coefficients of g, f, c."""
    keep = _Keep()
    o = _olinear(P, keep, boundary_shift)
    nodes = keep.arr(nodes, np.float64)
    paths = keep.arr(paths, np.int64)
    w = keep.arr(w, np.float64)
    n = len(paths)
    nd = P.ndim
    grads = {}
    for name, F in (("g", P.g), ("f", P.f), ("c", P.c)):
        grads[name + "_coef"] = np.zeros(max(1, F.n_terms))
        grads[name + "_poly"] = np.zeros(max(1, F.n_mono(nd)))
    out = (OStat * max(1, n))()
    rc = lib().orc_walk_adjoint(C.byref(o), _ptr(nodes, C.c_double), n, _ptr(paths, C.c_int64), dt, seed,
                                layout, default_max_steps(dt) if max_steps is None else max_steps,
                                default_threads() if n_threads is None else n_threads, _ptr(w, C.c_double),
                                *[_ptr(grads[k], C.c_double) for k in
                                  ("g_coef", "g_poly", "f_coef", "f_poly", "c_coef", "c_poly")], out)
    if rc != 0:
        raise ValueError("oracle rejected the adjoint arguments")
    res = {k: v[:max(0, (P.g if k[0] == "g" else P.f if k[0] == "f" else P.c).n_terms if k.endswith("coef")
                     else (P.g if k[0] == "g" else P.f if k[0] == "f" else P.c).n_mono(nd))]
           for k, v in grads.items()}
    res["stats"] = _stats(out[:n])
    return res


def walk_jacobian(P: LinearProblem, nodes, paths, dt: float, seed: int, layout: int = PAIR52,
                  max_steps: Optional[int] = None, n_threads: Optional[int] = None, node_ids=None,
                  boundary_shift: float = 0.0) -> dict:
    """Per-node Jacobian d mean_i / d theta (columns: g coef, g poly, f coef,
    f poly, c coef, c poly) and the standard error of every entry, from the
    spread of the per-path derivatives over the node's paths.  node_ids as in
    walk()."""
    keep = _Keep()
    o = _olinear(P, keep, boundary_shift)
    nodes = keep.arr(nodes, np.float64)
    paths = keep.arr(paths, np.int64)
    n = len(paths)
    npar = sum(F.n_terms + F.n_mono(P.ndim) for F in (P.g, P.f, P.c))
    mean = np.zeros((max(1, n), max(1, npar)))
    m2 = np.zeros((max(1, n), max(1, npar)))
    out = (OStat * max(1, n))()
    rc = lib().orc_walk_jacobian(C.byref(o), _ptr(nodes, C.c_double), n, _ptr(paths, C.c_int64), dt, seed, layout,
                                 default_max_steps(dt) if max_steps is None else max_steps,
                                 default_threads() if n_threads is None else n_threads,
                                 _ptr(mean, C.c_double), _ptr(m2, C.c_double), out,
                                 _ptr(keep.arr(node_ids, np.int64), C.c_int64) if node_ids is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the Jacobian arguments")
    N = paths[:, None].astype(np.float64)
    var = np.where(N > 1, m2[:n, :npar] / np.maximum(N - 1, 1), 0.0)
    return {"jac": mean[:n, :npar], "jac_se": np.sqrt(var / np.maximum(N, 1)), "stats": _stats(out[:n])}


def _obranching(B: BranchingProblem, keep: _Keep) -> OBranching:
    o = OBranching()
    o.dim, o.max_segments = int(B.ndim), int(B.max_segments)
    o.sigma, o.beta, o.T = float(B.sigma), float(B.beta), float(B.T)
    for k in range(5):
        o.alpha[k] = float(B.alpha[k]) if k < len(B.alpha) else 0.0
        o.q[k] = float(B.q[k]) if k < len(B.q) else 0.0
    o.psi = _ofun(B.psi, B.ndim, keep)
    return o


def branching(B: BranchingProblem, points, trees: int, seed: int, layout: int = PAIR52,
              n_threads: Optional[int] = None, dump: bool = False) -> dict:
    """Marked branching estimator, per-particle (depth-first) simulation."""
    keep = _Keep()
    o = _obranching(B, keep)
    pts = keep.arr(points, np.float64)
    n = len(pts)
    out = (OStat * max(1, n))()
    val = np.zeros(n * trees if dump else 1)
    segs = np.zeros(n * trees if dump else 1, np.int64)
    red = C.c_int64(0)
    rc = lib().orc_branching_dfs(C.byref(o), _ptr(pts, C.c_double), n, trees, seed, layout,
                                 default_threads() if n_threads is None else n_threads, out,
                                 _ptr(val, C.c_double) if dump else None, _ptr(segs, C.c_int64) if dump else None,
                                 C.byref(red))
    if rc != 0:
        raise ValueError("oracle rejected the branching arguments")
    res = _stats(out[:n])
    res["redrawn"] = int(red.value)
    if dump:
        res["value"], res["segments"] = val.reshape(n, trees), segs.reshape(n, trees)
    return res


def branching_alg31(B: BranchingProblem, points, trees: int, seed: int, max_particles: int = 64,
                    n_threads: Optional[int] = None) -> dict:
    """Same estimator in the global-clock form of Algorithm 3.1."""
    keep = _Keep()
    o = _obranching(B, keep)
    pts = keep.arr(points, np.float64)
    n = len(pts)
    out = (OStat * max(1, n))()
    red = C.c_int64(0)
    rc = lib().orc_branching_alg31(C.byref(o), _ptr(pts, C.c_double), n, trees, seed, max_particles,
                                   default_threads() if n_threads is None else n_threads, out, C.byref(red))
    if rc != 0:
        raise ValueError("oracle rejected the branching arguments")
    res = _stats(out[:n])
    res["redrawn"] = int(red.value)
    return res


def branching_bvp(B: BranchingProblem, Bd: BranchingBoundary, points, trees: int, seed: int, layout: int = PAIR52,
                  n_threads: Optional[int] = None, dump: bool = False, boundary_shift: float = 0.0) -> dict:
    """Branching estimator with particles stopped on a Dirichlet boundary
    (eq. 3.2), evaluated at every output time of one tree (Algorithm 3.1).
    Statistics have shape (n_times, n_points); dumps (n_points, trees,
    n_times) values and (n_points, trees) segment counts."""
    keep = _Keep()
    o = _obranching(B, keep)
    ob = OBranchBoundary()
    ob.dom = _odomain(Bd.domain)
    ob.g = _ofun(Bd.g, B.ndim, keep)
    ob.dt = float(Bd.dt)
    times = keep.arr(np.asarray(Bd.times, np.float64), np.float64)
    ob.n_times = len(times)
    ob.times = _ptr(times, C.c_double)
    ob.boundary_shift = float(boundary_shift)
    pts = keep.arr(points, np.float64)
    n = len(pts)
    nt = len(times)
    out = (OStat * max(1, n * nt))()
    val = np.zeros(n * trees * nt if dump else 1)
    segs = np.zeros(n * trees if dump else 1, np.int64)
    red = C.c_int64(0)
    rc = lib().orc_branching_bvp(C.byref(o), C.byref(ob), _ptr(pts, C.c_double), n, trees, seed, layout,
                                 default_threads() if n_threads is None else n_threads, out,
                                 _ptr(val, C.c_double) if dump else None, _ptr(segs, C.c_int64) if dump else None,
                                 C.byref(red))
    if rc != 0:
        raise ValueError("oracle rejected the branching-with-boundary arguments")
    per_time = [_stats(out[k * n:(k + 1) * n]) for k in range(nt)]
    res = {key: np.stack([r[key] for r in per_time]) for key in per_time[0]} if n else {}
    res["redrawn"] = int(red.value)
    if dump:
        res["value"], res["segments"] = val.reshape(n, trees, nt), segs.reshape(n, trees)
    return res
