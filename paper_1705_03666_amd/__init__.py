"""MI355X (gfx950) library for the Monte Carlo hot path of Probabilistic Domain
Decomposition (Bernal, dos Reis, Smith, arXiv 1705.03666).

Thin Python binding of libpdd.so (C ABI in include/pdd.h): it marshals
arguments, hands over torch device pointers and the current stream, and turns
status codes into exceptions.  Every step of the computation runs in the HIP
kernels; there is no CPU fallback.  If the library or a GPU is missing the
calls raise.

Problem objects are duck-typed: a linear problem has `domain` (kind, ndim,
lo, hi, center, radius), `sigma`, `b` (list of functions), `c`, `f`, `g`; a
function has the term-table arrays `fn, dim, power, a, b, coef` and
`poly_degree, poly` (graded-lex dense polynomial), as produced by the
`workloads` package.  A branching problem has `ndim, sigma, beta, T, alpha,
q, psi, psi_sup, max_segments`.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from . import nonlinear  # noqa: F401  (host-side driver of Sec. 3.3)

__all__ = ["mc_interface", "mc_interface_noalloc", "mc_interface_batch", "wos_interface_batch", "mc_interface_many", "mc_adjoint", "mc_value_jacobian", "branching_eval", "branching_bvp", "wos_interface",
           "item_count", "set_schedule", "get_schedule", "save_schedules", "load_schedules",
           "PDDInterface", "PddError",
           "release_workspace", "query_warnings", "library", "version", "param_layout", "jacobian_blocks",
           "jacobian_apply", "misfit_gradient", "merge_estimates", "cached_plan_count", "nonlinear"]


class PddError(RuntimeError):
    pass


_lib = None


def library():
    """The loaded libpdd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(A.LIB_PATH):
            raise RuntimeError(f"{A.LIB_PATH} is missing: build it with `python -m paper_1705_03666_amd.build`")
        _lib = A.load(A.LIB_PATH)
    return _lib


def version() -> int:
    return int(library().pdd_version())


def _need_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1705_03666_amd needs a ROCm GPU (torch.cuda.is_available() is False)")


def _check(status: int, what: str):
    L = library()
    if status < 0:
        msg = L.pdd_last_error().decode(errors="replace")
        raise PddError(f"{what}: {L.pdd_status_string(status).decode()} ({msg})")
    if status > 0:
        warnings.warn(f"{what}: {L.pdd_status_string(status).decode()}")


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


_PREC = {"fp64_plain": A.PDD_FP64_PLAIN, "fp64": A.PDD_FP64, "fp32": A.PDD_FP32_STEP}
_LAYOUT = {"pair52": A.PDD_RNG_PAIR52, "quad24": A.PDD_RNG_QUAD24}
_SCHED = {"auto": A.PDD_SCHED_AUTO, "persistent": A.PDD_SCHED_PERSISTENT, "graph": A.PDD_SCHED_PERSISTENT_GRAPH}
# problem-specialised kernels for generic terms in b, c, f (walks) and psi, g
# (branching) (pdd_options.specialize)
_SPEC = {"auto": 0, "on": 1, "off": -1}


def _options(precision: str, layout: Optional[str], max_steps: int, schedule: str, chunk_paths: int,
             blocks_per_cu: int, refill_groups: int, dump_phi=None, dump_steps=None,
             boundary_correction: bool = False, specialize: str = "auto") -> A.pdd_options:
    if precision not in _PREC:
        raise ValueError(f"precision must be one of {list(_PREC)}")
    if specialize not in _SPEC:
        raise ValueError(f"specialize must be one of {list(_SPEC)}")
    if layout is None:
        layout = "quad24" if precision == "fp32" else "pair52"
    o = A.pdd_options()
    o.precision = _PREC[precision]
    o.rng_layout = _LAYOUT[layout]
    o.max_steps = int(max_steps)
    o.dump_phi = dump_phi.data_ptr() if dump_phi is not None else None
    o.dump_steps = dump_steps.data_ptr() if dump_steps is not None else None
    o.schedule = _SCHED[schedule]
    o.chunk_paths = int(chunk_paths)
    o.blocks_per_cu = int(blocks_per_cu)
    o.refill_groups = int(refill_groups)
    o.boundary_correction = 1 if boundary_correction else 0
    o.specialize = _SPEC[specialize]
    return o


def _dev_f64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        t = x.detach()
        if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
            t = t.to(device="cuda", dtype=torch.float64).contiguous()
        return t
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


# Device copies of the constant arrays of problem data (coefficients) passed
# as host arrays, keyed by their content: a repeated call with the same data
# reuses the copy instead of a blocking host-to-device copy, so calls queue on
# the stream without waiting for earlier GPU work.  The library only reads
# these buffers.
_CONST_CACHE: "Dict[bytes, torch.Tensor]" = {}
_CONST_CACHE_MAX = 512


def _dev_const_f64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return _dev_f64(x)
    a = np.ascontiguousarray(x, dtype=np.float64)
    key = a.tobytes() + bytes(str(a.shape), "ascii")
    t = _CONST_CACHE.get(key)
    if t is None:
        if len(_CONST_CACHE) >= _CONST_CACHE_MAX:
            _CONST_CACHE.pop(next(iter(_CONST_CACHE)))
        t = torch.as_tensor(a, device="cuda")
        _CONST_CACHE[key] = t
    return t


class _Keep(list):
    pass


def _fun(F, keep: _Keep, coef=None, poly=None) -> A.pdd_fun:
    f = A.pdd_fun()
    T = int(np.asarray(F.coef).shape[0])
    nf = int(F.fn.shape[1]) if (T > 0 and np.asarray(F.fn).ndim == 2) else 0
    f.n_terms = T
    f.n_factors = nf
    if T > 0 and nf > 0:
        facs = (A.pdd_factor * (T * nf))()
        for t in range(T):
            for j in range(nf):
                k = t * nf + j
                facs[k].fn = int(F.fn[t, j]); facs[k].dim = int(F.dim[t, j]); facs[k].power = int(F.power[t, j])
                facs[k].a = float(F.a[t, j]); facs[k].b = float(F.b[t, j])
        keep.append(facs)
        f.factors = C.cast(facs, C.POINTER(A.pdd_factor))
    if T > 0:
        ct = _dev_const_f64(F.coef if coef is None else coef)
        if ct.numel() != T:
            raise ValueError("coefficient count does not match the term table")
        keep.append(ct)
        f.coef = ct.data_ptr()
    f.poly_degree = int(F.poly_degree)
    if F.poly_degree >= 0:
        pt = _dev_const_f64(F.poly if poly is None else poly)
        keep.append(pt)
        f.poly = pt.data_ptr()
    return f


def _zero_fun() -> A.pdd_fun:
    f = A.pdd_fun()
    f.poly_degree = -1
    return f


def _linear(P, keep: _Keep, coefs: Optional[Dict[str, torch.Tensor]] = None) -> A.pdd_linear_problem:
    coefs = coefs or {}
    p = A.pdd_linear_problem()
    D = P.domain
    p.domain.kind = int(D.kind)
    p.domain.dim = int(D.ndim)
    for k in range(3):
        p.domain.lo[k] = float(D.lo[k]); p.domain.hi[k] = float(D.hi[k]); p.domain.center[k] = float(D.center[k])
    p.domain.radius = float(D.radius)
    p.sigma = float(P.sigma)
    for k in range(3):
        p.b[k] = _fun(P.b[k], keep) if k < len(P.b) else _zero_fun()
    for name in ("c", "f", "g"):
        setattr(p, name, _fun(getattr(P, name), keep, coefs.get(name + "_coef"), coefs.get(name + "_poly")))
    return p


def _stats(raw: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Views of a pdd_node_stat array [n, 5] (FP64 words), plus the variance and
    standard error computed by the library (pdd_node_moments)."""
    raw = raw.contiguous()
    n = raw.shape[0]
    ints = raw[:, 2:].view(torch.int64)
    var = torch.empty(max(n, 1), dtype=torch.float64, device=raw.device)
    se = torch.empty(max(n, 1), dtype=torch.float64, device=raw.device)
    if n:
        _check(library().pdd_node_moments(raw.data_ptr(), n, var.data_ptr(), se.data_ptr(), _stream_handle()),
               "pdd_node_moments")
    return {"mean": raw[:, 0], "m2": raw[:, 1], "n": ints[:, 0], "steps": ints[:, 1], "censored": ints[:, 2],
            "var": var[:n], "se": se[:n], "_raw": raw}


def _nodes_tensor(nodes, ndim: int) -> torch.Tensor:
    t = _dev_f64(nodes)
    if t.dim() != 2 or t.shape[1] != ndim:
        raise ValueError(f"nodes must have shape (n, {ndim})")
    return t


def mc_interface(problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32",
                 layout: Optional[str] = None, max_steps: int = 0, dump: bool = False, schedule: str = "auto",
                 chunk_paths: int = 0, blocks_per_cu: int = 0, refill_groups: int = 0,
                 coefs: Optional[Dict[str, torch.Tensor]] = None,
                 boundary_correction: bool = False, specialize: str = "auto",
                 partials: Optional[torch.Tensor] = None, skip_items=None) -> Dict[str, torch.Tensor]:
    """Monte Carlo value of the linear problem at every node (pdd_mc_interface).
    Returns device tensors mean, m2, n, steps, censored, var, se (and, with
    dump=True, the per-path values `phi` and step counts `path_steps`,
    node-major).  `partials` (float64 device tensor [item_count(...), 6], the
    pdd_item_stat slots) and `skip_items` (bool array [item_count(...)])
    checkpoint and resume a call item by item."""
    _need_gpu()
    keep = _Keep()
    p = _linear(problem, keep, coefs)
    nt = _nodes_tensor(nodes, problem.domain.ndim)
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    if ph.shape[0] != n:
        raise ValueError("paths must have one entry per node")
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    dphi = dst = None
    if dump:
        total = int(ph.sum())
        dphi = torch.empty(max(total, 1), dtype=torch.float64, device="cuda")
        dst = torch.empty(max(total, 1), dtype=torch.int64, device="cuda")
    o = _options(precision, layout, max_steps, schedule, chunk_paths, blocks_per_cu, refill_groups, dphi, dst,
                 boundary_correction, specialize)
    if partials is not None:
        if not (partials.is_cuda and partials.dtype == torch.float64 and partials.is_contiguous()
                and partials.dim() == 2 and partials.shape[1] == 6):
            raise ValueError("partials must be a contiguous float64 CUDA tensor of shape [n_items, 6]")
        o.partials = partials.data_ptr()
    if skip_items is not None:
        sk = np.ascontiguousarray(np.asarray(skip_items, dtype=np.uint8).reshape(-1))
        keep.append(sk)
        o.skip_items = sk.ctypes.data
    st = library().pdd_mc_interface(C.byref(p), nt.data_ptr() if n else None, n,
                                    ph.ctypes.data_as(C.POINTER(C.c_int64)), float(dt), int(seed) & (2 ** 64 - 1),
                                    C.byref(o), raw.data_ptr(), _stream_handle())
    _check(st, "pdd_mc_interface")
    res = _stats(raw[:n])
    if dump:
        total = int(ph.sum())
        res["phi"], res["path_steps"] = dphi[:total], dst[:total]
    res["_keep"] = keep
    return res


def mc_interface_noalloc(problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32",
                         layout: Optional[str] = None, max_steps: int = 0, chunk_paths: int = 0,
                         blocks_per_cu: int = 0, refill_groups: int = 0,
                         coefs: Optional[Dict[str, torch.Tensor]] = None, boundary_correction: bool = False,
                         out: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """mc_interface through pdd_mc_interface_noalloc: the library maps no device
    memory for the call (its scratch is a fixed per-device area).  `out`, if
    given, is the caller's float64 CUDA tensor [n, 5] that receives the
    pdd_node_stat records (so that a caller who cannot allocate passes its own)."""
    _need_gpu()
    keep = _Keep()
    p = _linear(problem, keep, coefs)
    nt = _nodes_tensor(nodes, problem.domain.ndim)
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    if ph.shape[0] != n:
        raise ValueError("paths must have one entry per node")
    if out is None:
        out = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.dim() == 2
              and out.shape[1] == 5 and out.shape[0] >= n):
        raise ValueError("out must be a contiguous float64 CUDA tensor [>= n, 5]")
    o = _options(precision, layout, max_steps, "persistent", chunk_paths, blocks_per_cu, refill_groups,
                 boundary_correction=boundary_correction, specialize="off")
    st = library().pdd_mc_interface_noalloc(C.byref(p), nt.data_ptr() if n else None, n,
                                            ph.ctypes.data_as(C.POINTER(C.c_int64)), float(dt),
                                            int(seed) & (2 ** 64 - 1), C.byref(o), out.data_ptr(),
                                            _stream_handle())
    _check(st, "pdd_mc_interface_noalloc")
    res = _stats(out[:n])
    res["_keep"] = keep
    return res


def _batch(entry: str, problems, node_problem, nodes, paths, step: float, seed: int, precision: str,
           layout: Optional[str], max_steps: int, dump: bool, schedule: str, chunk_paths: int, blocks_per_cu: int,
           refill_groups: int, boundary_correction: bool) -> Dict[str, torch.Tensor]:
    _need_gpu()
    keep = _Keep()
    n_probs = len(problems)
    arr = (A.pdd_linear_problem * max(1, n_probs))()
    for k, P in enumerate(problems):
        arr[k] = _linear(P, keep)
    keep.append(arr)
    nt = _dev_f64(nodes)
    if nt.dim() != 2 or nt.shape[1] != 3:
        raise ValueError("nodes must have shape (n, 3) (rows padded to three coordinates)")
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    npb = np.ascontiguousarray(np.asarray(node_problem, dtype=np.int32).reshape(-1))
    if ph.shape[0] != n or npb.shape[0] != n:
        raise ValueError("paths and node_problem must have one entry per node")
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    dphi, dst = _dumps(dump, ph)
    o = _options(precision, layout, max_steps, schedule, chunk_paths, blocks_per_cu, refill_groups, dphi, dst,
                 boundary_correction)
    st = getattr(library(), entry)(arr, n_probs, npb.ctypes.data_as(C.POINTER(C.c_int32)),
                                   nt.data_ptr() if n else None, n, ph.ctypes.data_as(C.POINTER(C.c_int64)),
                                   float(step), int(seed) & (2 ** 64 - 1), C.byref(o), raw.data_ptr(),
                                   _stream_handle())
    _check(st, entry)
    res = _stats(raw[:n])
    if dump:
        total = int(ph.sum())
        res["phi"], res["path_steps"] = dphi[:total], dst[:total]
    res["_keep"] = (keep, nt)
    return res


def mc_interface_batch(problems, node_problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32",
                       layout: Optional[str] = None, max_steps: int = 0, dump: bool = False, schedule: str = "auto",
                       chunk_paths: int = 0, blocks_per_cu: int = 0, refill_groups: int = 0,
                       boundary_correction: bool = False) -> Dict[str, torch.Tensor]:
    """Interface values of a heterogeneous batch of linear problems in one
    persistent launch (pdd_mc_interface_batch): node i belongs to
    problems[node_problem[i]] and sits at nodes[i, :dim] (nodes is (n, 3)).
    Outputs as mc_interface."""
    return _batch("pdd_mc_interface_batch", problems, node_problem, nodes, paths, dt, seed, precision, layout,
                  max_steps, dump, schedule, chunk_paths, blocks_per_cu, refill_groups, boundary_correction)


def wos_interface_batch(problems, node_problem, nodes, paths, eps: float, seed: int = 0, precision: str = "fp32",
                        layout: Optional[str] = None, max_steps: int = 0, dump: bool = False, schedule: str = "auto",
                        chunk_paths: int = 0, blocks_per_cu: int = 0,
                        refill_groups: int = 0) -> Dict[str, torch.Tensor]:
    """Walk on Spheres over a heterogeneous batch (pdd_wos_interface_batch)."""
    return _batch("pdd_wos_interface_batch", problems, node_problem, nodes, paths, eps, seed, precision, layout,
                  max_steps, dump, schedule, chunk_paths, blocks_per_cu, refill_groups, False)


def wos_interface(problem, nodes, paths, eps: float, seed: int = 0, precision: str = "fp32",
                 layout: Optional[str] = None, max_steps: int = 0, dump: bool = False, schedule: str = "auto",
                 chunk_paths: int = 0, blocks_per_cu: int = 0, refill_groups: int = 0,
                 coefs: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
    """Walk on Spheres for Laplace's equation (pdd_wos_interface): b, c, f
    must be zero; eps is the width of the stopping shell.  Same outputs as
    mc_interface, with steps counting jumps."""
    _need_gpu()
    keep = _Keep()
    p = _linear(problem, keep, coefs)
    nt = _nodes_tensor(nodes, problem.domain.ndim)
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    if ph.shape[0] != n:
        raise ValueError("paths must have one entry per node")
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    dphi = dst = None
    if dump:
        total = int(ph.sum())
        dphi = torch.empty(max(total, 1), dtype=torch.float64, device="cuda")
        dst = torch.empty(max(total, 1), dtype=torch.int64, device="cuda")
    o = _options(precision, layout, max_steps, schedule, chunk_paths, blocks_per_cu, refill_groups, dphi, dst)
    st = library().pdd_wos_interface(C.byref(p), nt.data_ptr() if n else None, n,
                                     ph.ctypes.data_as(C.POINTER(C.c_int64)), float(eps), int(seed) & (2 ** 64 - 1),
                                     C.byref(o), raw.data_ptr(), _stream_handle())
    _check(st, "pdd_wos_interface")
    res = _stats(raw[:n])
    if dump:
        total = int(ph.sum())
        res["phi"], res["path_steps"] = dphi[:total], dst[:total]
    res["_keep"] = keep
    return res


_STREAM_POOL: Dict[int, list] = {}


def mc_interface_many(calls, max_streams: int = 8) -> list:
    """Several independent mc_interface calls (for instance the subdomain
    layouts of one batch, each with its own domain and data), issued on a pool
    of HIP streams so that one launch's tail overlaps the next launch; the
    current stream waits for all of them.  `calls` is a list of
    (args, kwargs) for mc_interface.  Every call computes exactly what it
    computes alone (same paths, same item order), so the results are
    identical to issuing the calls one after the other."""
    _need_gpu()
    dev = torch.cuda.current_device()
    pool = _STREAM_POOL.setdefault(dev, [])
    n = max(1, min(int(max_streams), len(calls)))
    while len(pool) < n:
        pool.append(torch.cuda.Stream(device=dev))
    cur = torch.cuda.current_stream()
    out = []
    for i, (args, kwargs) in enumerate(calls):
        s = pool[i % n]
        s.wait_stream(cur)
        with torch.cuda.stream(s):
            r = mc_interface(*args, **kwargs)
        # results are read on the current stream: tell the caching allocator
        for v in r.values():
            if isinstance(v, torch.Tensor) and v.is_cuda:
                v.record_stream(cur)
        out.append(r)
    for s in pool[:n]:
        cur.wait_stream(s)
    return out


def _dumps(dump: bool, paths: np.ndarray):
    if not dump:
        return None, None
    total = int(paths.sum())
    return (torch.empty(max(total, 1), dtype=torch.float64, device="cuda"),
            torch.empty(max(total, 1), dtype=torch.int64, device="cuda"))


def mc_adjoint(problem, nodes, paths, dt: float, seed: int, w, precision: str = "fp32",
               layout: Optional[str] = None, max_steps: int = 0, schedule: str = "auto", chunk_paths: int = 0,
               blocks_per_cu: int = 0, refill_groups: int = 0, coefs: Optional[Dict[str, torch.Tensor]] = None,
               with_stats: bool = False, boundary_correction: bool = False,
               specialize: str = "auto", dump: bool = False) -> Dict[str, torch.Tensor]:
    """Gradient of sum_i w_i u_i with respect to the coefficient arrays of g, f
    and c (pdd_mc_adjoint).  Returns device tensors g_coef, g_poly, f_coef,
    f_poly, c_coef, c_poly (and the per-node statistics with with_stats; with
    dump=True the per-path values `phi` and step counts `path_steps` of the
    adjoint kernel's own walk, node-major)."""
    _need_gpu()
    keep = _Keep()
    p = _linear(problem, keep, coefs)
    nt = _nodes_tensor(nodes, problem.domain.ndim)
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    if ph.shape[0] != n:
        raise ValueError("paths must have one entry per node")
    wt = _dev_f64(w).reshape(-1)
    if wt.numel() != n:
        raise ValueError("w must have one entry per node")
    ndim = problem.domain.ndim
    grads = {}
    gstruct = (A.pdd_fun_grad * 3)()
    for k, name in enumerate(("g", "f", "c")):
        F = getattr(problem, name)
        T = int(np.asarray(F.coef).shape[0])
        from math import comb
        M = comb(F.poly_degree + ndim, ndim) if F.poly_degree >= 0 else 0
        grads[name + "_coef"] = torch.zeros(max(T, 1), dtype=torch.float64, device="cuda")
        grads[name + "_poly"] = torch.zeros(max(M, 1), dtype=torch.float64, device="cuda")
        gstruct[k].dcoef = grads[name + "_coef"].data_ptr() if T else None
        gstruct[k].dpoly = grads[name + "_poly"].data_ptr() if M else None
        grads[name + "_coef"] = grads[name + "_coef"][:T]
        grads[name + "_poly"] = grads[name + "_poly"][:M]
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda") if with_stats else None
    dphi, dst = _dumps(dump, ph)
    o = _options(precision, layout, max_steps, schedule, chunk_paths, blocks_per_cu, refill_groups, dphi, dst,
                 boundary_correction=boundary_correction, specialize=specialize)
    st = library().pdd_mc_adjoint(C.byref(p), nt.data_ptr() if n else None, n,
                                  ph.ctypes.data_as(C.POINTER(C.c_int64)), float(dt), int(seed) & (2 ** 64 - 1),
                                  C.byref(o), wt.data_ptr() if n else None, gstruct,
                                  raw.data_ptr() if raw is not None else None, _stream_handle())
    _check(st, "pdd_mc_adjoint")
    if with_stats:
        grads["stats"] = _stats(raw[:n])
    if dump:
        total = int(ph.sum())
        grads["phi"], grads["path_steps"] = dphi[:total], dst[:total]
    grads["_keep"] = (keep, wt)
    return grads


def param_layout(problem):
    """(name, count) of the Jacobian column blocks, in column order."""
    from math import comb
    ndim = problem.domain.ndim
    out = []
    for name in ("g", "f", "c"):
        F = getattr(problem, name)
        out.append((name + "_coef", int(np.asarray(F.coef).shape[0])))
        out.append((name + "_poly", comb(F.poly_degree + ndim, ndim) if F.poly_degree >= 0 else 0))
    return out


def mc_value_jacobian(problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32",
                      layout: Optional[str] = None, max_steps: int = 0, schedule: str = "auto", chunk_paths: int = 0,
                      blocks_per_cu: int = 0, refill_groups: int = 0,
                      coefs: Optional[Dict[str, torch.Tensor]] = None,
                      boundary_correction: bool = False, specialize: str = "auto",
                      dump: bool = False) -> Dict[str, torch.Tensor]:
    """Per-node statistics and the Jacobian d mean_i / d coefficients in one
    pass (pdd_mc_value_jacobian).  Returns the statistics of mc_interface plus
    `jac` [n, n_params] (column blocks in `param_layout(problem)` order); with
    dump=True also the per-path values `phi` and step counts `path_steps`."""
    _need_gpu()
    keep = _Keep()
    p = _linear(problem, keep, coefs)
    nt = _nodes_tensor(nodes, problem.domain.ndim)
    n = nt.shape[0]
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    if ph.shape[0] != n:
        raise ValueError("paths must have one entry per node")
    npar = int(library().pdd_param_count(C.byref(p)))
    if npar < 0:
        raise PddError("pdd_param_count rejected the problem")
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    jac = torch.zeros((max(n, 1), max(npar, 1)), dtype=torch.float64, device="cuda")
    dphi, dst = _dumps(dump, ph)
    o = _options(precision, layout, max_steps, schedule, chunk_paths, blocks_per_cu, refill_groups, dphi, dst,
                 boundary_correction=boundary_correction, specialize=specialize)
    st = library().pdd_mc_value_jacobian(C.byref(p), nt.data_ptr() if n else None, n,
                                         ph.ctypes.data_as(C.POINTER(C.c_int64)), float(dt),
                                         int(seed) & (2 ** 64 - 1), C.byref(o), raw.data_ptr(), jac.data_ptr(),
                                         max(npar, 1), _stream_handle())
    _check(st, "pdd_mc_value_jacobian")
    res = _stats(raw[:n])
    res["jac"] = jac[:n, :npar]
    res["jac_ld"] = max(npar, 1)
    if dump:
        total = int(ph.sum())
        res["phi"], res["path_steps"] = dphi[:total], dst[:total]
    res["_keep"] = keep
    return res


def merge_estimates(acc: Dict[str, torch.Tensor], add: Dict[str, torch.Tensor], index) -> Dict[str, torch.Tensor]:
    """Merges `add` (the result of a call over some nodes, with an independent
    sample: another seed) into `acc` (a result over all nodes) in place, node
    acc[index[k]] receiving add's node k (pdd_merge_estimates); Jacobians are
    merged too when both results carry one.  Returns acc's statistics
    recomputed from the merged records (with acc's Jacobian)."""
    _need_gpu()
    idx = torch.as_tensor(np.asarray(index, dtype=np.int64), device="cuda").contiguous()
    n_add = idx.numel()
    ra, rb = acc["_raw"], add["_raw"]
    if rb.shape[0] != n_add:
        raise ValueError("index must have one entry per node of `add`")
    ja, jb = acc.get("jac"), add.get("jac")
    both = ja is not None and jb is not None
    npar = ja.shape[1] if both else 0
    st = library().pdd_merge_estimates(ra.data_ptr(), ja.data_ptr() if both else None,
                                       int(acc.get("jac_ld", npar)) if both else 0, rb.data_ptr(),
                                       jb.data_ptr() if both else None, int(add.get("jac_ld", npar)) if both else 0,
                                       npar, idx.data_ptr(), n_add, _stream_handle())
    _check(st, "pdd_merge_estimates")
    out = _stats(ra)
    for k in ("jac", "jac_ld"):
        if k in acc:
            out[k] = acc[k]
    out["_keep"] = (acc.get("_keep"), idx)
    return out


def jacobian_apply(jac: torch.Tensor, w) -> torch.Tensor:
    """J^T w on the device (pdd_jacobian_apply): the gradient of sum_i w_i u_i
    from a Jacobian of mc_value_jacobian, summed in a fixed order."""
    _need_gpu()
    if not (jac.is_cuda and jac.dtype == torch.float64 and jac.dim() == 2 and jac.stride(1) == 1):
        raise ValueError("jac must be a float64 CUDA matrix with unit column stride")
    n, npar = jac.shape
    wt = _dev_f64(w).reshape(-1).contiguous()
    if wt.numel() != n:
        raise ValueError("w must have one entry per Jacobian row")
    grad = torch.empty(max(npar, 1), dtype=torch.float64, device="cuda")
    st = library().pdd_jacobian_apply(jac.data_ptr() if n else None, n, max(jac.stride(0), npar), npar,
                                      wt.data_ptr() if n else None, grad.data_ptr(), _stream_handle())
    _check(st, "pdd_jacobian_apply")
    return grad[:npar]


def misfit_gradient(result: Dict[str, torch.Tensor], data) -> Dict[str, torch.Tensor]:
    """Least-squares misfit of the interface values to `data` and its gradient
    with respect to the coefficients (pdd_misfit_gradient), from the result of
    mc_value_jacobian: loss = sum_i (u_i - d_i)^2, grad = J^T 2 (u - d).
    Returns {"loss": [1] tensor, "grad": [n_params] tensor}."""
    _need_gpu()
    raw, jac = result["_raw"], result["jac"]
    n, npar = jac.shape
    dt = _dev_f64(data).reshape(-1).contiguous()
    if dt.numel() != n:
        raise ValueError("data must have one entry per node")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(max(npar, 1), dtype=torch.float64, device="cuda")
    st = library().pdd_misfit_gradient(raw.data_ptr() if n else None, dt.data_ptr() if n else None, n,
                                       jac.data_ptr() if n else None, int(result.get("jac_ld", npar)), npar,
                                       loss.data_ptr(), grad.data_ptr(), _stream_handle())
    _check(st, "pdd_misfit_gradient")
    return {"loss": loss, "grad": grad[:npar], "_keep": dt}


def jacobian_blocks(problem, jac: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Split Jacobian columns (or a gradient vector) into per-array blocks."""
    out, c = {}, 0
    for name, k in param_layout(problem):
        out[name] = jac[..., c:c + k]
        c += k
    return out


def branching_eval(problem, points, trees: int, seed: int = 0, precision: str = "fp32",
                   layout: Optional[str] = None, dump: bool = False, schedule: str = "persistent",
                   chunk_paths: int = 0, blocks_per_cu: int = 0, specialize: str = "auto") -> Dict[str, torch.Tensor]:
    """Marked branching estimator at every point (pdd_branching_eval).  With
    dump=True also the per-tree values `value` [n, trees] and segment counts.
    `specialize` ("auto", "on", "off"): when psi has generic terms, run a
    kernel compiled at run time with psi's factor structure written in (same
    results as the table-driven kernel)."""
    _need_gpu()
    keep = _Keep()
    b = A.pdd_branching_problem()
    b.dim = int(problem.ndim)
    b.max_segments = int(problem.max_segments)
    b.sigma, b.beta, b.T = float(problem.sigma), float(problem.beta), float(problem.T)
    for k in range(5):
        b.alpha[k] = float(problem.alpha[k]) if k < len(problem.alpha) else 0.0
        b.q[k] = float(problem.q[k]) if k < len(problem.q) else 0.0
    b.psi_sup = float(problem.psi_sup)
    b.psi = _fun(problem.psi, keep)
    pt = _nodes_tensor(points, b.dim)
    n = pt.shape[0]
    raw = torch.empty((max(n, 1), 5), dtype=torch.float64, device="cuda")
    dv = ds = None
    if dump:
        dv = torch.empty(max(n * trees, 1), dtype=torch.float64, device="cuda")
        ds = torch.empty(max(n * trees, 1), dtype=torch.int64, device="cuda")
    o = _options(precision, layout, 0, schedule, chunk_paths, blocks_per_cu, 0, dv, ds, specialize=specialize)
    st = library().pdd_branching_eval(C.byref(b), pt.data_ptr() if n else None, n, int(trees),
                                      int(seed) & (2 ** 64 - 1), C.byref(o), raw.data_ptr(), _stream_handle())
    _check(st, "pdd_branching_eval")
    res = _stats(raw[:n])
    if dump:
        res["value"] = dv[:n * trees].reshape(n, trees)
        res["segments"] = ds[:n * trees].reshape(n, trees)
    res["_keep"] = keep
    return res


def branching_bvp(problem, boundary, points, trees: int, seed: int = 0, precision: str = "fp32",
                  layout: Optional[str] = None, dump: bool = False, chunk_paths: int = 0,
                  blocks_per_cu: int = 0, boundary_correction: bool = False,
                  specialize: str = "auto") -> Dict[str, torch.Tensor]:
    """Branching estimator with particles stopped on a Dirichlet boundary,
    evaluated at every output time of one tree (pdd_branching_bvp).
    `boundary` is a workloads.problem.BranchingBoundary.  Statistics have
    shape [n_times, n_points]; with dump=True also `value` [n, trees, n_times]
    and `segments` [n, trees].  `specialize` as for branching_eval (psi or g
    with generic terms)."""
    _need_gpu()
    keep = _Keep()
    b = A.pdd_branching_problem()
    b.dim = int(problem.ndim)
    b.max_segments = int(problem.max_segments)
    b.sigma, b.beta, b.T = float(problem.sigma), float(problem.beta), float(problem.T)
    for k in range(5):
        b.alpha[k] = float(problem.alpha[k]) if k < len(problem.alpha) else 0.0
        b.q[k] = float(problem.q[k]) if k < len(problem.q) else 0.0
    b.psi_sup = float(problem.psi_sup)
    b.psi = _fun(problem.psi, keep)
    bd = A.pdd_branching_boundary()
    D = boundary.domain
    bd.domain.kind, bd.domain.dim = int(D.kind), int(D.ndim)
    for k in range(3):
        bd.domain.lo[k], bd.domain.hi[k], bd.domain.center[k] = float(D.lo[k]), float(D.hi[k]), float(D.center[k])
    bd.domain.radius = float(D.radius)
    bd.g = _fun(boundary.g, keep)
    bd.g_sup = float(boundary.g_sup)
    bd.dt = float(boundary.dt)
    times = np.ascontiguousarray(np.asarray(boundary.times, dtype=np.float64).reshape(-1))
    keep.append(times)
    bd.n_times = int(times.shape[0])
    bd.times = times.ctypes.data_as(C.POINTER(C.c_double))
    nt = bd.n_times
    pt = _nodes_tensor(points, b.dim)
    n = pt.shape[0]
    raw = torch.empty((max(n * nt, 1), 5), dtype=torch.float64, device="cuda")
    dv = ds = None
    if dump:
        dv = torch.empty(max(n * trees * nt, 1), dtype=torch.float64, device="cuda")
        ds = torch.empty(max(n * trees, 1), dtype=torch.int64, device="cuda")
    o = _options(precision, layout, 0, "persistent", chunk_paths, blocks_per_cu, 0, dv, ds, boundary_correction,
                 specialize)
    st = library().pdd_branching_bvp(C.byref(b), C.byref(bd), pt.data_ptr() if n else None, n, int(trees),
                                     int(seed) & (2 ** 64 - 1), C.byref(o), raw.data_ptr(), _stream_handle())
    _check(st, "pdd_branching_bvp")
    res = {k: (v if k == "_raw" else v.reshape(nt, n)) for k, v in _stats(raw[:n * nt]).items()}
    if dump:
        res["value"] = dv[:n * trees * nt].reshape(n, trees, nt)
        res["segments"] = ds[:n * trees].reshape(n, trees)
    res["_keep"] = keep
    return res


_KERNELS = {"walk": A.PDD_KERNEL_WALK, "walk_adjoint": A.PDD_KERNEL_WALK_ADJOINT, "wos": A.PDD_KERNEL_WOS,
            "walk_batch": A.PDD_KERNEL_WALK_BATCH, "wos_batch": A.PDD_KERNEL_WOS_BATCH,
            "branch": A.PDD_KERNEL_BRANCH, "branch_bvp": A.PDD_KERNEL_BRANCH_BVP}


def item_count(paths, dim: int, kernel: str = "walk", precision: str = "fp32", layout: Optional[str] = None,
               schedule: str = "auto", chunk_paths: int = 0, blocks_per_cu: int = 0, refill_groups: int = 0) -> int:
    """Work items (partials slots) a forward call of `kernel` ("walk", "wos",
    "walk_batch", "wos_batch") in dimension `dim` (0 for the batch kernels)
    cuts these budgets into with these schedule options on the current device
    (pdd_item_count)."""
    ph = np.ascontiguousarray(np.asarray(paths, dtype=np.int64).reshape(-1))
    o = _options(precision, layout, 0, schedule, chunk_paths, blocks_per_cu, refill_groups)
    n = int(library().pdd_item_count(_KERNELS[kernel], int(dim), ph.shape[0],
                                     ph.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(o)))
    if n < 0:
        _check(n, "pdd_item_count")
    return n


def _prec_key(precision: str) -> int:
    if precision not in ("fp32", "fp64"):
        raise ValueError("schedules are kept for precision 'fp32' or 'fp64'")
    return A.PDD_FP32_STEP if precision == "fp32" else A.PDD_FP64


def set_schedule(kernel: str, dim: int, precision: str, chunk_paths: Optional[int] = None,
                 blocks_per_cu: Optional[int] = None, refill_groups: Optional[int] = None):
    """Sets the current device's schedule-table entry (kernel, dim, precision)
    (pdd_set_schedule); with every knob None, removes it."""
    if chunk_paths is None and blocks_per_cu is None and refill_groups is None:
        st = library().pdd_set_schedule(_KERNELS[kernel], int(dim), _prec_key(precision), None)
    else:
        s = A.pdd_launch_schedule(int(chunk_paths), int(blocks_per_cu), int(refill_groups), 0)
        st = library().pdd_set_schedule(_KERNELS[kernel], int(dim), _prec_key(precision), C.byref(s))
    _check(st, "pdd_set_schedule")


def get_schedule(kernel: str, dim: int, precision: str) -> dict:
    """The schedule a call would start from (pdd_get_schedule): the table's
    tuned entry or the built-in default, with `tuned` telling which."""
    s = A.pdd_launch_schedule()
    t = C.c_int32(0)
    _check(library().pdd_get_schedule(_KERNELS[kernel], int(dim), _prec_key(precision), C.byref(s), C.byref(t)),
           "pdd_get_schedule")
    return {"chunk_paths": s.chunk_paths, "blocks_per_cu": s.blocks_per_cu, "refill_groups": s.refill_groups,
            "tuned": bool(t.value)}


def save_schedules(path: Optional[str] = None):
    _check(library().pdd_save_schedules(path.encode() if path else None), "pdd_save_schedules")


def load_schedules(path: Optional[str] = None):
    _check(library().pdd_load_schedules(path.encode() if path else None), "pdd_load_schedules")


def query_warnings():
    """Synchronizes the current stream; returns (censored paths, redrawn trees)
    since the last query."""
    c, r = C.c_int64(0), C.c_int64(0)
    st = library().pdd_query_warnings(_stream_handle(), C.byref(c), C.byref(r))
    if st < 0:
        _check(st, "pdd_query_warnings")
    return int(c.value), int(r.value)


def release_workspace():
    _check(library().pdd_release_workspace(), "pdd_release_workspace")


def cached_plan_count() -> int:
    """Graph launch plans the library currently caches (at most 16)."""
    return int(library().pdd_cached_plan_count())


_COEF_KEYS = ("g_coef", "g_poly", "f_coef", "f_poly", "c_coef", "c_poly")


class PDDInterface(torch.autograd.Function):
    """u = PDDInterface.apply(problem, nodes, paths, dt, seed, opts,
    g_coef, g_poly, f_coef, f_poly, c_coef, c_poly): interface values,
    differentiable in the six coefficient tensors (None = take the problem's
    own array, not differentiated).

    opts["gradient"] selects how the backward pass is formed:
      "recompute" (default): backward re-simulates the same paths from their
          counters with w = grad_u (pdd_mc_adjoint); nothing per path is kept.
      "jacobian": forward runs pdd_mc_value_jacobian, keeping the per-node
          Jacobian (n x n_params FP64); backward is J^T grad_u (no second pass).
    Both give the same derivative of the same discrete estimator."""

    @staticmethod
    def forward(ctx, problem, nodes, paths, dt, seed, opts, *coef_tensors):
        coefs = {k: v for k, v in zip(_COEF_KEYS, coef_tensors) if v is not None}
        opts = dict(opts or {})
        mode = opts.pop("gradient", "recompute")
        if mode not in ("recompute", "jacobian"):
            raise ValueError("opts['gradient'] must be 'recompute' or 'jacobian'")
        ctx.jac = None
        if mode == "jacobian" and any(ctx.needs_input_grad[6:]):
            r = mc_value_jacobian(problem, nodes, paths, dt, seed, coefs=coefs, **opts)
            ctx.jac = r["jac"]
        else:
            r = mc_interface(problem, nodes, paths, dt, seed, coefs=coefs, **opts)
        ctx.problem, ctx.nodes, ctx.paths, ctx.dt, ctx.seed, ctx.opts = problem, nodes, paths, dt, seed, opts
        ctx.present = [v is not None for v in coef_tensors]
        ctx.save_for_backward(*[v for v in coef_tensors if v is not None])
        return r["mean"].clone()

    @staticmethod
    def backward(ctx, grad_u):
        saved = list(ctx.saved_tensors)
        coefs = {}
        for k, present in zip(_COEF_KEYS, ctx.present):
            if present:
                coefs[k] = saved.pop(0)
        if ctx.jac is not None:
            g = jacobian_blocks(ctx.problem, jacobian_apply(ctx.jac, grad_u.detach()))
        else:
            opts = {k: v for k, v in ctx.opts.items() if k not in ("dump",)}
            g = mc_adjoint(ctx.problem, ctx.nodes, ctx.paths, ctx.dt, ctx.seed, grad_u.detach(), coefs=coefs, **opts)
        out = [None] * 6
        for i, k in enumerate(_COEF_KEYS):
            if ctx.present[i] and ctx.needs_input_grad[6 + i]:
                out[i] = g[k].to(coefs[k].dtype)
        return (None, None, None, None, None, None, *out)
