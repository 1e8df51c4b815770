"""Schedule autotuner for the persistent kernels.

Searches the launch schedule (work-item size `chunk_paths`, persistent grid
`blocks_per_cu`, lane-refill interval `refill_groups`) by coordinate descent,
timing each candidate with HIP events on a subsample of the caller's workload
sized so that every resident wavefront sees the item granularity the full
workload will see.  The winner goes into the library's schedule table for
(kernel, dimension, precision) on this kind of device (pdd_set_schedule) and
into its file (pdd_save_schedules), so every later call with the schedule
options left at 0, from any caller and process, runs with it.  Results never
depend on the schedule (per-path arithmetic is the same), only speed does.
"""
from __future__ import annotations

from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import (branching_bvp, branching_eval, get_schedule, mc_adjoint, mc_interface, mc_interface_batch,
               save_schedules, set_schedule, wos_interface_batch)

WALK_SPACE = {
    "chunk_paths": [2048, 4096, 8192, 16384, 32768],
    "blocks_per_cu": [1, 2, 3, 4, 6, 8],
    "refill_groups": [1, 2, 3, 4, 6, 8],
}
# item sizes between the powers of two as well: with a few items per
# wavefront the end of a launch depends on how the trees divide into items
# (C4: 3.17 ms with 14336-tree items against 3.24 with 16384)
BRANCH_SPACE = {
    "chunk_paths": [2048, 4096, 8192, 12288, 14336, 16384, 24576, 32768],
    "blocks_per_cu": [2, 3, 4, 6, 8],
}


def items_per_node(paths: int, chunk: int) -> int:
    """Work items the library cuts one node's paths into (guided sizes: items
    of `chunk` paths, the last eighth in items of chunk/8, at least 256)."""
    big = max(1, chunk)
    small = max(min(256, big), big // 8)
    n_big = (paths - paths // 8) // big if paths > big else 0
    rest = paths - n_big * big
    return n_big + (rest + small - 1) // small


def _n_cu() -> int:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


# a candidate replaces the current schedule only when it is at least this
# much faster, so that timing noise between near-equal schedules does not
# move the table from run to run
MIN_GAIN = 1.01


def _search(run: Callable[[dict], float], start: dict, space: Dict[str, list], log=None, tag="") -> tuple:
    """Coordinate descent from `start` over `space`; run(cfg) returns a rate
    (work units per second, higher is better)."""
    cur = dict(start)
    r_cur = run(cur)
    r0 = r_cur
    for knob, values in space.items():
        for v in values:
            if v == cur[knob]:
                continue
            cand = dict(cur)
            cand[knob] = v
            r = run(cand)
            if log:
                log(f"autotune {tag} {cand}: {r:.4g}/s")
            if r > r_cur * MIN_GAIN:
                cur, r_cur = cand, r
    return cur, r_cur, r0


def _timed_rate(call: Callable[[], float], repeats: int) -> float:
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 0.0
    for _ in range(repeats + 1):      # the first run warms up (and compiles, for specialised kernels)
        ev0.record()
        work = call()
        ev1.record()
        torch.cuda.synchronize()
        best = max(best, work() / (ev0.elapsed_time(ev1) * 1e-3))
    return best


def _store(kernel: str, dim: int, precision: str, cfg: dict):
    set_schedule(kernel, dim, precision, cfg["chunk_paths"], cfg["blocks_per_cu"], cfg.get("refill_groups", 1))
    save_schedules()


def _start(kernel: str, dim: int, precision: str) -> Optional[dict]:
    s = get_schedule(kernel, dim, precision)
    return s


def tune_walk(problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32", adjoint: bool = False,
              coefs=None, items_per_wave: int = 4, sample_paths: int = 100000, repeats: int = 2,
              force: bool = False, log=None) -> dict:
    """Best schedule of the batched walk (forward, or adjoint / value+Jacobian)
    for this dimension and precision; stored in the library's table."""
    kernel = "walk_adjoint" if adjoint else "walk"
    dim = problem.domain.ndim
    s = _start(kernel, dim, precision)
    if s["tuned"] and not force:
        return {k: s[k] for k in ("chunk_paths", "blocks_per_cu", "refill_groups")}
    n = len(nodes)
    n_cu = _n_cu()
    all_paths = np.minimum(np.asarray(paths, dtype=np.int64), sample_paths)
    typical = int(np.median(all_paths)) if n else 0

    def run(cfg) -> float:
        per_node = max(1, items_per_node(typical, cfg["chunk_paths"]))
        want = items_per_wave * cfg["blocks_per_cu"] * 4 * n_cu
        k = int(min(n, max(1, -(-want // per_node))))
        idx = np.linspace(0, n - 1, k).round().astype(int)
        sub = nodes[torch.as_tensor(idx, device=nodes.device)] if isinstance(nodes, torch.Tensor) else nodes[idx]
        pa = all_paths[idx]
        kw = dict(precision=precision, schedule="persistent", coefs=coefs, **cfg)
        w = torch.ones(len(idx), dtype=torch.float64, device="cuda")

        def call():
            if adjoint:
                r = mc_adjoint(problem, sub, pa, dt, seed, w, with_stats=True, **kw)["stats"]
            else:
                r = mc_interface(problem, sub, pa, dt, seed, **kw)
            return lambda: float(r["steps"].sum().item())
        return _timed_rate(call, repeats)

    start = {k: s[k] for k in ("chunk_paths", "blocks_per_cu", "refill_groups")}
    best, r_best, r0 = _search(run, start, WALK_SPACE, log, kernel)
    _store(kernel, dim, precision, best)
    if log:
        log(f"autotune {kernel} d{dim} {precision}: {best} at {r_best:.4g} path-steps/s (start {r0:.4g})")
    return best


# the previous name of tune_walk
tune = tune_walk


def tune_batch(problems, node_problem, nodes, paths, dt_or_eps: float, seed: int = 0, precision: str = "fp32",
               wos: bool = False, repeats: int = 2, force: bool = False, log=None) -> dict:
    """Best schedule of the heterogeneous batch entry point (walk or walk on
    spheres) on the caller's whole batch (batches are short, so the full
    batch is the sample); stored under dimension 0."""
    kernel = "wos_batch" if wos else "walk_batch"
    s = _start(kernel, 0, precision)
    if s["tuned"] and not force:
        return {k: s[k] for k in ("chunk_paths", "blocks_per_cu", "refill_groups")}
    fn = wos_interface_batch if wos else mc_interface_batch

    def run(cfg) -> float:
        def call():
            r = fn(problems, node_problem, nodes, paths, dt_or_eps, seed, precision=precision, schedule="persistent",
                   **cfg)
            return lambda: float(r["steps"].sum().item())
        return _timed_rate(call, repeats)

    start = {k: s[k] for k in ("chunk_paths", "blocks_per_cu", "refill_groups")}
    best, r_best, r0 = _search(run, start, WALK_SPACE, log, kernel)
    _store(kernel, 0, precision, best)
    if log:
        log(f"autotune {kernel} {precision}: {best} at {r_best:.4g} steps/s (start {r0:.4g})")
    return best


def tune_branching(problem, points, trees: int, seed: int = 0, precision: str = "fp32", boundary=None,
                   items_per_wave: int = 8, repeats: int = 1, force: bool = False, log=None) -> dict:
    """Best schedule of the branching estimator (free space, or with a
    boundary when `boundary` is given) for this dimension and precision,
    compared by simulated segments (sub-steps) per second; stored in the
    library's table.  The sample gives every resident wavefront at least
    `items_per_wave` items, so it sees the imbalance at the end of a launch
    that the caller's workload will see (with 1024 points x 1e5 trees it is
    the whole workload)."""
    kernel = "branch_bvp" if boundary is not None else "branch"
    dim = int(problem.ndim)
    s = _start(kernel, dim, precision)
    if s["tuned"] and not force:
        return {k: s[k] for k in ("chunk_paths", "blocks_per_cu", "refill_groups")}
    n = len(points)
    n_cu = _n_cu()

    def run(cfg) -> float:
        per_point = max(1, -(-int(trees) // cfg["chunk_paths"]))
        want = items_per_wave * cfg["blocks_per_cu"] * 4 * n_cu
        k = int(min(n, max(1, -(-want // per_point))))
        idx = np.linspace(0, n - 1, k).round().astype(int)
        sub = points[torch.as_tensor(idx, device=points.device)] if isinstance(points, torch.Tensor) else points[idx]

        def call():
            if boundary is not None:
                r = branching_bvp(problem, boundary, sub, trees, seed, precision=precision,
                                  chunk_paths=cfg["chunk_paths"], blocks_per_cu=cfg["blocks_per_cu"])
                return lambda: float(r["steps"][0].sum().item())
            r = branching_eval(problem, sub, trees, seed, precision=precision, chunk_paths=cfg["chunk_paths"],
                               blocks_per_cu=cfg["blocks_per_cu"])
            return lambda: float(r["steps"].sum().item())
        return _timed_rate(call, repeats)

    start = {k: s[k] for k in ("chunk_paths", "blocks_per_cu")}
    best, r_best, r0 = _search(run, start, BRANCH_SPACE, log, kernel)
    best["refill_groups"] = 1
    _store(kernel, dim, precision, best)
    if log:
        log(f"autotune {kernel} d{dim} {precision}: {best} at {r_best:.4g} segments/s (start {r0:.4g})")
    return best
