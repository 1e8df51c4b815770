"""Schedule autotuner for the persistent walk kernels.

Searches the launch schedule (work-item size `chunk_paths`, persistent grid
`blocks_per_cu`, lane-refill interval `refill_groups`) by coordinate descent,
timing each candidate with HIP events on a subsample of the caller's
workload, and caches the winner in a JSON file keyed by device, dimension,
domain, precision, direction (forward / adjoint) and the sizes of the
coefficient tables.  Results never depend on the schedule (the per-path
arithmetic is the same), so tuning only changes speed.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import numpy as np
import torch

from . import mc_adjoint, mc_interface

CACHE = os.environ.get("PDD_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pdd_autotune.json"))

SPACE = {
    "blocks_per_cu": [1, 2, 3, 4, 6, 8],
    "refill_groups": [1, 2, 3, 4, 6, 8],
    "chunk_paths": [2048, 4096, 8192, 16384, 32768],
}
DEFAULT = {"blocks_per_cu": 8, "refill_groups": 3, "chunk_paths": 16384}
VERSION = 2


def items_per_node(paths: int, chunk: int) -> int:
    """Work items the library cuts one node's paths into (guided sizes: items
    of `chunk` paths, the last eighth in items of chunk/8, at least 256)."""
    big = max(1, chunk)
    small = max(min(256, big), big // 8)
    n_big = (paths - paths // 8) // big if paths > big else 0
    rest = paths - n_big * big
    return n_big + (rest + small - 1) // small


def _key(problem, precision: str, adjoint: bool) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    f = lambda F: f"{int(np.asarray(F.coef).shape[0])}t{int(F.poly_degree)}p"
    parts = [f"v{VERSION}", props.name, str(props.multi_processor_count), f"d{problem.domain.ndim}",
             f"k{problem.domain.kind}",
             precision, "adj" if adjoint else "fwd", "g" + f(problem.g), "f" + f(problem.f), "c" + f(problem.c),
             "b" + "".join(f(b) for b in problem.b)]
    return "|".join(parts)


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(cache: Dict[str, dict]):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def lookup(problem, precision: str = "fp32", adjoint: bool = False) -> Optional[dict]:
    return _load().get(_key(problem, precision, adjoint))


def tune(problem, nodes, paths, dt: float, seed: int = 0, precision: str = "fp32", adjoint: bool = False,
         coefs=None, items_per_wave: int = 4, sample_paths: int = 100000, repeats: int = 2, force: bool = False,
         log=None) -> dict:
    """Best schedule for this problem shape (cached).  Each candidate runs on
    a node subsample sized so that every resident wavefront gets about
    `items_per_wave` work items (at most `sample_paths` paths per node, the
    caller's own path counts otherwise), and candidates are compared by
    path-steps per second, so work-item size is judged at the granularity
    the full workload will see."""
    key = _key(problem, precision, adjoint)
    cache = _load()
    if not force and key in cache:
        return cache[key]["schedule"]
    n = len(nodes)
    n_cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
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
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = 0.0
        for _ in range(repeats + 1):
            ev0.record()
            if adjoint:
                r = mc_adjoint(problem, sub, pa, dt, seed, w, with_stats=True, **kw)["stats"]
            else:
                r = mc_interface(problem, sub, pa, dt, seed, **kw)
            ev1.record()
            torch.cuda.synchronize()
            rate = float(r["steps"].sum().item()) / (ev0.elapsed_time(ev1) * 1e-3)
            best = max(best, rate)
        return best

    cur = dict(DEFAULT)
    r_cur = run(cur)
    trials = [(dict(cur), r_cur)]
    for knob in ("chunk_paths", "blocks_per_cu", "refill_groups"):
        for v in SPACE[knob]:
            if v == cur[knob]:
                continue
            cand = dict(cur)
            cand[knob] = v
            r = run(cand)
            trials.append((dict(cand), r))
            if log:
                log(f"autotune {'adj' if adjoint else 'fwd'} {cand}: {r:.4g} path-steps/s")
            if r > r_cur:
                cur, r_cur = cand, r
    cache = _load()
    cache[key] = {"schedule": cur, "path_steps_per_s": r_cur, "default_path_steps_per_s": trials[0][1],
                  "when": time.time()}
    _save(cache)
    return cur
