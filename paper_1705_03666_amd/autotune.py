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
    "chunk_paths": [1024, 2048, 4096, 8192],
}
DEFAULT = {"blocks_per_cu": 2, "refill_groups": 1, "chunk_paths": 4096}


def _key(problem, precision: str, adjoint: bool) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    f = lambda F: f"{int(np.asarray(F.coef).shape[0])}t{int(F.poly_degree)}p"
    parts = [props.name, str(props.multi_processor_count), f"d{problem.domain.ndim}", f"k{problem.domain.kind}",
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
         coefs=None, sample_nodes: int = 1024, sample_paths: int = 20000, repeats: int = 2, force: bool = False,
         log=None) -> dict:
    """Best schedule for this problem shape (cached).  Times forward or adjoint
    launches on `sample_nodes` nodes x `sample_paths` paths of the workload."""
    key = _key(problem, precision, adjoint)
    cache = _load()
    if not force and key in cache:
        return cache[key]["schedule"]
    n = len(nodes)
    idx = np.linspace(0, n - 1, min(sample_nodes, n)).round().astype(int)
    sub = nodes[torch.as_tensor(idx, device=nodes.device)] if isinstance(nodes, torch.Tensor) else nodes[idx]
    pa = np.minimum(np.asarray(paths)[idx], sample_paths).astype(np.int64)
    w = torch.ones(len(idx), dtype=torch.float64, device="cuda")

    def run(cfg) -> float:
        kw = dict(precision=precision, schedule="persistent", coefs=coefs, **cfg)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(repeats + 1):
            ev0.record()
            if adjoint:
                mc_adjoint(problem, sub, pa, dt, seed, w, **kw)
            else:
                mc_interface(problem, sub, pa, dt, seed, **kw)
            ev1.record()
            torch.cuda.synchronize()
            best = min(best, ev0.elapsed_time(ev1))
        return best

    cur = dict(DEFAULT)
    t_cur = run(cur)
    trials = [(dict(cur), t_cur)]
    for knob in ("blocks_per_cu", "refill_groups", "chunk_paths"):
        for v in SPACE[knob]:
            if v == cur[knob]:
                continue
            cand = dict(cur)
            cand[knob] = v
            t = run(cand)
            trials.append((dict(cand), t))
            if log:
                log(f"autotune {'adj' if adjoint else 'fwd'} {cand}: {t:.2f} ms")
            if t < t_cur:
                cur, t_cur = cand, t
    cache = _load()
    cache[key] = {"schedule": cur, "ms": t_cur, "default_ms": trials[0][1], "when": time.time(),
                  "sample": [len(idx), int(pa.max()) if len(pa) else 0]}
    _save(cache)
    return cur
