"""Benchmark of the interface-node Monte Carlo hot path on one MI355X.

Headline workload (C5): 3-D unit ball, 1/2 Lap u - c u = -f with boundary data
g = sum_{k<64} theta_k r^l Y_k and 16-term polynomial c, f; 4096 interface
nodes on the three discs x_k = 0, |x| < 0.95; 1e5 paths per node; dt = 1e-3;
FP32 stepping and transforms, FP64 accumulation.  One step = the batched
forward pass at theta plus the adjoint of the loss sum_i (u_i - d_i)^2
(persistent kernels replayed from a cached hipGraph).

value = path-steps of the estimator (forward pass) per second of the whole
forward + adjoint step.  Also reported: forward-only and adjoint-only rates,
interface nodes per second at a standard error of 1e-3 (derived from the
measured per-node variances and step counts), the speed-up over the plain
FP64 one-node-per-launch kernel, the ALU roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published FP32 vector peak 157.3 TFLOP/s = 256 CUs x 128 FP32 lanes x
# 2.4 GHz x 2 flops per FMA; one VALU lane operation (FMA, multiply, add,
# integer op, conversion, transcendental) is counted as one op.
PEAK_LANE_OPS = 256 * 128 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Algorithmic VALU lane-ops per path-step of the C5 walk (3-D ball, b = 0,
# cubic c and f, QUAD24 Gaussians); each op is one VALU lane operation:
#   Philox4x32-10 block: 10 rounds x (2 32x32->64 products + 2 three-input
#     xors) + 2 counter ops = 42, x 3/4 block per step                  31.5
#   QUAD24 uniforms: 4 words x (funnel shift, add) = 8, x 3/4            6
#   Box-Muller pair: log2, mul, sqrt, sin, cos, 2 mul = 7, x 1.5        10.5
#   cubic monomials of X                                                16
#   f and c: 2 x 19 FMA                                                 38
#   Z += f Y dt (2), Y *= exp2(-c dt log2 e) (4)                          6
#   X += sigma sqrt(dt) z                                                3
#   ball exit test: 3 sub, mul, 2 fma, compare                           7
#   step count and cap                                                   2
# forward: 120.  The adjoint adds the 3 x 20 tangent updates F/dt += m Y,
# S/dt += m, B/dt += m Z (the factor dt is applied once per fold): 180.
OPS_PER_PS_FWD = 120.0
OPS_PER_PS_ADJ = 180.0
# The same step in the survey's unit: lane-op slots with a quarter-rate
# operation (32x32->64 multiply, transcendental) counted as 4 slots; its
# estimate for a C5 adjoint path-step is 230.
OPS_PER_PS_ADJ_SURVEY = 230.0

# HBM bytes per launch of the dominant kernel (C5 value+Jacobian walk),
# from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the 256 MiB copy
# calibration (x 2.000 / x 1.000), counted at the schedule below (the item
# count, and with it the per-item writes, depends on it).  Valid only for the
# kernel sources and the schedule they were counted on: otherwise the bench
# reports null.
TRAFFIC_SOURCES = ['paper_1705_03666_amd/csrc/walk_kernels.hpp', 'paper_1705_03666_amd/csrc/pdd_device.hpp', 'paper_1705_03666_amd/csrc/pdd_internal.hpp', 'paper_1705_03666_amd/csrc/walk_adj_f32.hip']
TRAFFIC_SHA256 = "2be92012d1389510fa494e35ddad7e11c09923fcce68f3ddbc21ac6344958726"
TRAFFIC_SCHEDULE = {"chunk_paths": 32768, "blocks_per_cu": 8, "refill_groups": 3}
TRAFFIC_BYTES = 60.83e6 + 238.86e6


def traffic_bytes(schedule=None):
    """TRAFFIC_BYTES when the kernel sources hash to TRAFFIC_SHA256 and the
    adjoint schedule (if given) is TRAFFIC_SCHEDULE, else None."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC_SHA256:
        return None
    if schedule is not None and any(int(schedule.get(k, -1)) != v for k, v in TRAFFIC_SCHEDULE.items()):
        return None
    return TRAFFIC_BYTES


class ClockSampler:
    """Samples the GPU shader clock while the timed steps run, from the
    amdgpu driver's sysfs table (the active DPM level is marked '*'), or once
    from amd-smi when sysfs is not readable.  Reports MHz, or None."""

    def __init__(self, period: float = 0.05):
        import glob
        import threading
        self.files = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
        self.period = period
        self.samples = []
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._run, daemon=True)

    def _read(self):
        vals = []
        for f in self.files:
            try:
                for line in open(f):
                    if "*" in line:
                        vals.append(float(line.split(":")[1].strip().lower().replace("*", "").replace("mhz", "")))
            except (OSError, ValueError, IndexError):
                pass
        return max(vals) if vals else None

    def _run(self):
        while not self._stop.is_set():
            v = self._read()
            if v is not None:
                self.samples.append(v)
            self._stop.wait(self.period)

    def __enter__(self):
        if self.files:
            self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self.files:
            self._t.join()

    def result(self):
        if self.samples:
            return {"source": "sysfs pp_dpm_sclk", "median_mhz": float(np.median(self.samples)),
                    "min_mhz": float(min(self.samples)), "samples": len(self.samples)}
        import subprocess
        try:
            txt = subprocess.run(["amd-smi", "metric", "-g", "0", "--clock"], capture_output=True, text=True,
                                 timeout=20).stdout
            return {"source": "amd-smi metric --clock (after the steps)", "text": txt.strip()[:600]}
        except (OSError, subprocess.SubprocessError):
            return None


def run(args):
    import torch
    import paper_1705_03666_amd as pdd
    from workloads import configs as CF

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = CF.c5(scale=args.scale, n_nodes=args.nodes)
    P = w.problem_template
    nodes = torch.tensor(w.nodes, device=dev)
    paths = w.paths
    n = len(paths)
    sh = torch.tensor(w.sh_matrix, device=dev)
    sel = torch.tensor(w.fc_matrix, device=dev)
    theta = {k: torch.tensor(v, device=dev) for k, v in (("g", w.theta_g), ("f", w.theta_f), ("c", w.theta_c))}
    coefs = {"g_poly": (sh @ theta["g"]).contiguous(), "f_poly": (sel @ theta["f"]).contiguous(),
             "c_poly": (sel @ theta["c"]).contiguous()}
    star = {k: torch.tensor(v, device=dev) for k, v in w.theta_star.items()}
    coefs_star = {"g_poly": (sh @ star["g"]).contiguous(), "f_poly": (sel @ star["f"]).contiguous(),
                  "c_poly": (sel @ star["c"]).contiguous()}
    opts = dict(precision="fp32", schedule="graph")

    log(f"bench: C5 {n} nodes x {int(paths[0])} paths, dt={w.dt}; synthetic data at theta* (seed {w.data_seed})")
    t0 = time.time()
    d = pdd.mc_interface(P, nodes, paths, w.dt, w.data_seed, coefs=coefs_star, **opts)["mean"].clone()
    torch.cuda.synchronize()
    log(f"bench: data ready ({time.time() - t0:.1f} s)")

    from paper_1705_03666_amd import autotune

    def parse_sched(text):
        b, r, c = (int(v) for v in text.split(","))
        return {"blocks_per_cu": b, "refill_groups": r, "chunk_paths": c}

    # schedules live in the library's table: the timed calls pass none and the
    # library applies the table's entry (tuned here, or from an earlier run's
    # schedule file, else its defaults)
    if args.schedule_adj:
        sa = parse_sched(args.schedule_adj)
        sf = parse_sched(args.schedule_fwd) if args.schedule_fwd else dict(sa)
        pdd.set_schedule("walk_adjoint", 3, "fp32", **sa)
        pdd.set_schedule("walk", 3, "fp32", **sf)
        log(f"bench: given schedules: forward {sf}, adjoint {sa}")
    elif args.tune:
        t0 = time.time()
        autotune.tune_walk(P, nodes, paths, w.dt, w.seed, "fp32", False, coefs, log=log)
        autotune.tune_walk(P, nodes, paths, w.dt, w.seed, "fp32", True, coefs, log=log)
        log(f"bench: autotuned in {time.time() - t0:.1f} s")
    sched_f = pdd.get_schedule("walk", 3, "fp32")
    sched_a = pdd.get_schedule("walk_adjoint", 3, "fp32")
    log(f"bench: schedules from the library table: forward {sched_f}, adjoint {sched_a}")

    stats = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    ev_vj = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def step():
        # forward + adjoint in one pass: values and per-node Jacobian, then
        # the misfit loss sum (u - d)^2 and its gradient J^T 2 (u - d), both in
        # the library.  It launches on torch's current stream, so these events
        # bracket the value+Jacobian graph (walk kernel + its small reductions).
        ev_vj[0].record()
        r = pdd.mc_value_jacobian(P, nodes, paths, w.dt, w.seed, coefs=coefs, **opts)
        ev_vj[1].record()
        m = pdd.misfit_gradient(r, d)
        return r, m["grad"]

    def step_recompute():
        r = pdd.mc_interface(P, nodes, paths, w.dt, w.seed, coefs=coefs, **opts)
        ev[1].record()
        g = pdd.mc_adjoint(P, nodes, paths, w.dt, w.seed, 2.0 * (r["mean"] - d), coefs=coefs, **opts)
        return r, g

    for i in range(args.warmup):
        step()
        if not args.steps_only:
            step_recompute()
        torch.cuda.synchronize()
        log(f"bench: warmup {i + 1}/{args.warmup} done")

    step_ms, vj_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    with ClockSampler() as clock:
        for i in range(args.steps):
            ev[0].record()
            r, grad = step()
            ev[2].record()
            torch.cuda.synchronize()
            step_ms.append(ev[0].elapsed_time(ev[2]))
            vj_ms.append(ev_vj[0].elapsed_time(ev_vj[1]))
            stats["fwd"] = r
            log(f"bench: step {i + 1}/{args.steps}: value+jacobian+gradient {step_ms[-1]:.1f} ms")
        torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    sclk = clock.result()
    ms_step = wall * 1e3 / args.steps

    if args.steps_only:
        # profiling mode: only the timed value+Jacobian steps above
        r = stats["fwd"]
        ps = float(r["steps"].sum().item())
        dur = np.median(vj_ms) / 1e3
        return {"metric": "path-steps/s (batched FP32 forward+adjoint, C5)", "value": ps / (ms_step / 1e3),
                "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": ms_step, "mode": "steps-only", "schedule_adjoint": sched_a,
                "gpu_clock_during_steps": sclk,
                "roofline": {"bound": "alu", "achieved": ps * OPS_PER_PS_ADJ / dur / 1e12,
                             "achieved_survey_unit": ps * OPS_PER_PS_ADJ_SURVEY / dur / 1e12,
                             "peak": PEAK_LANE_OPS / 1e12, "unit": "Top/s", "launch_ms": dur * 1e3}}

    # the path-recomputing route (forward kernel, then adjoint kernel), timed
    # separately with the same schedule
    fwd_ms, adj_ms = [], []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        ev[0].record()
        step_recompute()
        ev[2].record()
        torch.cuda.synchronize()
        fwd_ms.append(ev[0].elapsed_time(ev[1]))
        adj_ms.append(ev[1].elapsed_time(ev[2]))
        log(f"bench: recompute route {i + 1}: forward {fwd_ms[-1]:.1f} ms, adjoint {adj_ms[-1]:.1f} ms")
    r = stats["fwd"]
    ps = float(r["steps"].sum().item())
    mean_steps = r["steps"].double() / r["n"].double()
    var = r["var"]
    fwd_s, adj_s = np.median(fwd_ms) / 1e3, np.median(adj_ms) / 1e3
    value = ps / (ms_step / 1e3)

    # ---- interface nodes per second at a standard error of 1e-3 (SE-target
    # mode): a pilot of 1e3 paths per node estimates s_i, then each node runs
    # N_i = clamp(ceil(s_i^2 / 1e-6), 1e3, 1e7) paths through the value+Jacobian
    # pass; nodes whose standard error still comes out above 1e-3 (the pilot
    # underestimated s_i) are run again with N_i scaled by (SE_i / 1e-3)^2 and
    # 5% more, up to 1e7, until every node meets the target.  The wall time
    # covers all of it.  Batched FP32 on every node; the plain FP64 one-node-
    # per-launch forward+adjoint on an evenly spaced subset of them.
    def se_target(idx, precision, extra):
        sub = nodes[torch.as_tensor(idx, device=dev)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        pilot = pdd.mc_interface(P, sub, np.full(len(idx), 1000, np.int64), w.dt, w.seed, precision=precision,
                                 coefs=coefs, **extra)
        s2 = pilot["var"].cpu().numpy()
        budget = np.clip(np.ceil(s2 / 1e-6), 1e3, 1e7).astype(np.int64)
        res = pdd.mc_value_jacobian(P, sub, budget, w.dt, w.seed, precision=precision, coefs=coefs, **extra)
        se = res["se"].cpu().numpy()
        rounds, topped = 0, np.zeros(len(idx), bool)
        while True:
            # nodes still above the target get more paths (an independent
            # sample: seed + 1 + round), merged into their estimate
            over = (se > 1e-3) & (budget < 10_000_000)
            if not over.any() or rounds >= 4:
                break
            sel = np.nonzero(over)[0]
            extra_n = np.minimum(10_000_000 - budget[sel],
                                 np.ceil(budget[sel] * ((se[sel] / 1e-3) ** 2 - 1.0) * 1.05) + 64).astype(np.int64)
            r2 = pdd.mc_value_jacobian(P, sub[torch.as_tensor(sel, device=dev)], extra_n, w.dt, w.seed + 1 + rounds,
                                       precision=precision, coefs=coefs, **extra)
            res = pdd.merge_estimates(res, r2, sel)
            se = res["se"].cpu().numpy()
            budget[sel] += extra_n
            topped[sel] = True
            rounds += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return el, budget, {"paths_run": float(budget.sum()) + 1000.0 * len(idx),
                            "path_steps": float(res["steps"].sum().item()), "top_up_rounds": rounds,
                            "topped_up_nodes": int(topped.sum())}, float(se.max())

    k_se = min(args.se_nodes, n)
    idx_se = np.linspace(0, n - 1, k_se).round().astype(int)
    se_target(idx_se[:64], "fp32", dict(schedule="persistent"))        # warm-up
    el_b, budget_b, info_b, se_max_b = se_target(idx_se, "fp32", dict(schedule="persistent"))
    nodes_per_s = k_se / el_b
    log(f"bench: SE-target batched FP32 fwd+adj: {k_se} nodes, {info_b['paths_run']:.3e} paths "
        f"({info_b['top_up_rounds']} top-up rounds, {info_b['topped_up_nodes']} nodes topped up), {el_b:.2f} s "
        f"-> {nodes_per_s:.1f} nodes/s (max SE {se_max_b:.3e})")
    k_pl = min(args.plain_nodes, k_se)
    idx_pl = idx_se[np.linspace(0, k_se - 1, k_pl).round().astype(int)]
    el_p, budget_p, info_p, se_max_p = se_target(idx_pl, "fp64_plain", {})
    plain_nodes_per_s = k_pl / el_p
    plain_ps_s = info_p["path_steps"] / el_p
    log(f"bench: SE-target plain FP64 fwd+adj: {k_pl} nodes, {info_p['paths_run']:.3e} paths, {el_p:.2f} s "
        f"-> {plain_nodes_per_s:.2f} nodes/s (max SE {se_max_p:.3e})")

    fwd_ps_s = ps / fwd_s
    adj_ps_s = ps / adj_s

    # roofline of the dominant kernel: the adjoint walk run by the value+Jacobian
    # call (the call's other kernels take microseconds), algorithmic ops
    dominant = "adjoint"
    ops = ps * OPS_PER_PS_ADJ
    dur = np.median(vj_ms) / 1e3
    achieved = ops / dur / 1e12
    peak = PEAK_LANE_OPS / 1e12

    out = {
        "metric": "path-steps/s (batched FP32 forward+adjoint, C5)",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C5 3-D unit-ball adjoint: 4096 nodes x 1e5 paths, dt=1e-3, fwd+adjoint",
                   "nodes": n, "paths_per_node": int(paths[0]), "dt": w.dt, "seed": w.seed,
                   "schedule": "persistent+hipGraph", "accumulation": "f64",
                   "schedule_forward": sched_f, "schedule_adjoint": sched_a},
        "step": "one value+Jacobian pass (pdd_mc_value_jacobian) + misfit loss and gradient J^T w "
                "(pdd_misfit_gradient)",
        "forward_path_steps_per_s": fwd_ps_s,
        "adjoint_path_steps_per_s": adj_ps_s,
        "forward_plus_recomputing_adjoint_path_steps_per_s": ps / (fwd_s + adj_s),
        "interface_nodes_per_s_at_se_1e-3": nodes_per_s,
        "se_target": {"nodes": k_se, "paths": info_b["paths_run"], "path_steps": info_b["path_steps"],
                      "seconds": el_b, "max_se": se_max_b, "top_up_rounds": info_b["top_up_rounds"],
                      "topped_up_nodes": info_b["topped_up_nodes"],
                      "budget_rule": "pilot 1e3 paths; N_i = clamp(ceil(s_i^2/1e-6), 1e3, 1e7); nodes above SE "
                                     "1e-3 get N_i ((SE_i/1e-3)^2 - 1) x 1.05 + 64 more paths (independent seed, "
                                     "merged; N_i <= 1e7) until all meet it; paths include the pilot's"},
        "plain_se_target": {"nodes": k_pl, "paths": info_p["paths_run"], "path_steps": info_p["path_steps"],
                            "seconds": el_p, "max_se": se_max_p, "top_up_rounds": info_p["top_up_rounds"]},
        "plain_fp64_fwd_adj_nodes_per_s_at_se_1e-3": plain_nodes_per_s,
        "plain_fp64_fwd_adj_path_steps_per_s": plain_ps_s,
        "plain_sample_nodes": k_pl,
        "speedup_vs_plain_fp64_at_se_1e-3": nodes_per_s / plain_nodes_per_s,
        "mean_steps_per_path": float(mean_steps.mean().item()),
        "gpu_clock_during_steps": sclk,
        "roofline": {"bound": "alu", "kernel": f"k_walk ({dominant}, FP32, DIM 3)", "achieved": achieved,
                     "peak": peak, "unit": "Top/s", "frac": achieved / peak, "traffic": traffic_bytes(sched_a),
                     "ops_per_path_step": OPS_PER_PS_ADJ if dominant == "adjoint" else OPS_PER_PS_FWD,
                     "ops_per_path_step_survey_unit": OPS_PER_PS_ADJ_SURVEY,
                     "achieved_survey_unit": ps * OPS_PER_PS_ADJ_SURVEY / dur / 1e12,
                     "frac_survey_unit": ps * OPS_PER_PS_ADJ_SURVEY / dur / 1e12 / peak,
                     "launch_ms": dur * 1e3},
    }
    if args.extras:
        out["other_workloads"] = other_workloads(pdd, dev, tune=args.tune)
    if args.cpu_baseline:
        out["cpu_baseline"], out["fp32_vs_fp64_oracle"] = cpu_baseline(w, args.cpu_seconds, pdd, coefs, dev)
    return out


def cva_problem(pdd, w):
    """The branching problem of a CVA workload, built by the library's
    host-side driver (rescaling by psi_sup, quartic fit, marks); returns
    (problem, scale) with u = scale * the estimate."""
    return pdd.nonlinear.rescaled_problem(w.points.shape[1], w.sigma, w.nonlinearity, w.psi, w.psi_sup, w.T,
                                          beta=w.beta)


def other_workloads(pdd, dev, tune=True):
    """Throughput of the other synthetic workloads (FP32 stepping, the
    library's tuned schedules, cached graphs; one warm-up call each): C3's
    4096-node batch over 8 layouts with variance-targeted budgets in one
    launch, C2's drift/killing/source problem on the disk and C4's KPP
    branching estimator, both at full size; C6, the branching estimator with
    a Dirichlet boundary at 11 output times; C7, the CVA construction."""
    import torch
    from workloads import configs as CF

    last_dev = [0.0]

    def timed(fn):
        """Wall time of the second of two calls (host side included), and in
        last_dev the device time between events recorded on the current
        stream, the library's stream, around it."""
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        last_dev[0] = e0.elapsed_time(e1) / 1e3
        return r, time.perf_counter() - t

    res = {}
    from paper_1705_03666_amd import autotune
    # C3: 4096 nodes over 8 layouts (2-D and 3-D, box, disk and ball) in one
    # persistent launch per call, the library's tuned batch schedule
    cb = CF.c3_batch()
    nb = torch.tensor(cb.nodes, device=dev)
    if tune:
        autotune.tune_batch(cb.problems, cb.node_problem, nb, cb.paths, cb.dt, cb.seed, "fp32", log=log)
        autotune.tune_batch(cb.problems, cb.node_problem, nb, cb.paths, 1e-4, cb.seed, "fp32", wos=True, log=log)

    def err_se(r):
        z = np.abs(r["mean"].cpu().numpy() - cb.exact) / r["se"].cpu().numpy()
        return float(z.max()), float(np.sqrt(np.mean(z ** 2)))

    run_c3 = lambda: pdd.mc_interface_batch(cb.problems, cb.node_problem, nb, cb.paths, cb.dt, cb.seed,
                                            precision="fp32")
    rb, el = timed(run_c3)
    ps = float(rb["steps"].sum().item())
    nn = len(cb.paths)
    zmax, zrms = err_se(rb)
    res["c3_batch"] = {"nodes": nn, "paths": int(cb.paths.sum()), "path_steps": ps, "seconds": el,
                       "device_seconds": last_dev[0],
                       "path_steps_per_s": ps / el, "nodes_per_s": nn / el, "launches": 1,
                       "schedule": pdd.get_schedule("walk_batch", 0, "fp32"),
                       "err_vs_exact_max_se": zmax, "err_vs_exact_rms_se": zrms}
    log(f"bench: C3 batch (Euler, one launch): {nn} nodes in {el * 1e3:.1f} ms, {ps / el:.3e} path-steps/s, "
        f"error vs exact max {zmax:.1f} SE, rms {zrms:.1f} SE")
    # the same batch with the boundary-corrected exit test: the O(sqrt dt)
    # exit bias that dominates the plain test's error at this budget
    rbc, elc = timed(lambda: pdd.mc_interface_batch(cb.problems, cb.node_problem, nb, cb.paths, cb.dt, cb.seed,
                                                    precision="fp32", boundary_correction=True))
    # nodes closer to the boundary than the shift c0 sigma sqrt(dt) exit at
    # once with phi = g(P x): no spread (SE 0), so their error is reported in
    # absolute terms, the others' in SE units
    mc, sc = rbc["mean"].cpu().numpy(), rbc["se"].cpu().numpy()
    band = sc == 0.0
    zc = np.abs(mc[~band] - cb.exact[~band]) / sc[~band]
    res["c3_batch"]["corrected"] = {"seconds": elc, "path_steps_per_s": float(rbc["steps"].sum().item()) / elc,
                                    "err_vs_exact_max_se": float(zc.max()),
                                    "err_vs_exact_rms_se": float(np.sqrt(np.mean(zc ** 2))),
                                    "nodes_exiting_at_start": int(band.sum()),
                                    "their_max_abs_err": float(np.abs(mc[band] - cb.exact[band]).max()) if band.any()
                                    else 0.0}
    log(f"bench: C3 batch, boundary-corrected: {elc * 1e3:.1f} ms, error vs exact max {zc.max():.1f} SE, "
        f"rms {np.sqrt(np.mean(zc ** 2)):.1f} SE ({int(band.sum())} nodes inside the shift exit at once)")

    # the same batch by walk on spheres (b = c = f = 0), eps = 1e-4
    run_c3_wos = lambda: pdd.wos_interface_batch(cb.problems, cb.node_problem, nb, cb.paths, 1e-4, cb.seed,
                                                 precision="fp32")
    rw, elw = timed(run_c3_wos)
    jumps = float(rw["steps"].sum().item())
    zmax, zrms = err_se(rw)
    res["c3_batch_walk_on_spheres"] = {"eps": 1e-4, "jumps": jumps, "seconds": elw, "device_seconds": last_dev[0],
                                       "jumps_per_s": jumps / elw,
                                       "nodes_per_s": nn / elw, "launches": 1,
                                       "schedule": pdd.get_schedule("wos_batch", 0, "fp32"),
                                       "err_vs_exact_max_se": zmax, "err_vs_exact_rms_se": zrms}
    log(f"bench: C3 batch (walk on spheres, one launch): {elw * 1e3:.1f} ms, {jumps / elw:.3e} jumps/s, "
        f"error vs exact max {zmax:.1f} SE, rms {zrms:.1f} SE")
    # C2 at its full size (256 nodes x 1e6 paths, dt = 1e-4); the first call
    # also compiles the problem-specialised kernel (timed separately)
    c2 = CF.c2()
    n2 = torch.tensor(c2.nodes, device=dev)
    c2call = lambda: pdd.mc_interface(c2.problem, n2, c2.paths, c2.dt, c2.seed, precision="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c2call()
    torch.cuda.synchronize()
    first2 = time.perf_counter() - t0
    r2, el2 = timed(c2call)
    ps2 = float(r2["steps"].sum().item())
    z2 = np.abs(r2["mean"].cpu().numpy() - CF.c2_exact(c2.nodes)) / r2["se"].cpu().numpy()
    res["c2"] = {"nodes": len(c2.paths), "paths_per_node": int(c2.paths[0]), "dt": c2.dt, "path_steps": ps2,
                 "seconds": el2, "device_seconds": last_dev[0], "path_steps_per_s": ps2 / el2,
                 "nodes_per_s": len(c2.paths) / el2,
                 "first_call_seconds_incl_kernel_compile": first2, "max_se": float(r2["se"].max().item()),
                 "err_vs_exact_max_se": float(z2.max()), "err_vs_exact_rms_se": float(np.sqrt(np.mean(z2 ** 2)))}
    log(f"bench: C2: {ps2:.3e} path-steps in {el2 * 1e3:.1f} ms, {ps2 / el2:.3e} path-steps/s (first call "
        f"{first2:.2f} s); error vs exact max {z2.max():.1f} SE, rms {np.sqrt(np.mean(z2 ** 2)):.1f} SE")
    r2c, el2c = timed(lambda: pdd.mc_interface(c2.problem, n2, c2.paths, c2.dt, c2.seed, precision="fp32",
                                               boundary_correction=True))
    z2c = np.abs(r2c["mean"].cpu().numpy() - CF.c2_exact(c2.nodes)) / r2c["se"].cpu().numpy()
    res["c2"]["corrected"] = {"seconds": el2c, "path_steps_per_s": float(r2c["steps"].sum().item()) / el2c,
                              "err_vs_exact_max_se": float(z2c.max()),
                              "err_vs_exact_rms_se": float(np.sqrt(np.mean(z2c ** 2)))}
    log(f"bench: C2, boundary-corrected: error vs exact max {z2c.max():.1f} SE, rms {np.sqrt(np.mean(z2c ** 2)):.1f} SE")
    # boundary-corrected exit test vs the plain one: C1 (harmonic data, exact
    # u = g) at dt = 4e-3 with 1e6 FP32 paths per node; error in SE units
    c1 = CF.c1(scale=100.0, dt=4e-3)
    n1 = torch.tensor(c1.nodes, device=dev)
    exact = CF.c1_exact(c1.nodes)
    acc = {}
    for name, corr in (("plain", False), ("corrected", True)):
        r1, el1 = timed(lambda: pdd.mc_interface(c1.problem, n1, c1.paths, c1.dt, c1.seed, precision="fp32",
                                                 boundary_correction=corr))
        err = np.abs(r1["mean"].cpu().numpy() - exact) / r1["se"].cpu().numpy()
        acc[name] = {"max_err_se": float(err.max()), "mean_err_se": float(err.mean()),
                     "path_steps_per_s": float(r1["steps"].sum().item()) / el1}
    res["c1_boundary_correction_dt_4e-3"] = acc
    log(f"bench: C1 dt=4e-3 error vs exact (SE units): plain max {acc['plain']['max_err_se']:.1f}, "
        f"corrected max {acc['corrected']['max_err_se']:.1f}")
    c4 = CF.c4()
    p4 = torch.tensor(c4.points, device=dev)
    if tune:
        autotune.tune_branching(c4.problem, p4, c4.trees, c4.seed, "fp32", log=log)
    r4, el4 = timed(lambda: pdd.branching_eval(c4.problem, p4, c4.trees, c4.seed, precision="fp32"))
    segs = float(r4["steps"].sum().item())
    trees = float(len(c4.points) * c4.trees)
    res["c4"] = {"points": len(c4.points), "trees_per_point": c4.trees, "segments": segs, "seconds": el4,
                 "device_seconds": last_dev[0],
                 "trees_per_s": trees / el4, "segments_per_s": segs / el4,
                 "schedule": pdd.get_schedule("branch", 3, "fp32")}
    log(f"bench: C4: {trees:.3e} trees, {segs:.3e} segments in {el4 * 1e3:.1f} ms")
    # C7: the CVA construction of Sec. 3.3 (signed quartic, marks q ~ |alpha|),
    # 1024 points x 1e5 trees, compared with the method-of-lines solution of
    # the same polynomial PDE
    c7 = CF.c7()
    prob7, scale7 = cva_problem(pdd, c7)
    p7 = torch.tensor(c7.points, device=dev)
    if tune:
        autotune.tune_branching(prob7, p7, c7.trees, c7.seed, "fp32", log=log)
    r7, el7 = timed(lambda: pdd.branching_eval(prob7, p7, c7.trees, c7.seed, precision="fp32"))
    segs7 = float(r7["steps"].sum().item())
    ref7 = CF.c7_reference(c7.points[:, 0])
    z7 = np.abs(scale7 * r7["mean"].cpu().numpy() - ref7) / (scale7 * r7["se"].cpu().numpy())
    res["c7_cva_marked"] = {"points": len(c7.points), "trees_per_point": c7.trees, "segments": segs7,
                            "seconds": el7, "device_seconds": last_dev[0],
                            "trees_per_s": len(c7.points) * c7.trees / el7,
                            "segments_per_s": segs7 / el7, "err_vs_pde_max_se": float(z7.max()),
                            "err_vs_pde_rms_se": float(np.sqrt(np.mean(z7 ** 2)))}
    log(f"bench: C7 (CVA, marked signed quartic): {len(c7.points) * c7.trees:.3e} trees, {segs7:.3e} segments in "
        f"{el7 * 1e3:.1f} ms; error vs PDE solve max {z7.max():.1f} SE, rms {np.sqrt(np.mean(z7 ** 2)):.1f} SE")
    # C6: KPP with a Dirichlet boundary and 11 output times (eq. 3.2,
    # Algorithm 3.1); the travelling wave is the exact solution
    c6 = CF.c6()
    p6 = torch.tensor(c6.points, device=dev)
    if tune:
        autotune.tune_branching(c6.problem, p6, c6.trees, c6.seed, "fp32", boundary=c6.boundary, log=log)
    r6, el6 = timed(lambda: pdd.branching_bvp(c6.problem, c6.boundary, p6, c6.trees, c6.seed, precision="fp32"))
    sub = float(r6["steps"][0].sum().item())
    tr6 = float(len(c6.points) * c6.trees)
    ex6 = np.array([CF.travelling_wave(c6.points[:, 0], t) for t in c6.boundary.times])
    z6 = (np.abs(r6["mean"].cpu().numpy() - ex6) / np.maximum(r6["se"].cpu().numpy(), 1e-300))[1:]
    res["c6_branching_boundary"] = {"points": len(c6.points), "trees_per_point": c6.trees,
                                    "output_times": len(c6.boundary.times), "dt": c6.boundary.dt,
                                    "particle_substeps": sub, "seconds": el6, "device_seconds": last_dev[0],
                                    "trees_per_s": tr6 / el6,
                                    "substeps_per_s": sub / el6, "schedule": pdd.get_schedule("branch_bvp", 1, "fp32"),
                                    "err_vs_exact_max_se": float(z6.max()),
                                    "err_vs_exact_rms_se": float(np.sqrt(np.mean(z6 ** 2)))}
    log(f"bench: C6: {tr6:.3e} trees x {len(c6.boundary.times)} times, {sub:.3e} particle sub-steps in "
        f"{el6 * 1e3:.1f} ms ({sub / el6:.3e}/s); error vs exact max {z6.max():.1f} SE, "
        f"rms {np.sqrt(np.mean(z6 ** 2)):.1f} SE")
    r6c, el6c = timed(lambda: pdd.branching_bvp(c6.problem, c6.boundary, p6, c6.trees, c6.seed, precision="fp32",
                                                boundary_correction=True))
    z6c = (np.abs(r6c["mean"].cpu().numpy() - ex6) / np.maximum(r6c["se"].cpu().numpy(), 1e-300))[1:]
    res["c6_branching_boundary"]["corrected"] = {"seconds": el6c, "err_vs_exact_max_se": float(z6c.max()),
                                                 "err_vs_exact_rms_se": float(np.sqrt(np.mean(z6c ** 2)))}
    log(f"bench: C6 with the per-sub-step boundary correction: {el6c * 1e3:.1f} ms; error vs exact max "
        f"{z6c.max():.1f} SE, rms {np.sqrt(np.mean(z6c ** 2)):.1f} SE")
    return res


def run_only(name, scale):
    """One workload of the other_workloads section, called twice (the first
    call of C2 also compiles its specialised kernel); for profiler runs."""
    import torch
    import paper_1705_03666_amd as pdd
    from workloads import configs as CF
    dev = "cuda"
    if name in ("c3", "c3wos"):
        cb = CF.c3_batch(scale=scale)
        nb = torch.tensor(cb.nodes, device=dev)
        if name == "c3":
            call = lambda: pdd.mc_interface_batch(cb.problems, cb.node_problem, nb, cb.paths, cb.dt, cb.seed,
                                                  precision="fp32")
        else:
            call = lambda: pdd.wos_interface_batch(cb.problems, cb.node_problem, nb, cb.paths, 1e-4, cb.seed,
                                                   precision="fp32")
        work = lambda r: float(r["steps"].sum().item())
        unit = "path_steps" if name == "c3" else "jumps"
    elif name == "c2":
        w = CF.c2(scale=scale)
        nd = torch.tensor(w.nodes, device=dev)
        call = lambda: pdd.mc_interface(w.problem, nd, w.paths, w.dt, w.seed, precision="fp32")
        work = lambda r: float(r["steps"].sum().item())
        unit = "path_steps"
    elif name in ("c4", "c7"):
        w = CF.c4(scale=scale) if name == "c4" else CF.c7(scale=scale)
        prob = w.problem if name == "c4" else cva_problem(pdd, w)[0]
        pt = torch.tensor(w.points, device=dev)
        call = lambda: pdd.branching_eval(prob, pt, w.trees, w.seed, precision="fp32")
        work = lambda r: float(r["steps"].sum().item())
        unit = "segments"
    else:
        w = CF.c6(scale=scale)
        pt = torch.tensor(w.points, device=dev)
        call = lambda: pdd.branching_bvp(w.problem, w.boundary, pt, w.trees, w.seed, precision="fp32")
        work = lambda r: float(r["steps"][0].sum().item())
        unit = "particle_substeps"
    for i in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = call()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n = work(r)
        print(json.dumps({"workload": name.upper(), "call": i + 1, unit: n, "seconds": el,
                          unit + "_per_s": n / el}), flush=True)


def host_cpu():
    """(threads to use, description) of the host CPU share this process may
    use: the CPUs in its affinity mask, bounded by a cgroup CPU quota and by
    OMP_NUM_THREADS when either is set, and the CPU model."""
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    omp = os.environ.get("OMP_NUM_THREADS")
    limits = [affinity] + ([quota] if quota else []) + ([int(omp)] if omp and omp.isdigit() and int(omp) > 0 else [])
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(limits), {"model": model, "affinity_cpus": affinity, "cgroup_quota_cpus": quota,
                         "omp_num_threads": omp, "os_cpu_count": os.cpu_count()}


def cpu_baseline(w, seconds, pdd, coefs, dev):
    """The FP64 oracle (forward + adjoint) on a bounded sample of the same
    workload, timed on the host's CPU share; the GPU FP32 path is then run on
    the same sample (same nodes, paths and seed) and its node values and
    gradient are compared with the oracle's."""
    import torch
    import oracle
    threads, cpu = host_cpu()
    P = w.problem_template
    # calibrate on a tiny sample, then size the sample for ~`seconds`
    nc = 2 * threads
    idx = np.linspace(0, len(w.nodes) - 1, nc).round().astype(int)
    pa = np.full(nc, 200, np.int64)
    t = time.perf_counter()
    r = oracle.walk_adjoint(P, w.nodes[idx], pa, w.dt, w.seed, np.ones(nc), layout=oracle.QUAD24,
                            n_threads=threads)
    rate = r["stats"]["steps"].sum() / (time.perf_counter() - t)
    per_node = max(200, int(seconds * rate / (4 * threads) / 180.0))
    nn = 4 * threads
    idx = np.linspace(0, len(w.nodes) - 1, nn).round().astype(int)
    pa = np.full(nn, per_node, np.int64)
    log(f"bench: cpu baseline: oracle fwd+adjoint on {nn} nodes x {per_node} paths, {threads} threads")
    t = time.perf_counter()
    r = oracle.walk_adjoint(P, w.nodes[idx], pa, w.dt, w.seed, np.ones(nn), layout=oracle.QUAD24,
                            n_threads=threads)
    el = time.perf_counter() - t
    ps = float(r["stats"]["steps"].sum())
    base = {"value": ps / el, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"C5 forward+adjoint, {nn} nodes x {per_node} paths ({ps:.3e} path-steps, {el:.1f} s), FP64",
            "cpu": cpu}
    # error of the FP32-stepping GPU path against the FP64 oracle on this sample
    sub = torch.tensor(w.nodes[idx], device=dev)
    g = pdd.mc_adjoint(P, sub, pa, w.dt, w.seed, torch.ones(nn, dtype=torch.float64, device=dev), precision="fp32",
                       coefs=coefs, with_stats=True)
    mean_g = g["stats"]["mean"].cpu().numpy()
    om = r["stats"]["mean"]
    se = np.sqrt(r["stats"]["m2"] / (r["stats"]["n"] - 1) / r["stats"]["n"])
    z = np.abs(mean_g - om) / se
    grad_err = {}
    for k in ("g_poly", "f_poly", "c_poly"):
        a, b = g[k].cpu().numpy(), np.asarray(r[k])
        grad_err[k] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    err = {"nodes": nn, "paths_per_node": per_node, "mean_err_max_se": float(z.max()),
           "mean_err_rms_se": float(np.sqrt(np.mean(z ** 2))), "gradient_rel_l2_err": grad_err}
    log(f"bench: FP32 GPU vs FP64 oracle: node values max {z.max():.3f} SE, rms {np.sqrt(np.mean(z ** 2)):.3f} SE; "
        f"gradient rel err {grad_err}")
    return base, err


def reap_children(timeout: float = 10.0) -> int:
    """Waits for (then ends) every child process this run started, so none
    outlives it; returns how many were still there.  The only children the
    bench itself starts are short host commands run to completion (uname for
    the CPU name, amd-smi when sysfs has no clock table)."""
    try:
        import psutil
    except ImportError:
        return -1
    kids = psutil.Process().children(recursive=True)
    if kids:
        _, alive = psutil.wait_procs(kids, timeout=timeout)
        for p in alive:
            p.terminate()
        psutil.wait_procs(alive, timeout=timeout)
    return len(kids)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0, help="path budget scale (1 = 1e5 paths/node)")
    ap.add_argument("--nodes", type=int, default=4096)
    ap.add_argument("--plain-nodes", type=int, default=32, help="plain FP64 nodes in the SE-target comparison")
    ap.add_argument("--se-nodes", type=int, default=4096, help="nodes in the SE-target run")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--no-extras", dest="extras", action="store_false", help="skip the C2/C3/C4 throughput lines")
    ap.add_argument("--no-tune", dest="tune", action="store_false", help="use the default schedule")
    ap.add_argument("--schedule-adj", default="", help="blocks_per_cu,refill_groups,chunk_paths (skips tuning)")
    ap.add_argument("--schedule-fwd", default="", help="as --schedule-adj, for the forward kernel")
    ap.add_argument("--steps-only", action="store_true",
                    help="run only the timed value+Jacobian steps (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 256 MiB (reference for the FETCH/WRITE counters)")
    ap.add_argument("--c2-only", action="store_true",
                    help="only run C2 at full size twice (the first call compiles its kernel; for profiler runs)")
    ap.add_argument("--c6-only", action="store_true",
                    help="only run C6 (branching with a boundary, 11 output times) twice (for profiler runs)")
    ap.add_argument("--only", default="", choices=["", "c2", "c3", "c3wos", "c4", "c6", "c7"],
                    help="only run this workload at full size (times --scale) twice, one JSON line per call "
                         "(for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library drives a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}), flush=True)
        return
    if args.c2_only:
        args.only = "c2"
    if args.c6_only:
        args.only = "c6"
    if args.only:
        run_only(args.only, args.scale)
        return
    out = run(args)
    out["child_processes_at_exit"] = reap_children()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
