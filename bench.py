"""Benchmark: propagated edges/s of Kino-PAX+ queries on one MI355X.

A step is one query: a planner run of --iters iterations (select ->
propagate -> prune -> insert, 200 by default) from the root, on the seeded
scene of that query.  --steps queries (seeds 0 .. steps-1) are timed after
--warmup untimed ones; each query's tree and scene are resident in HBM before
its run starts, and every count stays on the device.

value = the median over the timed queries of that query's propagated edges
(every expansion integrated, valid or not: the sum over its iterations of
selected nodes x samples per node) divided by its device-timed span (the
device wall clock from the first iteration's start to the last one's end).
The default workload is the 12D quadrotor (4096 nodes x 32 samples per
iteration, 64-box wall with two slots, 16^3 x 2^3 regions, tree capacity 2^21).

`roofline` covers the dominant kernel (propagate, bound by float32 ALU work),
from HIP events around the kernels of every `--timing-every`-th iteration of
the timed queries; `steady_state` repeats the measurement over a window of
iterations in which the selection is full; `cpu_baseline` is the float64
oracle running the first query from its root on every host core (and on one).
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic float32 FLOPs of one RK4 substep (FMA = 2, each transcendental,
# reciprocal or square root = 1): 13 per integrated component for the stage
# and combination updates plus four evaluations of f.
#   DI6      6 components, f has no arithmetic                  -> 78
#   QUAD12  12 components, f = 6 sin/cos + 1 rcp + 35 mul/FMA   -> 156 + 4 * 42 = 324
#   DUBINS6  6 components, f = 4 sin/cos + 4 mul                 -> 78 + 4 * 8 = 110
# The path-length cost integrates one more component and its rate
# (speed: 3 FMA-equivalents + sqrt for DI6/QUAD12, none for DUBINS6).
FLOPS_PER_SUBSTEP = {
    ("DI6", "TIME"): 78, ("DI6", "PATH_LENGTH"): 78 + 13 + 4 * 6,
    ("QUAD12", "TIME"): 324, ("QUAD12", "PATH_LENGTH"): 324 + 13 + 4 * 6,
    ("DUBINS6", "TIME"): 110, ("DUBINS6", "PATH_LENGTH"): 110 + 13,
}
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 FLOP/clk, packed)
PEAK_FP32_UNPACKED = 78.6     # ... without packed FP32 (the kernels are compiled without it)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2602_02846_amd/csrc/kpx.hip", "paper_2602_02846_amd/csrc/kpx_device.hpp")
KERNELS = ("propagate", "prune_flags", "insert", "finalize_select")
DIMS = {"DI6": (6, 3), "QUAD12": (12, 4), "DUBINS6": (6, 3)}
BUDGETS_MS = (5.0, 10.0, 20.0, 40.0)
# the small-delta workloads (10^8 slots) take 7 to 50 ms per iteration
BUDGETS_SMALL_DELTA_MS = (200.0, 500.0, 1000.0, 2000.0)


def budgets_for(workload):
    return BUDGETS_SMALL_DELTA_MS if workload.endswith("_paper_small") else BUDGETS_MS


def kernel_bytes(prob, prm, st):
    """Algorithmic bytes per launch of each iteration kernel, per iteration of
    the stats records `st` (what the step must read and write, not what this
    implementation happens to move):
      prune_flags  every region: table key 8 + activity byte 1; every region a
                   tree node still owns: status and I_count read and written 4;
                   every survivor (named by its region's key): survivor byte 1,
                   and its tile's count 4 per tile holding one (the ancestor
                   checks of Alg. 3 are left out: a lower bound)
      insert       every slot: survivor byte 1; per 256-slot tile: count 4;
                   every survivor: end state 4d, key 8, region 4, parent 4
                   read; state 4d, control 4m, steps 2, parent 4, cost 4,
                   region 4, status 1, I_count 1, table entry 8 written
      finalize     every region: activity 1 + owner 4; every selected node
                   of the next iteration: its index 4"""
    d, m = DIMS[prob.dynamics]
    cells = float(prm.n_cells)
    S = st["n_select"].astype(np.float64) * st["samples_per_node"]
    ns = st["n_survivors"].astype(np.float64)
    nl = st["n_live"].astype(np.float64)
    nsel_next = np.append(st["n_select"][1:], st["n_select"][-1:]).astype(np.float64)
    prune = cells * 9 + nl * 4 + ns + np.minimum(ns, np.ceil(S / 256)) * 4
    insert = S + np.ceil(S / 256) * 4 + ns * (4 * d + 16 + 4 * d + 4 * m + 28)
    final = cells * 5 + nsel_next * 4
    return {"prune_flags": prune, "insert": insert, "finalize_select": final}


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def bench_args_key(a):
    """The arguments that decide which kernels run (a counter profile of the
    same command covers the same launches)."""
    return (f"--workload {a.workload} --steps {a.steps} --warmup {a.warmup} --iters {a.iters}"
            + (f" --cost {a.cost}" if a.cost else "")
            + (f" --polish {a.polish}" if a.polish else "") + (" --polish-goal-only" if a.polish_goal_only else "")
            + (" --cost-first" if a.cost_first else "")
            + (f" --refine-at {a.refine_at}" if a.refine_at else "")
            + (f" --timing-every {a.timing_every}" if a.timing_every != 16 else ""))


def profile_fields(a, kind):
    """key: value lines of the committed profile summary profiles/<workload>_<kind>.txt,
    or None unless it was taken on the current kernel sources with the same
    bench arguments."""
    path = os.path.join(ROOT, "profiles", f"{a.workload}_{kind}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            k, sep, v = line.partition(":")
            if sep:
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != source_sha() or fields.get("bench_args") != bench_args_key(a):
        return None
    return fields


def measured_trace(a):
    """Average kernel-trace duration (us) per launch of each iteration kernel
    over the timed queries, from the committed rocprofv3 summary of the same
    command, or None."""
    f = profile_fields(a, "kernel_trace")
    if f is None:
        return None
    out = {}
    for k in KERNELS:
        try:
            out[k] = float(f[f"{k}_trace_us_per_launch"])
        except (KeyError, ValueError):
            pass
    return out or None


def measured_traffic(a):
    """HBM bytes per launch of each iteration kernel from the committed
    rocprofv3 counter summary of the same bench command (FETCH_SIZE and
    WRITE_SIZE, calibrated against a plain copy), or None when there is none,
    the kernel sources changed since it was taken or it profiled other
    arguments."""
    fields = profile_fields(a, "traffic")
    if fields is None:
        return None
    out = {}
    for k in KERNELS:
        try:
            out[k] = int(fields[f"{k}_hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            pass
    return out or None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed queries: seeds 0 .. steps-1, each a run of --iters iterations")
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed queries before them (seeds 0 .. warmup-1 on planners of their own)")
    ap.add_argument("--iters", type=int, default=200, help="iterations of every query")
    ap.add_argument("--workload", default="quad12",
                    choices=["di6", "quad12", "dubins6", "di6_paper", "quad12_paper", "dubins6_paper",
                             "di6_paper_small", "quad12_paper_small", "dubins6_paper_small",
                             "batch256", "diff65536"])
    ap.add_argument("--queries", type=int, default=256, help="queries of the batch256 workload")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch256: skip the sequential per-query comparison")
    ap.add_argument("--seed", type=int, default=0, help="batch256 and diff65536: scene seed")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="bound on the oracle CPU-baseline sample on every host core")
    ap.add_argument("--cpu-seconds-single", type=float, default=8.0,
                    help="bound on the oracle sample on one core")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--polish", type=int, default=0,
                    help="edge polish steps of every inserted node (quadrotor); 0 = plain")
    ap.add_argument("--polish-w-len", type=float, default=1.0,
                    help="weight of the path length in the polish loss (path-length cost)")
    ap.add_argument("--polish-goal-only", action="store_true",
                    help="polish only the nodes inserted in the goal set")
    ap.add_argument("--cost", choices=["TIME", "PATH_LENGTH"], default=None,
                    help="the workload's cost instead of its own")
    ap.add_argument("--cost-first", action="store_true",
                    help="propagate in the exact cost-first form (obstacle tests only for edges "
                         "that can still be their region's minimum)")
    ap.add_argument("--tree-growth", type=int, default=0,
                    help="also run the first query this many iterations and time every kernel in "
                         "windows as the tree grows (prune and insert against tree size)")
    ap.add_argument("--refine-at", type=int, default=0,
                    help="halve the region cells per axis after this many iterations of each query")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--timing-every", type=int, default=16,
                    help="bracket the kernels with HIP events in every n-th iteration of each query")
    ap.add_argument("--steady-window", type=int, default=20,
                    help="iterations of the steady-state window (0: none)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported "
              "(a planner query runs on a single device)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2602_02846_amd as K

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    K.lib()  # fails loudly when the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_bytes > 0:
        src = torch.ones(a.copy_bytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "batch256":
        return bench_batch(a)
    if a.workload == "diff65536":
        return bench_diff(a)
    return bench_queries(a)


def key_cost(key, cost_kind, dt):
    """Cost of a solution key: the high word is the total RK4 step count
    (TIME cost, times dt) or the float32 bits of the path length."""
    field = int(key) >> 32
    if cost_kind == "TIME":
        return field * dt
    return float(np.array([field], np.uint32).view(np.float32)[0])


def make_workload(W, a, seed):
    return W.make_workload(a.workload, seed, **({"cost": a.cost} if a.cost else {}))


def make_planner(K, W, a, seed, polish):
    w = make_workload(W, a, seed)
    if a.refine_at:
        w.params.refine_max = 2
    p = K.Planner(w.problem, w.params)
    if polish:
        p.set_polish(polish, w_len=a.polish_w_len if w.problem.cost == "PATH_LENGTH" else 0.0,
                     goal_only=a.polish_goal_only)
    if a.cost_first:
        p.set_cost_first(True)
    return w, p


def run_query(p, a):
    """Enqueues one query's run (with the optional mid-run refinement)."""
    if 0 < a.refine_at < a.iters:
        p.iterate(a.refine_at)
        p.refine(2)
        p.iterate(a.iters - a.refine_at)
    else:
        p.iterate(a.iters)


def run_queries(K, W, a, polish, timing):
    """Runs the timed queries one after another (each created, with its scene
    uploaded, before its timed run) and gathers per-query device-timed rates,
    solutions, cost at budgets and the sampled per-kernel times."""
    import torch

    from paper_2602_02846_amd.autotune import first_solution_ms

    for s in range(a.warmup):
        _, p = make_planner(K, W, a, s, polish)
        run_query(p, a)
        p.sync()
        p.close()
    rates, spans, edges_all, iters_all, wall, full = [], [], 0, 0, 0.0, 0
    t_first, costs, unsolved = [], [], []
    budgets = budgets_for(a.workload)
    at_budget = {b: [] for b in budgets}
    ksum = {k: 0.0 for k in KERNELS}
    klaunch = {k: 0 for k in KERNELS}
    flops = 0.0
    kbytes = {k: 0.0 for k in KERNELS[1:]}
    w = None
    for seed in range(a.steps):
        w, p = make_planner(K, W, a, seed, polish)
        if timing:
            p.set_timing(True, every=a.timing_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_query(p, a)
        p.sync()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        c = p.counters()
        done = int(c["iteration"])
        full += int(c["full"])
        st = p.stats(0, done)
        rate_hz = p.clock_rate_khz() * 1e3
        e = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
        span = (int(st["t_end"][-1]) - int(st["t_begin"][0])) / rate_hz
        rates.append(e / span)
        spans.append(span)
        edges_all += e
        iters_all += done
        t = first_solution_ms(p, a.iters)
        if t is not None:
            t_first.append(t)
            costs.append(p.solution()["cost"])
        else:
            unsolved.append(seed)
        t_ms = (st["t_end"].astype(np.float64) - float(st["t_begin"][0])) / rate_hz * 1e3
        for b in budgets:
            keys = st["solution_key"][t_ms <= b]
            best = int(keys.min()) if keys.size else (1 << 64) - 1
            at_budget[b].append(np.inf if best == (1 << 64) - 1 else key_cost(best, w.problem.cost, w.params.dt))
        if timing:
            ms, launches = p.read_timing()
            # the bracketed launches are those of iterations 0, E, 2E, ... that ran
            idx = np.arange(0, done, a.timing_every)
            n_t = min(len(idx), launches[0])
            if n_t == launches[0] and all(n == launches[0] for n in launches):
                idx = idx[:n_t]
                for i, k in enumerate(KERNELS):
                    ksum[k] += ms[i]
                    klaunch[k] += launches[i]
                flops += FLOPS_PER_SUBSTEP[(w.problem.dynamics, w.problem.cost)] * float(st["substeps"][idx].sum())
                kb = kernel_bytes(w.problem, w.params, st)
                for k in kbytes:
                    kbytes[k] += float(kb[k][idx].sum())
        p.close()
        if seed % 10 == 9:
            print(f"[bench] {seed + 1} queries timed", file=sys.stderr, flush=True)
    sols = {
        "queries": a.steps, "iterations": a.iters, "polish_steps": polish, "refine_at": a.refine_at,
        "solved": len(t_first), "unsolved_seeds": unsolved,
        "time_to_first_solution_ms_median": round(float(np.median(t_first)), 3) if t_first else None,
        "cost_median": round(float(np.median(costs)), 4) if costs else None,
        "cost_at_budget_median": {f"{b:g}ms": (None if not np.isfinite(np.median(v)) else
                                               round(float(np.median(v)), 4)) for b, v in at_budget.items()},
        "solved_at_budget": {f"{b:g}ms": int(np.isfinite(v).sum()) for b, v in at_budget.items()},
        "cost_unit": "s" if w.problem.cost == "TIME" else "length",
    }
    return {"rates": rates, "spans": spans, "edges": edges_all, "iterations": iters_all, "wall": wall,
            "full": full, "solutions": sols, "ksum": ksum, "klaunch": klaunch, "flops": flops,
            "kbytes": kbytes, "w": w}


def roofline_of(flops, ms, launches, traffic=None):
    if not launches or ms <= 0:
        return None
    achieved = flops / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "frac_of_unpacked_peak": round(achieved / PEAK_FP32_UNPACKED, 4),
            "launches": launches, "flops_per_launch": round(flops / launches, 1)}


def kernels_summary(ksum, klaunch, kbytes, traffic, trace=None):
    """Per iteration kernel: HIP-event microseconds per launch (which include
    the dispatch around the kernel, a few us), the kernel-trace time of the
    committed profile of the same command when there is one, and for prune,
    insert and finalize their algorithmic bytes per launch and the rate at
    either time."""
    out = {}
    for k in KERNELS:
        if not klaunch[k]:
            continue
        us = ksum[k] / klaunch[k] * 1e3
        e = {"us": round(us, 3)}
        if trace and k in trace:
            e["trace_us"] = round(trace[k], 3)
        if k in kbytes:
            b = kbytes[k] / klaunch[k]
            e["algorithmic_bytes_per_launch"] = round(b)
            e["algorithmic_gbs"] = round(b / us / 1e3, 2)
            e["frac_of_hbm"] = round(b / us / 1e3 / PEAK_HBM_GBS, 4)
            if trace and k in trace:
                e["algorithmic_gbs_trace"] = round(b / trace[k] / 1e3, 2)
                e["frac_of_hbm_trace"] = round(b / trace[k] / 1e3 / PEAK_HBM_GBS, 4)
        if traffic and k in traffic:
            e["counter_bytes_per_launch"] = traffic[k]
            if k in kbytes:
                e["counter_over_algorithmic"] = round(traffic[k] / (kbytes[k] / klaunch[k]), 2)
        out[k] = e
    return out


def steady_state(K, W, a, polish):
    """The first query once its selection is full: per-kernel HIP-event times
    and the propagate roofline over a window of iterations."""
    w, p = make_planner(K, W, a, 0, polish)
    target = w.params.n_select if w.params.samples_per_node else None
    done = 0
    while done < 400:
        p.iterate(5)
        done += 5
        c = p.counters()
        if c["full"] or target is None or int(c["n_select"]) >= target:
            break
    c0 = p.counters()
    if c0["full"] or (target is not None and int(c0["n_select"]) < target):
        p.close()
        return None
    p.set_timing(True, every=1)
    p.iterate(a.steady_window)
    p.sync()
    c1 = p.counters()
    n = int(c1["iteration"] - c0["iteration"])
    ms, launches = p.read_timing()
    st = p.stats(int(c0["iteration"]), n)
    p.close()
    if n != a.steady_window or launches[0] != n:
        return None
    e = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
    fl = FLOPS_PER_SUBSTEP[(w.problem.dynamics, w.problem.cost)] * float(st["substeps"].sum())
    kb = kernel_bytes(w.problem, w.params, st)
    return {"first_iteration": int(c0["iteration"]), "iterations": n,
            "edges_per_iteration": e // n, "substeps_per_iteration": int(st["substeps"].sum()) // n,
            "note": "HIP events around every kernel of every iteration of the window",
            "kernels": kernels_summary(dict(zip(KERNELS, ms)), dict(zip(KERNELS, launches)),
                                       {k: float(v.sum()) for k, v in kb.items()}, None),
            "roofline": roofline_of(fl, ms[0], launches[0])}


def bench_queries(a):
    import paper_2602_02846_amd as K
    import workloads as W

    w0 = make_workload(W, a, 0)
    prob, prm = w0.problem, w0.params
    print(f"[bench] {a.workload}: {prm.n_select} x {prm.samples_per_node} slots, {prm.n_cells} regions, "
          f"cap {prm.tree_cap}; {a.warmup} + {a.steps} queries of {a.iters} iterations", file=sys.stderr,
          flush=True)
    timing = not a.no_timing
    R = run_queries(K, W, a, a.polish, timing)
    value = float(np.median(R["rates"]))
    traffic = measured_traffic(a)
    roof = roofline_of(R["flops"], R["ksum"]["propagate"], R["klaunch"]["propagate"],
                       traffic.get("propagate") if traffic and not a.cost_first else None) if timing else None
    trace = measured_trace(a)
    kern = kernels_summary(R["ksum"], R["klaunch"], R["kbytes"], traffic, trace) if timing else None
    steady = steady_state(K, W, a, a.polish) if timing and a.steady_window > 0 else None
    print(f"[bench] {a.steps} queries: median {value:.4g} edges/s; whole job {R['edges']} edges in "
          f"{R['wall'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    growth = tree_growth(K, W, a) if a.tree_growth > 0 else None
    plain = None
    if a.polish or a.refine_at:
        class _A:  # the same queries with the plain planner
            pass
        b = _A()
        b.__dict__.update(vars(a))
        b.refine_at = 0
        plain = run_queries(K, W, b, 0, False)["solutions"]
    cpu = None if a.no_cpu_baseline else cpu_baseline(w0, a)

    out = {
        "metric": "propagated edges/s", "value": round(value, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(float(np.median(R["spans"])) * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {prob.dynamics} {prob.n_boxes} boxes, "
                   + (f"{prm.n_select}x{prm.samples_per_node} expansions/iteration, "
                      if prm.samples_per_node else
                      f"every active node sharing {prm.n_select} expansion slots per iteration, ")
                   + f"{prm.n_cells} regions, cap {prm.tree_cap}"
                   + (f", edge polish {a.polish} steps per inserted node" if a.polish else "")
                   + (f" (path-length weight {a.polish_w_len})" if a.polish and prob.cost == "PATH_LENGTH" else "")
                   + (" of the nodes inserted in the goal set" if a.polish and a.polish_goal_only else "")
                   + (", cost-first propagate" if a.cost_first else "")
                   + (f", regions refined after {a.refine_at} iterations" if a.refine_at else ""),
                   "step": f"one query: {a.iters} iterations from the root (seed = query index)",
                   "value": "median over queries of edges / device-timed span of the query",
                   "iterations_timed": R["iterations"], "edges_timed": R["edges"],
                   "queries_full": R["full"], "cost": prob.cost},
        "whole_job_edges_per_s": round(R["edges"] / R["wall"], 1) if R["wall"] > 0 else None,
        "whole_job_ms_per_iteration": round(R["wall"] * 1e3 / max(R["iterations"], 1), 5),
        "roofline": roof,
        "kernels": kern,
        "timing_every": a.timing_every if timing else None,
        "steady_state": steady,
        "solutions": R["solutions"],
        "solutions_plain": plain,
        "cpu_baseline": cpu,
    }
    if growth is not None:
        out["tree_growth"] = growth
    print(json.dumps(out))


def tree_growth(K, W, a, window=50):
    """Per-kernel HIP-event times over windows of `window` iterations at
    geometrically spaced points of a run of a.tree_growth iterations, with the
    tree size and live regions at each window: prune works per region and per
    slot, so its time should follow the region count, not the tree."""
    w = make_workload(W, a, 0)
    p = K.Planner(w.problem, w.params)
    if a.cost_first:
        p.set_cost_first(True)
    out, done, start = [], 0, window
    while done < a.tree_growth:
        p.iterate(max(0, start - done))
        done = start
        c0 = p.counters()
        if c0["full"]:
            break
        p.set_timing(True)
        p.iterate(window)
        ms, launches = p.read_timing()
        p.set_timing(False)
        c1 = p.counters()
        st = p.stats(int(c0["iteration"]), int(c1["iteration"] - c0["iteration"]))
        out.append({"iteration": int(c0["iteration"]), "n_tree": int(c1["n_tree"]),
                    "live_regions": int(st["n_live"][-1] + st["n_survivors"][-1]) if st.size else 0,
                    "survivors_per_iteration": float(st["n_survivors"].mean()) if st.size else 0.0,
                    "us": {n: round(ms[i] / launches[i] * 1e3, 2) for i, n in enumerate(KERNELS) if launches[i]}})
        done += window
        start = max(done, 2 * start)
        print(f"[bench] tree growth: iteration {done}, n_tree {c1['n_tree']}", file=sys.stderr, flush=True)
    p.close()
    return {"window_iterations": window, "capacity": int(w.params.tree_cap), "windows": out}


BATCH_BUDGETS_MS = (2.0, 5.0, 10.0, 20.0, 50.0, 100.0)


def query_trace(p, iters):
    """Per-iteration (t_end tick, solution key) of a planner's run and its
    first iteration's start tick, from the device statistics ring."""
    c = p.counters()
    done = min(int(c["iteration"]), iters)
    st = p.stats(0, done)
    return st, (int(st["t_begin"][0]) if done else None)


def cost_at_budgets(st, t0, rate_hz, offset_ms, w, budgets):
    """Cost of the best plan whose iteration ended within each budget (ms)
    after the job's start, for a query that started offset_ms after it."""
    if st.size == 0:
        return [np.inf] * len(budgets)
    t_ms = offset_ms + (st["t_end"].astype(np.float64) - float(t0)) / rate_hz * 1e3
    out = []
    for b in budgets:
        keys = st["solution_key"][t_ms <= b]
        best = int(keys.min()) if keys.size else (1 << 64) - 1
        out.append(np.inf if best == (1 << 64) - 1 else key_cost(best, w.problem.cost, w.params.dt))
    return out


def budget_summary(costs, budgets):
    """Per budget: the median cost over all queries (an unsolved one counts
    as infinite), over the solved ones, and how many are solved."""
    c = np.asarray(costs, np.float64)  # queries x budgets; unsolved = inf
    out = {}
    for i, b in enumerate(budgets):
        col = c[:, i]
        fin = col[np.isfinite(col)]
        med = float(np.median(col))
        out[f"{b:g}ms"] = {"cost_median": round(med, 4) if np.isfinite(med) else None,
                           "cost_median_solved": round(float(np.median(fin)), 4) if fin.size else None,
                           "solved": int(fin.size)}
    return out


def bench_batch(a):
    """Independent queries (half double integrators, half quadrotors, seeded
    scenes of 4..256 boxes, capacities 2^10..2^18) iterated as one batch of
    graph-replayed launches, against the same queries run one after another:
    queries per second, and each query's plan cost at budgets of device time
    counted from the start of the job (every batched query starts at once;
    the sequential query q starts when queries 0..q-1 have finished)."""
    import torch

    import paper_2602_02846_amd as K
    import workloads as W
    from paper_2602_02846_amd.autotune import autotune, first_solution_ms, with_samples

    K.lib()
    torch.cuda.set_device(0)
    ws = W.batch_workloads(a.seed, a.queries)
    chosen, scores = autotune(ws)
    ws = [with_samples(w, chosen[w.problem.dynamics][0]) for w in ws]
    print(f"[bench] batch of {len(ws)} queries; samples per node and propagate threads {chosen} "
          f"(autotuner medians, ms: {scores})", file=sys.stderr, flush=True)
    n_iter = a.iters

    # warmup: a short batched run of the same queries on planners of their own
    if a.warmup > 0:
        wp = [K.Planner(w.problem, w.params) for w in ws]
        wb = K.Batch(wp, graph=True)
        for model, (_, nt) in chosen.items():
            wb.set_threads(model, nt)
        wb.iterate(2 * a.warmup)
        wb.sync()
        wb.close()
        for p in wp:
            p.close()

    planners = [K.Planner(w.problem, w.params) for w in ws]
    batch = K.Batch(planners, graph=True)
    for model, (_, nt) in chosen.items():
        batch.set_threads(model, nt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.iterate(n_iter)
    batch.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rate_hz = planners[0].clock_rate_khz() * 1e3
    traces = [query_trace(p, n_iter) for p in planners]
    starts = [t for _, t in traces if t is not None]
    job0 = min(starts)
    span = (max(int(st["t_end"][-1]) for st, _ in traces if st.size) - job0) / rate_hz
    edges = substeps = 0
    flops = 0.0
    batch_costs = []
    for (st, _), w in zip(traces, ws):
        edges += int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
        sub = int(st["substeps"].sum())
        substeps += sub
        flops += FLOPS_PER_SUBSTEP[(w.problem.dynamics, w.problem.cost)] * sub
        batch_costs.append(cost_at_budgets(st, job0, rate_hz, 0.0, w, BATCH_BUDGETS_MS))
    t_first = [first_solution_ms(p, n_iter) for p in planners]
    solved = [t for t in t_first if t is not None]
    costs = [p.solution()["cost"] for p in planners if p.counters()["first_solution_iteration"] >= 0]
    batch.close()
    for p in planners:
        p.close()
    print(f"[bench] batch: {n_iter} iterations of {len(ws)} queries in {span * 1e3:.1f} ms of device time, "
          f"{edges} edges", file=sys.stderr, flush=True)

    seq = None
    if not a.no_sequential:
        seq_costs, offset_ms, seq_span, seq_wall, seq_edges = [], 0.0, 0.0, 0.0, 0
        seq_first = []
        for w in ws:
            p = K.Planner(w.problem, w.params)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            p.iterate(n_iter)
            p.sync()
            torch.cuda.synchronize()
            seq_wall += time.perf_counter() - s0
            st, q0 = query_trace(p, n_iter)
            qspan = (int(st["t_end"][-1]) - q0) / rate_hz if st.size else 0.0
            seq_costs.append(cost_at_budgets(st, q0, rate_hz, offset_ms, w, BATCH_BUDGETS_MS))
            seq_edges += int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
            tf = first_solution_ms(p, n_iter)
            if tf is not None:
                seq_first.append(tf)
            offset_ms += qspan * 1e3
            seq_span += qspan
            p.close()
        seq = {"device_span_s": round(seq_span, 4), "host_wall_s": round(seq_wall, 4),
               "queries_per_s": round(len(ws) / seq_span, 2), "edges_per_s": round(seq_edges / seq_span, 1),
               "solved": len(seq_first),
               "time_to_first_solution_ms_median": round(float(np.median(seq_first)), 3) if seq_first else None,
               "cost_at_budget_from_job_start": budget_summary(seq_costs, BATCH_BUDGETS_MS)}

    achieved = flops / span / 1e12 if span > 0 else 0.0
    out = {
        "metric": "propagated edges/s", "value": round(edges / span, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": n_iter, "warmup": a.warmup,
        "ms_per_step": round(span * 1e3 / max(n_iter, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}: {len(ws) // 2} DI6 + {len(ws) - len(ws) // 2} QUAD12 "
                               "queries, 4..256 boxes, caps 2^10..2^18, graph-replayed batch",
                   "step": "one batched iteration of every query", "seed": a.seed,
                   "samples_per_node": {m: kt[0] for m, kt in chosen.items()},
                   "propagate_threads": {m: kt[1] for m, kt in chosen.items()},
                   "autotune_ms": {m: {f"K{k}/{nt}": round(v, 3) for (k, nt), v in sc.items()}
                                   for m, sc in scores.items()},
                   "edges_timed": edges, "substeps_timed": substeps},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "scope": "RK4 FLOPs over the whole batched run (all kernels)"},
        "queries_per_s": round(len(ws) / span, 2),
        "batch_device_span_s": round(span, 4), "batch_host_wall_s": round(wall, 4),
        "sequential": seq,
        "speedup_vs_sequential": round(seq["device_span_s"] / span, 2) if seq else None,
        "solved": len(solved), "queries": len(ws),
        "time_to_first_solution_ms_median": round(float(np.median(solved)), 3) if solved else None,
        "solution_cost_median": round(float(np.median(costs)), 4) if costs else None,
        "cost_at_budget_from_job_start": budget_summary(batch_costs, BATCH_BUDGETS_MS),
        "cost_unit": "s (time)",
    }
    print(json.dumps(out))


# Algorithmic float32 FLOPs of the differentiable rollout (same counting as
# above), per RK4 step of one edge:
#   forward:  the RK4 step (324), the nearest-box scan (19 per box: 6 for q,
#             2 max for max q, 3 max and 3 FMA for the key, 1 min, 1 compare)
#             and the penalty at the new state (26: the box's signed distance
#             with its square root, softplus with one exp and one log);
#   adjoint:  the three stage states (3 evaluations of f, 126, and 36 FMA),
#             four vector-Jacobian products of f (120 each: 6 sin/cos, 1 rcp
#             and about 56 mul/FMA), the stage-adjoint combinations (144) and
#             the penalty gradient (30), 852 in all; plus one RK4 step of
#             recomputation for every step that does not start at a checkpoint.
DIFF_RK4, DIFF_SCAN_PER_BOX, DIFF_PENALTY, DIFF_ADJOINT = 324, 19, 26, 852
DIFF_CKPT = 8


def diff_flops(n, n_boxes, grad):
    n = np.asarray(n, np.int64)
    fwd = n * (DIFF_RK4 + DIFF_SCAN_PER_BOX * n_boxes + DIFF_PENALTY)
    if not grad:
        return float(fwd.sum())
    recompute = n - (n + DIFF_CKPT - 1) // DIFF_CKPT
    return float((fwd + n * DIFF_ADJOINT + recompute * DIFF_RK4).sum())


def diff_traffic():
    """HBM bytes per loss-and-gradient launch from the committed counter
    summary, or None when absent or taken on other kernel sources."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "diff_quad12_65536_traffic.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("paper_2602_02846_amd/csrc/kpx_diff.hip", "paper_2602_02846_amd/csrc/kpx_diff_device.hpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()
    fields = {}
    with open(path) as fh:
        for line in fh:
            k, sep, v = line.partition(":")
            if sep:
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != digest:
        return None
    try:
        return int(fields["diff_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_diff(a):
    """Loss and control gradient of 65,536 quadrotor edges (20..40 RK4 steps,
    4 control segments, 64-box wall scene) per step, then 3 projected-gradient
    polish steps on the same edges; HIP events on the launching stream."""
    import torch

    import paper_2602_02846_amd as K
    import workloads as W
    from paper_2602_02846_amd.diff import Rollout

    K.lib()
    torch.cuda.set_device(0)
    b = W.diff_workload(a.seed, n_edges=65536)
    E = b.n.size
    R = Rollout(b.problem, b.dt)
    x0 = torch.from_numpy(np.ascontiguousarray(b.x0.T)).cuda()
    u = torch.from_numpy(np.ascontiguousarray(b.u.T)).cuda()
    n = torch.from_numpy(np.ascontiguousarray(b.n)).cuda()
    loss = torch.empty(E, dtype=torch.float32, device="cuda")
    grad = torch.empty((16, E), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, k):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(k):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev0.elapsed_time(ev1) / 1e3 / max(k, 1)

    step = lambda: R.loss_grad_into(x0, u, n, loss, grad)  # noqa: E731
    for _ in range(a.warmup):
        step()
    elapsed, kern_s = timed(step, a.steps)
    loss_only = lambda: R.loss_grad_into(x0, u, n, loss, None)  # noqa: E731
    loss_only()
    _, kern_loss_s = timed(loss_only, max(1, a.steps // 2))
    _, bad0 = R.polish(x0, u.clone(), n, steps=0, validity=True)
    up = u.clone()
    res = {}
    _, polish_s = timed(lambda: res.setdefault("r", R.polish(x0, up, n, steps=3, lr=0.01, loss=loss,
                                                             validity=True)), 1)
    valid_before, valid_after = int((bad0 == 0).sum()), int((res["r"][1] == 0).sum())

    nb = int(np.asarray(b.problem.boxes).reshape(-1, 6).shape[0])
    fl = diff_flops(b.n, nb, grad=True)
    achieved = fl / kern_s / 1e12
    value = E * a.steps / elapsed if elapsed > 0 else 0.0

    cpu = None
    if not a.no_cpu_baseline:
        from oracle import oracle as O

        D = O.DiffProblem(b.problem, b.dt)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < a.cpu_seconds and done < E:
            O.diff_loss(D, b.x0[done], b.u[done], int(b.n[done]))
            O.diff_grad(D, b.x0[done], b.u[done], int(b.n[done]))
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 1) if el > 0 else None, "unit": "edges/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the first {done} edges of the same batch, loss and complex-step gradient "
                         f"(16 complex rollouts per edge), float64, one thread, {el:.1f} s"}
    R.close()
    out = {
        "metric": "edge loss+gradient evaluations/s", "value": round(value, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / max(a.steps, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"diff65536: {E} quadrotor edges, {int(b.n.min())}..{int(b.n.max())} RK4 steps "
                               f"of dt {b.dt}, 4 control segments, {nb} boxes; loss and gradient per step",
                   "seed": a.seed, "edges_per_step": E, "rk4_steps_per_step": int(b.n.sum())},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": diff_traffic(), "flops_per_launch": fl},
        "kernel_ms": {"loss_grad": round(kern_s * 1e3, 4), "loss": round(kern_loss_s * 1e3, 4),
                      "polish3": round(polish_s * 1e3, 4)},
        "polish": {"steps": 3, "lr": 0.01, "valid_edges_before": valid_before,
                   "valid_edges_after": valid_after},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))




def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(w, a):
    """The float64 oracle running the first query (seed 0) from its root, as
    the GPU does: on every host core (the OpenMP build of the same source,
    expansions shared among threads), then on one, each for a bounded sample
    of its iterations."""
    from oracle import oracle as O

    def sample(threaded, seconds):
        P = O.Problem(w.problem, w.params)
        tr = O.Tree(P)
        assert tr.init() == O.OK
        edges = iters = 0
        t0 = time.perf_counter()
        while iters < a.iters and time.perf_counter() - t0 < seconds:
            if tr.step(threaded=threaded) != O.OK:
                break
            edges += tr.cands.n_slots
            iters += 1
        return edges, iters, time.perf_counter() - t0

    threads = int(O.lib_threads().ora_threads())
    e_all, i_all, t_all = sample(True, a.cpu_seconds)
    e_one, i_one, t_one = sample(False, a.cpu_seconds_single)
    host = host_cpu()
    return {"value": round(e_all / t_all, 1) if t_all > 0 else None, "unit": "edges/s", "cores": threads,
            "kind": "oracle",
            "sample": f"iterations 0..{i_all - 1} of query 0 from its root ({e_all} expansions, "
                      f"{t_all:.1f} s, float64, {threads} threads)",
            "single_thread": {"value": round(e_one / t_one, 1) if t_one > 0 else None,
                              "sample": f"iterations 0..{i_one - 1} of query 0 ({e_one} expansions, "
                                        f"{t_one:.1f} s, one thread)"},
            **host}


if __name__ == "__main__":
    main()
