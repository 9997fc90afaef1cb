"""Benchmark: propagated edges/s of the Kino-PAX+ iteration on one MI355X.

A step is one planner iteration (select -> propagate -> prune -> insert) of one
query on the 12D quadrotor workload (4096 nodes x 32 samples per iteration,
64-box wall with two slots, 16^3 x 2^3 regions, tree capacity 2^21).  Inputs
live in HBM before timing starts; every count stays on the device.

Prints one JSON line.  `roofline` covers the dominant kernel (propagate, bound
by float32 ALU work); `cpu_baseline` is the float64 oracle replaying the same
workload on the host from the GPU tree at the start of the timed region.
"""

from __future__ import annotations

import argparse
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
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2602_02846_amd/csrc/kpx.hip", "paper_2602_02846_amd/csrc/kpx_device.hpp")


def measured_traffic(workload):
    """HBM bytes per propagate launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy), or
    None when there is none or the kernel sources changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"propagate_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    with open(path) as fh:
        for line in fh:
            k, sep, v = line.partition(":")
            if sep:
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    try:
        return int(fields["propagate_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="quad12",
                    choices=["di6", "quad12", "dubins6", "di6_paper", "quad12_paper", "dubins6_paper",
                             "di6_paper_small", "quad12_paper_small", "dubins6_paper_small",
                             "batch256", "diff65536"])
    ap.add_argument("--queries", type=int, default=256, help="queries of the batch256 workload")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch256: skip the sequential per-query comparison")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="bound on the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solution-seeds", type=int, default=100,
                    help="queries (seeds) for the median time to first solution and cost")
    ap.add_argument("--solution-iters", type=int, default=200,
                    help="iteration budget of each of those queries")
    ap.add_argument("--polish", type=int, default=0,
                    help="edge polish steps of every inserted node (quadrotor, TIME cost); 0 = plain")
    ap.add_argument("--cost-first", action="store_true",
                    help="propagate in the exact cost-first form (obstacle tests only for edges "
                         "that can still be their region's minimum)")
    ap.add_argument("--tree-growth", type=int, default=0,
                    help="also run the workload this many iterations and time every kernel in "
                         "windows as the tree grows (prune and insert against tree size)")
    ap.add_argument("--refine-at", type=int, default=0,
                    help="solution runs: halve the region cells per axis after this many iterations")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--timing-every", type=int, default=8,
                    help="bracket the kernels with HIP events in every n-th timed iteration")
    ap.add_argument("--time-all", action="store_true",
                    help="HIP events around all four kernels (default: propagate only)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported "
              "(the planner query runs on a single device)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2602_02846_amd as K
    import workloads as W

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
    w = W.make_workload(a.workload, a.seed)
    prob, prm = w.problem, w.params

    planner = K.Planner(prob, prm, device="cuda:0")
    if a.polish:
        planner.set_polish(a.polish)
    if a.cost_first:
        planner.set_cost_first(True)
    print(f"[bench] {a.workload}: {prm.n_select} x {prm.samples_per_node} slots, "
          f"{prm.n_cells} regions, cap {prm.tree_cap}; warmup {a.warmup}", file=sys.stderr,
          flush=True)
    planner.iterate(a.warmup)
    planner.sync()
    snap_start = planner.snapshot() if not a.no_cpu_baseline else None
    c0 = planner.counters()
    if not a.no_timing:
        # HIP events around propagate (the roofline kernel), or all four
        # kernels, in every timing_every-th iteration of the timed region
        planner.set_timing(15 if a.time_all else 1, every=a.timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    planner.iterate(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc = planner.sync()
    c1 = planner.counters()
    done = int(c1["iteration"] - c0["iteration"])
    st = planner.stats(int(c0["iteration"]), done) if done > 0 else None
    edges = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum()) if done else 0
    substeps = int(st["substeps"].sum()) if done else 0
    elapsed = t1 - t0
    value = edges / elapsed if elapsed > 0 else 0.0
    print(f"[bench] timed {done} iterations in {elapsed * 1e3:.2f} ms, {edges} edges, "
          f"status {rc}", file=sys.stderr, flush=True)

    roofline = None
    kernel_ms = None
    if not a.no_timing:
        ms, launches = planner.read_timing()
        kernel_ms = {name: (ms[i] / launches[i] if launches[i] else None)
                     for i, name in enumerate(["propagate", "prune_flags", "insert",
                                               "finalize_select"]) if launches[i]}
        if launches[0] and done:
            # the FLOPs of the launches the events bracketed (every
            # timing_every-th timed iteration, from the first), over their time
            sampled = st["substeps"][:: max(1, a.timing_every)][: launches[0]]
            fl = FLOPS_PER_SUBSTEP[(prob.dynamics, prob.cost)] * float(sampled.sum()) / launches[0]
            avg_s = ms[0] / launches[0] / 1e3
            achieved = fl / avg_s / 1e12
            roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                        # the counters were taken on the plain form's kernel
                        "traffic": None if a.cost_first else measured_traffic(a.workload)}

    # time to first solution and cost, from device timestamps of this query
    it_done = int(c1["iteration"])
    all_st = planner.stats(max(0, it_done - 65536), min(it_done, 65536))
    rate = planner.clock_rate_khz() * 1e3
    first_it = int(c1["first_solution_iteration"])
    sol = planner.solution()
    t_first = None
    if first_it >= 0 and all_st.size and all_st["iteration"][0] == 0:
        t_first = float((int(all_st["t_end"][first_it]) - int(all_st["t_begin"][0])) / rate * 1e3)

    planner.close()
    sols = solution_medians(K, W, a, a.polish, a.refine_at) if a.solution_seeds > 0 else None
    growth = tree_growth(K, W, a) if a.tree_growth > 0 else None
    sols_plain = (solution_medians(K, W, a, 0) if a.solution_seeds > 0 and (a.polish or a.refine_at)
                  else None)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(w, snap_start, a.cpu_seconds)

    out = {
        "metric": "propagated edges/s", "value": round(value, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / max(done, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {prob.dynamics} {prob.n_boxes} boxes, "
                   + (f"{prm.n_select}x{prm.samples_per_node} expansions/iteration, "
                      if prm.samples_per_node else
                      f"every active node sharing {prm.n_select} expansion slots per iteration, ")
                   + f"{prm.n_cells} regions, cap {prm.tree_cap}"
                   + (f", edge polish {a.polish} steps per inserted node" if a.polish else "")
                   + (", cost-first propagate" if a.cost_first else ""),
                   "seed": a.seed, "iterations_timed": done, "edges_timed": edges,
                   "substeps_timed": substeps, "cost": prob.cost},
        "roofline": roofline,
        "kernel_ms": kernel_ms,
        "time_to_first_solution_ms": t_first,
        "first_solution_iteration": first_it,
        "solution_cost": sol["cost"] if sol["found"] else None,
        "solutions": sols,
        "solutions_plain": sols_plain,
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
    w = W.make_workload(a.workload, a.seed)
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
        snap = p.snapshot()
        live = int((snap["cell_table"] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())
        st = p.stats(int(c0["iteration"]), int(c1["iteration"] - c0["iteration"]))
        out.append({"iteration": int(c0["iteration"]), "n_tree": int(c1["n_tree"]),
                    "live_regions": live, "survivors_per_iteration": float(st["n_survivors"].mean()) if st.size else 0.0,
                    "us": {n: round(ms[i] / launches[i] * 1e3, 2) for i, n in enumerate(
                        ["propagate", "prune_flags", "insert", "finalize_select"]) if launches[i]}})
        done += window
        start = max(done, 2 * start)
        print(f"[bench] tree growth: iteration {done}, n_tree {c1['n_tree']}", file=sys.stderr, flush=True)
    p.close()
    return {"window_iterations": window, "capacity": int(w.params.tree_cap), "windows": out}


BUDGETS_MS = (5.0, 10.0, 20.0, 40.0)


def key_cost(key, cost_kind, dt):
    """Cost of a solution key: the high word is the total RK4 step count
    (TIME cost, times dt) or the float32 bits of the path length."""
    field = int(key) >> 32
    if cost_kind == "TIME":
        return field * dt
    return float(np.array([field], np.uint32).view(np.float32)[0])


def solution_medians(K, W, a, polish=0, refine_at=0):
    """Median device-timed time to first solution and median solution cost
    over seeds 0 .. solution_seeds - 1 of the workload, each run for
    solution_iters iterations (or until its tree is full), with edge polish
    of `polish` steps (0: the plain planner).  Also the cost of the best plan
    known at fixed device-time budgets (median over all seeds, an unsolved
    seed counting as infinite) and the number of seeds solved by then.  With
    refine_at > 0 the region grid is halved per axis after that many
    iterations (adaptive decomposition)."""
    from paper_2602_02846_amd.autotune import first_solution_ms

    times, costs, refine_ms = [], [], []
    at_budget = {b: [] for b in BUDGETS_MS}
    dt = None
    for seed in range(a.solution_seeds):
        w = W.make_workload(a.workload, seed)
        dt = w.params.dt
        if refine_at:
            w.params.refine_max = 2
        p = K.Planner(w.problem, w.params)
        if polish:
            p.set_polish(polish)
        if a.cost_first:
            p.set_cost_first(True)
        if 0 < refine_at < a.solution_iters:
            import torch

            p.iterate(refine_at)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            p.refine(2)
            e1.record()
            p.iterate(a.solution_iters - refine_at)
            torch.cuda.synchronize()
            refine_ms.append(e0.elapsed_time(e1))
        else:
            p.iterate(a.solution_iters)
        p.sync()
        t = first_solution_ms(p, a.solution_iters)
        if t is not None:
            times.append(t)
            costs.append(p.solution()["cost"])
        c = p.counters()
        st = p.stats(0, min(int(c["iteration"]), 65536))
        rate = p.clock_rate_khz() * 1e3
        t_ms = (st["t_end"].astype(np.float64) - float(st["t_begin"][0])) / rate * 1e3 if st.size else np.zeros(0)
        for b in BUDGETS_MS:
            keys = st["solution_key"][t_ms <= b]
            best = int(keys.min()) if keys.size else (1 << 64) - 1
            at_budget[b].append(np.inf if best == (1 << 64) - 1 else key_cost(best, w.problem.cost, dt))
        p.close()
    return {"queries": a.solution_seeds, "iterations": a.solution_iters, "polish_steps": polish,
            "refine_at": refine_at,
            "refine_ms_median": round(float(np.median(refine_ms)), 4) if refine_ms else None,
            "solved": len(times),
            "time_to_first_solution_ms_median": round(float(np.median(times)), 3) if times else None,
            "cost_median": round(float(np.median(costs)), 4) if costs else None,
            "cost_at_budget_median": {f"{b:g}ms": (None if not np.isfinite(np.median(v)) else
                                                   round(float(np.median(v)), 4))
                                      for b, v in at_budget.items()},
            "solved_at_budget": {f"{b:g}ms": int(np.isfinite(v).sum()) for b, v in at_budget.items()},
            "cost_unit": "s" if W.make_workload(a.workload, 0).problem.cost == "TIME" else "length"}


def bench_batch(a):
    """Independent queries (half double integrators, half quadrotors, seeded
    scenes of 4..256 boxes, capacities 2^10..2^18) iterated as one batch of
    graph-replayed launches, against the same queries run one after another."""
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
    n_iter = a.warmup + a.steps

    planners = [K.Planner(w.problem, w.params) for w in ws]
    batch = K.Batch(planners, graph=True)
    for model, (_, nt) in chosen.items():
        batch.set_threads(model, nt)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    batch.iterate(a.warmup)
    batch.sync()
    c0 = [p.counters() for p in planners]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.iterate(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    batch.sync()
    elapsed, whole = t1 - t0, t1 - tb0
    edges = substeps = 0
    flops = 0.0
    for p, w, c in zip(planners, ws, c0):
        c1 = p.counters()
        done = int(c1["iteration"] - c["iteration"])
        if done > 0:
            st = p.stats(int(c["iteration"]), done)
            e = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
            sub = int(st["substeps"].sum())
            edges += e
            substeps += sub
            flops += FLOPS_PER_SUBSTEP[(w.problem.dynamics, w.problem.cost)] * sub
    t_first = [first_solution_ms(p, n_iter) for p in planners]
    solved = [t for t in t_first if t is not None]
    costs = [p.solution()["cost"] for p in planners if p.counters()["first_solution_iteration"] >= 0]
    batch.close()
    for p in planners:
        p.close()
    print(f"[bench] batch: {a.steps} iterations in {elapsed * 1e3:.1f} ms, {edges} edges", file=sys.stderr,
          flush=True)

    seq = None
    if not a.no_sequential:
        t_seq, seq_edges_timed = 0.0, 0
        for w in ws:
            p = K.Planner(w.problem, w.params)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            p.iterate(n_iter)
            p.sync()
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - s0
            p.close()
        seq = {"whole_run_s": round(t_seq, 4), "queries_per_s": round(len(ws) / t_seq, 2)}

    achieved = flops / elapsed / 1e12 if elapsed > 0 else 0.0
    out = {
        "metric": "propagated edges/s", "value": round(edges / elapsed, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / max(a.steps, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}: {len(ws) // 2} DI6 + {len(ws) - len(ws) // 2} QUAD12 "
                               "queries, 4..256 boxes, caps 2^10..2^18, graph-replayed batch",
                   "seed": a.seed, "samples_per_node": {m: kt[0] for m, kt in chosen.items()},
                   "propagate_threads": {m: kt[1] for m, kt in chosen.items()},
                   "autotune_ms": {m: {f"K{k}/{nt}": round(v, 3) for (k, nt), v in sc.items()}
                                   for m, sc in scores.items()},
                   "edges_timed": edges,
                   "substeps_timed": substeps},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "scope": "RK4 FLOPs over whole iterations (all kernels)"},
        "queries_per_s": round(len(ws) / whole, 2),
        "batch_whole_run_s": round(whole, 4),
        "sequential": seq,
        "speedup_vs_sequential": round(seq["whole_run_s"] / whole, 2) if seq else None,
        "solved": len(solved), "queries": len(ws),
        "time_to_first_solution_ms_median": round(float(np.median(solved)), 3) if solved else None,
        "solution_cost_median": round(float(np.median(costs)), 4) if costs else None,
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


def cpu_baseline(w, snap, seconds):
    """The float64 oracle (single thread, as written) stepping the same tree."""
    from oracle import oracle as O
    from oracle import parity

    P = O.Problem(w.problem, w.params)
    tr = parity.oracle_tree_from_snapshot(O, P, snap)
    edges = 0
    iters = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        rc = tr.step()
        if rc != O.OK:
            break
        edges += tr.cands.n_slots
        iters += 1
    el = time.perf_counter() - t0
    return {"value": round(edges / el, 1) if el > 0 else None, "unit": "edges/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} iterations of the same query from the GPU tree at the start of "
                      f"the timed region ({edges} expansions, {el:.1f} s, float64, one thread)"}


if __name__ == "__main__":
    main()
